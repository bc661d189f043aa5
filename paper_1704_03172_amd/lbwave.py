"""ctypes binding of liblbwave.so (C-ABI in include/lbwave.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch supplies device memory (the workspace, trace and field
buffers) and the stream.  There is no CPU fallback: if the library is not
built, importing the binding's entry points raises.
"""
import collections
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbwave.so")

LB_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "value out of range",
          -3: "unsupported combination", -4: "workspace", -5: "HIP runtime error",
          -6: "call out of order"}
F32, F64, F16S = 0, 1, 2
PRECISION = {"f32": F32, "f64": F64, "f16s": F16S}
FIELD = {"p": 1, "rho": 2, "jx": 4, "jy": 8}
FIELD_ORDER = ("p", "rho", "jx", "jy")
COLLISION = {"bgk": 0, "mrt": 1}

# every symbol the header declares (the ABI test checks the export table)
EXPORTS = ("lb_default_desc", "lb_validate_desc", "lb_blocked_steps", "lb_workspace_bytes",
           "lb_create_grid", "lb_destroy_grid", "lb_set_medium",
           "lb_set_medium_fine", "lb_set_state", "lb_set_state_fine",
           "lb_set_source", "lb_record", "lb_record_sum_rho", "lb_step_n", "lb_set_graph",
           "lb_get_time", "lb_get_field", "lb_get_field_fine",
           "lb_state_bytes", "lb_get_state", "lb_set_raw_state", "lb_sync",
           "lb_status_string", "lb_device_copy",
           "lb_batch_workspace_bytes", "lb_batch_create", "lb_shot_workspace_bytes",
           "lb_batch_add_shot", "lb_batch_remove_shot", "lb_batch_tick", "lb_batch_times", "lb_batch_completed",
           "lb_batch_sync", "lb_batch_destroy", "lb_misfit", "lb_adjoint", "lb_trace_misfit",
           "lb_trace_misfit_static")

TRACE_MISFIT_WORKSPACE_BYTES = 16384   # LB_TRACE_MISFIT_WORKSPACE_BYTES


class LBError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(code, "?"), code))
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("lattice", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("nbatch", ctypes.c_int32),
        ("tau", ctypes.c_double), ("s", ctypes.c_double * 9),
        ("d2q9_ratio", ctypes.c_double),
        ("sponge_width", ctypes.c_int32), ("_pad0", ctypes.c_int32),
        ("sponge_sigma_max", ctypes.c_double),
        ("patch_enable", ctypes.c_int32),
        ("patch_x0", ctypes.c_int32), ("patch_y0", ctypes.c_int32),
        ("patch_nx", ctypes.c_int32), ("patch_ny", ctypes.c_int32),
        ("patch_refine", ctypes.c_int32),
        ("patch_overlap_out", ctypes.c_int32), ("patch_overlap_in", ctypes.c_int32),
        ("trace_capacity", ctypes.c_int64),
        ("max_receivers", ctypes.c_int32),
        ("ckpt_every", ctypes.c_int32), ("ckpt_capacity", ctypes.c_int32),
        ("steps_per_launch", ctypes.c_int32),
        ("rho_tape", ctypes.c_int32), ("_pad1", ctypes.c_int32),
    ]


class ShotDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("src_x", ctypes.c_int32), ("src_y", ctypes.c_int32),
        ("nsteps", ctypes.c_int64),
        ("sponge_width", ctypes.c_int32), ("nrec", ctypes.c_int32),
        ("sponge_sigma_max", ctypes.c_double),
    ]


_LIB = None


def lib():
    """Load liblbwave.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbwave.so is not built (%s); run "
                           "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    PD = ctypes.POINTER(Desc)
    sig = {
        "lb_default_desc": (None, [PD]),
        "lb_validate_desc": (ctypes.c_int, [PD]),
        "lb_blocked_steps": (ctypes.c_int, [PD, ctypes.POINTER(ctypes.c_int32)]),
        "lb_workspace_bytes": (ctypes.c_size_t, [PD]),
        "lb_create_grid": (ctypes.c_int, [PD, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "lb_destroy_grid": (ctypes.c_int, [vp]),
        "lb_set_medium": (ctypes.c_int, [vp, vp, ctypes.c_int, ctypes.c_int]),
        "lb_set_medium_fine": (ctypes.c_int, [vp, vp, ctypes.c_int, ctypes.c_int]),
        "lb_set_state": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "lb_set_state_fine": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "lb_set_source": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(ctypes.c_double), i64]),
        "lb_record": (ctypes.c_int, [vp, ctypes.POINTER(i32), i32, vp, u32]),
        "lb_record_sum_rho": (ctypes.c_int, [vp, vp]),
        "lb_step_n": (ctypes.c_int, [vp, i64]),
        "lb_set_graph": (ctypes.c_int, [vp, ctypes.c_int32]),
        "lb_get_time": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
        "lb_get_field": (ctypes.c_int, [vp, u32, vp]),
        "lb_get_field_fine": (ctypes.c_int, [vp, u32, vp]),
        "lb_state_bytes": (ctypes.c_size_t, [vp]),
        "lb_get_state": (ctypes.c_int, [vp, vp]),
        "lb_set_raw_state": (ctypes.c_int, [vp, vp]),
        "lb_sync": (ctypes.c_int, [vp]),
        "lb_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "lb_device_copy": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp]),
        "lb_trace_misfit": (ctypes.c_int, [vp, vp, vp, i32, i64, i64, ctypes.c_int, vp, vp, ctypes.c_size_t, vp]),
        "lb_trace_misfit_static": (ctypes.c_int, [vp, vp, vp, i32, i64, i64, ctypes.c_int, vp, vp]),
        "lb_batch_workspace_bytes": (ctypes.c_size_t, [i32]),
        "lb_batch_create": (ctypes.c_int, [PD, i32, vp, ctypes.c_size_t, vp, ctypes.c_int,
                                           ctypes.POINTER(vp)]),
        "lb_shot_workspace_bytes": (ctypes.c_size_t, [vp, ctypes.POINTER(ShotDesc)]),
        "lb_batch_add_shot": (ctypes.c_int, [vp, ctypes.POINTER(ShotDesc), vp, ctypes.c_size_t, vp,
                                             ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                             i64, ctypes.POINTER(i32), vp, ctypes.POINTER(i32)]),
        "lb_batch_remove_shot": (ctypes.c_int, [vp, i32]),
        "lb_batch_tick": (ctypes.c_int, [vp, i64]),
        "lb_batch_times": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
        "lb_batch_completed": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
        "lb_batch_sync": (ctypes.c_int, [vp]),
        "lb_batch_destroy": (ctypes.c_int, [vp]),
        "lb_misfit": (ctypes.c_int, [vp, vp, i64, vp, vp]),
        "lb_adjoint": (ctypes.c_int, [vp, vp, i64, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = L
    return L


def _check(code, what):
    if code != LB_OK:
        raise LBError(code, what)


def make_desc(nx, ny, lattice=5, collision="bgk", precision="f32", tau=0.5,
              s=None, ratio=0.25, sponge_width=0, sponge_sigma_max=0.0,
              patch=None, overlap_out=2, overlap_in=2, trace_capacity=0,
              max_receivers=0, ckpt_every=0, ckpt_capacity=0, steps_per_launch=0, rho_tape=0):
    d = Desc()
    lib().lb_default_desc(ctypes.byref(d))
    d.nx, d.ny = int(nx), int(ny)
    d.lattice = int(lattice)
    d.collision = COLLISION[collision]
    d.precision = PRECISION[precision]
    d.tau = float(tau)
    if s is not None:
        for k, v in enumerate(s):
            d.s[k] = float(v)
    d.d2q9_ratio = float(ratio)
    d.sponge_width = int(sponge_width)
    d.sponge_sigma_max = float(sponge_sigma_max)
    if patch is not None:
        d.patch_enable = 1
        d.patch_x0, d.patch_y0, d.patch_nx, d.patch_ny = (int(v) for v in patch)
        d.patch_overlap_out, d.patch_overlap_in = int(overlap_out), int(overlap_in)
    d.trace_capacity = int(trace_capacity)
    d.max_receivers = int(max_receivers)
    d.ckpt_every = int(ckpt_every)
    d.ckpt_capacity = int(ckpt_capacity)
    d.steps_per_launch = int(steps_per_launch)
    d.rho_tape = int(rho_tape)
    return d


def workspace_bytes(**kw):
    d = make_desc(**kw)
    return int(lib().lb_workspace_bytes(ctypes.byref(d)))


def validate(**kw):
    d = make_desc(**kw)
    return int(lib().lb_validate_desc(ctypes.byref(d)))


def blocked_steps(**kw):
    """Most time steps one launch of lb_step_n takes for this descriptor."""
    d = make_desc(**kw)
    ns = ctypes.c_int32()
    _check(lib().lb_blocked_steps(ctypes.byref(d), ctypes.byref(ns)), "lb_blocked_steps")
    return int(ns.value)


class Grid:
    """One lattice (optionally with a refinement patch) on one HIP stream."""

    def __init__(self, nx, ny, device=None, stream=None, **kw):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.desc = make_desc(nx, ny, **kw)
        self.nx, self.ny = int(nx), int(ny)
        self.lattice = self.desc.lattice
        self.precision = kw.get("precision", "f32")
        self.dtype = torch.float64 if self.precision == "f64" else torch.float32
        self.trace_capacity = int(kw.get("trace_capacity", 0))
        L = lib()
        nbytes = L.lb_workspace_bytes(ctypes.byref(self.desc))
        if nbytes == 0:
            _check(L.lb_validate_desc(ctypes.byref(self.desc)), "lb_validate_desc")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = ctypes.c_void_p()
        _check(L.lb_create_grid(ctypes.byref(self.desc), ctypes.c_void_p(self.workspace.data_ptr()),
                                ctypes.c_size_t(int(nbytes)), ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(h)), "lb_create_grid")
        self._h = h
        self.traces = None
        self.sum_rho = None
        self.fine_shape = None
        if self.desc.patch_enable:
            W = self.desc.patch_nx + 2 * self.desc.patch_overlap_out
            H = self.desc.patch_ny + 2 * self.desc.patch_overlap_out
            self.fine_shape = (2 * H + 1, 2 * W + 1)

    # ---- marshalling helpers ------------------------------------------------
    def _arg(self, a, keep):
        """(pointer, dtype code, on_device) for a numpy array or torch tensor."""
        torch = self._torch
        if a is None:
            return None, F64, 0
        if isinstance(a, torch.Tensor):
            if a.is_cuda:
                if a.dtype not in (torch.float32, torch.float64):
                    raise TypeError("device inputs must be float32 or float64")
                a = a.contiguous()
                keep.append(a)
                return ctypes.c_void_p(a.data_ptr()), (F64 if a.dtype == torch.float64 else F32), 1
            a = a.numpy()
        arr = np.ascontiguousarray(a)
        if arr.dtype not in (np.float32, np.float64):
            arr = arr.astype(np.float64)
        keep.append(arr)
        return ctypes.c_void_p(arr.ctypes.data), (F64 if arr.dtype == np.float64 else F32), 0

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("grid is closed")
        return self._h

    # ---- C-ABI calls ----------------------------------------------------------
    def set_medium(self, c2, fine=False):
        keep = []
        p, t, dev = self._arg(c2, keep)
        fn = lib().lb_set_medium_fine if fine else lib().lb_set_medium
        _check(fn(self.handle, p, t, dev), "lb_set_medium")

    def set_state(self, rho, jx=None, jy=None, fine=False):
        keep = []
        pr, t, dev = self._arg(rho, keep)
        px, tx, _ = self._arg(jx, keep)
        py, ty, _ = self._arg(jy, keep)
        if (jx is not None and tx != t) or (jy is not None and ty != t):
            raise TypeError("rho, jx, jy must share one dtype")
        fn = lib().lb_set_state_fine if fine else lib().lb_set_state
        _check(fn(self.handle, pr, px, py, t, dev), "lb_set_state")

    def set_source(self, x, y, wavelet):
        w = np.ascontiguousarray(wavelet, dtype=np.float64)
        _check(lib().lb_set_source(self.handle, int(x), int(y),
                                   w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(w.size)),
               "lb_set_source")

    def record(self, receivers, fields=("p",)):
        """Register receivers (int array (nrec, 2) of (x, y)); returns the
        device trace tensor [nfields][nrec][trace_capacity]."""
        torch = self._torch
        rec = np.ascontiguousarray(receivers, dtype=np.int32).reshape(-1, 2)
        nrec = rec.shape[0]
        if nrec == 0:
            _check(lib().lb_record(self.handle, None, 0, None, 0), "lb_record")
            self.traces = None
            return None
        what = 0
        for f in fields:
            what |= FIELD[f]
        nf = bin(what).count("1")
        self.traces = torch.zeros((nf, nrec, self.trace_capacity), dtype=self.dtype, device=self.device)
        self.trace_fields = tuple(f for f in FIELD_ORDER if what & FIELD[f])
        _check(lib().lb_record(self.handle, rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), nrec,
                               ctypes.c_void_p(self.traces.data_ptr()), what), "lb_record")
        return self.traces

    def record_sum_rho(self):
        torch = self._torch
        self.sum_rho = torch.zeros(self.trace_capacity, dtype=torch.float64, device=self.device)
        _check(lib().lb_record_sum_rho(self.handle, ctypes.c_void_p(self.sum_rho.data_ptr())),
               "lb_record_sum_rho")
        return self.sum_rho

    def step(self, n=1):
        _check(lib().lb_step_n(self.handle, int(n)), "lb_step_n")

    def set_graph(self, steps):
        """Replay whole chunks of `steps` steps of each step() call from a
        captured HIP graph (0: off)."""
        _check(lib().lb_set_graph(self.handle, int(steps)), "lb_set_graph")

    @property
    def time(self):
        t = ctypes.c_int64()
        _check(lib().lb_get_time(self.handle, ctypes.byref(t)), "lb_get_time")
        return int(t.value)

    def field(self, what="rho", fine=False):
        torch = self._torch
        shape = self.fine_shape if fine else (self.ny, self.nx)
        out = torch.empty(shape, dtype=self.dtype, device=self.device)
        fn = lib().lb_get_field_fine if fine else lib().lb_get_field
        _check(fn(self.handle, FIELD[what], ctypes.c_void_p(out.data_ptr())), "lb_get_field")
        return out

    def get_state(self):
        torch = self._torch
        n = lib().lb_state_bytes(self.handle)
        out = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        _check(lib().lb_get_state(self.handle, ctypes.c_void_p(out.data_ptr())), "lb_get_state")
        return out

    def set_raw_state(self, blob):
        _check(lib().lb_set_raw_state(self.handle, ctypes.c_void_p(blob.data_ptr())), "lb_set_raw_state")

    def _trace_shaped(self, a, name):
        """a as a contiguous device tensor [nrec][trace_capacity] of the
        arithmetic type; ValueError (before any launch) for any other shape,
        since the kernels index it as r * trace_capacity + n."""
        torch = self._torch
        if self.traces is None:
            raise ValueError("%s: no receivers recorded" % name)
        nrec = int(self.traces.shape[1])
        shape = tuple(a.shape)
        if shape not in ((nrec, self.trace_capacity), (1, nrec, self.trace_capacity)):
            raise ValueError("%s must have shape (%d, %d) = (nrec, trace_capacity), got %s"
                             % (name, nrec, self.trace_capacity, shape))
        return torch.as_tensor(a).to(device=self.device, dtype=self.dtype).reshape(
            nrec, self.trace_capacity).contiguous()

    def misfit(self, d_obs, nt):
        """(phi, residual) of the recorded pressure traces against d_obs
        [nrec][trace_capacity] (device tensor of the arithmetic type)."""
        torch = self._torch
        d_obs = self._trace_shaped(d_obs, "d_obs")
        res = torch.zeros_like(d_obs)
        phi = torch.zeros((), dtype=torch.float64, device=self.device)
        _check(lib().lb_misfit(self.handle, ctypes.c_void_p(d_obs.data_ptr()), int(nt),
                               ctypes.c_void_p(res.data_ptr()), ctypes.c_void_p(phi.data_ptr())), "lb_misfit")
        return phi, res

    def adjoint(self, res, nt):
        """dL/dc^2 [ny][nx] (FP64) for trace sensitivities res
        [nrec][trace_capacity] after a forward run of nt steps."""
        torch = self._torch
        res = self._trace_shaped(res, "res")
        grad = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        _check(lib().lb_adjoint(self.handle, ctypes.c_void_p(res.data_ptr()), int(nt),
                                ctypes.c_void_p(grad.data_ptr())), "lb_adjoint")
        return grad

    def sync(self):
        _check(lib().lb_sync(self.handle), "lb_sync")

    def close(self):
        if getattr(self, "_h", None) is not None:
            code = lib().lb_destroy_grid(self._h)
            self._h = None
            _check(code, "lb_destroy_grid")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_copy(dst, src, nbytes, stream=None):
    """The library's plain 16-byte vector copy kernel (bandwidth reference)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    _check(lib().lb_device_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                ctypes.c_size_t(int(nbytes)), ctypes.c_void_p(s.cuda_stream)),
           "lb_device_copy")


def _misfit_args(traces, obs, ncols):
    """Checked (traces, obs, res, phi, nrec, cap, ncols, dtype code) for the
    trace-misfit entry points: traces and obs device tensors of one shape
    [nrec][cap] and one dtype (float32 or float64)."""
    import torch
    if not (isinstance(traces, torch.Tensor) and isinstance(obs, torch.Tensor) and traces.is_cuda and obs.is_cuda):
        raise TypeError("traces and obs must be CUDA tensors")
    if traces.dim() != 2 or tuple(obs.shape) != tuple(traces.shape) or obs.dtype != traces.dtype:
        raise ValueError("traces and obs must be [nrec][cap] tensors of one shape and dtype")
    if traces.dtype not in (torch.float32, torch.float64):
        raise TypeError("traces must be float32 or float64")
    nrec, cap = (int(v) for v in traces.shape)
    ncols = cap if ncols is None else int(ncols)
    traces, obs = traces.contiguous(), obs.contiguous()
    res = torch.zeros_like(traces)
    phi = torch.zeros((), dtype=torch.float64, device=traces.device)
    return traces, obs, res, phi, nrec, cap, ncols, (F64 if traces.dtype == torch.float64 else F32)


def trace_misfit(traces, obs, ncols=None, stream=None):
    """(phi, res) of lb_trace_misfit: res = traces - obs over the first
    ncols columns (default all) and phi = 1/2 sum res^2 (FP64), with a
    workspace tensor for the block partials."""
    import torch
    traces, obs, res, phi, nrec, cap, ncols, t = _misfit_args(traces, obs, ncols)
    s = torch.cuda.current_stream(traces.device) if stream is None else stream
    ws = torch.empty(TRACE_MISFIT_WORKSPACE_BYTES, dtype=torch.uint8, device=traces.device)
    _check(lib().lb_trace_misfit(ctypes.c_void_p(traces.data_ptr()), ctypes.c_void_p(obs.data_ptr()),
                                 ctypes.c_void_p(res.data_ptr()), nrec, cap, ncols, t,
                                 ctypes.c_void_p(phi.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                 ctypes.c_size_t(TRACE_MISFIT_WORKSPACE_BYTES), ctypes.c_void_p(s.cuda_stream)),
           "lb_trace_misfit")
    return phi, res


def trace_misfit_static(traces, obs, ncols=None, stream=None):
    """lb_trace_misfit_static: trace_misfit() with the block partials in the
    library's static device array (no workspace).  Calls whose execution
    overlaps on one GPU race; the output tensors are the caller's, as in
    trace_misfit()."""
    import torch
    traces, obs, res, phi, nrec, cap, ncols, t = _misfit_args(traces, obs, ncols)
    s = torch.cuda.current_stream(traces.device) if stream is None else stream
    _check(lib().lb_trace_misfit_static(ctypes.c_void_p(traces.data_ptr()), ctypes.c_void_p(obs.data_ptr()),
                                        ctypes.c_void_p(res.data_ptr()), nrec, cap, ncols, t,
                                        ctypes.c_void_p(phi.data_ptr()), ctypes.c_void_p(s.cuda_stream)),
           "lb_trace_misfit_static")
    return phi, res


def shot_desc(nx, ny, src, nsteps, nrec, sponge_width=0, sponge_sigma_max=0.0):
    d = ShotDesc()
    d.nx, d.ny = int(nx), int(ny)
    d.src_x, d.src_y = int(src[0]), int(src[1])
    d.nsteps = int(nsteps)
    d.nrec = int(nrec)
    d.sponge_width = int(sponge_width)
    d.sponge_sigma_max = float(sponge_sigma_max)
    return d


class Batch:
    """Batched executor: many shots advance together, several steps per
    launch (as lb_blocked_steps gives; steps_per_launch caps it), captured as
    a HIP graph per tick (lb_batch_* calls).

    Runs on its own (default-priority) stream so that ticks can be captured.
    """

    def __init__(self, max_shots, lattice=5, collision="bgk", precision="f32", tau=0.5,
                 s=None, ratio=0.25, use_graph=True, device=None, steps_per_launch=0):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.scheme = make_desc(1, 1, lattice=lattice, collision=collision, precision=precision,
                                tau=tau, s=s, ratio=ratio, steps_per_launch=steps_per_launch)
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.max_shots = int(max_shots)
        self.stream = torch.cuda.Stream(self.device)
        L = lib()
        nbytes = L.lb_batch_workspace_bytes(self.max_shots)
        if nbytes == 0:
            raise LBError(-2, "lb_batch_workspace_bytes")
        with torch.cuda.stream(self.stream):
            self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(L.lb_batch_create(ctypes.byref(self.scheme), self.max_shots,
                                 ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_size_t(int(nbytes)),
                                 ctypes.c_void_p(self.stream.cuda_stream), 1 if use_graph else 0,
                                 ctypes.byref(h)), "lb_batch_create")
        self._h = h
        self.shots = {}
        self._inflight = collections.deque()   # completion events of the ticks

    def shot_bytes(self, desc):
        return int(lib().lb_shot_workspace_bytes(self._h, ctypes.byref(desc)))

    def add(self, desc, c2, wavelet, receivers):
        """Admit a shot; returns its slot.  c2: numpy array or CUDA tensor."""
        torch = self._torch
        nbytes = self.shot_bytes(desc)
        if nbytes == 0:
            raise LBError(-2, "lb_shot_workspace_bytes")
        rec = np.ascontiguousarray(receivers, dtype=np.int32).reshape(-1, 2)
        if rec.shape[0] != desc.nrec:
            raise ValueError("receiver count does not match the shot description")
        w = np.ascontiguousarray(wavelet, dtype=np.float64)
        keep = []
        if isinstance(c2, torch.Tensor) and c2.is_cuda:
            c2 = c2.contiguous()
            keep.append(c2)
            cp, ct, dev = ctypes.c_void_p(c2.data_ptr()), (F64 if c2.dtype == torch.float64 else F32), 1
        else:
            arr = np.ascontiguousarray(c2, dtype=np.float64)
            keep.append(arr)
            cp, ct, dev = ctypes.c_void_p(arr.ctypes.data), F64, 0
        with torch.cuda.stream(self.stream):
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        traces = torch.zeros((max(desc.nrec, 1), desc.nsteps + 1), dtype=self.dtype, device=self.device)
        # the library reads c2 and writes the traces on a stream of its own:
        # both must be complete (the caller's stream, not the ticks, is waited on)
        torch.cuda.current_stream(self.device).synchronize()
        slot = ctypes.c_int32(-1)
        _check(lib().lb_batch_add_shot(self._h, ctypes.byref(desc), ctypes.c_void_p(ws.data_ptr()),
                                       ctypes.c_size_t(nbytes), cp, ct, dev,
                                       w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(w.size),
                                       rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       ctypes.c_void_p(traces.data_ptr()), ctypes.byref(slot)),
               "lb_batch_add_shot")
        self.shots[slot.value] = {"ws": ws, "traces": traces, "nsteps": int(desc.nsteps), "bytes": nbytes}
        return slot.value

    def remove(self, slot):
        """Retire a shot; returns its trace tensor [nrec][nsteps + 1].  Work
        queued afterwards on the caller's stream runs after the ticks
        enqueued so far (no host wait)."""
        _check(lib().lb_batch_remove_shot(self._h, int(slot)), "lb_batch_remove_shot")
        info = self.shots.pop(int(slot))
        self._torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return info["traces"]

    def tick(self, k):
        _check(lib().lb_batch_tick(self._h, int(k)), "lb_batch_tick")
        ev = self._torch.cuda.Event()
        ev.record(self.stream)
        self._inflight.append(ev)

    def in_flight(self):
        """Ticks enqueued and not yet completed (no wait)."""
        while self._inflight and self._inflight[0].query():
            self._inflight.popleft()
        return len(self._inflight)

    def wait_oldest(self):
        """Wait for the oldest tick in flight; False if there is none."""
        if not self._inflight:
            return False
        self._inflight.popleft().synchronize()
        return True

    def times(self):
        """Times the slots reach once the enqueued ticks have run."""
        out = (ctypes.c_int64 * self.max_shots)()
        _check(lib().lb_batch_times(self._h, out), "lb_batch_times")
        return np.frombuffer(out, dtype=np.int64).copy()

    def completed(self):
        """Times the slots have reached on the device (newest completed
        tick; -1 where none has completed since admission).  No wait."""
        out = (ctypes.c_int64 * self.max_shots)()
        _check(lib().lb_batch_completed(self._h, out), "lb_batch_completed")
        return np.frombuffer(out, dtype=np.int64).copy()

    def sync(self):
        _check(lib().lb_batch_sync(self._h), "lb_batch_sync")

    def close(self):
        if getattr(self, "_h", None) is not None:
            code = lib().lb_batch_destroy(self._h)
            self._h = None
            _check(code, "lb_batch_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
