"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/lbwave.h declares, and validates descriptors and arguments before
touching the device."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "lbwave.h")


@pytest.fixture(scope="module")
def lw():
    from paper_1704_03172_amd import lbwave
    if not os.path.exists(lbwave.LIB_PATH):
        from paper_1704_03172_amd import build
        build.build()
    lbwave.lib()
    return lbwave


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", text)))


def test_header_declarations_are_exported(lw):
    names = _declared_functions()
    assert len(names) >= 20
    L = lw.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(lw.EXPORTS) == names


def test_desc_layout_matches_c(lw):
    # lb_default_desc writes exactly sizeof(lb_grid_desc) bytes; a sentinel
    # after the ctypes struct must survive and the fields must read back.
    class Padded(ctypes.Structure):
        _fields_ = [("d", lw.Desc), ("tail", ctypes.c_uint8 * 64)]
    p = Padded()
    for i in range(64):
        p.tail[i] = 0xAB
    lw.lib().lb_default_desc(ctypes.byref(p.d))
    assert all(b == 0xAB for b in p.tail)
    d = p.d
    assert (d.nx, d.ny, d.lattice, d.collision, d.precision, d.nbatch) == (64, 64, 5, 0, 0, 1)
    assert d.tau == 0.5 and list(d.s) == [1, 1, 1, 2, 2, 2, 1, 1, 2]
    assert d.d2q9_ratio == 0.25 and d.sponge_width == 0 and d.sponge_sigma_max == 0.0
    assert (d.patch_enable, d.patch_refine, d.patch_overlap_out, d.patch_overlap_in) == (0, 2, 2, 2)
    assert d.trace_capacity == 0 and d.max_receivers == 0 and d.steps_per_launch == 0
    assert ctypes.sizeof(lw.Desc) == 192


@pytest.mark.parametrize("kw,code", [
    (dict(), 0),
    (dict(lattice=7), -1),
    (dict(nx=0), -2),
    (dict(ny=70000), -2),
    (dict(tau=0.49), -2),
    (dict(collision="mrt", s=[1, 1, 1, 2.5, 2]), -2),
    (dict(collision="mrt", s=[1, 1, 1, 0.0, 2]), -2),
    (dict(collision="mrt", s=[0, 0, 0, 2, 2]), 0),           # conserved rates ignored
    (dict(lattice=9, ratio=-0.1), -2),
    (dict(sponge_width=-1), -2),
    (dict(sponge_sigma_max=1.5), -2),
    (dict(nx=256, ny=256, patch=(96, 96, 64, 64)), 0),
    (dict(nx=256, ny=256, patch=(96, 96, 64, 64), tau=0.6), -3),
    (dict(nx=256, ny=256, patch=(96, 96, 64, 64), lattice=9), -3),
    (dict(nx=256, ny=256, patch=(96, 96, 64, 64), collision="mrt", s=[1, 1, 1, 2, 2]), 0),
    (dict(nx=256, ny=256, patch=(96, 96, 64, 64), collision="mrt", s=[1, 1, 1, 1.9, 2]), -3),
    (dict(nx=256, ny=256, patch=(2, 96, 64, 64)), -2),
    (dict(nx=256, ny=256, patch=(96, 96, 64, 64), sponge_width=100), -2),
    (dict(nx=256, ny=256, patch=(96, 96, 4, 64)), -2),
    (dict(steps_per_launch=1), 0),
    (dict(steps_per_launch=3), 0),
    (dict(steps_per_launch=4), 0),
    (dict(steps_per_launch=5), 0),
    (dict(steps_per_launch=8), 0),
    (dict(steps_per_launch=9), -2),
    (dict(steps_per_launch=-1), -2),
])
def test_validate(lw, kw, code):
    args = dict(nx=64, ny=64)
    args.update(kw)
    assert lw.validate(**args) == code
    nb = lw.workspace_bytes(**args)
    assert (nb > 0) == (code == 0)


@pytest.mark.parametrize("q,coll,prec,ns,nsm,ly", [
    (5, "bgk", "f32", 4, 7, 20), (5, "mrt", "f32", 4, 7, 20), (5, "bgk", "f64", 4, 8, 20), (5, "mrt", "f16s", 3, 5, 20),
    (9, "bgk", "f32", 3, 6, 20), (9, "mrt", "f32", 3, 5, 20), (9, "mrt", "f64", 4, 4, 20), (5, "mrt", "f64", 4, 7, 20), (9, "bgk", "f16s", 1, 1, 0)])
def test_blocked_steps(lw, q, coll, prec, ns, nsm, ly):
    """Steps per launch of lb_step_n for each configuration: ns with the
    short-segment kernel, nsm where the marching kernel (segments of ly
    rows) takes the grid (ny >= ly + 2 nsm; FP32: seven steps for D2Q5, six
    for D2Q9 BGK, five for D2Q9 MRT) and, by default, only where the grid
    fills the GPU with its waves (a 4096^2 grid does, a 64^2 one does not,
    except FP64 D2Q9, whose two kernels take the same count); a cap of
    steps_per_launch at or above nsm asks for it on any grid it takes; the
    cap (rounded down to a count a kernel takes), one step with a patch,
    and the validation errors."""
    kw = dict(nx=64, ny=64, lattice=q, collision=coll, precision=prec, s=[1, 1, 1, 2, 2, 2, 1, 1, 2][:q])
    assert lw.blocked_steps(**dict(kw, nx=4096, ny=4096)) == nsm
    assert lw.blocked_steps(**kw) == ns
    cap8 = dict(kw, steps_per_launch=8)
    assert lw.blocked_steps(**cap8) == nsm
    if ly:
        assert lw.blocked_steps(**dict(cap8, ny=ly + 2 * nsm)) == nsm
        assert lw.blocked_steps(**dict(cap8, ny=ly + 2 * nsm - 1)) == ns   # too short for the marching kernel
    # odd width: no vector accesses (FP64 takes one column per lane anyway)
    assert lw.blocked_steps(**dict(cap8, nx=63)) == (nsm if prec == "f64" else ns)
    for cap in range(1, 9):
        want = nsm if cap >= nsm else min(cap, ns)
        assert lw.blocked_steps(steps_per_launch=cap, **kw) == want
    kw.update(nx=256, ny=256)
    if lw.validate(patch=(96, 96, 64, 64), **kw) == 0:   # patches take D2Q5
        assert lw.blocked_steps(patch=(96, 96, 64, 64), **kw) == 1
    with pytest.raises(lw.LBError):
        lw.blocked_steps(steps_per_launch=9, **kw)
    assert lw.lib().lb_blocked_steps(None, None) == -1


def test_workspace_accounting(lw):
    # two population buffers dominate: 2 * Q * N * sizeof(storage)
    for prec, sz in (("f32", 4), ("f64", 8), ("f16s", 2)):
        for q in (5, 9):
            nb = lw.workspace_bytes(nx=1024, ny=512, lattice=q, precision=prec)
            pops = 2 * q * 1024 * 512 * sz
            c2 = 1024 * 512 * (8 if prec == "f64" else 4)
            assert pops + c2 <= nb <= pops + c2 + 4 * 1024 * 1024


def test_create_rejects_bad_workspace_before_touching_gpu(lw):
    d = lw.make_desc(64, 64)
    h = ctypes.c_void_p()
    L = lw.lib()
    assert L.lb_create_grid(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == -4
    assert L.lb_create_grid(ctypes.byref(d), ctypes.c_void_p(256), 16, None, ctypes.byref(h)) == -4
    assert L.lb_create_grid(ctypes.byref(d), ctypes.c_void_p(257), 1 << 30, None, ctypes.byref(h)) == -4
    bad = lw.make_desc(64, 64, tau=0.1)
    assert L.lb_create_grid(ctypes.byref(bad), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h)) == -2
    assert not h.value


def test_null_handles(lw):
    L = lw.lib()
    assert L.lb_destroy_grid(None) == 0
    assert L.lb_step_n(None, 1) == -1
    assert L.lb_sync(None) == -1
    assert L.lb_set_medium(None, None, 0, 0) == -1
    t = ctypes.c_int64()
    assert L.lb_get_time(None, ctypes.byref(t)) == -1
    assert L.lb_state_bytes(None) == 0
    assert L.lb_device_copy(None, None, 16, None) == -1
    assert L.lb_device_copy(ctypes.c_void_p(256), ctypes.c_void_p(272), 15, None) == -1


def test_status_strings(lw):
    L = lw.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        s = L.lb_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.lb_status_string(17).decode() == "unknown status"


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    from paper_1704_03172_amd import lbwave
    monkeypatch.setattr(lbwave, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(lbwave, "_LIB", None)
    with pytest.raises(RuntimeError):
        lbwave.lib()


def test_trace_shaped_arrays_are_checked_before_any_launch(lw):
    """Grid.misfit and Grid.adjoint take [nrec][trace_capacity] arrays that
    the kernels index as r * trace_capacity + n; any other shape must raise
    ValueError on the host before the library is called."""
    import torch

    class NoLib:
        def __getattr__(self, name):
            raise AssertionError("library called with a mis-shaped array: " + name)

    g = object.__new__(lw.Grid)
    g._torch = torch
    g.device = torch.device("cpu")
    g.dtype = torch.float32
    g.trace_capacity = 11
    g.traces = torch.zeros((1, 3, 11))
    g._h = ctypes.c_void_p(1)
    saved = lw._LIB
    lw._LIB = NoLib()
    try:
        for bad in ((3, 10), (3, 12), (2, 11), (33,), (1, 3, 10), (2, 3, 11)):
            with pytest.raises(ValueError):
                g.misfit(torch.zeros(bad), 10)
            with pytest.raises(ValueError):
                g.adjoint(torch.zeros(bad), 10)
        ok = g._trace_shaped(torch.arange(33.0).reshape(1, 3, 11), "d_obs")
        assert tuple(ok.shape) == (3, 11) and float(ok[2, 10]) == 32.0
        g.traces = None
        with pytest.raises(ValueError):
            g.misfit(torch.zeros((3, 11)), 10)
    finally:
        lw._LIB = saved
        g._h = None


def test_trace_misfit_rejects_bad_arguments_before_any_launch(lw):
    """lb_trace_misfit validates pointers, sizes, dtype and workspace on the
    host; these calls fail before anything is enqueued (no GPU needed)."""
    L = lw.lib()
    p = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)
    nbytes = ctypes.c_size_t(lw.TRACE_MISFIT_WORKSPACE_BYTES)
    call = lambda tr, ob, re, nrec, cap, ncols, t, phi, w, wb: L.lb_trace_misfit(
        tr, ob, re, nrec, cap, ncols, t, phi, w, wb, None)
    assert call(None, p, p, 3, 10, 10, 0, p, ws, nbytes) == -1
    assert call(p, None, p, 3, 10, 10, 0, p, ws, nbytes) == -1
    assert call(p, p, None, 3, 10, 10, 0, p, ws, nbytes) == -1
    assert call(p, p, p, 3, 10, 10, 0, None, ws, nbytes) == -1
    assert call(p, p, p, 3, 10, 10, 7, p, ws, nbytes) == -1          # no such dtype
    assert call(p, p, p, 0, 10, 10, 0, p, ws, nbytes) == -2          # no receivers
    assert call(p, p, p, 3, 10, 11, 0, p, ws, nbytes) == -2          # ncols > cap
    assert call(p, p, p, 3, 10, 0, 0, p, ws, nbytes) == -2
    assert call(p, p, p, 3, 0, 0, 0, p, ws, nbytes) == -2
    assert call(p, p, p, 2, 2 ** 62, 10, 0, p, ws, nbytes) == -2     # nrec x cap beyond int64
    assert call(p, p, p, 3, 10, 10, 0, p, None, nbytes) == -4
    assert call(p, p, p, 3, 10, 10, 0, p, ws, ctypes.c_size_t(16383)) == -4
    assert call(p, p, p, 3, 10, 10, 0, p, ctypes.c_void_p(0x200004), nbytes) == -4
