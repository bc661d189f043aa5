"""Python driver of the FP64 oracle recurrence (lb_oracle.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

What each piece follows in arXiv:1704.03172:
  VELOCITIES      Table I; ordering of Appendix A (the columns of M).
  M_D2Q5, M_D2Q9  Appendix A, typed from the paper.
  collision_matrix
                  C = M^-1 S M (eq. MRT-LB), M^-1 by a general linear solve;
                  S = diag(s) in the moment order of eq. D2Q5 moments /
                  eq. D2Q9 moments.  BGK is C = I / tau (eq. BGK-LB).
  OracleGrid.step one update n -> n+1 (moments, weights, eq. linear eqm dist,
                  collision, source w_i S(n) of eq. MRT-LB linear acoustic,
                  sponge, periodic streaming), done in C.
  records         p = c^2 rho (eq. state), rho, J of the pre-collision state
                  at integer times (eq. macroscopic density / velocity).

Time labelling (a reading; the paper only says that macroscopic variables are
evaluated after the step): the state g(n) is the pre-collision state at time
n; S(n) is added in the step n -> n+1; records at time n are taken from g(n).
A run of N steps therefore records times 0..N.

Pins (tests/test_oracle_*.py): Fourier-space exactness and plane-wave
eigenmodes against dispersion.py, conservation of sum rho, time reversal for
omega = 2, the printed matrices of Appendices A/B, the equivalences stated in
Sec. III, brute-force operator spectra on tiny grids, the analytic point
source solution, sponge and interface reflection coefficients.
"""
import ctypes
import numpy as np

from . import build as _build

VELOCITIES = {
    5: np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1)], dtype=np.int64),
    9: np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
                 (1, 1), (-1, 1), (-1, -1), (1, -1)], dtype=np.int64),
}

# Appendix A, D2Q5: rows are the moments {rho, rho0 vx, rho0 vy, e, pxx}.
M_D2Q5 = np.array([
    [1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0],
    [0, 0, 1, 0, -1],
    [-4, 1, 1, 1, 1],
    [0, 1, -1, 1, -1],
], dtype=np.float64)

# Appendix A, D2Q9: rows {rho, rho0 vx, rho0 vy, e, pxx, eps, qx, qy, pxy}.
M_D2Q9 = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)


def transformation_matrix(q):
    """Moment transformation matrix M of Appendix A."""
    return {5: M_D2Q5, 9: M_D2Q9}[q]


def collision_matrix(q, collision, tau=None, s=None):
    """Collision matrix C of eq. MRT-LB.

    collision='bgk': C = I / tau (eq. BGK-LB).
    collision='mrt': C = M^-1 diag(s) M with s the q relaxation rates in the
    moment order of Sec. II B (D2Q5: s_rho, s_v, s_v, s_e, s_p; D2Q9:
    s_rho, s_v, s_v, s_e, s_p, s_eps, s_q, s_q, s_p).
    """
    if collision == "bgk":
        return np.eye(q) / float(tau)
    if collision != "mrt":
        raise ValueError("collision must be 'bgk' or 'mrt'")
    M = transformation_matrix(q)
    s = np.asarray(s, dtype=np.float64)
    if s.shape != (q,):
        raise ValueError("MRT needs %d relaxation rates" % q)
    Minv = np.linalg.solve(M, np.eye(q))
    return Minv @ np.diag(s) @ M


def weights(q, c2, ratio=0.25):
    """Lattice weights for squared sound speed c2 (same rule as the C code).

    Returns an array of shape (q,) + shape(c2).
    """
    c2 = np.asarray(c2, dtype=np.float64)
    if q == 5:
        w1 = 0.5 * c2
        return np.stack([1.0 - 4.0 * w1] + [w1] * 4)
    w1 = c2 / (2.0 + 4.0 * ratio)
    w5 = ratio * w1
    return np.stack([1.0 - 4.0 * w1 - 4.0 * w5] + [w1] * 4 + [w5] * 4)


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("q", ctypes.c_int32),
        ("cx", ctypes.c_int32 * 9), ("cy", ctypes.c_int32 * 9),
        ("coll", ctypes.c_double * 81),
        ("ratio", ctypes.c_double),
        ("sponge_width", ctypes.c_int32),
        ("sponge_sigma_max", ctypes.c_double),
        ("src_x", ctypes.c_int32), ("src_y", ctypes.c_int32),
    ]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        lib = ctypes.CDLL(_build.ensure_built())
        P = ctypes.POINTER(_Params)
        D = ctypes.POINTER(ctypes.c_double)
        lib.orc_step.argtypes = [P, D, D, D, ctypes.c_double]
        lib.orc_step.restype = None
        lib.orc_equilibrium_field.argtypes = [P, D, D, D, D, D]
        lib.orc_equilibrium_field.restype = None
        lib.orc_collide_node.argtypes = [P, D, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, D]
        lib.orc_collide_node.restype = None
        lib.orc_sponge_sigma.argtypes = [P, ctypes.c_int, ctypes.c_int]
        lib.orc_sponge_sigma.restype = ctypes.c_double
        lib.orc_node_weights.argtypes = [P, ctypes.c_double, D]
        lib.orc_node_weights.restype = None
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        lib.orc_set_num_threads.restype = None
        _LIB = lib
    return _LIB


def _dptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads():
    """OpenMP threads the C step runs on."""
    return int(_lib().orc_num_threads())


def set_num_threads(n):
    """OpenMP threads of later C steps (for timing; results do not depend on it)."""
    _lib().orc_set_num_threads(int(n))


class OracleGrid:
    """One periodic lattice advanced by the plain FP64 recurrence.

    g has shape (q, ny, nx) and holds the pre-collision state at time n.
    """

    def __init__(self, nx, ny, q=5, collision="bgk", tau=0.5, s=None,
                 ratio=0.25, sponge_width=0, sponge_sigma_max=0.0,
                 source=None, wavelet=None, coll=None):
        self.nx, self.ny, self.q = int(nx), int(ny), int(q)
        self.ratio = float(ratio)
        self.coll = (np.asarray(coll, dtype=np.float64) if coll is not None
                     else collision_matrix(q, collision, tau, s))
        self.c = VELOCITIES[q]
        self.g = np.zeros((q, ny, nx))
        self._gn = np.zeros_like(self.g)
        self.c2 = None
        self.n = 0
        self.source = None if source is None else (int(source[0]), int(source[1]))
        self.wavelet = (np.zeros(0) if wavelet is None
                        else np.ascontiguousarray(wavelet, dtype=np.float64))
        p = _Params()
        p.nx, p.ny, p.q = self.nx, self.ny, self.q
        for i in range(9):
            p.cx[i] = int(self.c[i, 0]) if i < q else 0
            p.cy[i] = int(self.c[i, 1]) if i < q else 0
        flat = self.coll.reshape(-1)
        for i in range(q * q):
            p.coll[i] = float(flat[i])
        p.ratio = self.ratio
        p.sponge_width = int(sponge_width)
        p.sponge_sigma_max = float(sponge_sigma_max)
        p.src_x, p.src_y = self.source if self.source is not None else (-1, -1)
        self._p = p

    # -- set-up -----------------------------------------------------------
    def set_medium(self, c2):
        c2 = np.ascontiguousarray(c2, dtype=np.float64)
        assert c2.shape == (self.ny, self.nx)
        self.c2 = c2

    def set_state(self, rho, jx=None, jy=None):
        """g(0) = g^eq(rho, J) at every node; resets the step counter."""
        assert self.c2 is not None, "set_medium first"
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        jx = None if jx is None else np.ascontiguousarray(jx, dtype=np.float64)
        jy = None if jy is None else np.ascontiguousarray(jy, dtype=np.float64)
        lib = _lib()
        lib.orc_equilibrium_field(ctypes.byref(self._p), _dptr(self.c2),
                                  _dptr(rho),
                                  _dptr(jx) if jx is not None else None,
                                  _dptr(jy) if jy is not None else None,
                                  _dptr(self.g))
        self.n = 0

    def set_raw(self, g, n=0):
        self.g[...] = g
        self.n = int(n)

    # -- stepping ---------------------------------------------------------
    def source_value(self, n):
        return float(self.wavelet[n]) if 0 <= n < self.wavelet.size else 0.0

    def step(self, nsteps=1):
        lib = _lib()
        for _ in range(nsteps):
            lib.orc_step(ctypes.byref(self._p), _dptr(self.g), _dptr(self._gn),
                         _dptr(self.c2), self.source_value(self.n))
            self.g, self._gn = self._gn, self.g
            self.n += 1

    # -- observables ------------------------------------------------------
    def rho(self):
        return self.g.sum(axis=0)

    def jx(self):
        return np.tensordot(self.c[:, 0].astype(np.float64), self.g, axes=1)

    def jy(self):
        return np.tensordot(self.c[:, 1].astype(np.float64), self.g, axes=1)

    def pressure(self):
        return self.c2 * self.rho()

    def field(self, what):
        return {"p": self.pressure, "rho": self.rho, "jx": self.jx,
                "jy": self.jy}[what]()

    def fields_at(self, xs, ys):
        """p, rho, jx, jy at the nodes (xs[k], ys[k]) only."""
        gsel = self.g[:, ys, xs]                       # (q, k)
        rho = gsel.sum(axis=0)
        jx = self.c[:, 0].astype(np.float64) @ gsel
        jy = self.c[:, 1].astype(np.float64) @ gsel
        return {"p": self.c2[ys, xs] * rho, "rho": rho, "jx": jx, "jy": jy}

    def collide_node(self, gi, c2, s_here=0.0, sigma=0.0):
        """Steps 1-6 of the update at one node (used by the refinement)."""
        gi = np.ascontiguousarray(gi, dtype=np.float64)
        out = np.zeros(self.q)
        _lib().orc_collide_node(ctypes.byref(self._p), _dptr(gi), float(c2),
                                float(s_here), float(sigma), _dptr(out))
        return out

    def sponge_sigma(self, x, y):
        return float(_lib().orc_sponge_sigma(ctypes.byref(self._p), int(x), int(y)))


def run(grid, nsteps, receivers=None, fields=("p",), sum_rho=False,
        snapshots=()):
    """Advance `grid` by nsteps, recording like the product does.

    receivers: int array (nrec, 2) of (x, y).  Returns a dict with
      traces   (len(fields), nrec, nsteps + 1): field value at receivers at
               times n0 .. n0 + nsteps
      sum_rho  (nsteps + 1,) sum of rho over the grid at the same times
      snap     {time: {field: array}} for times listed in `snapshots`
    """
    rec = None if receivers is None else np.asarray(receivers, dtype=np.int64)
    out = {}
    nrec = 0 if rec is None else rec.shape[0]
    traces = np.zeros((len(fields), nrec, nsteps + 1))
    sums = np.zeros(nsteps + 1)
    snap = {}
    snaps = set(int(t) for t in snapshots)

    def record(k):
        if nrec:
            vals = grid.fields_at(rec[:, 0], rec[:, 1])
            for f, name in enumerate(fields):
                traces[f, :, k] = vals[name]
        if sum_rho:
            sums[k] = grid.rho().sum()
        if grid.n in snaps:
            snap[grid.n] = {name: grid.field(name).copy() for name in ("rho", "jx", "jy", "p")}

    record(0)
    for k in range(1, nsteps + 1):
        grid.step()
        record(k)
    out["traces"] = traces
    out["sum_rho"] = sums
    out["snap"] = snap
    return out
