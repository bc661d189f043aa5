"""Coarse/fine grid refinement composite (arXiv:1704.03172, Sec. IV,
eq. grid refinement eqm dist, eq. coarse-fine dist connect).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper fixes: refinement factor n (a multiple of 2; here n = 2), two fine
sub-steps per coarse step, equilibrium parts equal on both grids, the
non-equilibrium part multiplied by n going fine -> coarse and by 1/n going
coarse -> fine, spatial and temporal interpolation of coarse values at the
intermediate fine time, and overlap regions.  It leaves open the geometry of
the overlap, the interpolation orders and the per-edge direction logic; the
reading implemented here (bidirectional two-line exchange) is:

  * the fine grid covers the patch [px0, px0+pnx] x [py0, py0+pny] (coarse
    units) dilated by `overlap_out` coarse cells; fine node (i, j) sits at
    coarse coordinate (X0 + i/2, Y0 + j/2);
  * after each fine sub-step, every node of the outermost fine ring is
    overwritten with R_{1/2}(g_hat), where g_hat is the coarse state at the
    matching time: at the intermediate time the mean of the coarse states
    at T and T+2 (temporal interpolation), at T+2 the coarse state itself;
    ring nodes that coincide with coarse nodes take the coarse node,
    mid-edge nodes the 4-point cubic Lagrange value (-1, 9, 9, -1)/16 along
    the edge (spatial interpolation);
  * after the second sub-step, the coarse ring `overlap_in` cells inside the
    patch is overwritten with R_2(g^f) of the coincident fine nodes;
  * R_f(g) = g^eq(rho(g), J(g)) + f (g - g^eq), with the weights of the
    node that receives the value (eq. coarse-fine dist connect);
  * at time 0 the same two overwrites are applied once to the initial state.

Pins (tests/test_oracle_refine.py): R_f keeps rho and J and R_2 o R_1/2 is
the identity; the fine ring reproduces a bicubic coarse state exactly (the
4-point interpolant's exactness) and, at the intermediate time, a state
linear in time exactly (the temporal mean's exactness); the restriction
copies the coincident fine nodes to the coarse inner ring and nothing else;
planted mistakes (linear weights, a shifted stencil, no temporal mean) fail
those pins; a wide pulse in a homogeneous medium shows a spurious interface
signal below 1e-3 of the recorded one, and at least ten times more without
the rescaling; a uniform pressure at rest stays exact.
"""
import numpy as np

from .lb_oracle import OracleGrid, VELOCITIES, weights


def rescale(g, c2, f, q=5, ratio=0.25):
    """R_f(g) = g^eq + f (g - g^eq) for population vectors g of shape (q, ...)."""
    c = VELOCITIES[q].astype(np.float64)
    rho = g.sum(axis=0)
    jx = np.tensordot(c[:, 0], g, axes=1)
    jy = np.tensordot(c[:, 1], g, axes=1)
    w = weights(q, c2, ratio)
    cj = c[:, 0].reshape((q,) + (1,) * rho.ndim) * jx + \
        c[:, 1].reshape((q,) + (1,) * rho.ndim) * jy
    geq = w / c2 * (c2 * rho + cj)
    return geq + f * (g - geq)


class OracleRefined:
    """A coarse OracleGrid with one refined rectangular patch (factor 2)."""

    def __init__(self, coarse, c2_fine, patch, overlap_out=2, overlap_in=2,
                 factor=2, rescale_noneq=True):
        assert factor == 2, "only refinement factor 2 is implemented"
        assert coarse.q == 5
        px0, py0, pnx, pny = (int(v) for v in patch)
        self.patch = (px0, py0, pnx, pny)
        self.oo, self.oi = int(overlap_out), int(overlap_in)
        self.X0, self.Y0 = px0 - self.oo, py0 - self.oo
        self.W, self.H = pnx + 2 * self.oo, pny + 2 * self.oo
        self.nxf, self.nyf = 2 * self.W + 1, 2 * self.H + 1
        assert self.X0 >= 2 and self.Y0 >= 2
        assert self.X0 + self.W + 2 < coarse.nx and self.Y0 + self.H + 2 < coarse.ny
        assert 2 * self.oi < min(pnx, pny)
        self.coarse = coarse
        self.fine = OracleGrid(self.nxf, self.nyf, q=5, coll=coarse.coll)
        self.fine.set_medium(c2_fine)
        self.f_cf = 1.0 / factor if rescale_noneq else 1.0   # coarse -> fine
        self.f_fc = float(factor) if rescale_noneq else 1.0  # fine -> coarse
        self._ring = self._fine_ring_nodes()
        self._inner = self._coarse_inner_ring_nodes()
        self._ring_i = np.array([i for i, _ in self._ring], dtype=np.int64)
        self._ring_j = np.array([j for _, j in self._ring], dtype=np.int64)
        self._inner_x = np.array([x for x, _ in self._inner], dtype=np.int64)
        self._inner_y = np.array([y for _, y in self._inner], dtype=np.int64)
        self._stencil = self._ring_stencils()

    # -- geometry ---------------------------------------------------------
    def _fine_ring_nodes(self):
        nodes = []
        for i in range(self.nxf):
            nodes.append((i, 0))
            nodes.append((i, self.nyf - 1))
        for j in range(1, self.nyf - 1):
            nodes.append((0, j))
            nodes.append((self.nxf - 1, j))
        return nodes

    def _coarse_inner_ring_nodes(self):
        px0, py0, pnx, pny = self.patch
        xa, xb = px0 + self.oi, px0 + pnx - self.oi
        ya, yb = py0 + self.oi, py0 + pny - self.oi
        nodes = []
        for x in range(xa, xb + 1):
            nodes.append((x, ya))
            nodes.append((x, yb))
        for y in range(ya + 1, yb):
            nodes.append((xa, y))
            nodes.append((xb, y))
        return nodes

    def inside_patch(self, x, y):
        px0, py0, pnx, pny = self.patch
        return px0 <= x < px0 + pnx and py0 <= y < py0 + pny

    # -- interface operations -----------------------------------------------
    def _ring_stencils(self):
        """Per ring node: 4 coarse (x, y) stencil nodes and their weights.

        Coincident nodes use weights (0, 1, 0, 0); mid-edge nodes the cubic
        (-1, 9, 9, -1)/16 along the edge they lie on."""
        X0, Y0 = self.X0, self.Y0
        xs = np.zeros((len(self._ring), 4), dtype=np.int64)
        ys = np.zeros_like(xs)
        wt = np.zeros((len(self._ring), 4))
        for r, (i, j) in enumerate(self._ring):
            if i % 2 == 0 and j % 2 == 0:
                xs[r] = X0 + i // 2
                ys[r] = Y0 + j // 2
                wt[r] = (0.0, 1.0, 0.0, 0.0)
            elif i % 2 == 1:
                a = X0 + (i - 1) // 2
                xs[r] = (a - 1, a, a + 1, a + 2)
                ys[r] = Y0 + j // 2
                wt[r] = np.array([-1.0, 9.0, 9.0, -1.0]) / 16.0
            else:
                b = Y0 + (j - 1) // 2
                xs[r] = X0 + i // 2
                ys[r] = (b - 1, b, b + 1, b + 2)
                wt[r] = np.array([-1.0, 9.0, 9.0, -1.0]) / 16.0
        return xs, ys, wt

    def _coarse_at_ring(self, gc):
        """Coarse state interpolated to every fine ring node: (q, nring)."""
        xs, ys, wt = self._stencil
        vals = gc[:, ys, xs]                      # (q, nring, 4)
        return np.einsum("qrs,rs->qr", vals, wt)

    def prolong(self, gc):
        """Outer fine ring <- R_{1/2}(coarse state gc interpolated)."""
        ghat = self._coarse_at_ring(gc)
        fi, fj = self._ring_i, self._ring_j
        self.fine.g[:, fj, fi] = rescale(ghat, self.fine.c2[fj, fi], self.f_cf)

    def restrict(self):
        """Inner coarse ring <- R_2(coincident fine state)."""
        x, y = self._inner_x, self._inner_y
        i, j = 2 * (x - self.X0), 2 * (y - self.Y0)
        self.coarse.g[:, y, x] = rescale(self.fine.g[:, j, i],
                                         self.coarse.c2[y, x], self.f_fc)

    # -- stepping -----------------------------------------------------------
    def initialize(self):
        """Apply the interface overwrites to the state at time 0."""
        self.prolong(self.coarse.g)
        self.restrict()

    def step(self):
        """One coarse step T -> T+2 (fine times), Sec. IV procedure."""
        gc_then = self.coarse.g.copy()
        self.coarse.step()
        self.fine.step()
        self.prolong(0.5 * (gc_then + self.coarse.g))
        self.fine.step()
        self.prolong(self.coarse.g)
        self.restrict()

    def field_at(self, what, receivers):
        """Field values at coarse receiver nodes; nodes inside the patch are
        read from the coincident fine node."""
        out = np.zeros(len(receivers))
        fc = self.coarse.field(what)
        ff = self.fine.field(what)
        for r, (x, y) in enumerate(receivers):
            if self.inside_patch(x, y):
                out[r] = ff[2 * (y - self.Y0), 2 * (x - self.X0)]
            else:
                out[r] = fc[y, x]
        return out


def run_refined(ref, ncoarse, receivers=None, fields=("p",)):
    """Initialize interface, advance ncoarse coarse steps, record at coarse
    times 0..ncoarse.  Returns traces (len(fields), nrec, ncoarse + 1)."""
    rec = [] if receivers is None else [tuple(int(v) for v in r) for r in receivers]
    traces = np.zeros((len(fields), len(rec), ncoarse + 1))
    ref.initialize()

    def record(k):
        for f, name in enumerate(fields):
            if rec:
                traces[f, :, k] = ref.field_at(name, rec)

    record(0)
    for k in range(1, ncoarse + 1):
        ref.step()
        record(k)
    return {"traces": traces}
