"""Oracle pins for the grid-refinement composite (arXiv:1704.03172, Sec. IV,
eq. grid refinement eqm dist, eq. coarse-fine dist connect)."""
import numpy as np
import pytest

from oracle import lb_oracle as lo
from oracle import refine as rf
from paper_1704_03172_amd import inputs


def test_rescale_keeps_moments_and_inverts():
    rng = np.random.default_rng(3)
    g = rng.standard_normal((5, 50))
    c2 = rng.uniform(0.05, 0.45, 50)
    c = lo.VELOCITIES[5].astype(float)
    for f in (0.5, 2.0, 1.0, 0.0):
        r = rf.rescale(g, c2, f)
        np.testing.assert_allclose(r.sum(0), g.sum(0), atol=1e-14)
        np.testing.assert_allclose(c[:, 0] @ r, c[:, 0] @ g, atol=1e-14)
        np.testing.assert_allclose(c[:, 1] @ r, c[:, 1] @ g, atol=1e-14)
    np.testing.assert_allclose(rf.rescale(rf.rescale(g, c2, 0.5), c2, 2.0), g, atol=1e-13)
    # f = 0 gives the equilibrium, f = 1 the identity
    np.testing.assert_allclose(rf.rescale(g, c2, 1.0), g, atol=1e-15)
    geq = rf.rescale(g, c2, 0.0)
    np.testing.assert_allclose(rf.rescale(geq, c2, 0.5), geq, atol=1e-15)


def _run(patch, c_lens, nsteps=420, rescale=True, refine=True, n=160, fc=0.025):
    wl = inputs.refined_workload(n=n, nsteps=nsteps, nrec=48, lens_speed=c_lens,
                                 c_bg=0.5, fc=fc, patch=patch, lens_inset=4,
                                 sponge_width=16)
    g = lo.OracleGrid(n, n, q=5, collision="bgk", tau=0.5, sponge_width=16,
                      sponge_sigma_max=0.1, source=wl["source"],
                      wavelet=wl["wavelet"])
    g.set_medium(wl["c2"])
    g.set_state(np.zeros((n, n)))
    if not refine:
        return lo.run(g, nsteps, wl["receivers"])["traces"][0]
    ref = rf.OracleRefined(g, wl["c2_fine"], patch, rescale_noneq=rescale)
    return rf.run_refined(ref, nsteps, wl["receivers"])["traces"][0]


@pytest.fixture(scope="module")
def refinement_runs():
    patch = (48, 56, 64, 40)
    return {
        "coarse": _run(patch, 0.5, refine=False),
        "homog": _run(patch, 0.5),
        "norescale": _run(patch, 0.5, rescale=False),
        "lens": _run(patch, 0.25),
    }


def test_homogeneous_interface_is_nearly_transparent(refinement_runs):
    """P11: with a homogeneous medium the refined run differs from the
    coarse-only run at the surface receivers only by the small spurious
    interface reflection; without the 1/n, n rescaling it is >5x larger."""
    a = refinement_runs["coarse"]
    e_ref = np.linalg.norm(refinement_runs["homog"] - a) / np.linalg.norm(a)
    e_no = np.linalg.norm(refinement_runs["norescale"] - a) / np.linalg.norm(a)
    assert e_ref < 5e-3
    assert e_no > 5 * e_ref


def test_lens_reflection_is_physical(refinement_runs):
    """A low-velocity lens under the patch sends back a reflection far
    larger than the spurious interface signal."""
    a = refinement_runs["coarse"]
    e_lens = np.linalg.norm(refinement_runs["lens"] - a) / np.linalg.norm(a)
    e_ref = np.linalg.norm(refinement_runs["homog"] - a) / np.linalg.norm(a)
    assert e_lens > 20 * e_ref


def test_refined_run_keeps_uniform_pressure_at_rest():
    """A medium at rest with uniform pressure p = c^2 rho (rho = p0 / c^2,
    J = 0) is a steady state of the scheme in any medium; the composite
    with the interface exchange must keep it exactly."""
    n = 64
    patch = (20, 22, 24, 16)
    p0 = 0.3
    wl = inputs.refined_workload(n=n, nsteps=10, nrec=4, patch=patch, lens_inset=4,
                                 sponge_width=0)
    g = lo.OracleGrid(n, n, q=5, collision="bgk", tau=0.5)
    g.set_medium(wl["c2"])
    g.set_state(p0 / wl["c2"])
    ref = rf.OracleRefined(g, wl["c2_fine"], patch)
    ref.fine.set_state(p0 / wl["c2_fine"])
    ref.initialize()
    for _ in range(20):
        ref.step()
    np.testing.assert_allclose(ref.coarse.pressure(), p0, rtol=1e-13)
    np.testing.assert_allclose(ref.fine.pressure(), p0, rtol=1e-13)
    np.testing.assert_allclose(ref.coarse.jx(), 0.0, atol=1e-14)


# ---- independent pins of the interface arithmetic ---------------------------
# Sec. IV asks for spatial and temporal interpolation of the coarse state on
# the fine outer ring.  Reading R18 fixes them as the 4-point Lagrange
# interpolant along the edge (exact for cubics) and the mean of the coarse
# states at T and T+2 (exact for states linear in time).  These pins check
# the oracle against those exactness properties, with polynomial states
# whose values at the fine nodes are known in closed form, and check that
# planted mistakes (linear weights, a stencil shifted by one node, no
# temporal mean) fail them.

def _bare_refined(n=64, patch=(20, 22, 24, 16), rescale=False):
    """An OracleRefined over a homogeneous medium; rescale=False makes R_f
    the identity so that the ring receives the interpolated state itself."""
    c2 = 0.25
    g = lo.OracleGrid(n, n, q=5, collision="bgk", tau=0.5)
    g.set_medium(np.full((n, n), c2))
    ref = rf.OracleRefined(g, np.full((2 * (patch[3] + 4) + 1, 2 * (patch[2] + 4) + 1), c2),
                           patch, rescale_noneq=rescale)
    return ref


def _bicubic(seed, xc, yc, scale=8.0, q=5):
    """q bicubic polynomials P_i(x, y) = sum_{k,l<=3} a_ikl u^k v^l with
    u = (x - xc)/scale, v = (y - yc)/scale (values of order one near the
    patch); returns an evaluator (x, y) -> (q, ...)."""
    a = np.random.default_rng(seed).uniform(-1.0, 1.0, (q, 4, 4))

    def ev(x, y):
        u = (np.asarray(x, dtype=np.float64) - xc) / scale
        v = (np.asarray(y, dtype=np.float64) - yc) / scale
        return np.stack([sum(a[i, k, l] * u ** k * v ** l for k in range(4) for l in range(4))
                         for i in range(q)])
    return ev


def _ring_error(ref, P, t_fine=None):
    """Relative max error of the fine outer ring against P at the fine node
    positions (X0 + i/2, Y0 + j/2)."""
    i, j = ref._ring_i, ref._ring_j
    x, y = ref.X0 + 0.5 * i, ref.Y0 + 0.5 * j
    want = P(x, y) if t_fine is None else P(x, y, t_fine)
    got = ref.fine.g[:, j, i]
    return np.max(np.abs(got - want)) / np.max(np.abs(want))


def _coarse_state(ref, P, *t):
    n = ref.coarse.nx
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    return P(x, y, *t)


def test_prolongation_reproduces_cubics_exactly():
    """Every fine outer-ring node (corners, coincident and mid-edge nodes)
    receives the exact value of a bicubic coarse state."""
    ref = _bare_refined()
    P = _bicubic(11, ref.X0 + ref.W / 2, ref.Y0 + ref.H / 2)
    ref.prolong(_coarse_state(ref, P))
    assert _ring_error(ref, P) < 1e-13


def test_prolongation_with_rescaling_is_r_half_of_the_exact_value():
    """With the 1/2 rescaling on, the ring holds R_1/2 of the exact
    interpolated value (rho and J of the exact value, non-equilibrium part
    halved)."""
    ref = _bare_refined(rescale=True)
    P = _bicubic(12, ref.X0 + ref.W / 2, ref.Y0 + ref.H / 2)
    ref.prolong(_coarse_state(ref, P))
    i, j = ref._ring_i, ref._ring_j
    exact = P(ref.X0 + 0.5 * i, ref.Y0 + 0.5 * j)
    got = ref.fine.g[:, j, i]
    c = lo.VELOCITIES[5].astype(np.float64)
    np.testing.assert_allclose(got.sum(0), exact.sum(0), rtol=0, atol=1e-12)
    np.testing.assert_allclose(c[:, 0] @ got, c[:, 0] @ exact, rtol=0, atol=1e-12)
    np.testing.assert_allclose(c[:, 1] @ got, c[:, 1] @ exact, rtol=0, atol=1e-12)
    # non-equilibrium part: (got - geq) = (exact - geq) / 2 with geq the
    # equilibrium of rho, J at the node's c^2 = 1/4 (w0 = 1/2, w_i = 1/8,
    # w_i / c^2 = 1/2 for the movers)
    rho, jx, jy = exact.sum(0), c[:, 0] @ exact, c[:, 1] @ exact
    geq = np.stack([0.5 * rho] + [0.125 * rho + 0.5 * (cx * jx + cy * jy)
                                  for cx, cy in c[1:]])
    np.testing.assert_allclose(got - geq, 0.5 * (exact - geq), rtol=0, atol=1e-12)


def test_restriction_copies_coincident_fine_nodes():
    """The coarse inner ring receives the coincident fine node (identity
    rescaling) and no other coarse node changes."""
    ref = _bare_refined()
    P = _bicubic(13, ref.X0 + ref.W / 2, ref.Y0 + ref.H / 2)
    jj, ii = np.mgrid[0:ref.nyf, 0:ref.nxf].astype(np.float64)
    ref.fine.g[...] = P(ref.X0 + 0.5 * ii, ref.Y0 + 0.5 * jj)
    before = ref.coarse.g.copy()
    ref.restrict()
    x, y = ref._inner_x, ref._inner_y
    np.testing.assert_allclose(ref.coarse.g[:, y, x], P(x, y), rtol=1e-13, atol=1e-13)
    mask = np.ones(ref.coarse.g.shape[1:], dtype=bool)
    mask[y, x] = False
    np.testing.assert_array_equal(ref.coarse.g[:, mask], before[:, mask])
    # the inner ring is the rectangle overlap_in cells inside the patch
    px0, py0, pnx, pny = ref.patch
    assert set(zip(x.tolist(), y.tolist())) == {
        (xx, yy) for xx in range(px0 + 2, px0 + pnx - 1) for yy in range(py0 + 2, py0 + pny - 1)
        if xx in (px0 + 2, px0 + pnx - 2) or yy in (py0 + 2, py0 + pny - 2)}


class _LinearInTime:
    """Replaces the two grids' time steps: the coarse state follows
    g(x, y, t) = P(x, y) + t Q(x, y) (t in fine time units, so one coarse
    step adds 2 Q) and the fine grid does not move, so the fine ring after
    each sub-step holds exactly what the interface wrote."""

    def __init__(self, ref, P, Q):
        self.ref, self.P, self.Q = ref, P, Q
        self.t = 0
        self.ring_after_first_substep = None
        self.fine_calls = 0
        ref.coarse.g[...] = _coarse_state(ref, self.state)
        ref.coarse.step = self.coarse_step
        ref.fine.step = self.fine_step

    def state(self, x, y, t=None):
        t = self.t if t is None else t
        return self.P(x, y) + t * self.Q(x, y)

    def coarse_step(self, nsteps=1):
        self.t += 2
        self.ref.coarse.g[...] = _coarse_state(self.ref, self.state)

    def fine_step(self, nsteps=1):
        self.fine_calls += 1
        if self.fine_calls % 2 == 0:     # second sub-step: the ring holds T+1
            i, j = self.ref._ring_i, self.ref._ring_j
            self.ring_after_first_substep = self.ref.fine.g[:, j, i].copy()


def _temporal_errors(ref_cls=rf.OracleRefined):
    ref = _bare_refined()
    if ref_cls is not rf.OracleRefined:
        ref.__class__ = ref_cls
    xc, yc = ref.X0 + ref.W / 2, ref.Y0 + ref.H / 2
    P = _bicubic(21, xc, yc)
    Q = _bicubic(22, xc, yc)
    lin = _LinearInTime(ref, P, Q)
    i, j = ref._ring_i, ref._ring_j
    x, y = ref.X0 + 0.5 * i, ref.Y0 + 0.5 * j
    errs = []
    for _ in range(3):
        T = lin.t
        ref.step()
        mid = lin.state(x, y, T + 1)
        end = lin.state(x, y, T + 2)
        errs.append(np.max(np.abs(lin.ring_after_first_substep - mid)) / np.max(np.abs(mid)))
        errs.append(np.max(np.abs(ref.fine.g[:, j, i] - end)) / np.max(np.abs(end)))
    return errs


def test_temporal_interpolation_is_exact_for_states_linear_in_time():
    """At the intermediate fine time T+1 the ring receives the coarse state
    of time T+1 exactly when the coarse state is linear in time (and cubic
    in space); at T+2 it receives that of T+2."""
    assert max(_temporal_errors()) < 1e-13


# planted mistakes: each must fail one of the exactness pins above

class _NoTemporalMean(rf.OracleRefined):
    def step(self):
        self.coarse.step()
        self.fine.step()
        self.prolong(self.coarse.g)        # mistake: coarse state of T+2
        self.fine.step()
        self.prolong(self.coarse.g)
        self.restrict()


def test_planted_mistakes_fail_the_exactness_pins():
    # linear weights (0, 1/2, 1/2, 0) on the mid-edge nodes
    ref = _bare_refined()
    P = _bicubic(11, ref.X0 + ref.W / 2, ref.Y0 + ref.H / 2)
    xs, ys, wt = ref._stencil
    mid = wt[:, 0] != 0.0
    assert mid.sum() > 0.4 * len(wt)
    wt[mid] = (0.0, 0.5, 0.5, 0.0)
    ref.prolong(_coarse_state(ref, P))
    assert _ring_error(ref, P) > 1e-4
    # the cubic stencil shifted by one coarse node along the edge
    for shift in (-1, 1):
        ref = _bare_refined()
        xs, ys, wt = ref._stencil
        along_x = (wt[:, 0] != 0.0) & (xs[:, 0] != xs[:, 1])
        along_y = (wt[:, 0] != 0.0) & (ys[:, 0] != ys[:, 1])
        xs[along_x] += shift
        ys[along_y] += shift
        ref.prolong(_coarse_state(ref, P))
        assert _ring_error(ref, P) > 1e-2
    # no temporal mean at the intermediate time
    assert max(_temporal_errors(_NoTemporalMean)) > 1e-2


def _pulse_traces(rescale=True, refine=True, n=192, patch=(64, 80, 64, 48),
                  center=(96, 40), sigma=8.0, nsteps=200, c=0.5):
    g = lo.OracleGrid(n, n, q=5, collision="bgk", tau=0.5, sponge_width=16,
                      sponge_sigma_max=0.1)
    g.set_medium(np.full((n, n), c * c))
    y, x = np.mgrid[0:n, 0:n]
    g.set_state(np.exp(-((x - center[0]) ** 2 + (y - center[1]) ** 2) / (2 * sigma ** 2)))
    recs = np.array([(xx, center[1]) for xx in range(20, n - 20, 4)], dtype=np.int64)
    if not refine:
        return lo.run(g, nsteps, recs)["traces"][0]
    fine_c2 = np.full((2 * (patch[3] + 4) + 1, 2 * (patch[2] + 4) + 1), c * c)
    ref = rf.OracleRefined(g, fine_c2, patch, rescale_noneq=rescale)
    return rf.run_refined(ref, nsteps, recs)["traces"][0]


def test_p11_spurious_reflection_of_a_wide_pulse():
    """P11: a Gaussian pulse (sigma = 8 nodes) in a homogeneous medium
    crosses into the patch and its wake returns to the receivers on its
    row; the refined run differs from the coarse-only run by at most 1e-3
    of the recorded signal, and the ablation without the 1/n, n rescaling
    of the non-equilibrium part (eq. coarse-fine dist connect) is at least
    ten times worse."""
    a = _pulse_traces(refine=False)
    e = np.linalg.norm(_pulse_traces() - a) / np.linalg.norm(a)
    e_no = np.linalg.norm(_pulse_traces(rescale=False) - a) / np.linalg.norm(a)
    assert e < 1e-3, e
    assert e_no > 10 * e, (e, e_no)
