"""Pins of the oracle's misfit gradient: the complex copy of the recurrence
equals the C step; the discrete adjoint equals complex-step derivatives
node by node, and central differences in a random direction."""
import numpy as np
import pytest

from oracle import adjoint as ad
from oracle import lb_oracle as lo
from paper_1704_03172_amd import inputs


def tiny_case(q=5, collision="bgk", tau=0.5, s=None, ratio=0.25, nx=9, ny=7, N=24, seed=0,
              sponge=2, state=True):
    rng = np.random.default_rng(seed)
    hi = 0.45 if q == 5 else 0.55
    c2 = rng.uniform(0.1, hi, (ny, nx))
    case = {"q": q, "nx": nx, "ny": ny, "nsteps": N, "ratio": ratio,
            "coll": lo.collision_matrix(q, collision, tau, s), "c2": c2,
            "sponge_width": sponge, "sponge_sigma_max": 0.1,
            "source": (4, 3), "wavelet": inputs.ricker_wavelet(N + 1, 0.12),
            "receivers": np.array([(1, 1), (7, 5), (3, 2), (3, 2), (0, 6)])}
    if state:
        r, jx, jy = inputs.random_fields(nx, ny, seed=seed + 1)
        case.update(rho0=r, jx0=jx, jy0=jy)
    tr, _ = ad.forward(case, c2)
    case["d_obs"] = tr + 0.05 * np.abs(tr).max() * rng.standard_normal(tr.shape)
    return case


CASES = [dict(), dict(tau=0.8), dict(collision="mrt", s=[1, 1, 1, 2, 2]),
         dict(collision="mrt", s=[0.7, 1.2, 1.2, 1.5, 1.8]),
         dict(q=9, collision="mrt", s=[1, 1, 1, 2, 2, 2, 1, 1, 2]), dict(q=9, ratio=24.0),
         dict(state=False)]


@pytest.mark.parametrize("kw", CASES[:6])
def test_complex_step_copy_equals_c_step(kw):
    case = tiny_case(**kw)
    q = case["q"]
    g = lo.OracleGrid(case["nx"], case["ny"], q=q, coll=case["coll"], ratio=case["ratio"],
                      sponge_width=2, sponge_sigma_max=0.1, source=case["source"],
                      wavelet=case["wavelet"])
    g.set_medium(case["c2"])
    g.set_state(case["rho0"], case["jx0"], case["jy0"])
    tr_c = lo.run(g, case["nsteps"], case["receivers"])["traces"][0]
    tr_p, _ = ad.forward(case, case["c2"])
    np.testing.assert_allclose(tr_p, tr_c, rtol=0, atol=1e-13 * np.abs(tr_c).max())


@pytest.mark.parametrize("kw", CASES)
def test_adjoint_equals_complex_step(kw):
    case = tiny_case(**kw)
    grad, phi = ad.adjoint_gradient(case)
    assert abs(phi - ad.misfit(case, case["c2"])) <= 1e-14 * abs(phi)
    cs = ad.complex_step_gradient(case).reshape(case["ny"], case["nx"])
    err = np.linalg.norm(grad - cs) / np.linalg.norm(cs)
    assert err < 1e-11, err


def test_adjoint_directional_central_difference():
    case = tiny_case(q=5, N=30, seed=3)
    grad, _ = ad.adjoint_gradient(case)
    v = np.random.default_rng(7).standard_normal(case["c2"].shape)
    eps = 1e-6
    fp = ad.misfit(case, case["c2"] + eps * v)
    fm = ad.misfit(case, case["c2"] - eps * v)
    fd = (fp - fm) / (2 * eps)
    assert abs(fd - np.sum(grad * v)) <= 1e-7 * abs(fd)


def test_adjoint_control_wrong_transpose_fails():
    """Control: applying E instead of E^T in the adjoint collision breaks the
    agreement with complex-step derivatives."""
    case = tiny_case(q=5, N=16, seed=5)
    good, _ = ad.adjoint_gradient(case)
    bad, _ = ad.adjoint_gradient(case, _plant_no_transpose=True)
    cs = ad.complex_step_gradient(case).reshape(case["ny"], case["nx"])
    assert np.linalg.norm(good - cs) / np.linalg.norm(cs) < 1e-11
    assert np.linalg.norm(bad - cs) / np.linalg.norm(cs) > 1e-3
