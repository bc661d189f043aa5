"""Oracle pins against the matrices and constants the paper prints.

arXiv:1704.03172: Table I and Appendix A (velocities, M), Sec. III B (the
matrix A of eq. MRT-LB vector), Sec. II C (weight constraints, equilibrium
moments e^(0), pxx^(0)), Appendix B (M^-1, E_x, E_y, m^eq), Appendix D
(Courant number vs rest weight).
"""
import json
import os

import numpy as np
import pytest

from oracle import lb_oracle as lo
from oracle import dispersion as ds
from tests.conftest import GOLDEN


def test_velocity_order_matches_appendix_a():
    # Rows 1 and 2 of M are the x and y momenta: they list c_ix and c_iy.
    for q in (5, 9):
        M = lo.transformation_matrix(q)
        c = lo.VELOCITIES[q]
        np.testing.assert_array_equal(M[1], c[:, 0])
        np.testing.assert_array_equal(M[2], c[:, 1])
        np.testing.assert_array_equal(M[0], np.ones(q))


def test_moment_basis_orthogonal():
    # The moment vectors of Appendix A are mutually orthogonal.
    for q in (5, 9):
        M = lo.transformation_matrix(q)
        G = M @ M.T
        np.testing.assert_allclose(G - np.diag(np.diag(G)), 0.0, atol=0)


def test_printed_minv_d2q5(golden):
    Minv = np.linalg.solve(lo.M_D2Q5, np.eye(5))
    np.testing.assert_allclose(Minv, golden("appB_d2q5_Minv.txt"), atol=1e-15)


def test_printed_ex_ey_d2q5(golden):
    M = lo.M_D2Q5
    Minv = np.linalg.solve(M, np.eye(5))
    c = lo.VELOCITIES[5]
    Ex = M @ np.diag(c[:, 0]) @ Minv
    Ey = M @ np.diag(c[:, 1]) @ Minv
    np.testing.assert_allclose(Ex, golden("appB_d2q5_Ex.txt"), atol=1e-15)
    np.testing.assert_allclose(Ey, golden("appB_d2q5_Ey.txt"), atol=1e-15)


def _printed_a_d2q5(w, c2):
    """The matrix A of Sec. III B as printed (entries transcribed)."""
    k = 1.0 / c2
    w0, w1, w2, w3, w4 = w
    return np.array([
        [1 - w0, -w0, -w0, -w0, -w0],
        [-w1, 1 - w1 * (1 + k), -w1, -w1 * (1 - k), -w1],
        [-w2, -w2, 1 - w2 * (1 + k), -w2, -w2 * (1 - k)],
        [-w3, -w3 * (1 - k), -w3, 1 - w3 * (1 + k), -w3],
        [-w4, -w4, -w4 * (1 - k), -w4, 1 - w4 * (1 + k)],
    ])


@pytest.mark.parametrize("c2", [0.1, 0.25, 1.0 / 3.0, 0.5])
def test_printed_a_matrix_d2q5(c2):
    w = lo.weights(5, c2)
    np.testing.assert_allclose(ds.a_matrix(5, c2), _printed_a_d2q5(w, c2),
                               atol=1e-14)


def test_d1q3_a_matrix_appendix_e():
    # Appendix E prints A for D1Q3 (w1 = w2 = w, w0 = 1 - 2w, c^2 = 2w);
    # build it from the D1Q3 velocities and weights by the same rule as the
    # 2D lattices (g^eq = E g, A = I - E) and compare entry-wise.
    for wv in (0.1, 0.2, 0.25):
        c2 = 2 * wv
        k = 1.0 / c2
        printed = np.array([
            [2 * wv, 2 * wv - 1, 2 * wv - 1],
            [-wv, 1 - wv * (1 + k), -wv * (1 - k)],
            [-wv, -wv * (1 - k), 1 - wv * (1 + k)],
        ])
        c = np.array([0.0, 1.0, -1.0])
        w = np.array([1 - 2 * wv, wv, wv])
        A = np.eye(3) - w[:, None] * (1 + np.outer(c, c) / c2)
        np.testing.assert_allclose(A, printed, atol=1e-14)


@pytest.mark.parametrize("c2", [0.05, 0.2, 0.3, 0.5])
def test_equilibrium_moments_d2q5(c2):
    # Sec. II C / App. B: M g^eq = (rho, Jx, Jy, -4 rho + 10 rho c^2, 0).
    g = lo.OracleGrid(1, 1, q=5)
    g.set_medium(np.full((1, 1), c2))
    rho, jx, jy = 0.7, -0.3, 0.11
    g.set_state(np.full((1, 1), rho), np.full((1, 1), jx), np.full((1, 1), jy))
    meq = lo.M_D2Q5 @ g.g[:, 0, 0]
    np.testing.assert_allclose(meq, [rho, jx, jy, -4 * rho + 10 * rho * c2, 0.0],
                               atol=1e-15)


@pytest.mark.parametrize("q,ratio", [(5, 0.25), (9, 0.25), (9, 24.0), (9, 0.0)])
def test_weight_constraints(q, ratio):
    # eq. LB lattice moments: sum w = 1, sum w c c = c^2 I, odd moments 0.
    c = lo.VELOCITIES[q].astype(float)
    for c2 in (0.05, 0.2, 1.0 / 3.0, 0.45):
        w = lo.weights(q, c2, ratio)
        assert abs(w.sum() - 1) < 1e-15
        T = np.einsum("i,ia,ib->ab", w, c, c)
        np.testing.assert_allclose(T, c2 * np.eye(2), atol=1e-15)
        np.testing.assert_allclose(w @ c, 0.0, atol=1e-15)
    # and the C implementation gives the same numbers
    g = lo.OracleGrid(1, 1, q=q, ratio=ratio)
    import ctypes
    for c2 in (0.1, 0.3):
        out = np.zeros(q)
        lo._lib().orc_node_weights(ctypes.byref(g._p), c2, lo._dptr(out))
        np.testing.assert_allclose(out, lo.weights(q, c2, ratio), rtol=1e-15)


def test_paper_weight_constants():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        k = json.load(f)
    # D2Q5 homogeneous eta = 1 (c^2 = c_max^2 = 1/2): w0 = 0, w1 = 1/4.
    w = lo.weights(5, 0.5)
    np.testing.assert_allclose([w[0], w[1]], k["d2q5_homogeneous_weights"]["value"], atol=1e-16)
    # conventional D2Q9 weights are the ratio-1/4 family at c^2 = 1/3
    w = lo.weights(9, 1.0 / 3.0, 0.25)
    np.testing.assert_allclose([w[0], w[1], w[5]], k["d2q9_conventional_weights"]["value"], atol=1e-16)
    # simulation weights (0, 0.01, 0.24) are ratio 24 at c^2 = 2*0.01 + 4*0.24
    for key in ("d2q9_simulation_weights", "d2q9_optimum_weights"):
        w0, w1, w5 = k[key]["value"]
        c2 = 2 * w1 + 4 * w5
        w = lo.weights(9, c2, w5 / w1)
        np.testing.assert_allclose([w[0], w[1], w[5]], [w0, w1, w5], atol=1e-15)


def test_courant_rest_weight_appendix_d():
    # C = sqrt((1 - w0) / 2); w0 = 0 gives C_max = 1/sqrt(2).
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        cmax = json.load(f)["d2q5_max_courant"]["value"]
    for c2 in (0.01, 0.1, 0.3, 0.5):
        w0 = lo.weights(5, c2)[0]
        assert abs(np.sqrt((1 - w0) / 2) - np.sqrt(c2)) < 1e-15
    assert abs(np.sqrt((1 - lo.weights(5, 0.5)[0]) / 2) - cmax) < 1e-15


def test_bgk_is_mrt_with_equal_rates():
    # Sec. II B: with all inverse relaxation times equal, MRT is BGK.
    for q in (5, 9):
        for tau in (0.5, 0.8, 1.0):
            C = lo.collision_matrix(q, "mrt", s=np.full(q, 1.0 / tau))
            np.testing.assert_allclose(C, np.eye(q) / tau, atol=1e-14)
