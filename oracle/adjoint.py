"""Gradient of a receiver-trace misfit with respect to the per-node c^2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The forward model is the recurrence of lb_oracle.c (eq. linear eqm dist,
eq. MRT-LB, eq. MRT-LB linear acoustic, Sec. IV sponge, periodic streaming),
with records p_r(n) = c^2(x_r) rho(x_r, n) (eq. state) for n = 0..N and the
misfit phi = 1/2 sum_r sum_n (p_r(n) - d_r(n))^2.  The paper does not
differentiate its scheme; this module supplies two independent routes to
d phi / d c^2:

complex_step_gradient
    phi(c^2 + i h e_x) evaluated with complex arithmetic through a complex
    copy of the recurrence (step_complex); Im(phi) / h is the derivative to
    machine precision (no subtractive cancellation).  Plain and slow: one
    full forward run per node.
adjoint_gradient
    the discrete adjoint: lambda(N) = r(N); for n = N-1 .. 0
      mu(n)     = (1 - sigma) P^T lambda(n+1)     (mu_i(x) = lambda_i(x + c_i))
      lambda(n) = K^T mu(n) + r(n),  K = I - C (I - E(c^2))
    with r(n) = c^2(x_r) (p_r(n) - d_r(n)) on every population at receiver
    nodes, and
      dphi/dc^2(x) = sum_n rho(x,n) (C^T mu(x,n)) . dw + [x = x_s] S(n) mu . dw
                     + sum_n [x = x_r] (p_r(n) - d_r(n)) rho(x_r, n)
                     + rho(x, 0) lambda(x, 0) . dw          (g(0) = g^eq(rho0, J0))
    where dw = d w / d c^2 (w_i / c^2 does not depend on c^2 for the D2Q5
    weights or the D2Q9 family, so d g^eq / d c^2 = dw rho).
The two are pinned against each other on tiny grids
(tests/test_oracle_adjoint.py); step_complex is pinned against the C step.
"""
import numpy as np

from .lb_oracle import VELOCITIES


def dweights(q, ratio=0.25):
    """d w_i / d c^2 for the weight rule of lb_oracle.c (constant in c^2)."""
    if q == 5:
        return np.array([-2.0, 0.5, 0.5, 0.5, 0.5])
    a = 1.0 / (2.0 + 4.0 * ratio)
    return np.array([-4.0 * a - 4.0 * ratio * a] + [a] * 4 + [ratio * a] * 4)


def weights_c(q, c2, ratio=0.25):
    """Weights for a real or complex c^2 array (same rule as the C code)."""
    if q == 5:
        w1 = 0.5 * c2
        return np.stack([1.0 - 4.0 * w1] + [w1] * 4)
    w1 = c2 / (2.0 + 4.0 * ratio)
    w5 = ratio * w1
    return np.stack([1.0 - 4.0 * w1 - 4.0 * w5] + [w1] * 4 + [w5] * 4)


def sponge_field(nx, ny, L, smax):
    """sigma(x, y) of lb_oracle.c, as an array."""
    if L <= 0:
        return np.zeros((ny, nx))
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    d = np.minimum(np.minimum(x, y), np.minimum(nx - 1 - x, ny - 1 - y))
    f = np.where(d < L, (L - d) / float(L), 0.0)
    return smax * f * f


def equilibrium_c(q, c2, rho, jx, jy, ratio=0.25):
    c = VELOCITIES[q]
    w = weights_c(q, c2, ratio)
    cj = c[:, 0, None, None] * jx[None] + c[:, 1, None, None] * jy[None]
    return w / c2 * (c2 * rho + cj)


def step_complex(g, c2, coll, q, ratio, sigma, src, s_n):
    """One update n -> n+1 on arrays (works for complex g and c^2)."""
    c = VELOCITIES[q]
    rho = g.sum(axis=0)
    jx = np.tensordot(c[:, 0].astype(float), g, axes=1)
    jy = np.tensordot(c[:, 1].astype(float), g, axes=1)
    geq = equilibrium_c(q, c2, rho, jx, jy, ratio)
    gs = g - np.einsum("ij,jyx->iyx", coll, g - geq)
    if src is not None:
        w = weights_c(q, c2, ratio)
        gs[:, src[1], src[0]] = gs[:, src[1], src[0]] + w[:, src[1], src[0]] * s_n
    gs = gs * (1.0 - sigma)
    out = np.empty_like(gs)
    for i in range(q):
        out[i] = np.roll(gs[i], shift=(int(c[i, 1]), int(c[i, 0])), axis=(0, 1))
    return out


def forward(case, c2, record_rho=False):
    """Run the case with the given c^2 (real or complex); returns the
    traces p [nrec][N+1] and optionally rho at every time [N+1][ny][nx]."""
    q, nx, ny, N = case["q"], case["nx"], case["ny"], case["nsteps"]
    ratio = case.get("ratio", 0.25)
    coll = case["coll"]
    sigma = sponge_field(nx, ny, case.get("sponge_width", 0), case.get("sponge_sigma_max", 0.0))
    rec = np.asarray(case["receivers"])
    rho0 = case.get("rho0", np.zeros((ny, nx)))
    jx0 = case.get("jx0", np.zeros((ny, nx)))
    jy0 = case.get("jy0", np.zeros((ny, nx)))
    g = equilibrium_c(q, c2, rho0 + 0 * c2, jx0 + 0 * c2, jy0 + 0 * c2, ratio)
    wav = case.get("wavelet", np.zeros(0))
    src = case.get("source")
    tr = np.zeros((len(rec), N + 1), dtype=g.dtype)
    rhos = [] if record_rho else None

    def record(k, g):
        rho = g.sum(axis=0)
        tr[:, k] = c2[rec[:, 1], rec[:, 0]] * rho[rec[:, 1], rec[:, 0]]
        if record_rho:
            rhos.append(rho.copy())

    record(0, g)
    for n in range(N):
        s_n = float(wav[n]) if n < len(wav) else 0.0
        g = step_complex(g, c2, coll, q, ratio, sigma, src, s_n)
        record(n + 1, g)
    return tr, (np.array(rhos) if record_rho else None)


def misfit(case, c2):
    tr, _ = forward(case, c2)
    r = tr - case["d_obs"]
    return 0.5 * np.sum(r * r)


def complex_step_gradient(case, nodes=None, h=1e-30):
    """d phi / d c^2 at the listed (x, y) nodes (all nodes by default)."""
    nx, ny = case["nx"], case["ny"]
    c2 = np.asarray(case["c2"], dtype=np.float64)
    if nodes is None:
        nodes = [(x, y) for y in range(ny) for x in range(nx)]
    out = np.zeros(len(nodes))
    for k, (x, y) in enumerate(nodes):
        cz = c2.astype(np.complex128)
        cz[y, x] += 1j * h
        out[k] = np.imag(misfit(case, cz)) / h
    return out


def adjoint_gradient(case, _plant_no_transpose=False):
    """Discrete adjoint gradient d phi / d c^2 over the whole grid (FP64).

    _plant_no_transpose applies E instead of E^T in K^T; it exists only for
    the control test that shows the pins catch such a mistake.  (Streaming
    the adjoint the wrong way is not a usable control: for these isotropic
    collisions the mirrored recursion yields exactly the velocity-reversed
    adjoint and the same gradient.)"""
    q, nx, ny, N = case["q"], case["nx"], case["ny"], case["nsteps"]
    ratio = case.get("ratio", 0.25)
    coll = case["coll"]
    c = VELOCITIES[q]
    c2 = np.asarray(case["c2"], dtype=np.float64)
    sigma = sponge_field(nx, ny, case.get("sponge_width", 0), case.get("sponge_sigma_max", 0.0))
    rec = np.asarray(case["receivers"])
    tr, rho = forward(case, c2, record_rho=True)
    res = tr - case["d_obs"]                        # dphi/dp_r(n)
    wav = case.get("wavelet", np.zeros(0))
    src = case.get("source")
    dw = dweights(q, ratio)
    w = weights_c(q, c2, ratio)
    woc = w / c2                                     # w_i / c^2
    grad = np.zeros((ny, nx))

    def inject(lam, n):
        for r, (x, y) in enumerate(rec):
            lam[:, y, x] += c2[y, x] * res[r, n]
            grad[y, x] += res[r, n] * rho[n][y, x]

    def KT(mu):
        # K^T mu = mu - (I - E^T) C^T mu,  (E^T v)_j = sum_i w_i v_i + c_j . sum_i (w_i/c^2) c_i v_i
        nu = np.einsum("ji,jyx->iyx", coll, mu)
        if _plant_no_transpose:   # (E v)_i = w_i (sum_j v_j + c_i . sum_j c_j v_j / c^2)
            s0 = nu.sum(axis=0)
            sx = (c[:, 0, None, None] * nu).sum(axis=0) / c2
            sy = (c[:, 1, None, None] * nu).sum(axis=0) / c2
            et = w * (s0[None] + c[:, 0, None, None] * sx[None] + c[:, 1, None, None] * sy[None])
            return mu - nu + et
        s0 = (w * nu).sum(axis=0)
        sx = (woc * c[:, 0, None, None] * nu).sum(axis=0)
        sy = (woc * c[:, 1, None, None] * nu).sum(axis=0)
        et = s0[None] + c[:, 0, None, None] * sx[None] + c[:, 1, None, None] * sy[None]
        return mu - nu + et

    lam = np.zeros((q, ny, nx))
    inject(lam, N)
    for n in range(N - 1, -1, -1):
        mu = np.empty_like(lam)
        for i in range(q):                         # mu_i(x) = lam_i(x + c_i)
            mu[i] = np.roll(lam[i], shift=(-int(c[i, 1]), -int(c[i, 0])), axis=(0, 1))
        mu *= (1.0 - sigma)
        nu = np.einsum("ji,jyx->iyx", coll, mu)    # C^T mu
        grad += rho[n] * np.tensordot(dw, nu, axes=1)
        if src is not None and n < len(wav):
            grad[src[1], src[0]] += float(wav[n]) * (dw @ mu[:, src[1], src[0]])
        lam = KT(mu)
        inject(lam, n)
    grad += rho[0] * np.tensordot(dw, lam, axes=1)
    return grad, 0.5 * np.sum(res * res)
