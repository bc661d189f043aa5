"""Fourier-space update operator and dispersion relations (arXiv:1704.03172,
Sec. III B and Appendix E).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

equilibrium_map   g^eq = E g for a homogeneous medium, from eq. D2Q5 dist to
                  eqm dist / eq. D2Q9 dist to eqm dist: E_ij = w_i (1 + c_i.c_j
                  / c^2).  A = I - E is the matrix A of eq. MRT-LB vector.
update_operator   one time step in Fourier space, G(k) = D(k) (I - C A) with
                  D(k) = diag(exp(-i k.c_j)).  The paper writes the product
                  as (I - C A) D(k) (eq. MRT-LB dispersion); the two are
                  similar matrices (same eigenvalues).  The order here is the
                  one a collide-then-stream step applies, so it can be used to
                  evolve a field exactly.
frequencies       omega from eigenvalues lambda = exp(-i omega).
d2q5_cos_omega    closed form of the D2Q5 acoustic pair for omega = 2:
                  cos(omega) = 1 - 2 c^2 [sin^2(kx/2) + sin^2(ky/2)]; at
                  theta = 0 this is Appendix E (eq. appD1Q3 dispersion).
d1q3_characteristic
                  the characteristic polynomial printed in Appendix E.
fourier_evolve    exact evolution of a homogeneous periodic field with a
                  point source, done per wavenumber.

Pins: the printed A of Sec. III B and the App. E polynomial
(tests/test_oracle_dispersion.py); the operator is in turn the pin of the
time stepping in lb_oracle.c.
"""
import numpy as np

from .lb_oracle import VELOCITIES, weights


def equilibrium_map(q, c2, ratio=0.25):
    """E with g^eq = E g for squared sound speed c2 (homogeneous)."""
    c = VELOCITIES[q].astype(np.float64)
    w = weights(q, c2, ratio)
    return w[:, None] * (1.0 + (c @ c.T) / c2)


def a_matrix(q, c2, ratio=0.25):
    """Matrix A of eq. MRT-LB vector: A g = g - g^eq."""
    return np.eye(q) - equilibrium_map(q, c2, ratio)


def collision_step_matrix(q, coll, c2, ratio=0.25):
    """K = I - C A: post-collision populations from pre-collision ones."""
    return np.eye(q) - coll @ a_matrix(q, c2, ratio)


def stream_phase(q, kx, ky):
    """D(k) = diag(exp(-i k.c_j)) (streaming by c_j in Fourier space)."""
    c = VELOCITIES[q]
    return np.diag(np.exp(-1j * (kx * c[:, 0] + ky * c[:, 1])))


def update_operator(q, kx, ky, coll, c2, ratio=0.25):
    """G(k) = D(k) K: one collide-then-stream step for wavenumber (kx, ky)."""
    return stream_phase(q, kx, ky) @ collision_step_matrix(q, coll, c2, ratio)


def paper_operator(q, kx, ky, coll, c2, ratio=0.25):
    """(I - C A) D(k), the product in the order eq. MRT-LB dispersion prints."""
    return collision_step_matrix(q, coll, c2, ratio) @ stream_phase(q, kx, ky)


def frequencies(G):
    """Complex omega of every eigenvalue lambda = exp(-i omega) of G.

    Re(omega) = -arg(lambda); Im(omega) = ln|lambda| (negative = attenuation).
    """
    lam = np.linalg.eigvals(G)
    return -np.angle(lam) + 1j * np.log(np.abs(lam)), lam


def d2q5_cos_omega(c2, kx, ky):
    """cos(omega) of the D2Q5 acoustic pair for omega_relax = 2."""
    return 1.0 - 2.0 * c2 * (np.sin(kx / 2.0) ** 2 + np.sin(ky / 2.0) ** 2)


def d1q3_characteristic(lam, c2, k):
    """Appendix E: (lambda + 1) [lambda^2 - 2 lambda (1 - 2 c^2 sin^2(k/2)) + 1]."""
    b = 1.0 - 2.0 * c2 * np.sin(k / 2.0) ** 2
    return (lam + 1.0) * (lam * lam - 2.0 * lam * b + 1.0)


def fourier_evolve(g0, nsteps, q, coll, c2, ratio=0.25, source=None,
                   wavelet=None):
    """Evolve a homogeneous periodic state g0 (q, ny, nx) by nsteps in
    Fourier space: g_hat(n+1) = D(k) [K g_hat(n) + w S(n) e^{-i k.x_s}].
    Returns the real-space pre-collision state at time nsteps."""
    q_, ny, nx = g0.shape
    assert q_ == q
    gh = np.fft.fft2(g0, axes=(1, 2))
    K = collision_step_matrix(q, coll, c2, ratio)
    w = weights(q, c2, ratio)
    c = VELOCITIES[q]
    kx = 2.0 * np.pi * np.fft.fftfreq(nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)
    KX, KY = np.meshgrid(kx, ky)                     # (ny, nx)
    phase = np.exp(-1j * (c[:, 0, None, None] * KX[None] +
                          c[:, 1, None, None] * KY[None]))   # D(k) diag
    if source is not None:
        xs, ys = source
        src_phase = np.exp(-1j * (KX * xs + KY * ys))
    for n in range(nsteps):
        post = np.einsum("ij,jyx->iyx", K, gh)
        if source is not None and wavelet is not None and n < len(wavelet):
            post = post + w[:, None, None] * wavelet[n] * src_phase[None]
        gh = phase * post
    return np.real(np.fft.ifft2(gh, axes=(1, 2)))
