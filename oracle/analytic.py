"""Analytic pressure of a point source in a homogeneous 2D medium
(arXiv:1704.03172, Sec. V A, eq. source, eq. tau, eq. exact solution).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

ricker / ricker_dot
    S(t) = -(1 - 4 xi^2) exp(-2 xi^2), xi = (2 pi f_c / 3)(t - 3 / (2 f_c)),
    and its time derivative (written out by hand).
pressure_freq
    eq. exact solution evaluated as printed: p_hat(omega) =
    -(i/4) FT[dS/dt](omega) H0^(2)(omega r / c), inverse-transformed with an
    FFT (time dependence exp(+i omega t), outgoing waves for H^(2)).
pressure_time
    the same solution in the time domain: the 2D Green's function of
    (1/c^2) p_tt - lap p = dS/dt delta(x) convolved with dS/dt, written with
    t' = (r/c) cosh(u):  p(r, t) = (1/2 pi) int_0^inf S'(t - (r/c) cosh u) du.
The two routes share nothing but the wavelet and pin each other
(tests/test_oracle_analytic.py); both are then the pin of the LB recurrence
at physics-level tolerance.
"""
import numpy as np
from scipy import special


def ricker(t, fc):
    """eq. source with eq. tau (source wavelet, without the delta)."""
    xi = (2.0 * np.pi * fc / 3.0) * (np.asarray(t, dtype=np.float64) - 1.5 / fc)
    return -(1.0 - 4.0 * xi * xi) * np.exp(-2.0 * xi * xi)


def ricker_dot(t, fc):
    """dS/dt of the wavelet: a * exp(-2 xi^2) (12 xi - 16 xi^3), a = 2 pi fc / 3."""
    a = 2.0 * np.pi * fc / 3.0
    xi = a * (np.asarray(t, dtype=np.float64) - 1.5 / fc)
    return a * np.exp(-2.0 * xi * xi) * (12.0 * xi - 16.0 * xi ** 3)


def pressure_time(r, c, t, fc, du=2e-4):
    """Time-domain point-source pressure at distance r, speed c, times t."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    tr = r / c
    tmax = t.max() + 8.0 / fc
    umax = np.arccosh(max(tmax / tr, 1.0 + 1e-12)) + 0.5
    u = np.arange(0.0, umax + du, du)
    delay = tr * np.cosh(u)                       # (nu,)
    vals = ricker_dot(t[:, None] - delay[None, :], fc)
    wts = np.full(u.size, du)
    wts[0] = wts[-1] = 0.5 * du
    return (vals @ wts) / (2.0 * np.pi)


def pressure_freq(r, c, t, fc, dt=0.25, nfft=1 << 18):
    """eq. exact solution by FFT: p = IFT[-(i/4) FT(S') H0^(2)(omega r / c)]."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    ts = np.arange(nfft) * dt
    sd = ricker_dot(ts, fc)
    sd_hat = np.fft.rfft(sd) * dt                 # continuous FT approximation
    omega = 2.0 * np.pi * np.fft.rfftfreq(nfft, d=dt)
    h = np.zeros_like(sd_hat)
    pos = omega > 0
    h[pos] = -0.25j * special.hankel2(0, omega[pos] * r / c)
    p = np.fft.irfft(sd_hat * h, n=nfft) / dt
    return np.interp(t, ts, p)
