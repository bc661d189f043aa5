"""Seeded synthetic inputs for the linear lattice Boltzmann acoustic workloads.

This module only builds input arrays (media, source wavelet samples, initial
fields, receiver lists); it holds none of the scheme's arithmetic.  Both the
GPU path and the CPU oracle are fed from here, so that the two see the same
inputs.  All speeds are lattice units (dx = dt = 1), y is depth with row 0 at
the top, and every random draw is seeded.

Workloads (scaled to the paper's experiments, Sec. V of arXiv:1704.03172,
which uses a homogeneous or two-medium setup, a Ricker-type point source and
at least ~16 points per wavelength):

  pulse_workload      periodic homogeneous grid with a Gaussian density
                      pulse (128 x 128, c^2 = 1/3, sigma = 6, amplitude 1e-3)
  layered_workload    two-layer medium with 2:1 speed contrast at mid-depth
                      plus 20 seeded Gaussian anomalies of +-10 % (4096^2 at
                      full size), 64-node sponge, source near the surface,
                      256 surface receivers
  refined_workload    2048^2 background c = 0.5 with a low-velocity lens
                      (c = 0.25) covered by a factor-2 refined patch
"""
import math
import numpy as np


# ---------------------------------------------------------------------------
# source wavelet (eq. source with eq. tau), sampled at integer steps
# ---------------------------------------------------------------------------
def ricker_wavelet(nt, fc, dt=1.0):
    """S(n dt) = -(1 - 4 xi^2) exp(-2 xi^2), xi = (2 pi fc / 3)(t - 3/(2 fc))."""
    t = np.arange(int(nt), dtype=np.float64) * dt
    xi = (2.0 * math.pi * fc / 3.0) * (t - 1.5 / fc)
    return -(1.0 - 4.0 * xi * xi) * np.exp(-2.0 * xi * xi)


# ---------------------------------------------------------------------------
# initial fields
# ---------------------------------------------------------------------------
def gaussian_pulse(nx, ny, sigma=6.0, amp=1e-3, center=None):
    """rho(x, 0) = amp exp(-|x - x0|^2 / (2 sigma^2)), 0-based nodes,
    plain (non-wrapped) distance; x0 defaults to (nx/2, ny/2)."""
    cx, cy = (nx // 2, ny // 2) if center is None else center
    x = np.arange(nx, dtype=np.float64)[None, :] - cx
    y = np.arange(ny, dtype=np.float64)[:, None] - cy
    return amp * np.exp(-(x * x + y * y) / (2.0 * sigma * sigma))


def random_fields(nx, ny, seed, amp=1e-3):
    """Seeded smooth-free random rho, Jx, Jy (for operator-level tests)."""
    rng = np.random.default_rng(seed)
    return (amp * rng.standard_normal((ny, nx)),
            amp * 0.1 * rng.standard_normal((ny, nx)),
            amp * 0.1 * rng.standard_normal((ny, nx)))


# ---------------------------------------------------------------------------
# media
# ---------------------------------------------------------------------------
def _add_anomalies(c, n_anom, seed, margin, sig_lo, sig_hi, amp=0.1):
    """c *= 1 + sum_k a_k exp(-|x - x_k|^2 / (2 s_k^2)), a_k ~ U[-amp, amp];
    centres at least `margin` nodes (at most a quarter of the axis) inside."""
    ny, nx = c.shape
    rng = np.random.default_rng(seed)
    mx, my = min(margin, nx / 4.0), min(margin, ny / 4.0)
    xs = rng.uniform(mx, nx - mx, n_anom)
    ys = rng.uniform(my, ny - my, n_anom)
    sg = rng.uniform(sig_lo, sig_hi, n_anom)
    aa = rng.uniform(-amp, amp, n_anom)
    bump = np.zeros_like(c)
    for k in range(n_anom):
        r = int(math.ceil(6.0 * sg[k]))
        x0, x1 = max(0, int(xs[k]) - r), min(nx, int(xs[k]) + r + 1)
        y0, y1 = max(0, int(ys[k]) - r), min(ny, int(ys[k]) + r + 1)
        xx = np.arange(x0, x1, dtype=np.float64)[None, :] - xs[k]
        yy = np.arange(y0, y1, dtype=np.float64)[:, None] - ys[k]
        bump[y0:y1, x0:x1] += aa[k] * np.exp(-(xx * xx + yy * yy) / (2.0 * sg[k] ** 2))
    return c * (1.0 + bump)


def two_layer_speed(nx, ny, c_top=0.25, c_bottom=0.5, n_anom=20, seed=1704):
    """Two layers (interface at mid-depth) plus seeded Gaussian anomalies.

    At 4096^2: centres U[64, 4032)^2, widths U[32, 128], amplitudes
    U[-0.1, 0.1]; sizes scale with the grid for smaller grids.
    """
    c = np.where(np.arange(ny)[:, None] < ny // 2, c_top, c_bottom) * np.ones((1, nx))
    s = nx / 4096.0
    return _add_anomalies(c, n_anom, seed, margin=max(2.0, 64.0 * s),
                          sig_lo=max(1.0, 32.0 * s), sig_hi=max(2.0, 128.0 * s))


def surface_receivers(nx, nrec, y, margin):
    """nrec receivers on row y, evenly spaced over [margin, nx - 1 - margin]."""
    span = nx - 1 - 2 * margin
    xs = [margin + int(round(r * span / (nrec - 1))) for r in range(nrec)]
    return np.array([(x, y) for x in xs], dtype=np.int32)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def pulse_workload(n=128, c2=1.0 / 3.0, sigma=6.0, amp=1e-3, nsteps=500):
    """Periodic homogeneous grid, Gaussian pulse at the centre, J = 0."""
    return {
        "nx": n, "ny": n, "c2": np.full((n, n), c2),
        "rho0": gaussian_pulse(n, n, sigma, amp), "nsteps": nsteps,
        "tau": 1.0, "sponge_width": 0, "sponge_sigma_max": 0.0,
    }


def layered_workload(n=4096, nsteps=4000, nrec=256, seed=1704):
    """Two-layer medium with anomalies, sponge, Ricker source, receivers.

    Full size: 4096^2, sponge 64 nodes (sigma_max 0.1), source at (n/2, 64),
    fc = c_min / 20 (>= 20 nodes per wavelength), 256 receivers on row 64.
    Smaller n scales the sponge, depth and receiver count down.
    """
    c = two_layer_speed(n, n, seed=seed)
    L = 64 if n >= 1024 else max(4, n // 16)
    depth = L
    nrec = min(nrec, n - 2 * L - 1)
    cmin = float(c.min())
    fc = cmin / 20.0
    return {
        "nx": n, "ny": n, "c2": c * c, "nsteps": nsteps,
        "sponge_width": L, "sponge_sigma_max": 0.1,
        "source": (n // 2, depth), "fc": fc,
        "wavelet": ricker_wavelet(nsteps + 1, fc),
        "receivers": surface_receivers(n, nrec, depth, L),
    }


def refined_workload(n=2048, nsteps=3000, nrec=128, lens_speed=0.25,
                     c_bg=0.5, fc=0.025, patch=None, lens_inset=16,
                     sponge_width=64):
    """Background c_bg with a low-velocity lens under a factor-2 patch.

    Full size: coarse 2048^2, patch coarse x in [768, 1280), y in [512, 768)
    (1024 x 512 fine nodes), lens = patch interior shrunk by 16 coarse cells,
    source at (n/2, 64), 128 receivers on row 64 over [64, n - 65].
    Returns coarse and fine c^2 (fine nodes sampled at their own positions).
    """
    if patch is None:
        patch = (3 * n // 8, n // 4, n // 4, n // 8)
    px0, py0, pnx, pny = patch
    oo = 2

    def speed_at(xc, yc):
        inside = ((xc >= px0 + lens_inset) & (xc < px0 + pnx - lens_inset) &
                  (yc >= py0 + lens_inset) & (yc < py0 + pny - lens_inset))
        return np.where(inside, lens_speed, c_bg)

    xc = np.arange(n, dtype=np.float64)[None, :]
    yc = np.arange(n, dtype=np.float64)[:, None]
    c_coarse = speed_at(xc, yc) * np.ones((n, n))
    X0, Y0 = px0 - oo, py0 - oo
    nxf, nyf = 2 * (pnx + 2 * oo) + 1, 2 * (pny + 2 * oo) + 1
    xf = X0 + np.arange(nxf, dtype=np.float64)[None, :] / 2.0
    yf = Y0 + np.arange(nyf, dtype=np.float64)[:, None] / 2.0
    c_fine = speed_at(xf, yf) * np.ones((nyf, nxf))
    L = sponge_width
    depth = L
    return {
        "nx": n, "ny": n, "c2": c_coarse ** 2, "c2_fine": c_fine ** 2,
        "patch": patch, "overlap_out": oo, "overlap_in": 2,
        "nsteps": nsteps, "sponge_width": L, "sponge_sigma_max": 0.1,
        "source": (n // 2, depth), "fc": fc,
        "wavelet": ricker_wavelet(nsteps + 1, fc),
        "receivers": surface_receivers(n, nrec, depth, L),
    }


# ---------------------------------------------------------------------------
# serving: a seeded trace of shot requests
# ---------------------------------------------------------------------------
def serving_trace(nreq=1000, rate=50.0, seed=4, sizes=None, steps=(1000, 4000)):
    """Poisson arrivals (mean `rate` per second) of shot requests.

    Each request: square grid n uniform over {256, 512, ..., 4096}; a layered
    medium of 3-8 layers (sorted interface depths U(0, n), speeds
    U[0.3, 0.57]) with 1-5 Gaussian blobs (+-10 %, sigma U[n/64, n/16]); a
    Ricker source at (U[L, n-L), L) with fc = c_min / 20; 128 receivers on
    row L; steps U{steps}; sponge L = min(64, n/8).
    """
    rng = np.random.default_rng(seed)
    sizes = list(range(256, 4097, 256)) if sizes is None else list(sizes)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
    reqs = []
    for i in range(nreq):
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        nl = int(rng.integers(3, 9))
        depths = np.sort(rng.uniform(0, n, nl - 1))
        speeds = rng.uniform(0.3, 0.57, nl)
        nb = int(rng.integers(1, 6))
        blobs = [(float(rng.uniform(0, n)), float(rng.uniform(0, n)),
                  float(rng.uniform(n / 64.0, n / 16.0)), float(rng.uniform(-0.1, 0.1)))
                 for _ in range(nb)]
        L = min(64, n // 8)
        sx = int(rng.integers(L, n - L))
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        reqs.append({"rid": i, "arrival": float(arrivals[i]), "n": n, "depths": depths,
                     "speeds": speeds, "blobs": blobs, "sponge": L, "src": (sx, L),
                     "nsteps": nsteps, "nrec": 128})
    return reqs


def serving_speed_numpy(req):
    """Sound speed of a serving request (host, FP64): layer speed times
    (1 + bump), bump = sum of blobs clipped to +-10 %."""
    n = req["n"]
    y = np.arange(n, dtype=np.float64)[:, None]
    x = np.arange(n, dtype=np.float64)[None, :]
    layer = np.searchsorted(req["depths"], np.arange(n), side="right")
    cl = np.asarray(req["speeds"])[layer][:, None]
    bump = np.zeros((n, n))
    for bx, by, sg, a in req["blobs"]:
        bump += a * np.exp(-((x - bx) ** 2 + (y - by) ** 2) / (2.0 * sg * sg))
    return cl * (1.0 + np.clip(bump, -0.1, 0.1))


def serving_speed_torch(req, device):
    """The same medium built with torch on a device (for the serving loop,
    where host-side generation would stall admission)."""
    import torch
    n = req["n"]
    y = torch.arange(n, dtype=torch.float64, device=device)[:, None]
    x = torch.arange(n, dtype=torch.float64, device=device)[None, :]
    layer = np.searchsorted(req["depths"], np.arange(n), side="right")
    cl = torch.as_tensor(np.asarray(req["speeds"])[layer], dtype=torch.float64, device=device)[:, None]
    bump = torch.zeros((n, n), dtype=torch.float64, device=device)
    for bx, by, sg, a in req["blobs"]:
        bump += a * torch.exp(-((x - bx) ** 2 + (y - by) ** 2) / (2.0 * sg * sg))
    return cl * (1.0 + torch.clamp(bump, -0.1, 0.1))


def serving_receivers(req):
    L = req["sponge"]
    return surface_receivers(req["n"], req["nrec"], L, L)


def serving_min_speed(req):
    """Lower bound of the request's sound speed: slowest layer, blobs at -10 %."""
    return float(np.min(req["speeds"])) * 0.9


def serving_wavelet(req):
    """Ricker wavelet at fc = c_min / 20 (>= 20 nodes per wavelength), from
    the request's speed bound so that no device read is needed."""
    return ricker_wavelet(req["nsteps"] + 1, serving_min_speed(req) / 20.0)


# ---------------------------------------------------------------------------
# adjoint workload: a multi-shot gradient of the trace misfit
# ---------------------------------------------------------------------------
def adjoint_workload(n=2048, nshots=16, nsteps=3000, nrec=128, seed=55, smooth=32.0):
    """True medium: 5 layers with speeds increasing 0.3 -> 0.55 with depth
    plus 20 seeded +-10 % anomalies; starting medium: the true one smoothed by
    a Gaussian of `smooth` nodes.  Sources on row 64 at x = 64 + (k + 1/2) *
    (n - 128) / nshots; shared receivers on row 64; fc = c_min / 20."""
    from scipy import ndimage
    speeds = np.linspace(0.3, 0.55, 5)
    layer = np.minimum((np.arange(n) * 5) // n, 4)
    c = speeds[layer][:, None] * np.ones((1, n))
    s = n / 4096.0
    c = _add_anomalies(c, 20, seed, margin=max(2.0, 64.0 * s), sig_lo=max(1.0, 32.0 * s),
                       sig_hi=max(2.0, 128.0 * s))
    c0 = ndimage.gaussian_filter(c, sigma=smooth * n / 2048.0, mode="nearest")
    L = 64 if n >= 1024 else max(4, n // 16)
    fc = float(min(c.min(), c0.min())) / 20.0
    xs = [int(L + (k + 0.5) * (n - 2 * L) / nshots) for k in range(nshots)]
    return {"nx": n, "ny": n, "c2_true": c * c, "c2_init": c0 * c0, "nsteps": nsteps,
            "sources": [(x, L) for x in xs], "receivers": surface_receivers(n, nrec, L, L),
            "sponge_width": L, "sponge_sigma_max": 0.1, "fc": fc,
            "wavelet": ricker_wavelet(nsteps + 1, fc)}
