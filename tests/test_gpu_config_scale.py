"""GPU parity at the sizes and lengths of the configured workloads.

* Layered workload (Sec. V A scaled: two-layer medium with 20 anomalies,
  sponge, Ricker source, 256 surface receivers) at 1024^2 for the full 4000
  steps, every lattice and collision, through the blocked path the benchmark
  times: the whole [field][receiver][4001] trace array and the rho and J
  snapshots at T/4 and T/2 against the FP64 oracle at the FP32 bar, and an
  FP64 run cut to 500 steps at the FP64 bar.
* Refinement (Sec. IV, Sec. V B) at its configured geometry: 2048^2 coarse
  grid, 1024 x 512 fine patch over a 0.5x-speed lens, MRT s = (1, 1, 1, 2, 2),
  FP32, from a random state on both grids so that the interface carries
  signal from the first step.
* Adjoint at scale: central differences of FP64 GPU forward runs at 10
  seeded nodes of one 2048^2 x 3000-step shot of the adjoint workload, and
  an FP64 dot-product test of the adjoint against the oracle's complex-step
  tangent.

Errors are printed; bars are relative L2 norms against the oracle
(FP32 1e-5, FP64 1e-12).
"""
import numpy as np
import pytest

from oracle import adjoint as ad
from oracle import lb_oracle as lo
from oracle import refine as rf
from paper_1704_03172_amd import inputs
from tests.harness import FIELDS, make_grid, rel_l2

pytestmark = pytest.mark.gpu

MRT5 = [1, 1, 1, 2, 2]
MRT9 = [1, 1, 1, 2, 2, 2, 1, 1, 2]
VARIANTS = [(5, "bgk", None), (5, "mrt", MRT5), (9, "bgk", None), (9, "mrt", MRT9)]


def layered_case(n, nsteps, q, collision, s):
    wl = inputs.layered_workload(n=n, nsteps=nsteps)
    return {"nx": n, "ny": n, "q": q, "collision": collision, "tau": 0.5, "s": s, "ratio": 0.25,
            "c2": wl["c2"], "nsteps": nsteps, "sponge_width": wl["sponge_width"],
            "sponge_sigma_max": wl["sponge_sigma_max"], "source": wl["source"],
            "wavelet": wl["wavelet"], "receivers": wl["receivers"]}


def oracle_layered(case, snapshots):
    g = lo.OracleGrid(case["nx"], case["ny"], q=case["q"], collision=case["collision"],
                      tau=case["tau"], s=case["s"], ratio=case["ratio"],
                      sponge_width=case["sponge_width"], sponge_sigma_max=case["sponge_sigma_max"],
                      source=case["source"], wavelet=case["wavelet"])
    g.set_medium(case["c2"])
    g.set_state(np.zeros((case["ny"], case["nx"])))
    return lo.run(g, case["nsteps"], case["receivers"], fields=FIELDS, snapshots=snapshots)


def gpu_layered(case, precision, snapshots):
    """The run as lb_step_n takes it without sum-of-rho recording (several
    steps per launch), stopping at the snapshot times to read the fields."""
    g = make_grid(case, precision)
    g.set_medium(case["c2"])
    g.set_source(case["source"][0], case["source"][1], case["wavelet"])
    tr = g.record(case["receivers"], fields=FIELDS)
    snap = {}
    for t in list(snapshots) + [case["nsteps"]]:
        g.step(t - g.time)
        if t in snapshots:
            snap[t] = {f: g.field(f).cpu().numpy() for f in ("rho", "jx", "jy")}
    g.sync()
    out = {"traces": tr.cpu().numpy(), "snap": snap}
    g.close()
    return out


def momentum_error(gx, gy, rx, ry):
    """Relative L2 error of the momentum J = (Jx, Jy) as a vector field:
    ||(gx - rx, gy - ry)|| / ||(rx, ry)||.  One component alone can be
    small by symmetry (Jy on the source row, where the direct wave runs
    along the row), and its error, set by the rounding of populations of
    the size of rho, is then not small relative to that component."""
    d = np.hypot(np.linalg.norm(np.asarray(gx, np.float64) - rx), np.linalg.norm(np.asarray(gy, np.float64) - ry))
    return d / np.hypot(np.linalg.norm(rx), np.linalg.norm(ry))


def layered_errors(case, precision, snapshots):
    """Errors that the bars apply to (p, rho, J as a vector, for the traces
    and the snapshots) and, for information, the J components alone and the
    ratio of their trace norms."""
    ref = oracle_layered(case, snapshots)
    gpu = gpu_layered(case, precision, snapshots)
    gt, rt = gpu["traces"], ref["traces"]
    errs = {"trace_p": rel_l2(gt[0], rt[0]), "trace_rho": rel_l2(gt[1], rt[1]),
            "trace_J": momentum_error(gt[2], gt[3], rt[2], rt[3])}
    info = {"trace_jx": rel_l2(gt[2], rt[2]), "trace_jy": rel_l2(gt[3], rt[3]),
            "|jy|/|jx|": np.linalg.norm(rt[3]) / np.linalg.norm(rt[2])}
    for t in snapshots:
        gs, rs = gpu["snap"][t], ref["snap"][t]
        errs["rho@%d" % t] = rel_l2(gs["rho"], rs["rho"])
        errs["J@%d" % t] = momentum_error(gs["jx"], gs["jy"], rs["jx"], rs["jy"])
        info["jx@%d" % t] = rel_l2(gs["jx"], rs["jx"])
        info["jy@%d" % t] = rel_l2(gs["jy"], rs["jy"])
    assert np.linalg.norm(rt[0]) > 0
    print("  components (not barred):", " ".join("%s %.2e" % kv for kv in sorted(info.items())))
    return errs


@pytest.mark.parametrize("q,collision,s", VARIANTS)
def test_layered_1024_full_length_f32(q, collision, s):
    """4000 steps, FP32 populations, blocked path: traces [4][256][4001] and
    rho / J at n = 1000 and 2000 within 1e-5 of the FP64 oracle."""
    case = layered_case(1024, 4000, q, collision, s)
    errs = layered_errors(case, "f32", (1000, 2000))
    print("D2Q%d %s FP32 1024^2 x 4000:" % (q, collision), " ".join("%s %.2e" % kv for kv in sorted(errs.items())))
    bad = {k: v for k, v in errs.items() if not v <= 1e-5}
    assert not bad, bad


@pytest.mark.parametrize("q,collision,s", VARIANTS)
def test_layered_1024_fp64_cut(q, collision, s):
    """The same workload in FP64, cut to 500 steps: within 1e-12."""
    case = layered_case(1024, 500, q, collision, s)
    errs = layered_errors(case, "f64", (250, 400))
    print("D2Q%d %s FP64 1024^2 x 500:" % (q, collision), " ".join("%s %.2e" % kv for kv in sorted(errs.items())))
    bad = {k: v for k, v in errs.items() if not v <= 1e-12}
    assert not bad, bad


def test_refinement_configured_geometry_f32():
    """2048^2 coarse D2Q5 MRT FP32, 1024 x 512 fine patch at coarse
    x in [768, 1280), y in [512, 768) over the 0.25 lens, from random
    (rho, J) states on both grids, 200 coarse steps: traces at the surface
    receivers and at nodes inside the patch, and the final coarse and fine
    fields, within 1e-5 of the oracle composite."""
    n, nsteps = 2048, 200
    wl = inputs.refined_workload(n=n, nsteps=nsteps)
    patch = wl["patch"]
    assert patch == (768, 512, 512, 256)
    px0, py0, pnx, pny = patch
    recs = np.concatenate([wl["receivers"], np.array(
        [(px0, py0), (px0 + 1, py0 + 1), (px0 + pnx - 1, py0 + pny - 1), (px0 + 2, py0 + 2),
         (px0 + pnx // 2, py0 + pny // 2), (px0 + 17, py0 + 17), (px0 - 1, py0 + 5), (px0 + 5, py0 - 1),
         (px0 + pnx, py0 + pny), (px0 + pnx + 2, py0 + 40)], dtype=np.int32)])
    rho, jx, jy = inputs.random_fields(n, n, seed=31)
    nyf, nxf = wl["c2_fine"].shape
    rf_, jxf, jyf = inputs.random_fields(nxf, nyf, seed=32)

    # oracle composite
    g = lo.OracleGrid(n, n, q=5, collision="mrt", s=MRT5, sponge_width=wl["sponge_width"],
                      sponge_sigma_max=wl["sponge_sigma_max"], source=wl["source"], wavelet=wl["wavelet"])
    g.set_medium(wl["c2"])
    g.set_state(rho, jx, jy)
    ref = rf.OracleRefined(g, wl["c2_fine"], patch)
    ref.fine.set_state(rf_, jxf, jyf)
    ref.initialize()
    inside = np.array([ref.inside_patch(x, y) for x, y in recs])
    rx, ry = recs[:, 0], recs[:, 1]
    fi, fj = 2 * (rx[inside] - ref.X0), 2 * (ry[inside] - ref.Y0)
    ref_tr = np.zeros((len(FIELDS), len(recs), nsteps + 1))

    def record(k):
        vc = ref.coarse.fields_at(rx[~inside], ry[~inside])
        vf = ref.fine.fields_at(fi, fj)
        for f, name in enumerate(FIELDS):
            ref_tr[f, ~inside, k] = vc[name]
            ref_tr[f, inside, k] = vf[name]

    record(0)
    for k in range(1, nsteps + 1):
        ref.step()
        record(k)

    # GPU
    case = {"nx": n, "ny": n, "q": 5, "collision": "mrt", "tau": 0.5, "s": MRT5, "ratio": 0.25,
            "c2": wl["c2"], "c2_fine": wl["c2_fine"], "patch": patch, "nsteps": nsteps,
            "sponge_width": wl["sponge_width"], "sponge_sigma_max": wl["sponge_sigma_max"],
            "receivers": recs}
    gg = make_grid(case, "f32")
    gg.set_medium(wl["c2"])
    gg.set_medium(wl["c2_fine"], fine=True)
    gg.set_state(rho, jx, jy)
    gg.set_state(rf_, jxf, jyf, fine=True)
    gg.set_source(wl["source"][0], wl["source"][1], wl["wavelet"])
    tr = gg.record(recs, fields=FIELDS)
    gg.step(nsteps)
    gg.sync()
    gpu_tr = tr.cpu().numpy()
    errs = {"trace_" + f: rel_l2(gpu_tr[k], ref_tr[k]) for k, f in enumerate(FIELDS)}
    for f in FIELDS:
        errs["coarse_" + f] = rel_l2(gg.field(f).cpu().numpy(), ref.coarse.field(f))
        errs["fine_" + f] = rel_l2(gg.field(f, fine=True).cpu().numpy(), ref.fine.field(f))
    gg.close()
    print("refinement 2048^2 + 1024x512 MRT FP32, %d coarse steps:" % nsteps,
          " ".join("%s %.2e" % kv for kv in sorted(errs.items())))
    bad = {k: v for k, v in errs.items() if not v <= 1e-5}
    assert not bad, bad


# ---- adjoint at scale -----------------------------------------------------------

def _adjoint_grid(wl, precision, K=0):
    from paper_1704_03172_amd import lbwave
    n, N = wl["nx"], wl["nsteps"]
    return lbwave.Grid(n, n, precision=precision, sponge_width=wl["sponge_width"],
                       sponge_sigma_max=wl["sponge_sigma_max"], trace_capacity=N + 1,
                       max_receivers=len(wl["receivers"]), ckpt_every=K,
                       ckpt_capacity=(N // K + 1) if K else 0)


def _forward_phi(g, wl, src, c2, d_obs):
    """phi of one FP64 forward run (fresh state at rest)."""
    g.set_medium(c2)
    g.set_state(np.zeros((wl["ny"], wl["nx"])))
    g.set_source(src[0], src[1], wl["wavelet"])
    g.record(wl["receivers"], fields=("p",))
    g.step(wl["nsteps"])
    phi, _ = g.misfit(d_obs, wl["nsteps"])
    return float(phi.item())


def test_adjoint_workload_central_differences_fp64():
    """One shot of the adjoint workload (2048^2, 3000 steps, D2Q5 BGK
    tau = 1/2, checkpoints every 55 steps): dphi/dc^2 from lb_adjoint against
    (phi(c2 + h e_x) - phi(c2 - h e_x)) / 2h of FP64 GPU forward runs,
    h = 1e-4 c^2(x), at 10 seeded nodes in the region the shot illuminates
    (within 600 nodes of the source along x and between the receiver row and
    the first layer interface), rel <= 1e-4."""
    import torch
    wl = inputs.adjoint_workload(n=2048, nshots=16, nsteps=3000)
    src = wl["sources"][8]
    N = wl["nsteps"]
    fwd = _adjoint_grid(wl, "f64")
    fwd.set_medium(wl["c2_true"])
    fwd.set_source(src[0], src[1], wl["wavelet"])
    obs = fwd.record(wl["receivers"], fields=("p",))
    fwd.step(N)
    d_obs = obs[0].clone()
    g = _adjoint_grid(wl, "f64", K=55)
    g.set_medium(wl["c2_init"])
    g.set_source(src[0], src[1], wl["wavelet"])
    g.record(wl["receivers"], fields=("p",))
    g.step(N)
    phi, res = g.misfit(d_obs, N)
    grad = g.adjoint(res, N).cpu().numpy()
    g.close()
    phi0 = float(phi.item())
    assert _forward_phi(fwd, wl, src, wl["c2_init"], d_obs) == phi0
    rng = np.random.default_rng(2048)
    c2 = wl["c2_init"]
    worst = 0.0
    gmax = np.abs(grad).max()
    for _ in range(10):
        x = int(rng.integers(src[0] - 600, src[0] + 600))
        y = int(rng.integers(wl["sponge_width"] + 8, 2048 // 5 - 8))
        h = 1e-4 * c2[y, x]
        cp = c2.copy(); cp[y, x] += h
        cm = c2.copy(); cm[y, x] -= h
        fd = (_forward_phi(fwd, wl, src, cp, d_obs) - _forward_phi(fwd, wl, src, cm, d_obs)) / (2 * h)
        e = abs(fd - grad[y, x]) / max(abs(fd), 1e-3 * gmax)
        print("node (%d, %d): adjoint %.6e  central difference %.6e  rel %.1e" % (x, y, grad[y, x], fd, e))
        worst = max(worst, e)
    fwd.close()
    del torch
    assert worst <= 1e-4, worst


def test_adjoint_dot_product_fp64():
    """<J dm, r> = <dm, J^T r> for the trace Jacobian J = dp/dc^2: J^T r is
    lb_adjoint's FP64 gradient for trace sensitivities r (random, not a
    misfit residual) and J dm the oracle's complex-step tangent
    Im(p(c^2 + i h dm)) / h, which has no cancellation error.  Within 1e-12;
    the adjoint is also linear in r to rounding."""
    import torch
    from tests.test_gpu_adjoint import make_case
    case = make_case(nx=96, ny=64, N=150, seed=9)
    N, nrec = case["nsteps"], len(case["receivers"])
    rng = np.random.default_rng(17)
    dm = rng.standard_normal(case["c2"].shape) * case["c2"]
    h = 1e-30
    tr_c, _ = ad.forward(case, case["c2"] + 1j * h * dm)
    jdm = tr_c.imag / h                                  # [nrec][N+1]
    from paper_1704_03172_amd import lbwave
    g = lbwave.Grid(case["nx"], case["ny"], lattice=5, collision="bgk", precision="f64", tau=0.5,
                    sponge_width=case["sponge_width"], sponge_sigma_max=case["sponge_sigma_max"],
                    trace_capacity=N + 1, max_receivers=nrec, ckpt_every=16, ckpt_capacity=N // 16 + 1)

    def jt(r):
        g.set_medium(case["c2"])
        g.set_state(case["rho0"], case["jx0"], case["jy0"])
        g.set_source(case["source"][0], case["source"][1], case["wavelet"])
        g.record(case["receivers"], fields=("p",))
        g.step(N)
        return g.adjoint(torch.as_tensor(r, device="cuda"), N).cpu().numpy()

    r1 = rng.standard_normal((nrec, N + 1))
    r2 = rng.standard_normal((nrec, N + 1))
    a1, a2 = jt(r1), jt(r2)
    lhs = float(np.sum(jdm * r1))
    rhs = float(np.sum(dm * a1))
    e_dot = abs(lhs - rhs) / abs(lhs)
    a12 = jt(0.75 * r1 - 1.5 * r2)
    e_lin = np.linalg.norm(a12 - (0.75 * a1 - 1.5 * a2)) / np.linalg.norm(a12)
    g.close()
    print("dot-product test: <J dm, r> %.15e  <dm, J^T r> %.15e  rel %.1e; linearity %.1e"
          % (lhs, rhs, e_dot, e_lin))
    assert e_dot <= 1e-12, e_dot
    assert e_lin <= 1e-12, e_lin
