"""Run one seeded case on the oracle and on the HIP library.

A case is a dict of inputs (from paper_1704_03172_amd.inputs) plus scheme
parameters.  Both sides receive the same arrays; neither side sees the
other's results.
"""
import numpy as np

from oracle import lb_oracle as lo
from oracle import refine as rf

FIELDS = ("p", "rho", "jx", "jy")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def scheme_kwargs(case):
    return dict(q=case.get("q", 5), collision=case.get("collision", "bgk"),
                tau=case.get("tau", 0.5), s=case.get("s"),
                ratio=case.get("ratio", 0.25))


def run_oracle(case):
    kw = scheme_kwargs(case)
    g = lo.OracleGrid(case["nx"], case["ny"], q=kw["q"], collision=kw["collision"],
                      tau=kw["tau"], s=kw["s"], ratio=kw["ratio"],
                      sponge_width=case.get("sponge_width", 0),
                      sponge_sigma_max=case.get("sponge_sigma_max", 0.0),
                      source=case.get("source"), wavelet=case.get("wavelet"))
    g.set_medium(case["c2"])
    ny, nx = case["ny"], case["nx"]
    g.set_state(case.get("rho0", np.zeros((ny, nx))), case.get("jx0"), case.get("jy0"))
    if "patch" in case:
        ref = rf.OracleRefined(g, case["c2_fine"], case["patch"],
                               case.get("overlap_out", 2), case.get("overlap_in", 2))
        out = rf.run_refined(ref, case["nsteps"], case.get("receivers"), fields=FIELDS)
        out["fields"] = {f: g.field(f) for f in FIELDS}
        out["fine_fields"] = {f: ref.fine.field(f) for f in FIELDS}
        return out
    out = lo.run(g, case["nsteps"], case.get("receivers"), fields=FIELDS,
                 sum_rho=True, snapshots=case.get("snapshots", ()))
    out["fields"] = {f: g.field(f) for f in FIELDS}
    return out


def make_grid(case, precision, steps_per_launch=0):
    from paper_1704_03172_amd import lbwave
    kw = scheme_kwargs(case)
    rec = case.get("receivers")
    nrec = 0 if rec is None else len(rec)
    extra = {}
    if "patch" in case:
        extra = dict(patch=case["patch"], overlap_out=case.get("overlap_out", 2),
                     overlap_in=case.get("overlap_in", 2))
    return lbwave.Grid(case["nx"], case["ny"], lattice=kw["q"], collision=kw["collision"],
                       precision=precision, tau=kw["tau"], s=kw["s"], ratio=kw["ratio"],
                       sponge_width=case.get("sponge_width", 0),
                       sponge_sigma_max=case.get("sponge_sigma_max", 0.0),
                       trace_capacity=case["nsteps"] + 1, max_receivers=max(nrec, 1),
                       steps_per_launch=steps_per_launch, **extra)


def run_gpu(case, precision="f32", chunks=None, on_device=False, sum_rho=False, steps_per_launch=0):
    """Run the case through the C-ABI.  chunks: list of step counts whose sum
    is nsteps (exercises repeated lb_step_n calls).  By default lb_step_n
    takes as many steps per launch as the blocked kernel offers (the path
    the benchmark times); recording the sum of rho (sum_rho=True) or
    steps_per_launch=1 keeps it at one step per launch."""
    import torch
    grid = make_grid(case, precision, steps_per_launch)
    ny, nx = case["ny"], case["nx"]
    c2 = case["c2"]
    rho0 = case.get("rho0", np.zeros((ny, nx)))
    jx0, jy0 = case.get("jx0"), case.get("jy0")
    if on_device:
        dev = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64, device="cuda")
        c2, rho0, jx0, jy0 = dev(c2), dev(rho0), dev(jx0), dev(jy0)
    grid.set_medium(c2)
    if "patch" in case:
        grid.set_medium(case["c2_fine"], fine=True)
    grid.set_state(rho0, jx0, jy0)
    if case.get("source") is not None:
        grid.set_source(case["source"][0], case["source"][1], case["wavelet"])
    traces = None
    if case.get("receivers") is not None:
        traces = grid.record(case["receivers"], fields=FIELDS)
    sums = None if ("patch" in case or not sum_rho) else grid.record_sum_rho()
    for n in (chunks or [case["nsteps"]]):
        grid.step(n)
    grid.sync()
    out = {"time": grid.time}
    if traces is not None:
        out["traces"] = traces.cpu().numpy()
    if sums is not None:
        out["sum_rho"] = sums.cpu().numpy()
    out["fields"] = {f: grid.field(f).cpu().numpy() for f in FIELDS}
    if "patch" in case:
        out["fine_fields"] = {f: grid.field(f, fine=True).cpu().numpy() for f in FIELDS}
    out["grid"] = grid
    return out
