"""Graph replay of lb_step_n (lb_set_graph) against the same grid stepped
launch by launch.

The multi-step kernels give the same bits as one step per launch, so a
replayed chunk, whatever its launch plan, must leave every field, trace and
sum of rho bitwise equal to the eager run.  Each case calls step() with
lengths that are not multiples of the chunk (the rest runs eagerly), reads
fields between the calls (eager work and synchronisation between replays),
and changes the source in the middle (the graph is captured again).
"""
import numpy as np
import pytest
import torch

from paper_1704_03172_amd import inputs, lbwave

pytestmark = pytest.mark.gpu

CALLS = (100, 37, 200, 5, 158)


def grid_pair(nx, ny, **kw):
    """Two identical grids, each on a stream of its own (graphs cannot be
    captured on the null stream)."""
    return [lbwave.Grid(nx, ny, stream=torch.cuda.Stream(), **kw) for _ in range(2)]


def snapshot(g):
    g.sync()
    out = {"rho": g.field("rho").cpu().numpy().copy(), "t": g.time}
    if g.traces is not None:
        out["traces"] = g.traces.cpu().numpy().copy()
    if g.sum_rho is not None:
        out["sum_rho"] = g.sum_rho.cpu().numpy().copy()
    return out


def assert_same(a, b, what):
    assert a["t"] == b["t"], what
    for k in a:
        if k != "t":
            assert np.array_equal(a[k], b[k]), "%s: %s differs (max %g)" % (
                what, k, float(np.max(np.abs(a[k] - b[k]))))


def run_pair(eager, graph, chunk, calls=CALLS, swap_source=None):
    graph.set_graph(chunk)
    for k, n in enumerate(calls):
        if swap_source is not None and k == 2:
            for g in (eager, graph):
                g.set_source(*swap_source)
        eager.step(n)
        graph.step(n)
        assert_same(snapshot(eager), snapshot(graph), "after call %d (%d steps, chunk %d)" % (k, n, chunk))
    print("chunk %d: %d steps bitwise equal" % (chunk, sum(calls)), flush=True)


def test_graph_pulse_fp64_sum_rho():
    """The 128^2 periodic pulse (D2Q5 BGK tau = 1, FP64), sum of rho every
    step: one step per launch plus the sum's finalize launch."""
    wl = inputs.pulse_workload()
    ev, gr = grid_pair(128, 128, lattice=5, collision="bgk", precision="f64", tau=1.0,
                       trace_capacity=sum(CALLS) + 1)
    for g in (ev, gr):
        g.set_medium(wl["c2"])
        g.set_state(wl["rho0"])
        g.record_sum_rho()
    run_pair(ev, gr, 64)
    ev.close()
    gr.close()


@pytest.mark.parametrize("q,collision,precision,chunk", [
    (5, "bgk", "f32", 32), (5, "mrt", "f32", 17), (9, "mrt", "f32", 16), (5, "bgk", "f64", 64),
    (5, "bgk", "f16s", 24), (9, "bgk", "f64", 2)])
def test_graph_layered_source_receivers(q, collision, precision, chunk):
    """A small layered case with sponge, source and receivers on the
    multi-step kernels (launches of up to four steps inside a chunk)."""
    nx, ny = 192, 96
    wl = inputs.layered_workload(n=192, nsteps=sum(CALLS) + 1)
    c2 = wl["c2"][:ny, :nx]
    rec = wl["receivers"][:40]
    other = (nx // 3, ny // 2, inputs.ricker_wavelet(sum(CALLS) + 1, wl["fc"] * 1.3))
    ev, gr = grid_pair(nx, ny, lattice=q, collision=collision, precision=precision, tau=0.5,
                       s=[1, 1, 1, 2, 2, 2, 1, 1, 2][:q], sponge_width=12, sponge_sigma_max=0.1,
                       trace_capacity=sum(CALLS) + 1, max_receivers=len(rec))
    for g in (ev, gr):
        g.set_medium(c2)
        g.set_source(nx // 2, 20, wl["wavelet"])
        g.record(rec, fields=("p", "rho", "jx", "jy") if precision != "f16s" else ("p",))
    run_pair(ev, gr, chunk, swap_source=other)
    ev.close()
    gr.close()


def test_graph_across_state_reset():
    """set_state resets the time to 0 and keeps the captured graph (its
    launches take the same params); the chunk table carries the new times.
    record_sum_rho then makes it capture again."""
    wl = inputs.pulse_workload(n=96, nsteps=300)
    ev, gr = grid_pair(96, 96, lattice=5, collision="bgk", precision="f64", tau=1.0, trace_capacity=400)
    for g in (ev, gr):
        g.set_medium(wl["c2"])
        g.set_state(wl["rho0"])
        g.record_sum_rho()
    run_pair(ev, gr, 40, calls=(90, 130))
    for g in (ev, gr):
        g.set_state(wl["rho0"] * 0.5)
    run_pair(ev, gr, 40, calls=(81, 120))
    for g in (ev, gr):
        g.set_state(wl["rho0"] * 0.25)
        g.record_sum_rho()
    run_pair(ev, gr, 40, calls=(45, 80))
    ev.close()
    gr.close()


def raises_code(code, fn, *a):
    with pytest.raises(lbwave.LBError) as e:
        fn(*a)
    assert e.value.code == code, str(e.value)


def test_graph_argument_errors():
    g = lbwave.Grid(64, 64, stream=torch.cuda.Stream(), precision="f32")
    for bad in (1, -1, 257):
        raises_code(-2, g.set_graph, bad)
    g.set_graph(256)
    g.set_graph(0)
    g.close()
    p = lbwave.Grid(128, 128, stream=torch.cuda.Stream(), precision="f32", patch=(48, 48, 32, 16))
    raises_code(-3, p.set_graph, 16)
    p.close()
    d = lbwave.Grid(64, 64, precision="f32", stream=torch.cuda.default_stream())
    raises_code(-3, d.set_graph, 16)
    d.close()
