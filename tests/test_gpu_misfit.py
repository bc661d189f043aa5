"""The trace misfit on the GPU (lb_misfit with a grid, lb_trace_misfit
without): res = p - d and phi = 1/2 sum res^2, reduced in FP64 through
block partials (wave64 shuffles) and one block adding them in order.
Checked against the definition in FP64 on the host, bit for bit between
the two entry points and between repeats, for sizes from one element to
more elements than 2048 blocks of 256 threads cover (grid-stride path)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (3, 10, 7), (128, 3001, 3001), (256, 4001, 2500), (700, 1001, 1001), (5, 300000, 299999)]


def _data(nrec, cap, dtype, seed):
    import torch
    rng = np.random.default_rng(seed)
    tr = rng.standard_normal((nrec, cap))
    ob = tr + 0.1 * rng.standard_normal((nrec, cap))
    return (torch.as_tensor(tr, dtype=dtype, device="cuda"), torch.as_tensor(ob, dtype=dtype, device="cuda"))


@pytest.mark.parametrize("nrec,cap,ncols", SHAPES)
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_trace_misfit_matches_definition(nrec, cap, ncols, prec):
    import torch
    from paper_1704_03172_amd import lbwave
    dt = torch.float64 if prec == "f64" else torch.float32
    tr, ob = _data(nrec, cap, dt, nrec * 7 + cap)
    phi, res = lbwave.trace_misfit(tr, ob, ncols)
    phi2, res2 = lbwave.trace_misfit(tr, ob, ncols)
    torch.cuda.synchronize()
    # residual: the same rounding as the arithmetic type's subtraction
    want_res = (tr - ob)[:, :ncols].cpu().numpy()
    got = res.cpu().numpy()
    np.testing.assert_array_equal(got[:, :ncols], want_res)
    assert not got[:, ncols:].any()                       # columns past ncols untouched
    d = want_res.astype(np.float64)
    want = 0.5 * np.sum(d * d)
    assert abs(phi.item() - want) <= 1e-13 * want, (phi.item(), want)
    assert phi.item() == phi2.item()
    np.testing.assert_array_equal(res.cpu().numpy(), res2.cpu().numpy())


def test_grid_misfit_equals_trace_misfit():
    """lb_misfit (partials in the grid's workspace) gives the bits of
    lb_trace_misfit on the grid's recorded traces."""
    import torch
    from paper_1704_03172_amd import inputs, lbwave
    n, N = 300, 200
    c = inputs.two_layer_speed(n, n, seed=5)
    g = lbwave.Grid(n, n, sponge_width=8, sponge_sigma_max=0.1, trace_capacity=N + 1, max_receivers=40)
    g.set_medium(c * c)
    g.set_source(n // 2, 10, inputs.ricker_wavelet(N + 1, float(c.min()) / 8))
    tr = g.record(inputs.surface_receivers(n, 40, 10, 8), fields=("p",))
    g.step(N)
    obs = (0.9 * tr[0]).contiguous()
    phi, res = g.misfit(obs, N)
    phi2, res2 = lbwave.trace_misfit(tr[0].contiguous(), obs, N + 1)
    torch.cuda.synchronize()
    assert phi.item() == phi2.item() and phi.item() > 0
    np.testing.assert_array_equal(res.cpu().numpy(), res2.cpu().numpy())
    g.close()
