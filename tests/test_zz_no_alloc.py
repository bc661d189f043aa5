"""lb_trace_misfit_static (no workspace: block partials in a static device
array) against lb_trace_misfit (caller workspace) through the C-ABI: the
same bits, on two calls in a row on the same GPU, the second with a smaller
input, and against the definition in FP64."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pair(nrec, cap, dtype, seed):
    import torch
    rng = np.random.default_rng(seed)
    tr = rng.standard_normal((nrec, cap))
    ob = tr + 0.05 * rng.standard_normal((nrec, cap))
    return torch.as_tensor(tr, dtype=dtype, device="cuda"), torch.as_tensor(ob, dtype=dtype, device="cuda")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_static_scratch_variant_equals_workspace_variant(prec):
    import torch
    from paper_1704_03172_amd import lbwave
    torch.cuda.set_device(0)
    dt = torch.float64 if prec == "f64" else torch.float32
    # first call: more elements than 2048 blocks of 256 threads cover (every
    # scratch slot written); second call: a smaller input (fewer slots read)
    for k, (nrec, cap, ncols) in enumerate([(256, 4001, 4001), (16, 301, 250), (1, 1, 1)]):
        tr, ob = _pair(nrec, cap, dt, 100 + k)
        phi_s, res_s = lbwave.trace_misfit_static(tr, ob, ncols)
        phi_w, res_w = lbwave.trace_misfit(tr, ob, ncols)
        torch.cuda.synchronize()
        print("%s nrec %d cap %d ncols %d: phi static %.17g workspace %.17g" % (prec, nrec, cap, ncols,
                                                                             phi_s.item(), phi_w.item()))
        assert phi_s.item() == phi_w.item()
        np.testing.assert_array_equal(res_s.cpu().numpy(), res_w.cpu().numpy())
        d = (tr - ob)[:, :ncols].cpu().numpy().astype(np.float64)
        want = 0.5 * np.sum(d * d)
        assert abs(phi_s.item() - want) <= 1e-13 * want


def test_static_variant_on_a_side_stream():
    """A stream other than the current one, on the same GPU."""
    import torch
    from paper_1704_03172_amd import lbwave
    torch.cuda.set_device(0)
    s = torch.cuda.Stream()
    tr, ob = _pair(40, 1001, torch.float32, 7)
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        phi_s, res_s = lbwave.trace_misfit_static(tr, ob, 999, stream=s)
    s.synchronize()
    phi_w, res_w = lbwave.trace_misfit(tr, ob, 999)
    torch.cuda.synchronize()
    assert phi_s.item() == phi_w.item()
    np.testing.assert_array_equal(res_s.cpu().numpy(), res_w.cpu().numpy())


def test_static_variant_rejects_bad_sizes():
    import ctypes
    from paper_1704_03172_amd import lbwave
    L = lbwave.lib()
    p = ctypes.c_void_p(0x100000)
    assert L.lb_trace_misfit_static(p, p, p, 0, 10, 10, 0, p, None) == -2
    assert L.lb_trace_misfit_static(p, p, p, 3, 10, 11, 0, p, None) == -2
    assert L.lb_trace_misfit_static(p, p, p, 2, 2 ** 62, 10, 0, p, None) == -2
    assert L.lb_trace_misfit_static(None, p, p, 3, 10, 10, 0, p, None) == -1
