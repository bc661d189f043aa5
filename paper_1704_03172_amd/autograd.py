"""torch.autograd.Function over the library's forward run and adjoint.

C2Misfit.apply(c2, d_obs, shot) returns phi = 1/2 sum_r sum_n (p_r(n) -
d_r(n))^2 for one shot (lb_step_n + lb_misfit) and, on backward, the gradient
with respect to the per-node c^2 from lb_adjoint (FP64 accumulation, cast to
the dtype of c2).  All arithmetic runs in the library's kernels; torch holds
the buffers.
"""
import torch

from . import lbwave


class C2Misfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c2, d_obs, shot):
        """shot: dict with nx, ny, nsteps, source (x, y), wavelet, receivers
        (nrec, 2); optional lattice, collision, tau, s, ratio, precision,
        sponge_width, sponge_sigma_max, ckpt_every."""
        n = int(shot["nsteps"])
        K = int(shot.get("ckpt_every", 64))
        rec = shot["receivers"]
        g = lbwave.Grid(shot["nx"], shot["ny"], lattice=shot.get("lattice", 5),
                        collision=shot.get("collision", "bgk"), precision=shot.get("precision", "f32"),
                        tau=shot.get("tau", 0.5), s=shot.get("s"), ratio=shot.get("ratio", 0.25),
                        sponge_width=shot.get("sponge_width", 0),
                        sponge_sigma_max=shot.get("sponge_sigma_max", 0.0),
                        trace_capacity=n + 1, max_receivers=len(rec),
                        ckpt_every=K, ckpt_capacity=n // K + 1, device=c2.device)
        g.set_medium(c2.detach())
        g.set_source(shot["source"][0], shot["source"][1], shot["wavelet"])
        g.record(rec, fields=("p",))
        g.step(n)
        phi, res = g.misfit(d_obs, n)
        ctx.grid, ctx.res, ctx.n, ctx.dtype = g, res, n, c2.dtype
        return phi

    @staticmethod
    def backward(ctx, gphi):
        grad = ctx.grid.adjoint(ctx.res, ctx.n)
        ctx.grid.close()
        ctx.grid = None
        return (gphi * grad).to(ctx.dtype), None, None


def misfit_and_gradient(c2, d_obs, shot):
    """Convenience: (phi, dphi/dc2) of one shot without building a graph."""
    c2 = c2.detach().requires_grad_(True)
    phi = C2Misfit.apply(c2, d_obs, shot)
    (grad,) = torch.autograd.grad(phi, c2)
    return phi.detach(), grad
