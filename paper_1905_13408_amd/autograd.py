"""torch.autograd.Function over an unrolled SPG solve on the HIP library.

    x_K = UnrolledSPG.apply(lam, mu, b, solver, w, K, C)

runs K SPG iterations from x = 0 (momentum restarted, the solver's current penalty
weights) with the given lambda, mu and data b, checkpointing every C iterations; the
backward pass calls the library's reverse mode (spg_vjp) for d/d(lam, mu, b).  The
gradient for the complex b follows torch's convention for real losses
(d loss = Re sum conj(grad) db).  Every step of both passes runs in libspg.
"""
import torch


class UnrolledSPG(torch.autograd.Function):
    @staticmethod
    def forward(ctx, lam, mu, b, solver, w, K, C):
        solver.set_params(float(lam), float(mu))
        solver.set_data(w, b)
        solver.set_map(None)
        solver.run_checkpointed(int(K), int(C))
        ctx.solver = solver
        ctx.w = w
        ctx.lam_dtype = lam.dtype if isinstance(lam, torch.Tensor) else torch.float64
        return solver.get_map()

    @staticmethod
    def backward(ctx, grad_x):
        lb, mb, bb = ctx.solver.vjp(ctx.w, grad_x.contiguous())
        dev = grad_x.device
        return (torch.tensor(lb, dtype=ctx.lam_dtype, device=dev), torch.tensor(mb, dtype=ctx.lam_dtype, device=dev),
                bb, None, None, None, None)
