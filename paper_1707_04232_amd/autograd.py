"""torch.autograd wrapper of the adjoint of the conservative dynamics (F/D
off): K Velocity-Verlet steps with density, entropy-conserving energies and
pressure forces, differentiated by the library's reverse pass.

    qK, pK = sdpd_dynamics(q0, p0, eps0, params, nsteps, checkpoint_every)

q0, p0: (3, n) float64 device tensors, eps0: (n,), all indexed by particle
id (0..n-1); params: an SdpdParams with fd = FD_NONE.  Gradients flow to q0,
p0 and eps0.  Reordering between id order and the library's cell order is
done here with index operations; every step of the dynamics and of its
adjoint runs in the library.
"""
import torch

from . import sdpd


class _Dynamics(torch.autograd.Function):
    @staticmethod
    def forward(fctx, q0, p0, eps0, params, nsteps, every):
        n = eps0.shape[0]
        ids = torch.arange(n, dtype=torch.int32, device=q0.device)
        S = sdpd.DeviceState(q0.detach().clone().contiguous(), p0.detach().clone().contiguous(),
                             eps0.detach().clone().contiguous(),
                             torch.zeros(n, dtype=torch.float64, device=q0.device),
                             torch.zeros((3, n), dtype=torch.float64, device=q0.device), ids)
        ctx = sdpd.Context(params)
        ctx.prepare(S)
        ctx.adjoint_forward(S, nsteps, every)
        ctx.sync()
        order = S.id.long()
        qK = torch.empty_like(S.q)
        pK = torch.empty_like(S.p)
        qK[:, order] = S.q
        pK[:, order] = S.p
        fctx.lib_ctx = ctx
        fctx.state = S
        return qK, pK

    @staticmethod
    def backward(fctx, gq, gp):
        ctx = fctx.lib_ctx
        gq = torch.zeros_like(fctx.state.q) if gq is None else gq.contiguous()
        gp = torch.zeros_like(fctx.state.p) if gp is None else gp.contiguous()
        dq0, dp0, de0, _ = ctx.adjoint_backward(gq, gp)
        ctx.sync()
        ctx.close()
        return dq0, dp0, de0, None, None, None


def sdpd_dynamics(q0, p0, eps0, params, nsteps, checkpoint_every=10):
    if params.fd != sdpd.FD_NONE:
        raise ValueError("the adjoint covers the conservative dynamics: params.fd must be FD_NONE")
    return _Dynamics.apply(q0, p0, eps0, params, nsteps, checkpoint_every)
