"""torch.autograd wrapper of the adjoint of the conservative dynamics (F/D
off): K Velocity-Verlet steps with density, entropy-conserving energies and
pressure forces, differentiated by the library's reverse pass.

    qK, pK = sdpd_dynamics(q0, p0, eps0, params, nsteps, checkpoint_every)
    qK, pK, epsK, rhoK = sdpd_dynamics(..., full=True, A=A, Cv=Cv)

q0, p0: (3, n) float64 device tensors, eps0: (n,), all indexed by particle
id (0..n-1); params: an SdpdParams with fd = FD_NONE.  Gradients flow to q0,
p0 and eps0, and to the closure coefficient A and the heat capacity Cv of
eq. (pg-eos) when they are given as 0-dim float64 tensors (their values
replace params.A and params.Cv).  Without A, the default A = Cv / (3 kB) is
formed here from Cv, so a Cv gradient follows the tie.  The final energies
and densities (full=True) let a loss read the closure of Sec. 2.1.2, e.g.
the mean pressure A kB rho eps / (m Cv).  Reordering between id order and
the library's cell order is done here with index operations; every step of
the dynamics and of its adjoint runs in the library.
"""
import dataclasses

import torch

from . import sdpd


class _Dynamics(torch.autograd.Function):
    @staticmethod
    def forward(fctx, q0, p0, eps0, A, Cv, params, nsteps, every):
        n = eps0.shape[0]
        prm = dataclasses.replace(params, A=float(A), Cv=float(Cv))
        ids = torch.arange(n, dtype=torch.int32, device=q0.device)
        S = sdpd.DeviceState(q0.detach().clone().contiguous(), p0.detach().clone().contiguous(),
                             eps0.detach().clone().contiguous(),
                             torch.zeros(n, dtype=torch.float64, device=q0.device),
                             torch.zeros((3, n), dtype=torch.float64, device=q0.device), ids)
        ctx = sdpd.Context(prm)
        ctx.prepare(S)
        ctx.adjoint_forward(S, nsteps, every)
        ctx.sync()
        order = S.id.long()
        qK = torch.empty_like(S.q)
        pK = torch.empty_like(S.p)
        epsK = torch.empty_like(S.eps)
        rhoK = torch.empty_like(S.rho)
        qK[:, order] = S.q
        pK[:, order] = S.p
        epsK[order] = S.eps
        rhoK[order] = S.rho
        fctx.lib_ctx = ctx
        fctx.state = S
        fctx.set_materialize_grads(False)   # unused outputs: no cotangent passed
        return qK, pK, epsK, rhoK

    @staticmethod
    def backward(fctx, gq, gp, geps, grho):
        ctx = fctx.lib_ctx
        gq = torch.zeros_like(fctx.state.q) if gq is None else gq.contiguous()
        gp = torch.zeros_like(fctx.state.p) if gp is None else gp.contiguous()
        out = ctx.adjoint_vjp(gq, gp, geps, grho)
        ctx.sync()
        ctx.close()
        dev = gq.device
        dA = torch.tensor(out["dA"], dtype=torch.float64, device=dev)
        dCv = torch.tensor(out["dCv"], dtype=torch.float64, device=dev)
        return out["dq0"], out["dp0"], out["deps0"], dA, dCv, None, None, None


def sdpd_dynamics(q0, p0, eps0, params, nsteps, checkpoint_every=10, A=None, Cv=None,
                  full=False):
    if params.fd != sdpd.FD_NONE:
        raise ValueError("the adjoint covers the conservative dynamics: params.fd must be FD_NONE")
    dev = q0.device
    if Cv is None:
        Cv = torch.tensor(float(params.Cv), dtype=torch.float64, device=dev)
    if A is None and params.A in (None, 0.0):
        # the default A = Cv / (3 kB): its value as the library resolves it
        # (one IEEE division), its derivative 1 / (3 kB) along the tie
        A = (Cv - Cv.detach()) / (3.0 * params.kB) + float(Cv) / (3.0 * params.kB)
    elif A is None:
        A = torch.tensor(float(params.A), dtype=torch.float64, device=dev)
    out = _Dynamics.apply(q0, p0, eps0, A, Cv, params, nsteps, checkpoint_every)
    return out if full else out[:2]
