"""torch.autograd.Function around one implicit step: forward = fg_assemble +
fg_step (Newton with partitioned CG), backward = fg_adjoint_solve.  Gradients of
any objective of the step's displacement and pressure with respect to the
per-tetrahedron log-permeability and Young modulus."""
from __future__ import annotations

import torch

from . import fg


class ImplicitStep(torch.autograd.Function):
    """U, P = ImplicitStep.apply(logk, E, system, params, t0, F_u, f_p, solver)

    logk, E: CUDA float64 [n_tets].  system: fg.System.  params: inputs.Params.
    t0 [3 nq], F_u [3N], f_p [N]: CUDA float64.  solver: dict of tolerances
    (newton_tol, inner_tol, outer_tol of the forward step; adjoint_outer_tol and
    adjoint_inner_tol of each defect-correction solve, defect_tol of the adjoint;
    precision of the K solves).
    The step starts from the initial state (U = P = 0, no inelastic slip)."""

    @staticmethod
    def forward(ctx, logk, E, system, params, t0, F_u, f_p, solver=None):
        s = dict(newton_tol=1e-12, inner_tol=1e-13, outer_tol=1e-12, defect_tol=1e-12, precision=fg.FG_F64,
                 newton_max_iter=80, adjoint_outer_tol=0.05, adjoint_inner_tol=1e-3)
        s.update(solver or {})
        system.assemble(params, E.detach(), logk.detach())
        U = torch.zeros(3 * system.N, dtype=torch.float64, device=E.device)
        P = torch.zeros(system.N, dtype=torch.float64, device=E.device)
        die = torch.zeros(2 * system.nq, dtype=torch.float64, device=E.device)
        ik = fg.opts(tol=s["inner_tol"], precision=s["precision"])
        ip = fg.opts(tol=s["inner_tol"])
        trac, flag, info = system.step(U, P, die, t0, F_u, f_p, newton_tol=s["newton_tol"],
                                       newton_max_iter=s["newton_max_iter"], inner_k=ik, inner_p=ip,
                                       outer_tol=s["outer_tol"])
        ctx.system, ctx.params, ctx.s = system, params, s
        ctx.info = info
        ctx.save_for_backward(logk.detach(), E.detach(), U, P, t0)
        return U, P

    @staticmethod
    def backward(ctx, gU, gP):
        logk, E, U, P, t0 = ctx.saved_tensors
        S, s = ctx.system, ctx.s
        S.assemble(ctx.params, E, logk)       # the operators of this step (another step may have run since)
        die0 = torch.zeros(2 * S.nq, dtype=torch.float64, device=E.device)
        gU = torch.zeros_like(U) if gU is None else gU.contiguous()
        gP = torch.zeros_like(P) if gP is None else gP.contiguous()
        ik = fg.opts(tol=s["adjoint_inner_tol"], precision=s["precision"])
        ip = fg.opts(tol=s["adjoint_inner_tol"])
        dE, dk, info = S.adjoint(U, P, die0, t0, logk, gU, gP, inner_k=ik, inner_p=ip,
                                 outer_tol=s["adjoint_outer_tol"], defect_tol=s["defect_tol"])
        ctx.adjoint_info = info
        return dk, dE, None, None, None, None, None, None


def fault_slip_uplift_objective(U, pairs, normal, uplift):
    """J = sum over fault node pairs of the squared tangential jump of U plus the sum of the
    squared vertical displacement at the `uplift` nodes (differentiable torch code)."""
    U3 = U.view(-1, 3)
    jump = U3[pairs[:, 1]] - U3[pairs[:, 0]]
    slip = jump - (jump @ normal)[:, None] * normal[None, :]
    return (slip * slip).sum() + (U3[uplift, 2] ** 2).sum()
