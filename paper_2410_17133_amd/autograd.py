"""torch.autograd.Functions around one implicit step (forward = fg_assemble +
fg_step, Newton with partitioned CG; backward = fg_adjoint_solve) and around a
loop of steps (backward = the checkpointed reverse sweep through the slip state).
Gradients of any objective of the displacements and pressures with respect to
the per-tetrahedron log-permeability and Young modulus."""
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


class ImplicitLoop(torch.autograd.Function):
    """U_all, P_all = ImplicitLoop.apply(logk, E, system, params, t0, F_u, f_p, steps, solver)

    `steps` implicit steps from the initial state with the state (U, P, inelastic
    slip) carried from step to step; U_all [steps, 3N] and P_all [steps, N] are the
    converged states of every step, so an objective may read any of them.  The
    backward pass is the checkpointed reverse sweep of paper_2410_17133_amd.trajectory
    (adjoint through the slip state).  solver: as ImplicitStep, plus
    max_defect_iters per step (default 1000)."""

    @staticmethod
    def forward(ctx, logk, E, system, params, t0, F_u, f_p, steps, solver=None):
        from . import trajectory
        s = dict(newton_tol=1e-12, inner_tol=1e-13, outer_tol=1e-12, defect_tol=1e-12, precision=fg.FG_F64,
                 newton_max_iter=80, adjoint_outer_tol=0.05, adjoint_inner_tol=1e-3, max_defect_iters=1000)
        s.update(solver or {})
        system.assemble(params, E.detach(), logk.detach())
        U = torch.zeros(3 * system.N, dtype=torch.float64, device=E.device)
        P = torch.zeros(system.N, dtype=torch.float64, device=E.device)
        die = torch.zeros(2 * system.nq, dtype=torch.float64, device=E.device)
        ik = fg.opts(tol=s["inner_tol"], precision=s["precision"])
        ip = fg.opts(tol=s["inner_tol"])
        ck, infos = trajectory.run(system, U, P, die, t0, F_u, f_p, int(steps), newton_tol=s["newton_tol"],
                                   newton_max_iter=s["newton_max_iter"], inner_k=ik, inner_p=ip,
                                   outer_tol=s["outer_tol"])
        ctx.system, ctx.params, ctx.s, ctx.ck, ctx.infos = system, params, s, ck, infos
        ctx.save_for_backward(logk.detach(), E.detach(), t0)
        return torch.stack([c[0] for c in ck]), torch.stack([c[1] for c in ck])

    @staticmethod
    def backward(ctx, gU, gP):
        from . import trajectory
        logk, E, t0 = ctx.saved_tensors
        S, s, ck = ctx.system, ctx.s, ctx.ck
        S.assemble(ctx.params, E, logk)
        zU = torch.zeros_like(ck[0][0])
        zP = torch.zeros_like(ck[0][1])

        def grad_y(n, U, P):
            return (zU if gU is None else gU[n].contiguous()), (zP if gP is None else gP[n].contiguous())
        ik = fg.opts(tol=s["adjoint_inner_tol"], precision=s["precision"])
        ip = fg.opts(tol=s["adjoint_inner_tol"])
        dE, dk, infos = trajectory.gradient(S, ck, t0, logk, grad_y, inner_k=ik, inner_p=ip,
                                            outer_tol=s["adjoint_outer_tol"], defect_tol=s["defect_tol"],
                                            max_defect_iters=s["max_defect_iters"])
        ctx.adjoint_infos = infos
        return dk, dE, None, None, None, None, None, None, None


def fault_slip_uplift_objective(U, pairs, normal, uplift):
    """J = sum over fault node pairs of the squared tangential jump of U plus the sum of the
    squared vertical displacement at the `uplift` nodes (differentiable torch code)."""
    U3 = U.view(-1, 3)
    jump = U3[pairs[:, 1]] - U3[pairs[:, 0]]
    slip = jump - (jump @ normal)[:, None] * normal[None, :]
    return (slip * slip).sum() + (U3[uplift, 2] ** 2).sum()
