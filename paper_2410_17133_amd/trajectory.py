"""Time loop of implicit steps and its reverse sweep (adjoint through the loop).

The forward loop checkpoints every step's converged state (U_n, P_n) and the
inelastic slip before and after it (die_{n-1}, die_n): a few vectors per step,
kept in device memory.  The reverse sweep runs n = T..1:

  J_n^T lam_n = dj_n/dy_n - (dR_{n+1}/dy_n)^T lam_{n+1} + (dPhi_n/dU_n)^T a_n
  a_{n-1}     = (dPhi_n/ddie_{n-1})^T a_n - (dR_n/ddie_{n-1})^T lam_n

where R_n is the step residual (total form, fg_step), whose flow part reads the
previous state through dR_{n+1,f}/dU_n = -A_up and dR_{n+1,f}/dP_n = -(A22 - dt C)
= -S, and Phi_n the return map that carries the slip (fg_slip_adjoint).  The
gradient sums -lam_n^T dR_n/dtheta over the steps (fg_adjoint_solve returns each
step's share).  Every operation is a libfg call on device tensors."""
from __future__ import annotations

from . import fg


def run(S, U, P, die, t0, F_u, f_p, steps: int, **step_kw):
    """Advance (U, P, die) in place through `steps` implicit steps; returns the
    checkpoints [(U_n, P_n, die_{n-1}, die_n)] and the per-step solve infos."""
    ck, infos = [], []
    for _ in range(steps):
        die_prev = die.clone()
        trac, flag, info = S.step(U, P, die, t0, F_u, f_p, **step_kw)
        if info.status != fg.FG_OK:
            raise fg.FgError(info.status, "a step of the time loop did not converge")
        ck.append((U.clone(), P.clone(), die_prev, die.clone()))
        infos.append(info)
    return ck, infos


def gradient(S, ck, t0, logk, grad_y, inner_k=None, inner_p=None, outer_tol=1e-12, defect_tol=1e-12,
             max_defect_iters=1000, log=None):
    """dJ/dE and dJ/dln k (per tetrahedron) of J = sum_n j_n(U_n, P_n) over the
    checkpointed loop.  grad_y(n, U, P) -> (dj/dU, dj/dP) as CUDA float64 tensors
    (n counted from 0).  Returns (dJ_dE, dJ_dlogk, per-step adjoint infos); log(str),
    if given, receives one line per step of the sweep.
    Every step of the sweep is one fg_adjoint_loop_step call; this function only
    allocates its buffers and passes them along."""
    import torch
    dev = t0.device
    f64 = dict(dtype=torch.float64, device=dev)
    a = torch.zeros(2 * S.nq, **f64)
    dE, dk = torch.zeros(S.ne, **f64), torch.zeros(S.ne, **f64)
    lam = [torch.zeros(S.N, **f64), torch.zeros(S.N, **f64)]
    lp_next = None
    infos = []
    for n in range(len(ck) - 1, -1, -1):
        U, P, die_prev, _ = ck[n]
        gu, gp = grad_y(n, U, P)
        lp = lam[n & 1]
        info = S.adjoint_loop_step(U, P, die_prev, t0, logk, gu.contiguous(), gp.contiguous(), lp_next, a, dE, dk,
                                   lp, inner_k=inner_k, inner_p=inner_p, outer_tol=outer_tol, defect_tol=defect_tol,
                                   max_defect_iters=max_defect_iters)
        if log:
            log(f"[sweep] step {n}: status {info.status}, defect iterations {info.newton_iters}, outer "
                f"{info.outer_iters}, K iterations {info.inner_k_iters}")
        if info.status != fg.FG_OK:
            raise fg.FgError(info.status, f"the adjoint of step {n} did not converge within {max_defect_iters} "
                                          "defect iterations")
        infos.append(info)
        lp_next = lp
    return dE, dk, infos[::-1]
