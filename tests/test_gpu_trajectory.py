"""Adjoint through a time loop on the GPU (fg_slip_adjoint and the reverse sweep of
paper_2410_17133_amd.trajectory) against the oracle's, on a 4^3 loop of four steps in
which slip starts, spreads and part of the fault opens; and the loop gradient against
central differences of the GPU's own loop."""
import dataclasses

import numpy as np
import pytest

from paper_2410_17133_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TIGHT_O = dict(tol_newton=1e-13, max_newton=80, tol_outer=1e-13, tol_inner=1e-14)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def instance():
    return I.make_instance(dataclasses.replace(I.cube_config(4), Q=2e-3))


def tight(fg, newton_tol=1e-13):
    # iteration caps about 100 times what these solves take (a stalled solve ends with an error)
    return dict(newton_tol=newton_tol, newton_max_iter=80, inner_k=fg.opts(tol=1e-14, max_iter=50000),
                inner_p=fg.opts(tol=1e-14, max_iter=50000), outer_tol=1e-13)


def objective(inst, uplift):
    m = inst.mesh
    X = m.xyz[m.coh[0, 3:]]
    n = np.cross(X[1] - X[0], X[2] - X[0])
    n /= np.linalg.norm(n)

    def j_and_grad(U):
        U3 = U.reshape(-1, 3)
        jump = U3[m.pairs[:, 1]] - U3[m.pairs[:, 0]]
        slip = jump - np.outer(jump @ n, n)
        g = np.zeros_like(U3)
        np.add.at(g, m.pairs[:, 1], 2 * slip)
        np.add.at(g, m.pairs[:, 0], -2 * slip)
        g[uplift, 2] += 2 * U3[uplift, 2]
        return np.sum(slip * slip) + np.sum(U3[uplift, 2] ** 2), g.reshape(-1)
    return j_and_grad


@pytest.fixture(scope="module")
def loop():
    from oracle import oracle as O
    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import trajectory as T
    inst = instance()
    P = O.Problem(inst)
    ck_o = P.trajectory(4, **TIGHT_O)
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    t0 = dev(inst.t0.reshape(-1))
    U, Pp, die = dev(np.zeros(3 * S.N)), dev(np.zeros(S.N)), dev(np.zeros(2 * S.nq))
    ck, infos = T.run(S, U, Pp, die, t0, dev(np.zeros(3 * S.N)), dev(inst.source), 4, **tight(fg))
    return inst, P, ck_o, S, ck, t0, fg, T


def test_loop_states_match_oracle(loop):
    inst, P, ck_o, S, ck, t0, fg, T = loop
    for n, ((Uo, Po, dpo, do), (U, Pg, dp, d)) in enumerate(zip(ck_o, ck)):
        print(f"[loop] step {n}: U {rel(host(U), Uo):.1e} P {rel(host(Pg), Po):.1e}", flush=True)
        assert rel(host(U), Uo) < 1e-9 and rel(host(Pg), Po) < 1e-9
        assert np.abs(host(d) - do.reshape(-1)).max() <= 1e-9 * max(np.abs(do).max(), 1e-300)


def test_slip_adjoint_matches_oracle(loop):
    inst, P, ck_o, S, ck, t0, fg, T = loop
    Uo, Po, dpo, do = ck_o[-1]
    r = np.random.default_rng(4)
    U2 = Uo + r.normal(0.0, 3e-7, Uo.size) * (1 - inst.dir_u)      # stick, slip and open points
    flag = P.cohesive(U2, dpo)[2]
    assert all((flag == k).sum() > 0 for k in (0, 1, 2))
    a_new = r.standard_normal((P.nq, 2))
    lam = r.standard_normal(3 * P.N) * (1 - inst.dir_u)
    gU_o, a_old_o = P.slip_adjoint(U2, dpo, a_new, lam)
    gU, a_old = S.slip_adjoint(dev(U2), dev(dpo.reshape(-1)), t0, dev(a_new.reshape(-1)), dev(lam))
    print(f"[slip adjoint] gU {rel(host(gU), gU_o):.1e} a_old {rel(host(a_old), a_old_o.reshape(-1)):.1e}", flush=True)
    assert rel(host(gU), gU_o) < 1e-12
    assert rel(host(a_old), a_old_o.reshape(-1)) < 1e-12
    _, a_old0 = S.slip_adjoint(dev(U2), dev(dpo.reshape(-1)), t0, dev(a_new.reshape(-1)))
    assert rel(host(a_old0), P.slip_adjoint(U2, dpo, a_new)[1].reshape(-1)) < 1e-12


def test_loop_gradient_matches_oracle_and_differences(loop):
    inst, P, ck_o, S, ck, t0, fg, T = loop
    uplift = I.uplift_nodes(inst, 8)
    jg = objective(inst, uplift)
    dE_o, dk_o = P.trajectory_gradient(ck_o, lambda n, U, Pp: (jg(U)[1], np.zeros(P.N)))
    print("[loop gradient] oracle reverse sweep done", flush=True)
    logk = dev(inst.logk)
    # iteration caps about 100 times the counts these solves take, so that a solve that
    # stalls at its floor ends with an error instead of running a million iterations
    dE, dk, infos = T.gradient(S, ck, t0, logk, lambda n, U, Pp: (dev(jg(host(U))[1]), torch.zeros_like(Pp)),
                               inner_k=fg.opts(tol=1e-14, max_iter=50000), inner_p=fg.opts(tol=1e-14, max_iter=50000),
                               outer_tol=1e-13, defect_tol=1e-12, max_defect_iters=100,
                               log=lambda s: print(s, flush=True))
    print(f"[loop gradient] dE {rel(host(dE), dE_o):.1e} dlnk {rel(host(dk), dk_o):.1e}; defect iterations "
          f"{[i.newton_iters for i in infos]}", flush=True)
    assert rel(host(dE), dE_o) < 1e-7 and rel(host(dk), dk_o) < 1e-7
    # central differences of the GPU loop along one seeded direction in (ln k, ln E)
    ne = inst.E.size
    d = I.fd_directions(2 * ne, count=1, seed=2)[0]
    grad = np.r_[host(dk), host(dE) * inst.E]

    def J(x):
        S.assemble(inst.params, inst.E * np.exp(x[ne:]), inst.logk + x[:ne])
        U, Pp, die = dev(np.zeros(3 * S.N)), dev(np.zeros(S.N)), dev(np.zeros(2 * S.nq))
        # 1e-12: the perturbed loops' Newton floors sit just above 1e-13; 1e-12 in J is
        # 1e-7 of the difference quotient at this step
        ckx, _ = T.run(S, U, Pp, die, t0, dev(np.zeros(3 * S.N)), dev(inst.source), 4, **tight(fg, 1e-12))
        print("[loop gradient] perturbed forward loop done", flush=True)
        return sum(jg(host(c[0]))[0] for c in ckx)
    eps = 1e-5
    fd = (J(eps * d) - J(-eps * d)) / (2 * eps)
    S.assemble(inst.params, inst.E, inst.logk)
    print(f"[loop gradient] fd {fd:.9e} adjoint {grad @ d:.9e}", flush=True)
    assert abs(fd - grad @ d) <= 1e-5 * abs(fd)


def test_autograd_loop_gradient_equals_reverse_sweep(loop):
    """ImplicitLoop (torch.autograd.Function) on the same 4-step loop: the objective summed
    over the steps in torch, backward through the loop, equals the oracle's reverse sweep."""
    inst, P, ck_o, S, ck, t0, fg, T = loop
    from paper_2410_17133_amd.autograd import ImplicitLoop, fault_slip_uplift_objective
    uplift = I.uplift_nodes(inst, 8)
    jg = objective(inst, uplift)
    dE_o, dk_o = P.trajectory_gradient(ck_o, lambda n, U, Pp: (jg(U)[1], np.zeros(P.N)))
    print("[autograd loop] oracle reverse sweep done", flush=True)
    m = inst.mesh
    X = m.xyz[m.coh[0, 3:]]
    nrm = np.cross(X[1] - X[0], X[2] - X[0])
    logk = dev(inst.logk).requires_grad_(True)
    E = dev(inst.E).requires_grad_(True)
    solver = dict(newton_tol=1e-13, inner_tol=1e-14, outer_tol=1e-13, adjoint_outer_tol=1e-13,
                  adjoint_inner_tol=1e-14)
    U_all, P_all = ImplicitLoop.apply(logk, E, S, inst.params, t0, dev(np.zeros(3 * S.N)), dev(inst.source), 4,
                                      solver)
    pairs = torch.as_tensor(m.pairs.astype(np.int64)).cuda()
    up = torch.as_tensor(uplift.astype(np.int64)).cuda()
    J = sum(fault_slip_uplift_objective(U_all[n], pairs, dev(nrm / np.linalg.norm(nrm)), up) for n in range(4))
    print("[autograd loop] forward loop done", flush=True)
    J.backward()
    print(f"[autograd loop] dE {rel(host(E.grad), dE_o):.1e} dlnk {rel(host(logk.grad), dk_o):.1e}", flush=True)
    assert rel(host(E.grad), dE_o) < 1e-7 and rel(host(logk.grad), dk_o) < 1e-7


def test_loop_with_mixed_amg_solves_matches_oracle(loop):
    """The same 4-step loop and its reverse sweep with every K solve by the FP64 CG whose
    AMG V-cycle runs in FP32 ("k_precond" 3 with FG_MIXED): states and gradient equal the
    oracle's to the bounds of the point-Jacobi runs (1e-9, 1e-7), since the preconditioner
    changes the iterations, not the solutions the tolerances fix; the AMG hierarchy's
    values and their FP32 copies are rebuilt at every change of the tangent."""
    inst, P, ck_o, S, ck, t0, fg, T = loop
    uplift = I.uplift_nodes(inst, 8)
    jg = objective(inst, uplift)
    dE_o, dk_o = P.trajectory_gradient(ck_o, lambda n, U, Pp: (jg(U)[1], np.zeros(P.N)))
    print("[mixed amg loop] oracle reverse sweep done", flush=True)
    mk = fg.opts(tol=1e-14, max_iter=50000, precision=fg.FG_MIXED)
    kw = tight(fg)
    kw["inner_k"] = mk
    S.tune("k_precond", 3)
    try:
        U, Pp, die = dev(np.zeros(3 * S.N)), dev(np.zeros(S.N)), dev(np.zeros(2 * S.nq))
        ck2, infos = T.run(S, U, Pp, die, t0, dev(np.zeros(3 * S.N)), dev(inst.source), 4, **kw)
        print(f"[mixed amg loop] forward loop done, K iterations {[i.inner_k_iters for i in infos]}", flush=True)
        for n, ((Uo, Po, dpo, do), (Un, Pn, dp, d)) in enumerate(zip(ck_o, ck2)):
            print(f"[mixed amg loop] step {n}: U {rel(host(Un), Uo):.1e} P {rel(host(Pn), Po):.1e}", flush=True)
            assert rel(host(Un), Uo) < 1e-9 and rel(host(Pn), Po) < 1e-9
            assert np.abs(host(d) - do.reshape(-1)).max() <= 1e-9 * max(np.abs(do).max(), 1e-300)
        dE, dk, ainfos = T.gradient(S, ck2, t0, dev(inst.logk),
                                    lambda n, Un, Pn: (dev(jg(host(Un))[1]), torch.zeros_like(Pn)),
                                    inner_k=mk, inner_p=fg.opts(tol=1e-14, max_iter=50000), outer_tol=1e-13,
                                    defect_tol=1e-12, max_defect_iters=100, log=lambda s: print(s, flush=True))
    finally:
        S.tune("k_precond", 0)
    print(f"[mixed amg loop] dE {rel(host(dE), dE_o):.1e} dlnk {rel(host(dk), dk_o):.1e}", flush=True)
    assert all(i.status == 0 for i in ainfos)
    assert rel(host(dE), dE_o) < 1e-7 and rel(host(dk), dk_o) < 1e-7
