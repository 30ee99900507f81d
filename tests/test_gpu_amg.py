"""The smoothed-aggregation AMG preconditioner of K ("k_precond" 3) on the GPU
against the oracle's, through the C-ABI: the same hierarchy (levels and nodes
per level), the same AMG-PCG iterates, the same converged solution, in a small
fraction of the block-Jacobi iterations.  Both sides take the level-0 smoother's
interval from their own Lanczos estimate (equal to about 1e-8), so the iterates
are compared to 1e-6 and the converged solutions to 1e-9."""
import numpy as np
import pytest

from paper_2410_17133_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n,dip,slip", [(8, 90.0, False), (12, 60.0, True), (16, 35.0, False)])
def test_amg_pcg_matches_oracle(n, dip, slip):
    from oracle import oracle as O
    from paper_2410_17133_amd import fg
    inst = I.make_instance(I.cube_config(n, dip_deg=dip, heterogeneous=n > 8))
    print(f"[case] AMG {n}^3 dip {dip} slip {slip}", flush=True)
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    P = O.Problem(inst)
    r = np.random.default_rng(40 + n)
    U = r.normal(0.0, 2e-5 / n, 3 * S.N) * (1 - inst.dir_u) if slip else np.zeros(3 * S.N)
    P.cohesive(U, np.zeros((P.nq, 2)))
    S.cohesive_update(dev(U), dev(np.zeros(2 * S.nq)), dev(inst.t0.reshape(-1)))
    hi0 = P.cheb_bounds(40, 1.1, 300)[1]
    b = r.standard_normal(3 * S.N) * (1 - inst.dir_u)
    xo20 = P.pcg_amg(b, hi0, tol=1e-300, maxit=20)[0]
    xo, st, ito, rro, levels, nodes = P.pcg_amg(b, hi0, tol=1e-12)
    _, _, itb, _ = P.pcg_block(b, tol=1e-12)
    S.tune("k_precond", 3)
    try:
        gl, gnodes = S.amg_levels()
        # the aggregation is integer work: every level's aggregate map equals the oracle's exactly
        for lev in range(gl - 1):
            np.testing.assert_array_equal(S.amg_aggregates(lev), P.amg_export(hi0, lev, 2))
        x20, i20 = S.pcg_solve(fg.FG_K, dev(b), tol=1e-300, max_iter=20)
        x, info = S.pcg_solve(fg.FG_K, dev(b), tol=1e-12)
    finally:
        S.tune("k_precond", 0)
    x20, x = x20.cpu().numpy(), x.cpu().numpy()
    print(f"[amg] levels gpu {gl} {list(gnodes)} oracle {levels} {list(nodes)}; iterations gpu {info.iters} "
          f"oracle {ito} (block Jacobi {itb}); 20 iterates {relerr(x20, xo20):.1e}, solution {relerr(x, xo):.1e}",
          flush=True)
    assert gl == levels and list(gnodes) == list(nodes)
    assert i20.iters == 20 and relerr(x20, xo20) < 1e-6
    assert info.status == 0 and st == 0 and abs(info.iters - ito) <= 1
    assert relerr(x, xo) < 1e-9
    assert np.linalg.norm(b - P.spmv(O.K_TANGENT, x)) <= 1e-11 * np.linalg.norm(b)
    assert 4 * info.iters < itb


@pytest.mark.parametrize("n,dip", [(12, 60.0), (16, 35.0)])
def test_mixed_amg_reaches_the_oracle_solution(n, dip):
    """FG_MIXED with the AMG preconditioner: FP64 CG whose V-cycle runs on FP32 copies
    of the hierarchy.  Rounding the cycle perturbs the preconditioner, not the FP64
    recurrence that decides the solution, so each solve to 1e-12 reaches the
    oracle's FP64 AMG-PCG solution to 1e-9 (the bound of the FP64 cycle) with its
    true residual (the oracle's product) within 1e-11, in at most 10% (+2) more
    iterations.  A second right-hand side after a change of the tangent (a
    displacement with slip points) checks that the FP32 copies follow K."""
    from oracle import oracle as O
    from paper_2410_17133_amd import fg
    inst = I.make_instance(I.cube_config(n, dip_deg=dip, heterogeneous=True))
    print(f"[case] mixed AMG {n}^3 dip {dip}", flush=True)
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    P = O.Problem(inst)
    r = np.random.default_rng(60 + n)
    U0 = np.zeros(3 * S.N)
    U1 = r.normal(0.0, 2e-5 / n, 3 * S.N) * (1 - inst.dir_u)
    S.tune("k_precond", 3)
    try:
        for k, U in enumerate((U0, U1)):
            P.cohesive(U, np.zeros((P.nq, 2)))
            S.cohesive_update(dev(U), dev(np.zeros(2 * S.nq)), dev(inst.t0.reshape(-1)))
            hi0 = P.cheb_bounds(40, 1.1, 300)[1]
            b = r.standard_normal(3 * S.N) * (1 - inst.dir_u)
            xo, st, ito, _, _, _ = P.pcg_amg(b, hi0, tol=1e-12)
            x, info = S.pcg_solve(fg.FG_K, dev(b), tol=1e-12, precision=fg.FG_MIXED)
            x = x.cpu().numpy()
            res = np.linalg.norm(b - P.spmv(O.K_TANGENT, x)) / np.linalg.norm(b)
            print(f"[mixed amg] tangent {k}: iterations fp32 cycle {info.iters}, oracle fp64 cycle {ito}; "
                  f"solution {relerr(x, xo):.1e}, true residual {res:.1e}", flush=True)
            assert st == 0 and info.status == 0 and info.cycles == 1
            assert info.iters <= 1.1 * ito + 2
            assert relerr(x, xo) < 1e-9 and res <= 1e-11
    finally:
        S.tune("k_precond", 0)


@pytest.mark.parametrize("cfg", ["cube8", "slip4", "cube8-mixed", "slip4-exact"])
def test_step_with_amg_reaches_the_same_state(cfg):
    """A full implicit step (Newton, partitioned CG) whose FP64 K solves are
    preconditioned by the AMG V-cycle ends in the oracle's converged state; the
    hierarchy's values are rebuilt at every change of the tangent.  -mixed: the
    V-cycle in FP32; -exact: Newton on the exact tangent K_t + N, whose BiCGStab
    solves take the V-cycle of K_t as preconditioner."""
    from oracle import oracle as O
    from paper_2410_17133_amd import fg
    import dataclasses
    if cfg.startswith("cube8"):
        inst = I.make_instance(I.cube_config(8))
    else:                                              # a higher injection rate: slip points in the step
        inst = I.make_instance(dataclasses.replace(I.cube_config(4), Q=4e-3))
    print(f"[case] AMG step {cfg}", flush=True)
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    P = O.Problem(inst)
    N, nq = S.N, S.nq
    Uo, Po, dieo = np.zeros(3 * N), np.zeros(N), np.zeros((nq, 2))
    _, flag_o, _, st = P.step(Uo, Po, dieo, tol_newton=1e-11, max_newton=60, tol_outer=1e-12, tol_inner=1e-13)
    assert st == 0
    S.tune("k_precond", 3)
    S.tune("exact_tangent", 1 if "exact" in cfg else 0)
    try:
        U, Pp, die = dev(np.zeros(3 * N)), dev(np.zeros(N)), dev(np.zeros(2 * nq))
        trac, flag, info = S.step(U, Pp, die, dev(inst.t0.reshape(-1)), dev(inst.load), dev(inst.source),
                                  newton_tol=1e-11, newton_max_iter=60,
                                  inner_k=fg.opts(tol=1e-13, precision=fg.FG_MIXED if "mixed" in cfg else fg.FG_F64),
                                  inner_p=fg.opts(tol=1e-13), outer_tol=1e-12)
    finally:
        S.tune("exact_tangent", 0)
        S.tune("k_precond", 0)
    eu, ep = relerr(U.cpu().numpy(), Uo), relerr(Pp.cpu().numpy(), Po)
    print(f"[amg step] {cfg}: newton {info.newton_iters}, K iterations {info.inner_k_iters}, slip points "
          f"{int((flag_o == 1).sum())}; rel err U {eu:.1e} P {ep:.1e}", flush=True)
    assert info.status == 0
    assert eu < 1e-9 and ep < 1e-9


def test_amg_on_a_mesh_below_the_coarsening_threshold_is_a_direct_solve():
    """A mesh of no more than "amg_coarse" nodes is the coarsest level itself: the
    preconditioner is the exact inverse (the slices' padding rows decoupled), PCG
    converges in one or two iterations, and the solution equals the oracle's."""
    from oracle import oracle as O
    from paper_2410_17133_amd import fg
    inst = I.make_instance(I.cube_config(2))
    print(f"[case] AMG one level, {inst.mesh.n_nodes} nodes", flush=True)
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    P = O.Problem(inst)
    P.cohesive(np.zeros(3 * P.N), np.zeros((P.nq, 2)))
    S.cohesive_update(dev(np.zeros(3 * S.N)), dev(np.zeros(2 * S.nq)), dev(inst.t0.reshape(-1)))
    hi0 = P.cheb_bounds(40, 1.1, 300)[1]
    b = np.random.default_rng(7).standard_normal(3 * S.N) * (1 - inst.dir_u)
    xo, st, ito, rro, levels, nodes = P.pcg_amg(b, hi0, tol=1e-12)
    S.tune("k_precond", 3)
    try:
        gl, gnodes = S.amg_levels()
        x, info = S.pcg_solve(fg.FG_K, dev(b), tol=1e-12)
        # the FP32 cycle: the exact inverse rounded to FP32 inside the FP64 CG
        xm, im = S.pcg_solve(fg.FG_K, dev(b), tol=1e-12, precision=fg.FG_MIXED)
    finally:
        S.tune("k_precond", 0)
    x, xm = x.cpu().numpy(), xm.cpu().numpy()
    print(f"[amg one level] levels gpu {gl} oracle {levels}; iterations gpu {info.iters} oracle {ito}; "
          f"solution {relerr(x, xo):.1e}; FP32 cycle {im.iters} iterations, solution {relerr(xm, xo):.1e}",
          flush=True)
    assert gl == levels == 1 and list(gnodes) == list(nodes)
    assert info.status == 0 and st == 0 and info.iters <= 2 and abs(info.iters - ito) <= 1
    assert relerr(x, xo) < 1e-9
    assert im.status == 0 and im.iters <= 8 and relerr(xm, xo) < 1e-9


def test_amg_edge_cases():
    """A zero right-hand side (x = 0 at once), an iteration cap (FG_NOT_CONVERGED with
    the iterate so far, as the oracle's capped AMG-PCG), a new "amg_coarse" (the
    hierarchy rebuilt, as the oracle builds it with the same threshold) and
    out-of-range knobs (rejected); the first three with the FP32 cycle too."""
    from oracle import oracle as O
    from paper_2410_17133_amd import fg
    inst = I.make_instance(I.cube_config(12, dip_deg=60.0, heterogeneous=True))
    print("[case] AMG edge cases 12^3", flush=True)
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    P = O.Problem(inst)
    P.cohesive(np.zeros(3 * P.N), np.zeros((P.nq, 2)))
    S.cohesive_update(dev(np.zeros(3 * S.N)), dev(np.zeros(2 * S.nq)), dev(inst.t0.reshape(-1)))
    hi0 = P.cheb_bounds(40, 1.1, 300)[1]
    b = np.random.default_rng(3).standard_normal(3 * S.N) * (1 - inst.dir_u)
    S.tune("k_precond", 3)
    try:
        for prec in (fg.FG_F64, fg.FG_MIXED):
            x0, i0 = S.pcg_solve(fg.FG_K, dev(np.zeros(3 * S.N)), tol=1e-10, precision=prec)
            assert i0.status == 0 and i0.iters == 0 and not x0.abs().max().item()
        xc, ic = S.pcg_solve(fg.FG_K, dev(b), tol=1e-14, max_iter=7)
        xoc, stc, itc, _, _, _ = P.pcg_amg(b, hi0, tol=1e-14, maxit=7)
        assert ic.status == fg.FG_NOT_CONVERGED and ic.iters == itc == 7 and stc == 1
        assert relerr(xc.cpu().numpy(), xoc) < 1e-6
        _, icm = S.pcg_solve(fg.FG_K, dev(b), tol=1e-14, max_iter=7, precision=fg.FG_MIXED)
        assert icm.status == fg.FG_NOT_CONVERGED and icm.iters == 7
        levels_64 = S.amg_levels()
        S.tune("amg_coarse", 200)                   # coarsening stops one level earlier
        gl, gnodes = S.amg_levels()
        _, st, ito, _, levels, nodes = P.pcg_amg(b, hi0, coarse_nodes=200, tol=1e-12)
        assert gl == levels < levels_64[0] and list(gnodes) == list(nodes)
        x, info = S.pcg_solve(fg.FG_K, dev(b), tol=1e-12)
        assert info.status == 0 and abs(info.iters - ito) <= 1
        xm, im = S.pcg_solve(fg.FG_K, dev(b), tol=1e-12, precision=fg.FG_MIXED)   # FP32 copies of the new hierarchy
        assert im.status == 0 and im.iters <= 1.1 * ito + 2
        assert relerr(xm.cpu().numpy(), x.cpu().numpy()) < 1e-9
        for bad in (0, 1001):
            with pytest.raises(fg.FgError):
                S.tune("amg_coarse", bad)
        with pytest.raises(fg.FgError):
            S.tune("k_precond", 4)
    finally:
        S.tune("amg_coarse", 64)
        S.tune("k_precond", 0)
    print(f"[amg edge] levels {levels_64[0]} -> {gl} with amg_coarse 200; capped at 7 iterations; zero rhs ok",
          flush=True)
