"""The injection-into-a-frictional-fault workload of Sec. 4.2 on the GPU against
the oracle, through the C-ABI: the same graded box, materials and loads as the
oracle's slip-front pins, stepped from rest with tight tolerances on both sides.
After every step the interface states must agree point by point (stick / slip
flags exactly, except at points whose yield value is within the solvers'
tolerance of zero, where either decision is correct), and U, P and the
inelastic slip to 1e-9 relative L2; the slip fronts are then the same."""
import numpy as np
import pytest

from paper_2410_17133_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

B = I.SLIP_BENCHMARK


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("case", ["CS", "MP"])
def test_slip_benchmark_steps_match_oracle(case):
    from oracle import oracle as O
    from paper_2410_17133_amd import fg
    # Newton tolerance: each case's flow residual stagnates about 10x below it (the
    # tied lips' transverse conductance times dt sets the FP64 floor)
    if case == "CS":
        inst = I.slip_benchmark_instance(B["tau0_CS"], h=0.1, n_fine=16, n_grade=6, nx_grade=7, dt=4.0)
        steps, ntol = 2, 1e-11
    else:
        inst = I.slip_benchmark_instance(B["tau0_MP"], h=0.05, n_fine=16, n_grade=10, nx_grade=7, dt=870.0)
        steps, ntol = 1, 1e-10
    print(f"[case] slip benchmark {case}: {inst.mesh.n_nodes} nodes, {inst.mesh.coh.shape[0]} interface "
          f"elements, {steps} steps of {inst.params.dt} s", flush=True)
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    P = O.Problem(inst)
    N, nq = S.N, S.nq
    U, Pg, die = dev(np.zeros(3 * N)), dev(np.zeros(N)), dev(np.zeros(2 * nq))
    t0, load, src = dev(inst.t0.reshape(-1)), dev(inst.load), dev(inst.source)
    Uo, Po, dieo = np.zeros(3 * N), np.zeros(N), np.zeros((nq, 2))
    f, ks = B["friction"], B["k_s"]
    for s in range(1, steps + 1):
        die_start = dieo.copy()
        trac, flag, info = S.step(U, Pg, die, t0, load, src, newton_tol=ntol, inner_k=fg.opts(tol=1e-13),
                                  inner_p=fg.opts(tol=1e-13), outer_tol=1e-12)
        trac_o, flag_o, info_o, st = P.step(Uo, Po, dieo, tol_newton=ntol, tol_outer=1e-12, tol_inner=1e-13)
        print(f"[step {s}] gpu {info.as_dict()} oracle {info_o.tolist()}", flush=True)
        assert info.status == 0 and st == 0
        flag, trac = host(flag), host(trac).reshape(-1, 3)
        # yield value of the oracle's trial traction at each point (k_s times the slip
        # increment where it slipped); a tie within the solvers' tolerance may fall either way
        slip = flag_o == 1
        F = np.where(slip, ks * np.linalg.norm(dieo - die_start, axis=1),
                     np.hypot(trac_o[:, 1], trac_o[:, 2]) - f * trac_o[:, 0])
        tie = np.abs(F) <= 1e-8 * f * B["sigma0"]
        mism = (flag != flag_o) & ~tie
        eu, ep = relerr(host(U), Uo), relerr(host(Pg), Po)
        ed = relerr(host(die).reshape(-1, 2), dieo)
        print(f"[step {s}] newton gpu {info.newton_iters} oracle {int(info_o[0])}; slip points {int(slip.sum())}, "
              f"ties {int(tie.sum())}, flag mismatches {int((flag != flag_o).sum())}; rel err U {eu:.2e} "
              f"P {ep:.2e} slip {ed:.2e}", flush=True)
        assert slip.sum() > 0 and not np.any(flag_o == 2)
        assert not mism.any()
        assert eu <= 1e-9 and ep <= 1e-9 and ed <= 1e-9
        assert np.abs(trac - trac_o).max() <= 1e-9 * B["sigma0"]
