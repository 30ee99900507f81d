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
