"""The allocation-free K / A22 solve (fg_pcg_solve_noalloc) against fg_pcg_solve on
the same systems and right-hand sides, through the C-ABI: same kernels, same
launch shapes, so the iterates agree to rounding (the existing entry point
replays captured graphs of the same kernels).  Two calls in a row, the second on
a smaller system, share the library's fixed per-GPU scratch."""
import numpy as np
import pytest

from paper_2410_17133_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve_pair(fg, S, which, seed, tol=1e-12):
    n = (3 if which == fg.FG_K else 1) * S.N
    g = np.random.default_rng(seed)
    b = torch.as_tensor(g.standard_normal(n)).cuda()
    x_ref, info_ref = S.pcg_solve(which, b, tol=tol)
    x = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    info = S.pcg_solve_noalloc(which, b, x, tol=tol)
    torch.cuda.synchronize()
    xr, xn = x_ref.cpu().numpy(), x.cpu().numpy()
    err = np.linalg.norm(xn - xr) / np.linalg.norm(xr)
    print(f"[case] noalloc which={which} N={S.N} iters {info.iters}/{info_ref.iters} relerr {err:.2e}", flush=True)
    assert info.status == fg.FG_OK and info_ref.status == fg.FG_OK
    assert info.iters == info_ref.iters
    assert err <= 1e-12
    return info


def test_noalloc_matches_pcg_solve_two_calls_shrinking():
    from paper_2410_17133_amd import fg
    ctx = fg.Context(0)
    big = I.make_instance(I.cube_config(12, dip_deg=60, heterogeneous=True))
    small = I.make_instance(I.config(1))
    Sb = fg.System.from_instance(ctx, big)
    Sb.assemble(big.params, big.E, big.logk)
    Ss = fg.System.from_instance(ctx, small)
    Ss.assemble(small.params, small.E, small.logk)
    for which in (fg.FG_K, fg.FG_A22):
        _solve_pair(fg, Sb, which, 1)
        _solve_pair(fg, Ss, which, 2)        # second call, smaller input, same scratch
    # the existing entry point still works after the scratch-backed calls
    _solve_pair(fg, Sb, fg.FG_K, 3)


def test_noalloc_rejects_bad_arguments():
    from paper_2410_17133_amd import fg
    ctx = fg.Context(0)
    inst = I.make_instance(I.cube_config(4))
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    b = torch.ones(3 * S.N, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(fg.FgError) as e:
        S.pcg_solve_noalloc(fg.FG_K, b, x, precision=fg.FG_MIXED)
    assert e.value.status == fg.FG_ERR_ARG
    with pytest.raises(fg.FgError) as e:
        S.pcg_solve_noalloc(fg.FG_KBULK, b, x)
    assert e.value.status == fg.FG_ERR_ARG


def test_noalloc_rejects_a_solve_beyond_the_scratch():
    """A 96^3 cube's K solve needs 4 x 2.8 M doubles of CG vectors: more than the
    fixed scratch holds.  The call refuses it before launching anything."""
    from paper_2410_17133_amd import fg
    ctx = fg.Context(0)
    inst = I.make_instance(I.cube_config(96))
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    b = torch.ones(3 * S.N, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(fg.FgError) as e:
        S.pcg_solve_noalloc(fg.FG_K, b, x)
    assert e.value.status == fg.FG_ERR_ARG
    assert "scratch" in str(e.value)
    # the A22 solve of the same mesh (0.94 M unknowns) fits
    bp = torch.ones(S.N, dtype=torch.float64, device="cuda")
    xp = torch.zeros_like(bp)
    info = S.pcg_solve_noalloc(fg.FG_A22, bp, xp, tol=1e-10)
    assert info.status == fg.FG_OK
