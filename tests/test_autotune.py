"""Autotuner search and cache (CPU), and tuning on a real system (GPU)."""
import numpy as np
import pytest

from paper_2410_17133_amd import autotune as AT


def test_coordinate_descent_finds_the_separable_minimum():
    cands = {"a": [0, 1, 2, 3], "b": [10, 20, 30], "c": [5, 6]}
    cost = lambda cfg: (cfg["a"] - 2) ** 2 + (cfg["b"] - 30) ** 2 / 100 + (cfg["c"] == 5)
    calls = []
    best, t, log = AT.coordinate_descent(cands, {"a": 0, "b": 10, "c": 5}, lambda c: calls.append(c) or cost(c))
    assert best == {"a": 2, "b": 30, "c": 6} and t == 0
    assert len(log) == len(calls)
    # the start is measured once and no candidate equal to the incumbent is re-measured within a pass
    assert calls[0] == {"a": 0, "b": 10, "c": 5}


def test_coordinate_descent_keeps_the_start_when_nothing_is_faster():
    best, t, log = AT.coordinate_descent({"a": [1, 2]}, {"a": 0}, lambda c: 1.0 + c["a"])
    assert best == {"a": 0} and t == 1.0 and len(log) == 3


def test_candidates():
    c = AT.single_candidates(238.0)
    assert c["halo_cap"][0] == 0 and 682 in c["halo_cap"] and c["halo_cap"] == sorted(c["halo_cap"])
    assert all(v % 32 == 0 for v in c["halo_cap"] if v not in (0, 682))
    assert AT.block_candidates(4)["rhs_tile"] == [0, 1, 2, 4]
    assert AT.block_candidates(4)["mr_form"] == []            # the row-group product needs 8 columns
    assert AT.DEFAULTS["mr_form"] in AT.block_candidates(32)["mr_form"]


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "tune.json")
    c = AT.Cache(p)
    assert c.get("k") is None
    c.put("k", {"config": {"rhs_tile": 0}, "us_per_iteration": 12.5})
    assert AT.Cache(p).get("k") == {"config": {"rhs_tile": 0}, "us_per_iteration": 12.5}


@pytest.mark.gpu
def test_tuning_a_system_keeps_its_results(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import inputs as I
    inst = I.make_instance(I.cube_config(16, dip_deg=60.0, heterogeneous=True))
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64)).cuda()
    S.cohesive_update(dev(np.zeros(3 * S.N)), dev(np.zeros(2 * S.nq)), dev(inst.t0.reshape(-1)))
    b = dev(np.random.default_rng(3).standard_normal(3 * S.N) * (1 - inst.dir_u))
    x0, i0 = S.pcg_solve(fg.FG_K, b, tol=1e-10)
    cache = AT.Cache(str(tmp_path / "tune.json"))
    rec = AT.tune_single(S, fg.FG_K, fg.FG_F64, iters=20, cache=cache)
    assert set(rec["config"]) == set(AT.SINGLE_KNOBS) and rec["us_per_iteration"] > 0
    x1, i1 = S.pcg_solve(fg.FG_K, b, tol=1e-10)
    torch.cuda.synchronize()
    # dot products may be grouped differently: the same convergence to rounding, and the
    # FP64 true residual meets the tolerance
    assert abs(i1.iters - i0.iters) <= 0.02 * i0.iters
    assert torch.linalg.norm(b - S.spmv(fg.FG_K, x1)) <= 2e-10 * torch.linalg.norm(b)
    assert AT.tune_single(S, fg.FG_K, fg.FG_F64, cache=cache) == rec   # served from the cache
    B = dev(np.random.default_rng(4).standard_normal((8, 3 * S.N)) * (1 - inst.dir_u))
    X0, _ = S.pcg_solve(fg.FG_K, B.reshape(-1), nrhs=8, tol=1e-10)
    rb = AT.tune_block(S, 8, fg.FG_F64, iters=10, cache=cache)
    assert rb["config"]["rhs_tile"] in AT.block_candidates(8)["rhs_tile"]
    assert rb["config"]["mr_form"] in AT.block_candidates(8)["mr_form"]
    X1, _ = S.pcg_solve(fg.FG_K, B.reshape(-1), nrhs=8, tol=1e-10)
    X0, X1 = X0.cpu().numpy().reshape(8, -1), X1.cpu().numpy().reshape(8, -1)
    for c in range(8):
        assert np.linalg.norm(X1[c] - X0[c]) <= 1e-8 * np.linalg.norm(X0[c])
