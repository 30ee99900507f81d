"""Autotuner for the launch parameters of the CG products (the fg_tune knobs).

The knobs change how the products stream memory, not what they compute
(spmv_wpb and vec_grid regroup the partial sums of the dot products, so results
agree to rounding; the others give bitwise the same iterates):

  single-vector CG (K FP64, K FP32, A22):  halo_cap, spmv_unroll, spmv_nt,
                                           spmv_wpb, vec_grid
  block CG (many right-hand sides on K):   rhs_tile, mr_form

Each candidate is timed on the system it will run on, a few dozen CG iterations
long; the search is coordinate descent from the library defaults (every value of
one knob with the others held, best kept, knobs in turn, twice over).  Results
are cached in a JSON file keyed by device, operator sizes and workload, so a
run tunes once per machine and problem shape.

Each candidate is timed as wall time per CG iteration over a fixed number of
graph-replayed iterations (after one untimed run that captures the graphs), the
better of two runs; this covers the product and the vector kernels alike.
"""
from __future__ import annotations

import json
import os
import time

from . import fg

SINGLE_KNOBS = ("halo_cap", "spmv_unroll", "spmv_nt", "spmv_wpb", "vec_grid")
BLOCK_KNOBS = ("rhs_tile", "mr_form")
DEFAULTS = {"spmv_unroll": 2, "spmv_nt": 23, "spmv_wpb": 4, "vec_grid": 512, "rhs_tile": 0, "mr_form": 2}


def single_candidates(mean_halo: float) -> dict:
    """Values tried per knob; halo caps are taken relative to the mean slice halo."""
    caps = sorted({0, 682, *(int(round(mean_halo * f / 32.0)) * 32 for f in (1.0, 1.25, 1.5, 2.0))})
    return {"halo_cap": caps, "spmv_unroll": [1, 2, 3, 4, 6], "spmv_nt": [0, 1, 3, 7, 15, 23], "spmv_wpb": [1, 2, 4],
            "vec_grid": [512, 1024, 2048]}


def block_candidates(nrhs: int) -> dict:
    forms = [0, 1, 2, 4, 9, 10, 12, 17, 18, 25, 26] if nrhs >= 8 else []
    return {"rhs_tile": [0] + [t for t in (1, 2, 4, 8, 16) if t <= nrhs], "mr_form": forms}


def coordinate_descent(candidates: dict, start: dict, measure, passes: int = 2) -> tuple:
    """Minimise measure(config) one knob at a time.  Returns (best config, best time, log)."""
    best = dict(start)
    best_t = measure(best)
    log = [(dict(best), best_t)]
    for _ in range(passes):
        improved = False
        for knob, values in candidates.items():
            for v in values:
                if v == best.get(knob):
                    continue
                trial = dict(best)
                trial[knob] = v
                t = measure(trial)
                log.append((dict(trial), t))
                if t < best_t:
                    best, best_t, improved = trial, t, True
        if not improved:
            break
    return best, best_t, log


class Cache:
    """JSON cache of tuned configurations (path None: in memory only)."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key):
        return self.data.get(key)

    def put(self, key, value):
        self.data[key] = value
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _device_name():
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


def _key(S, kind, **extra):
    npairs, nblk, nslices, nhalo = S.sizes()
    parts = [_device_name(), kind, f"N={S.N}", f"blocks={npairs}", f"slices={nslices}", f"halo={nhalo}",
             f"groups={S.ngroups}"] + [f"{k}={v}" for k, v in sorted(extra.items())]
    return "|".join(parts)


def apply(S, config: dict):
    for k, v in config.items():
        S.tune(k, int(v))


def _iteration_time(S, run, iters):
    import torch
    run()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(2):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) / iters * 1e6)
    return best


def tune_single(S, which: int = fg.FG_K, precision: int = fg.FG_F64, b=None, iters: int = 64,
                cache: Cache | None = None, passes: int = 2) -> dict:
    """Tune the single-vector CG on `which` of S (assembled); leaves the best
    configuration applied and returns it with its time per iteration in microseconds."""
    import torch
    op = "K" if which == fg.FG_K else "A22"
    if which == fg.FG_A22:
        precision = fg.FG_F64
    key = _key(S, "single", op=op, precision=precision)
    if cache is not None and cache.get(key):
        rec = cache.get(key)
        apply(S, rec["config"])
        return rec
    n = (3 if which == fg.FG_K else 1) * S.N
    if b is None:
        g = torch.Generator(device="cpu").manual_seed(0)
        b = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    npairs, nblk, nslices, nhalo = S.sizes()
    cands = single_candidates(nhalo / max(nslices, 1))
    start = {"halo_cap": 384, **{k: DEFAULTS[k] for k in ("spmv_unroll", "spmv_nt", "spmv_wpb", "vec_grid")}}

    def measure(cfg):
        apply(S, cfg)
        return _iteration_time(S, lambda: S.pcg_solve(which, b, tol=1e-300, max_iter=iters, check_every=iters,
                                                      precision=precision), iters)

    cfg, t, log = coordinate_descent({k: cands[k] for k in SINGLE_KNOBS}, start, measure, passes)
    apply(S, cfg)
    rec = {"config": cfg, "us_per_iteration": t, "trials": len(log)}
    if cache is not None:
        cache.put(key, rec)
    return rec


def tune_block(S, nrhs: int, precision: int = fg.FG_F64, B=None, iters: int = 30,
               cache: Cache | None = None) -> dict:
    """Tune the block product for nrhs columns on K; leaves the best applied and
    returns it with the wall time per block iteration in microseconds."""
    import torch
    key = _key(S, "block", nrhs=nrhs, precision=precision)
    if cache is not None and cache.get(key):
        rec = cache.get(key)
        apply(S, rec["config"])
        return rec
    if B is None:
        g = torch.Generator(device="cpu").manual_seed(0)
        B = torch.randn(nrhs * 3 * S.N, generator=g, dtype=torch.float64).cuda()
    inner = fg.FG_F32 if precision == fg.FG_MIXED else precision

    def measure(cfg):
        apply(S, cfg)
        return _iteration_time(S, lambda: S.pcg_solve(fg.FG_K, B, nrhs=nrhs, tol=1e-300, max_iter=iters,
                                                      check_every=iters, precision=inner), iters)

    cfg, t, log = coordinate_descent(block_candidates(nrhs), {k: DEFAULTS[k] for k in BLOCK_KNOBS}, measure, 1)
    apply(S, cfg)
    rec = {"config": cfg, "us_per_iteration": t, "trials": len(log)}
    if cache is not None:
        cache.put(key, rec)
    return rec
