#!/usr/bin/env python3
"""Benchmark of the partitioned-CG hot path on one MI355X.

Workload: the 128^3-hex unit cube (12,582,912 Kuhn tetrahedra, 2,163,330 nodes
after duplicating the 60-degree fault plane, 32,768 interface triangles),
seeded log-normal permeability and uniform E per tetrahedron.  One timed step
is one iteration of the partitioned (Prevost) CG of the first Newton
correction of an injection step, through the C-ABI:
  interface update with tangent (fg_cohesive_update), Newton residuals
  (fg_residual), then fg_flow_solve limited to one outer iteration: A22 solve,
  coupling A_pu, K solve to 1e-8 relative residual (FP64 Jacobi-PCG),
  coupling A_up, A22 product and the Schur-CG update.
value = K-PCG iterations per second of wall time over the whole step.
Also reported (outside the timed steps): time to a 1e-8 relative residual of
the same K solve in FP64 and in mixed precision, and the live HIP-event
duration of the CG SpMV kernel against the HBM roofline.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="hexes per cube edge (128 = the 12.6M-tet workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=25, help="oracle PCG iterations timed for the CPU baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the time-to-1e-8 comparison")
    ap.add_argument("--profile-iters", type=int, default=0,
                    help="profiling mode for hardware counters: run exactly this many FP64 K-PCG iterations and "
                         "one 1 GiB device copy (counter calibration), print a short JSON line, skip the rest")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver's multi-GPU sharding is not part of this build "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import inputs as I

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    n = args.n
    cfg = I.config(3) if n == 128 else I.cube_config(n, dip_deg=60.0, heterogeneous=True)
    t = time.perf_counter()
    inst = I.make_instance(cfg)
    log(f"instance n={n} nodes={inst.n_nodes} tets={inst.mesh.tets.shape[0]} coh={inst.mesh.coh.shape[0]} "
        f"({time.perf_counter() - t:.1f}s)")
    t = time.perf_counter()
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    npairs, nblk, nslices, nhalo = S.sizes()
    log(f"planned: {npairs} blocks ({nblk} padded), {nslices} slices ({time.perf_counter() - t:.1f}s)")
    t = time.perf_counter()
    S.assemble(inst.params, inst.E, inst.logk)
    torch.cuda.synchronize()
    log(f"assembled ({time.perf_counter() - t:.2f}s)")

    d = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64)).cuda()
    N, nq = S.N, S.nq
    if args.profile_iters > 0:
        S.cohesive_update(d(np.zeros(3 * N)), d(np.zeros(2 * nq)), d(inst.t0.reshape(-1)))
        b = d(np.random.default_rng(0).standard_normal(3 * N) * (1 - inst.dir_u))
        x, info = S.pcg_solve(fg.FG_K, b, tol=1e-30, max_iter=args.profile_iters, check_every=args.profile_iters)
        src_t = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        bytes_launch = 74.0 * npairs + 4.0 * nhalo + 52.0 * N
        print(json.dumps({"profile_iters": info.iters, "spmv_bytes_per_launch": bytes_launch,
                          "copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30}), flush=True)
        return
    t0, src, load = d(inst.t0.reshape(-1)), d(inst.source), d(inst.load)
    U, P, die = d(np.zeros(3 * N)), d(np.zeros(N)), d(np.zeros(2 * nq))
    ik = fg.opts(tol=1e-8, check_every=64)
    ip = fg.opts(tol=1e-8, check_every=64)

    def step():
        trac, die_new, flag, fcoh = S.cohesive_update(U, die, t0, write_tangent=True)
        Rm, Rf = S.residual(U, P, U, P, fcoh, load, src)
        du, dp, info = S.flow_solve(-Rm, -Rf, inner_k=ik, inner_p=ip, outer_tol=1e-10, outer_max_iter=1)
        return info

    for w in range(args.warmup):
        info = step()
        log(f"warmup {w}: K iters {info.inner_k_iters} A22 iters {info.inner_a22_iters}")
    # timed pass: production configuration (CG batches replayed as HIP graphs)
    torch.cuda.synchronize()
    k_iters = 0
    t = time.perf_counter()
    for s in range(args.steps):
        info = step()
        k_iters += info.inner_k_iters
        log(f"step {s}: K iters {info.inner_k_iters} A22 iters {info.inner_a22_iters}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    value = k_iters / elapsed
    # second timed pass of the same steps for the roofline: kernel-by-kernel launches with
    # timing-only HIP events around every CG SpMV on the stream it runs on
    S.profile(True)
    S.profile_read(0, reset=True)
    t = time.perf_counter()
    k_iters_p = 0
    for s in range(args.steps):
        k_iters_p += step().inner_k_iters
    torch.cuda.synchronize()
    elapsed_p = time.perf_counter() - t
    launches, ms = S.profile_read(0, reset=True)
    S.profile(False)
    # algorithmic bytes of one FP64 CG SpMV launch in this storage: each stored 3x3 block
    # (72 B) and its 16-bit halo-local column once, each halo list entry (4 B) once,
    # x read once, q written once (24 B each per node) and the diagonal slot (4 B per node)
    bytes_launch = 74.0 * npairs + 4.0 * nhalo + 52.0 * N
    avg_s = ms / 1e3 / max(launches, 1)
    achieved = bytes_launch / avg_s / 1e9 if launches else 0.0
    out = {
        "metric": "PCG iters/s + HBM GB/s at 128³ tets; time-to-1e-8 mixed vs FP64; adjoint grad/s",
        "value": value,
        "unit": "PCG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"cube{n}_dip60_hetero: {n}^3 hexes, {inst.mesh.tets.shape[0]} tets, {N} nodes, "
                        f"{inst.mesh.coh.shape[0]} interface tris; one partitioned-CG iteration of the first "
                        f"Newton correction (interface update, residuals, A22 solve, coupling, FP64 K solve to 1e-8)",
            "k_iters_per_step": k_iters / args.steps,
            "blocks": npairs,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_cg_spmv<3,double,double>",
            "bytes_per_launch": bytes_launch,
            "avg_launch_us": avg_s * 1e6,
            "launches": launches,
            "timed_pass_iters_per_s": k_iters_p / elapsed_p,
        },
    }

    if not args.no_extras:
        # time to 1e-8 of the step's K solve, FP64 vs mixed precision
        trac, die_new, flag, fcoh = S.cohesive_update(U, die, t0, write_tangent=True)
        Rm, Rf = S.residual(U, P, U, P, fcoh, load, src)
        z, _ = S.pcg_solve(fg.FG_A22, -Rf, tol=1e-8)
        b = S.coupling(z)
        res = {}
        for name, prec in (("f64", fg.FG_F64), ("mixed", fg.FG_MIXED)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = S.pcg_solve(fg.FG_K, b, tol=1e-8, precision=prec, check_every=64)
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t, info.iters, info.cycles, x)
            log(f"{name}: {res[name][0]:.3f}s iters {info.iters} cycles {info.cycles} relres {info.relres:.2e}")
        err = (torch.linalg.norm(res["mixed"][3] - res["f64"][3]) / torch.linalg.norm(res["f64"][3])).item()
        out["time_to_1e-8"] = {"f64_s": res["f64"][0], "mixed_s": res["mixed"][0], "f64_iters": res["f64"][1],
                               "mixed_inner_iters": res["mixed"][1], "mixed_cycles": res["mixed"][2],
                               "mixed_vs_f64_rel_l2": err, "speedup": res["f64"][0] / res["mixed"][0]}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_iters, log)
    print(json.dumps(out), flush=True)


def cpu_baseline(inst, iters, log):
    """The oracle (plain FP64 CSR Jacobi-PCG, OpenMP) on the same 128^3 tangent
    matrix: a bounded sample of `iters` iterations, reported as iterations/s."""
    import numpy as np

    from oracle import oracle as O

    t = time.perf_counter()
    P = O.Problem(inst)
    P.cohesive(np.zeros(3 * P.N), np.zeros((P.nq, 2)))
    log(f"oracle assembled ({time.perf_counter() - t:.1f}s)")
    b = np.random.default_rng(0).standard_normal(3 * P.N) * (1 - inst.dir_u)
    t = time.perf_counter()
    x, st, it, rr = P.pcg(O.K_TANGENT, b, tol=1e-30, maxit=iters)
    dt = time.perf_counter() - t
    log(f"oracle: {it} PCG iterations in {dt:.2f}s")
    return {"value": it / dt, "unit": "PCG iters/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{it} FP64 CSR Jacobi-PCG iterations of the oracle on the same {inst.mesh.tets.shape[0]}-tet "
                      f"tangent stiffness (assembly excluded)"}


if __name__ == "__main__":
    main()
