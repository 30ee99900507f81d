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
Also reported, outside the timed steps (--extras selects them):
  roofline  live HIP-event duration of the CG SpMV kernel against HBM peak
  tt8       time to a 1e-8 relative residual of the step's K solve, FP64 vs mixed
  adjoint   gradients/s of one implicit 64^3 step (forward timed separately)
  block     32 right-hand sides on one 64^3 K: block CG vs 32 separate solves
  batch     48 uneven instances (n 16..48, dip 30..90) in one grouped system vs
            48 separate systems
and the oracle on the same matrices (cpu_baseline at 128^3, and at 64^3).
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
    ap.add_argument("--cpu-iters", type=int, default=700,
                    help="oracle PCG iterations timed for the CPU baseline (about 10 s at 128^3)")
    ap.add_argument("--no-extras", action="store_true", help="skip every extra measurement")
    ap.add_argument("--extras", default="tt8,adjoint,steps,block,batch",
                    help="comma list of extra measurements: tt8, adjoint, steps, block, batch, and fd64 "
                         "(central differences of the 64^3 adjoint along 20 directions: about 10 minutes, "
                         "not in the default list)")
    ap.add_argument("--profile-iters", type=int, default=0,
                    help="profiling mode for hardware counters: run exactly this many FP64 K-PCG iterations and "
                         "one 1 GiB device copy (counter calibration), print a short JSON line, skip the rest")
    ap.add_argument("--profile-amg", type=int, default=0,
                    help="profiling mode for the AMG preconditioner: this many FP64 AMG-PCG solves to 1e-8 of the "
                         "benchmark's first K system (the first also builds the hierarchy); prints a short JSON line")
    ap.add_argument("--amg-mixed", action="store_true",
                    help="with --profile-amg: FG_MIXED solves (the V-cycle in FP32 inside the FP64 CG)")
    ap.add_argument("--profile-block", type=int, default=0,
                    help="profiling mode for the block product: this many FP64 block-CG iterations on 32 "
                         "right-hand sides at 64^3, then one 1 GiB device copy; prints a short JSON line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path, so --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import inputs as I

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.profile_block > 0:
        profile_block(args.profile_block)
        return
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
    if args.profile_amg > 0:
        S.cohesive_update(d(np.zeros(3 * N)), d(np.zeros(2 * nq)), d(inst.t0.reshape(-1)))
        z, _ = S.pcg_solve(fg.FG_A22, d(inst.source * inst.params.dt), tol=1e-12)
        b = S.coupling(z)
        S.tune("k_precond", 3)
        times = []
        prec = fg.FG_MIXED if args.amg_mixed else fg.FG_F64
        for _ in range(args.profile_amg):
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = S.pcg_solve(fg.FG_K, b, tol=1e-8, precision=prec)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        levels = S.amg_levels()
        S.tune("k_precond", 0)
        print(json.dumps({"profile_amg_solves": args.profile_amg, "fp32_cycle": args.amg_mixed,
                          "iters": info.iters, "seconds": times,
                          "levels": int(levels[0]), "nodes": [int(v) for v in levels[1]]}), flush=True)
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
    # timed pass: kernel-by-kernel launches with timing-only HIP events around every CG
    # SpMV on the stream it runs on, so the roofline's launch duration comes from the
    # same timed region as the rate
    torch.cuda.synchronize()
    S.profile(True)
    S.profile_read(0, reset=True)
    k_iters = 0
    per_step = []
    t = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        info = step()
        k_iters += info.inner_k_iters
        per_step.append(info.inner_k_iters / (time.perf_counter() - ts))   # the step ends on a host sync
        log(f"step {s}: K iters {info.inner_k_iters} A22 iters {info.inner_a22_iters} "
            f"({per_step[-1]:.0f} K iters/s)")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    value = k_iters / elapsed
    launches, ms = S.profile_read(0, reset=True)
    S.profile(False)
    # the same steps with the CG batches replayed as captured HIP graphs (no events)
    t = time.perf_counter()
    k_iters_g = 0
    for s in range(args.steps):
        k_iters_g += step().inner_k_iters
    torch.cuda.synchronize()
    elapsed_g = time.perf_counter() - t
    log(f"graph replay: {k_iters_g / elapsed_g:.0f} K iters/s")
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
            "traffic": measured_traffic(n),
            "kernel": "k_cg_spmv<3,double,double>",
            "bytes_per_launch": bytes_launch,
            "avg_launch_us": avg_s * 1e6,
            "launches": launches,
        },
        "graph_replay_iters_per_s": k_iters_g / elapsed_g,
        "per_step_iters_per_s": per_step,
        "median_step_iters_per_s": float(np.median(per_step)),
    }
    extras = set() if args.no_extras else set(e for e in args.extras.split(",") if e)

    if "tt8" in extras:
        # time to 1e-8 of the step's K solve, FP64 vs mixed precision
        trac, die_new, flag, fcoh = S.cohesive_update(U, die, t0, write_tangent=True)
        Rm, Rf = S.residual(U, P, U, P, fcoh, load, src)
        z, _ = S.pcg_solve(fg.FG_A22, -Rf, tol=1e-8)
        b = S.coupling(z)
        res = {}
        for name, prec in (("f64", fg.FG_F64), ("mixed", fg.FG_MIXED), ("mixed_f32val", fg.FG_MIXED_F32VAL),
                           ("f64_block_jacobi", fg.FG_F64), ("mixed_block_jacobi", fg.FG_MIXED),
                           ("f64_chebyshev_d2", fg.FG_F64), ("f64_chebyshev_d4", fg.FG_F64)):
            if name == "f64_block_jacobi":
                S.tune("k_precond", 1)
                S.pcg_solve(fg.FG_K, b, tol=1e-8, check_every=64)                 # blocks built, graphs captured
            if name.startswith("f64_chebyshev"):
                S.tune("k_precond", 2)
                S.tune("cheb_degree", int(name[-1]))
                if name.endswith("d2"):
                    S.tune("cheb_ratio", 300)                                      # drops the interval: time its estimate
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    cheb_lo, cheb_hi = S.cheb_interval()
                    cheb_est = time.perf_counter() - t
                    log(f"chebyshev interval [{cheb_lo:.4e}, {cheb_hi:.4e}] estimated in {cheb_est:.3f}s")
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = S.pcg_solve(fg.FG_K, b, tol=1e-8, precision=prec, check_every=64)
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t, info.iters, info.cycles, x)
            log(f"{name}: {res[name][0]:.3f}s iters {info.iters} cycles {info.cycles} relres {info.relres:.2e}")
        S.tune("k_precond", 0)
        S.tune("cheb_degree", 4)
        err = (torch.linalg.norm(res["mixed"][3] - res["f64"][3]) / torch.linalg.norm(res["f64"][3])).item()
        err2 = (torch.linalg.norm(res["mixed_f32val"][3] - res["f64"][3]) / torch.linalg.norm(res["f64"][3])).item()
        out["time_to_1e-8"] = {"f64_s": res["f64"][0], "mixed_s": res["mixed"][0], "f64_iters": res["f64"][1],
                               "mixed_inner_iters": res["mixed"][1], "mixed_cycles": res["mixed"][2],
                               "mixed_vs_f64_rel_l2": err, "speedup": res["f64"][0] / res["mixed"][0],
                               "mixed_f32val_s": res["mixed_f32val"][0],
                               "mixed_f32val_inner_iters": res["mixed_f32val"][1],
                               "mixed_f32val_cycles": res["mixed_f32val"][2],
                               "mixed_f32val_vs_f64_rel_l2": err2,
                               "speedup_f32val": res["f64"][0] / res["mixed_f32val"][0],
                               "f64_block_jacobi_s": res["f64_block_jacobi"][0],
                               "f64_block_jacobi_iters": res["f64_block_jacobi"][1],
                               "block_jacobi_vs_f64_rel_l2": (torch.linalg.norm(res["f64_block_jacobi"][3] - res["f64"][3])
                                                              / torch.linalg.norm(res["f64"][3])).item(),
                               "speedup_block_jacobi": res["f64"][0] / res["f64_block_jacobi"][0],
                               "mixed_block_jacobi_s": res["mixed_block_jacobi"][0],
                               "mixed_block_jacobi_iters": res["mixed_block_jacobi"][1],
                               "mixed_block_jacobi_cycles": res["mixed_block_jacobi"][2],
                               "mixed_block_jacobi_vs_f64_rel_l2": (
                                   torch.linalg.norm(res["mixed_block_jacobi"][3] - res["f64"][3])
                                   / torch.linalg.norm(res["f64"][3])).item(),
                               "speedup_mixed_block_jacobi": res["f64"][0] / res["mixed_block_jacobi"][0],
                               "chebyshev_interval": [cheb_lo, cheb_hi], "chebyshev_estimate_s": cheb_est}
        # smoothed-aggregation AMG (k_precond 3): the first solve builds the hierarchy (host
        # patterns once per mesh, values on the GPU), the second reuses it (K unchanged)
        S.tune("k_precond", 3)
        torch.cuda.synchronize()
        t = time.perf_counter()
        xa0, ia0 = S.pcg_solve(fg.FG_K, b, tol=1e-8)
        torch.cuda.synchronize()
        amg_first = time.perf_counter() - t
        t = time.perf_counter()
        xa, ia = S.pcg_solve(fg.FG_K, b, tol=1e-8)
        torch.cuda.synchronize()
        amg_s = time.perf_counter() - t
        amg_levels = S.amg_levels()
        # the same CG with the V-cycle in FP32 (FG_MIXED); the first call rounds the hierarchy
        S.pcg_solve(fg.FG_K, b, tol=1e-8, precision=fg.FG_MIXED)
        torch.cuda.synchronize()
        t = time.perf_counter()
        xam, iam = S.pcg_solve(fg.FG_K, b, tol=1e-8, precision=fg.FG_MIXED)
        torch.cuda.synchronize()
        amg32_s = time.perf_counter() - t
        S.tune("k_precond", 0)
        log(f"f64_amg: {amg_s:.3f}s iters {ia.iters} relres {ia.relres:.2e} (first solve with set-up {amg_first:.2f}s); "
            f"levels {amg_levels[0]} nodes {list(amg_levels[1])}; FP32 cycle {amg32_s:.3f}s iters {iam.iters}")
        out["time_to_1e-8"].update({
            "f64_amg_s": amg_s, "f64_amg_iters": ia.iters, "f64_amg_first_solve_with_setup_s": amg_first,
            "amg_levels": int(amg_levels[0]), "amg_nodes": [int(v) for v in amg_levels[1]],
            "amg_vs_f64_rel_l2": (torch.linalg.norm(xa - res["f64"][3]) / torch.linalg.norm(res["f64"][3])).item(),
            "speedup_amg": res["f64"][0] / amg_s,
            "mixed_amg_s": amg32_s, "mixed_amg_iters": iam.iters, "mixed_amg_status": iam.status,
            "mixed_amg_vs_f64_rel_l2": (torch.linalg.norm(xam - res["f64"][3])
                                        / torch.linalg.norm(res["f64"][3])).item(),
            "speedup_mixed_amg": res["f64"][0] / amg32_s})
        for d in (2, 4):
            r_ = res[f"f64_chebyshev_d{d}"]
            out["time_to_1e-8"].update({
                f"f64_chebyshev_d{d}_s": r_[0], f"f64_chebyshev_d{d}_iters": r_[1],
                f"f64_chebyshev_d{d}_products": r_[1] * d,
                f"chebyshev_d{d}_vs_f64_rel_l2": (torch.linalg.norm(r_[3] - res["f64"][3])
                                                  / torch.linalg.norm(res["f64"][3])).item(),
                f"speedup_chebyshev_d{d}": res["f64"][0] / r_[0]})

    del S
    torch.cuda.empty_cache()
    if "adjoint" in extras:
        out["adjoint_64"] = extra_adjoint(ctx, log)
    if "steps" in extras:
        out["steps_64"] = extra_steps(ctx, log)
    if "fd64" in extras:
        out["fd_64"] = extra_fd64(ctx, log)
    if "block" in extras:
        out["block_64"] = extra_block(ctx, log)
    if "batch" in extras:
        out["batch_48"] = extra_batch(ctx, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_iters, log)
        if extras:
            out["cpu_baseline_64"] = cpu_baseline(I.make_instance(I.config(2)), 8 * args.cpu_iters, log)
    print(json.dumps(out), flush=True)


def profile_block(iters):
    """Fixed-length FP64 block CG (32 columns, 64^3) for kernel-trace and counter runs."""
    import numpy as np
    import torch

    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import inputs as I

    inst = I.make_instance(I.config(5))
    ctx = fg.Context(0)
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    npairs, nblk, nslices, nhalo = S.sizes()
    B = torch.as_tensor(np.random.default_rng(0).standard_normal((32, 3 * S.N)) * (1 - inst.dir_u)).cuda()
    X, info = S.pcg_solve(fg.FG_K, B.reshape(-1).contiguous(), nrhs=32, tol=1e-300, max_iter=iters,
                          check_every=iters)
    src_t = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    dst_t = torch.empty_like(src_t)
    dst_t.copy_(src_t)
    torch.cuda.synchronize()
    # algorithmic bytes of one 32-column FP64 row-group product: each stored block (72 B) and its
    # column index (4 B) once; P read and Q written once (3 x 32 x 8 B per node each)
    print(json.dumps({"profile_block_iters": info.iters, "nrhs": 32, "nodes": S.N, "blocks": npairs,
                      "product_bytes_per_launch": 76.0 * npairs + 2 * 768.0 * S.N,
                      "copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30}), flush=True)


def measured_traffic(n):
    """HBM bytes per launch of the K product from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy), or None when the summary is for another
    workload or the sources the product is built from have changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_cg_spmv_cube128_counters.json")
    if n != 128 or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for s in rec["sources"]:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return rec["traffic_bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t, r


def extra_adjoint(ctx, log):
    """Gradient of J = sum over fault pairs of |tangential jump|^2 + squared uplift at 32 seeded top
    nodes, w.r.t. ln k and E of every tetrahedron, after one implicit injection step at 64^3."""
    import numpy as np
    import torch

    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import inputs as I
    from paper_2410_17133_amd.autograd import fault_slip_uplift_objective

    inst = I.make_instance(I.config(4))
    S = fg.System.from_instance(ctx, inst)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64)).cuda()
    E, logk = d(inst.E), d(inst.logk)
    S.assemble(inst.params, E, logk)
    U, P, die = d(np.zeros(3 * S.N)), d(np.zeros(S.N)), d(np.zeros(2 * S.nq))
    t0 = d(inst.t0.reshape(-1))
    # inexact Newton: residual 1e-8, each partitioned solve to 1e-2, inner K and A22 solves to 1e-4
    inner = fg.opts(tol=1e-4, check_every=64)
    t_fwd, (trac, flag, finfo) = _timed(lambda: S.step(U, P, die, t0, d(inst.load), d(inst.source), newton_tol=1e-8,
                                                       newton_max_iter=60, inner_k=inner, inner_p=inner,
                                                       outer_tol=1e-2))
    log(f"adjoint: forward step {t_fwd:.2f}s newton {finfo.newton_iters} outer {finfo.outer_iters} "
        f"K iters {finfo.inner_k_iters} status {finfo.status}; slip points {int((flag == 1).sum())}")
    m = inst.mesh
    X = m.xyz[m.coh[0, 3:]]
    nrm = np.cross(X[1] - X[0], X[2] - X[0])
    Uv = U.clone().requires_grad_(True)
    J = fault_slip_uplift_objective(Uv, torch.as_tensor(m.pairs.astype(np.int64)).cuda(),
                                    d(nrm / np.linalg.norm(nrm)),
                                    torch.as_tensor(I.uplift_nodes(inst, 32).astype(np.int64)).cuda())
    gU, = torch.autograd.grad(J, Uv)
    gP = torch.zeros_like(P)
    die0 = torch.zeros_like(die)
    res = {}
    for name, prec, kp, et in (("f64", fg.FG_F64, 0, 0), ("mixed", fg.FG_MIXED, 0, 0),
                               ("f64_block_jacobi", fg.FG_F64, 1, 0), ("mixed_block_jacobi", fg.FG_MIXED, 1, 0),
                               ("f64_block_jacobi_exact", fg.FG_F64, 1, 1), ("f64_amg", fg.FG_F64, 3, 0),
                               ("mixed_amg", fg.FG_MIXED, 3, 0), ("f64_amg_exact", fg.FG_F64, 3, 1),
                               ("mixed_amg_exact", fg.FG_MIXED, 3, 1)):
        # corrections solved loosely (outer 0.05, inner 1e-3); the defect tolerance sets the accuracy;
        # exact: the corrections solve with K_t + N^T (BiCGStab) instead of the symmetric tangent
        S.tune("k_precond", kp)
        S.tune("exact_tangent", et)
        ik = fg.opts(tol=1e-3, check_every=64, precision=prec)
        ip = fg.opts(tol=1e-3, check_every=64)
        t_adj, (dE, dk, ainfo) = _timed(lambda: S.adjoint(U, P, die0, t0, logk, gU, gP, inner_k=ik, inner_p=ip,
                                                           outer_tol=0.05, defect_tol=1e-8))
        log(f"adjoint {name}: {t_adj:.2f}s defect iters {ainfo.newton_iters} outer {ainfo.outer_iters} "
            f"K iters {ainfo.inner_k_iters} status {ainfo.status}")
        res[name] = (t_adj, ainfo, torch.cat([dE * E, dk]))
    S.tune("k_precond", 0)
    S.tune("exact_tangent", 0)
    g64 = res["f64"][2]
    bj = {name: {"s": res[name][0], "defect_iters": res[name][1].newton_iters, "k_iters": res[name][1].inner_k_iters,
                 "status": res[name][1].status,
                 "vs_f64_grad_rel_l2": (torch.linalg.norm(res[name][2] - g64) / torch.linalg.norm(g64)).item()}
          for name in ("f64_block_jacobi", "mixed_block_jacobi", "f64_block_jacobi_exact", "f64_amg", "mixed_amg",
                       "f64_amg_exact", "mixed_amg_exact")}
    # the exact tangent K_t + N at the converged state (slip points present): BiCGStab to 1e-8
    # on b = dJ/dU, against CG on the symmetric tangent
    S.cohesive_update(U, die0, t0, write_tangent=True)
    ex = {}
    for name, kp in (("bicgstab_block_jacobi", 1), ("bicgstab_point_jacobi", 0), ("cg_symmetric_block_jacobi", 1)):
        S.tune("k_precond", kp)
        solve = (lambda: S.pcg_solve(fg.FG_K, gU, tol=1e-8, check_every=64)) if name.startswith("cg") else \
            (lambda: S.exact_solve(gU, tol=1e-8))
        solve()
        t_ex, (x_ex, i_ex) = _timed(solve)
        ex[name] = (t_ex, i_ex.iters, x_ex, i_ex.status)
        log(f"exact tangent {name}: {t_ex:.3f}s iters {i_ex.iters} status {i_ex.status}")
    S.tune("k_precond", 0)
    xb = ex["bicgstab_block_jacobi"][2]
    # the forward step again, block-Jacobi K solves with the symmetric and with the exact tangent,
    # and AMG-preconditioned K solves (symmetric tangent; hierarchy values rebuilt at every change of K)
    fwd = {}
    inner32 = fg.opts(tol=1e-4, check_every=64, precision=fg.FG_MIXED)
    for kp, et, ik in ((1, 0, inner), (1, 1, inner), (3, 0, inner), (3, 0, inner32), (3, 1, inner)):
        S.tune("k_precond", kp)
        S.tune("exact_tangent", et)
        U2, P2, die2 = d(np.zeros(3 * S.N)), d(np.zeros(S.N)), d(np.zeros(2 * S.nq))
        t_f, (_, flag2, finfo2) = _timed(lambda: S.step(U2, P2, die2, t0, d(inst.load), d(inst.source),
                                                         newton_tol=1e-8, newton_max_iter=60, inner_k=ik,
                                                         inner_p=inner, outer_tol=1e-2))
        name = ("amg_exact" if et else "amg_mixed_symmetric" if ik is inner32 else "amg_symmetric") if kp == 3 else \
            "exact" if et else "symmetric"
        log(f"forward step, {'AMG' if kp == 3 else 'block Jacobi'}, {name} tangent: {t_f:.2f}s newton {finfo2.newton_iters} cuts "
            f"{finfo2.step_cuts} K iters {finfo2.inner_k_iters} status {finfo2.status}")
        fwd[name] = {"s": t_f, "newton": finfo2.newton_iters, "step_cuts": finfo2.step_cuts,
                     "k_iters": finfo2.inner_k_iters, "status": finfo2.status,
                     "vs_first_step_rel_l2": (torch.linalg.norm(U2 - U) / torch.linalg.norm(U)).item()}
    S.tune("exact_tangent", 0)
    S.tune("k_precond", 0)
    r_true = (torch.linalg.norm(gU - S.spmv(fg.FG_K_EXACT, xb)) / torch.linalg.norm(gU)).item()
    exact = {"rhs": "dJ/dU of the objective at the converged step", "tol": 1e-8, "true_relres_block_jacobi": r_true,
             "symmetric_vs_exact_rel_l2": (torch.linalg.norm(ex["cg_symmetric_block_jacobi"][2] - xb)
                                           / torch.linalg.norm(xb)).item()}
    for name, (t_ex, it_ex, _, st_ex) in ex.items():
        exact.update({f"{name}_s": t_ex, f"{name}_iters": it_ex, f"{name}_status": st_ex,
                      f"{name}_k_products": it_ex * (1 if name.startswith("cg") else 2)})
    return {"workload": f"cube64_dip60_hetero one implicit step, {inst.mesh.tets.shape[0]} tets, "
                        f"{2 * inst.mesh.tets.shape[0]} parameters (ln k, E); forward: Newton 1e-8, outer 1e-2, inner "
                        f"1e-4; adjoint: defect 1e-8, corrections outer 0.05 inner 1e-3",
            "forward_s": t_fwd, "forward_newton_iters": finfo.newton_iters, "forward_k_iters": finfo.inner_k_iters,
            "forward_status": finfo.status, "forward_step_cuts": finfo.step_cuts,
            "grad_per_s_f64": 1.0 / res["f64"][0], "grad_per_s_mixed": 1.0 / res["mixed"][0],
            "adjoint_s_f64": res["f64"][0], "adjoint_s_mixed": res["mixed"][0],
            "defect_iters": res["f64"][1].newton_iters, "adjoint_k_iters_f64": res["f64"][1].inner_k_iters,
            "mixed_vs_f64_grad_rel_l2": (torch.linalg.norm(res["mixed"][2] - g64) / torch.linalg.norm(g64)).item(),
            "slip_points": int((flag == 1).sum()), "exact_tangent_solve": exact,
            "forward_block_jacobi": fwd, "adjoint_block_jacobi": bj}


def extra_steps(ctx, log, nsteps=20):
    """The 20-step 64^3 trajectory (constant injection, the state U, P and inelastic slip
    carried from step to step, inexact Newton as in the adjoint, K solves by FP64 CG with the
    AMG V-cycle in FP32),
    checkpointed, then the reverse sweep: the gradient of J = sum over the steps of the
    fault-slip and uplift objective w.r.t. ln k and E through the whole loop, slip state
    included."""
    import numpy as np
    import torch

    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import inputs as I
    from paper_2410_17133_amd import trajectory as T
    from paper_2410_17133_amd.autograd import fault_slip_uplift_objective

    inst = I.make_instance(I.config(2))
    S = fg.System.from_instance(ctx, inst)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64)).cuda()
    E, logk = d(inst.E), d(inst.logk)
    S.assemble(inst.params, E, logk)
    U, P, die = d(np.zeros(3 * S.N)), d(np.zeros(S.N)), d(np.zeros(2 * S.nq))
    t0, load, src = d(inst.t0.reshape(-1)), d(inst.load), d(inst.source)
    inner = fg.opts(tol=1e-4, check_every=64)
    inner_k = fg.opts(tol=1e-4, check_every=64, precision=fg.FG_MIXED)
    S.tune("k_precond", 3)
    steps, ck = [], []
    for k in range(nsteps):
        ts, (c, infos) = _timed(lambda: T.run(S, U, P, die, t0, load, src, 1, newton_tol=1e-8, newton_max_iter=60,
                                              inner_k=inner_k, inner_p=inner, outer_tol=1e-2))
        ck += c
        info = infos[0]
        fl = S.cohesive_update(U, c[0][2], t0, write_tangent=False)[2].cpu().numpy()
        rec = {"s": ts, "newton": info.newton_iters, "step_cuts": info.step_cuts, "outer": info.outer_iters,
               "k_iters": info.inner_k_iters, "status": info.status, "slip": int((fl == 1).sum()),
               "open": int((fl == 2).sum())}
        steps.append(rec)
        log(f"step {k + 1}: {ts:.1f}s newton {info.newton_iters} cuts {info.step_cuts} K iters {info.inner_k_iters} "
            f"slip {rec['slip']} open {rec['open']} status {info.status}")
    m = inst.mesh
    X = m.xyz[m.coh[0, 3:]]
    nrm = np.cross(X[1] - X[0], X[2] - X[0])
    pairs = torch.as_tensor(m.pairs.astype(np.int64)).cuda()
    nrm_d = d(nrm / np.linalg.norm(nrm))
    up = torch.as_tensor(I.uplift_nodes(inst, 32).astype(np.int64)).cuda()

    def grad_y(n, Un, Pn):
        Uv = Un.clone().requires_grad_(True)
        g, = torch.autograd.grad(fault_slip_uplift_objective(Uv, pairs, nrm_d, up), Uv)
        return g, torch.zeros_like(Pn)
    # corrections solved loosely (outer 0.05, inner 1e-3); the defect tolerance sets the accuracy
    corr = fg.opts(tol=1e-3, check_every=64)
    corr_k = fg.opts(tol=1e-3, check_every=64, precision=fg.FG_MIXED)
    tr, (dE, dk, ainfos) = _timed(lambda: T.gradient(S, ck, t0, logk, grad_y, inner_k=corr_k, inner_p=corr,
                                                     outer_tol=0.05, defect_tol=1e-8))
    S.tune("k_precond", 0)
    defect = [i.newton_iters for i in ainfos]
    log(f"reverse sweep over {nsteps} steps: {tr:.1f}s, defect iterations per step {defect}, "
        f"K iters {sum(i.inner_k_iters for i in ainfos)}")
    fwd = float(sum(s["s"] for s in steps))
    return {"workload": f"cube64_dip60_hetero, {nsteps} consecutive 1 s steps (the 20-step trajectory); K solves by "
                        f"FP64 CG with the AMG V-cycle in FP32; Newton 1e-8, outer 1e-2, inner 1e-4; reverse sweep: "
                        f"defect 1e-8, corrections outer 0.05 inner 1e-3",
            "steps": steps, "mean_step_s": float(np.mean([s["s"] for s in steps])), "forward_s": fwd,
            "reverse_s": tr, "reverse_defect_iters": defect, "gradients_per_s": 1.0 / tr,
            "forward_and_reverse_s": fwd + tr,
            "reverse_k_iters": int(sum(i.inner_k_iters for i in ainfos)),
            "gradient_norm": float(torch.linalg.norm(torch.cat([dE * E, dk])).item())}


def extra_fd64(ctx, log, count=20, eps=1e-6):
    """Central differences of the 64^3 injection step's objective (squared fault slip plus
    squared uplift at 32 seeded top nodes) along `count` seeded random directions in
    (ln k, ln E) with standard normal components (every parameter moves by about eps),
    step eps, against the adjoint gradient in FP64 and in mixed precision.
    Every forward is a step from rest with block-Jacobi K solves, the exact interface
    tangent (quadratic Newton) and a tight Newton tolerance."""
    import numpy as np
    import torch

    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import inputs as I
    from paper_2410_17133_amd.autograd import fault_slip_uplift_objective

    inst = I.make_instance(I.config(4))
    S = fg.System.from_instance(ctx, inst)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64)).cuda()
    t0, load, src = d(inst.t0.reshape(-1)), d(inst.load), d(inst.source)
    m = inst.mesh
    X = m.xyz[m.coh[0, 3:]]
    nrm = np.cross(X[1] - X[0], X[2] - X[0])
    pairs, nrm_d = torch.as_tensor(m.pairs.astype(np.int64)).cuda(), d(nrm / np.linalg.norm(nrm))
    up = torch.as_tensor(I.uplift_nodes(inst, 32).astype(np.int64)).cuda()
    S.tune("k_precond", 1)
    S.tune("exact_tangent", 1)
    inner = fg.opts(tol=1e-6, check_every=64)

    def forward(logk, E):
        S.assemble(inst.params, E, logk)
        U, P, die = d(np.zeros(3 * S.N)), d(np.zeros(S.N)), d(np.zeros(2 * S.nq))
        _, flag, info = S.step(U, P, die, t0, load, src, newton_tol=1e-12, newton_max_iter=80, inner_k=inner,
                               inner_p=inner, outer_tol=1e-3)
        if info.status != 0:
            raise RuntimeError(f"forward step failed: status {info.status}, residuals {info.res_m:.1e} {info.res_f:.1e}")
        return U, P, flag, info

    E0, lk0 = d(inst.E), d(inst.logk)
    tf, (U, P, flag, info) = _timed(lambda: forward(lk0, E0))
    log(f"fd64: base forward {tf:.1f}s newton {info.newton_iters} cuts {info.step_cuts} slip {int((flag == 1).sum())}")
    Uv = U.clone().requires_grad_(True)
    J0 = fault_slip_uplift_objective(Uv, pairs, nrm_d, up)
    gU, = torch.autograd.grad(J0, Uv)
    die0 = torch.zeros(2 * S.nq, dtype=torch.float64, device="cuda")
    grads = {}
    for name, prec in (("f64", fg.FG_F64), ("mixed", fg.FG_MIXED)):
        S.tune("exact_tangent", 0)              # mixed K solves are symmetric; both refine on the exact residual
        ik = fg.opts(tol=1e-3, check_every=64, precision=prec)
        ip = fg.opts(tol=1e-3, check_every=64)
        ta, (dE, dk, ainfo) = _timed(lambda: S.adjoint(U, P, die0, t0, lk0, gU, torch.zeros_like(P), inner_k=ik,
                                                        inner_p=ip, outer_tol=0.05, defect_tol=1e-11))
        log(f"fd64: adjoint {name} {ta:.2f}s defect iterations {ainfo.newton_iters} status {ainfo.status}")
        grads[name] = (dk.cpu().numpy(), (dE * E0).cpu().numpy(), ta)   # dJ/dln k, dJ/dln E
    S.tune("exact_tangent", 1)
    ne = inst.E.size
    rows = []
    t = time.perf_counter()
    for j, dvec in enumerate(I.fd_directions(2 * ne, count=count, unit=False)):
        dlk, dlE = dvec[:ne], dvec[ne:]
        Jpm = []
        for sgn in (1.0, -1.0):
            Uj = forward(d(inst.logk + sgn * eps * dlk), d(inst.E * np.exp(sgn * eps * dlE)))[0]
            Jpm.append(fault_slip_uplift_objective(Uj, pairs, nrm_d, up).item())
        fd = (Jpm[0] - Jpm[1]) / (2 * eps)
        ad = {k: float(g[0] @ dlk + g[1] @ dlE) for k, g in grads.items()}
        rows.append({"fd": fd, "adjoint_f64": ad["f64"], "adjoint_mixed": ad["mixed"],
                     "rel_f64": abs(fd - ad["f64"]) / abs(ad["f64"]), "rel_mixed": abs(fd - ad["mixed"]) / abs(ad["mixed"])})
        log(f"fd64 direction {j}: fd {fd:.10e} adjoint f64 {ad['f64']:.10e} (rel {rows[-1]['rel_f64']:.1e}) mixed "
            f"{ad['mixed']:.10e} (rel {rows[-1]['rel_mixed']:.1e}) [{time.perf_counter() - t:.0f}s]")
    S.tune("k_precond", 0)
    S.tune("exact_tangent", 0)
    return {"workload": f"cube64_dip60_hetero one implicit step from rest, {2 * ne} parameters (ln k, ln E); "
                        f"{count} seeded random directions (standard normal components), central differences with step {eps}; forwards with "
                        f"block-Jacobi K solves, exact interface tangent, Newton 1e-12; adjoint defect 1e-11",
            "J": J0.item(), "base_forward_s": tf, "adjoint_f64_s": grads["f64"][2], "adjoint_mixed_s": grads["mixed"][2],
            "max_rel_f64": max(r["rel_f64"] for r in rows), "max_rel_mixed": max(r["rel_mixed"] for r in rows),
            "directions": rows}


def extra_block(ctx, log):
    """32 injection scenarios on one 64^3 tangent: the first K solve of each scenario's partitioned
    CG, b_s = A_pu A22^{-1} (dt q_s), solved to 1e-8 as one 32-column block and as 32 solves."""
    import numpy as np
    import torch

    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import inputs as I

    inst = I.make_instance(I.config(5))
    S = fg.System.from_instance(ctx, inst)
    S.assemble(inst.params, inst.E, inst.logk)
    pairs, rates = I.injection_scenarios(inst, 32)
    Q = I.source_matrix(inst, pairs, rates) * inst.params.dt
    cols = []
    for q in Q:
        z, _ = S.pcg_solve(fg.FG_A22, torch.as_tensor(q).cuda(), tol=1e-12)
        cols.append(S.coupling(z))
    B = torch.stack(cols).reshape(-1).contiguous()
    from paper_2410_17133_amd import autotune as AT
    res = {}
    tuned_by_prec = {}
    # point Jacobi (the paper's), then the nodal / fault-pair block-Jacobi preconditioner on every column
    for name, prec, kp in (("mixed", fg.FG_MIXED, 0), ("f64", fg.FG_F64, 0), ("mixed_block_jacobi", fg.FG_MIXED, 1),
                           ("f64_block_jacobi", fg.FG_F64, 1)):
        S.tune("k_precond", kp)
        if prec not in tuned_by_prec:
            tuned = AT.tune_block(S, 32, prec, B=B, iters=20)               # product tile from the autotuner
            tuned_by_prec[prec] = tuned
            log(f"block {name}: autotuner picked {tuned['config']} ({tuned['us_per_iteration']:.0f} us/iteration, "
                f"{tuned['trials']} trials)")
        tuned = tuned_by_prec[prec]
        AT.apply(S, tuned["config"])
        S.pcg_solve(fg.FG_K, B, nrhs=32, tol=1e-8, precision=prec)          # graphs captured
        tb, (Xb, ib) = _timed(lambda: S.pcg_solve(fg.FG_K, B, nrhs=32, tol=1e-8, precision=prec))
        n3 = 3 * S.N

        def separate():
            it = 0
            for c in range(32):
                x, i1 = S.pcg_solve(fg.FG_K, B[c * n3:(c + 1) * n3], tol=1e-8, precision=prec, check_every=64)
                it += i1.iters
            return it
        ts, its = _timed(separate)
        log(f"block {name}: 32 columns {tb:.2f}s ({ib.iters} iters, {ib.cycles} cycles) vs separate {ts:.2f}s "
            f"({its} iters)")
        res[name] = {"block_s": tb, "separate_s": ts, "speedup": ts / tb, "block_iters": ib.iters,
                     "block_cycles": ib.cycles, "separate_iters_total": its, "autotuned": tuned["config"]}
    S.tune("k_precond", 0)
    return {"workload": f"cube64_dip60_hetero, {S.N} nodes, 32 injection right-hand sides on one K, to 1e-8",
            **res}


def extra_batch(ctx, log):
    """48 seeded uneven instances in one grouped system against 48 separate systems: the first K
    solve of each instance's partitioned CG, b = A_pu A22^{-1} (dt q), to 1e-8 per instance."""
    import numpy as np
    import torch

    from paper_2410_17133_amd import fg
    from paper_2410_17133_amd import inputs as I

    t = time.perf_counter()
    insts = [I.make_instance(c) for c in I.batched_configs(48)]
    Bt = I.concat_instances(insts)
    G = fg.System.from_batch(ctx, Bt)
    G.assemble([i.params for i in insts], Bt.E, Bt.logk)
    log(f"batch: {len(insts)} instances, {Bt.xyz.shape[0]} nodes, {Bt.tets.shape[0]} tets "
        f"({time.perf_counter() - t:.1f}s)")
    dt = insts[0].params.dt
    z, _ = G.pcg_solve(fg.FG_A22, torch.as_tensor(Bt.source * dt).cuda(), tol=1e-12)
    b = G.coupling(z)
    res = {}
    singles = []
    for i, inst in enumerate(insts):
        Si = fg.System.from_instance(ctx, inst)
        Si.assemble(inst.params, inst.E, inst.logk)
        singles.append(Si)
    for name, prec, kp in (("f64", fg.FG_F64, 0), ("mixed", fg.FG_MIXED, 0), ("f64_block_jacobi", fg.FG_F64, 1),
                           ("mixed_block_jacobi", fg.FG_MIXED, 1)):
        G.tune("k_precond", kp)
        for Si in singles:
            Si.tune("k_precond", kp)
        G.pcg_solve(fg.FG_K, b, tol=1e-8, precision=prec, check_every=64)
        tg, (xg, ig) = _timed(lambda: G.pcg_solve(fg.FG_K, b, tol=1e-8, precision=prec, check_every=64))
        iters, rel, stt = G.group_stats()

        def separate():
            it = 0
            for i, Si in enumerate(singles):
                lo, hi = 3 * Bt.node_off[i], 3 * Bt.node_off[i + 1]
                x, i1 = Si.pcg_solve(fg.FG_K, b[lo:hi], tol=1e-8, precision=prec, check_every=64)
                it += i1.iters
            return it
        separate()
        ts, its = _timed(separate)
        log(f"batch {name}: grouped {tg:.2f}s (max {ig.iters} iters, worst relres {ig.relres:.1e}) vs separate "
            f"{ts:.2f}s ({its} iters)")
        res[name] = {"grouped_s": tg, "separate_s": ts, "speedup": ts / tg, "grouped_max_iters": ig.iters,
                     "group_iters_total": int(iters.sum()), "separate_iters_total": its,
                     "all_converged": bool(np.all(stt == 0))}
    G.tune("k_precond", 0)
    return {"workload": f"48 instances n~U{{16..48}} dip~U[30,90] heterogeneous: {Bt.xyz.shape[0]} nodes, "
                        f"{Bt.tets.shape[0]} tets; first K solve of each to 1e-8", **res}


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
    nnz = P.scipy(O.K_TANGENT).nnz
    # CSR value + column per stored entry, row pointers, and the vector passes of one iteration
    bytes_it = 12.0 * nnz + 8.0 * (3 * P.N + 1) + 8.0 * 3 * P.N * 12
    return {"value": it / dt, "unit": "PCG iters/s", "cores": O.num_threads(), "kind": "oracle",
            "gbs": bytes_it * it / dt / 1e9,
            "sample": f"{it} FP64 CSR Jacobi-PCG iterations of the oracle on the same {inst.mesh.tets.shape[0]}-tet "
                      f"tangent stiffness (assembly excluded)"}


if __name__ == "__main__":
    main()
