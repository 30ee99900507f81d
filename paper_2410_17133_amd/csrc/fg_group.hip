// Batched independent problems in one system: the mesh is a disjoint union of
// instances ("groups"), each padded to whole slices, and point-Jacobi CG runs on
// every group with its own alpha, beta, rho and stop test.  Every kernel works
// on slices (one wavefront each) and leaves per-slice partial sums; one-block
// finalize kernels per group add the partials of the group's slice range.
// A group that has stopped is skipped by all later kernels, so small instances
// stop costing bandwidth as soon as they converge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <vector>

#include "fg_device.h"
#include "fg_kernels.h"

namespace fg {

namespace {

// element k*64 + lane of slice s (BS values per row, stored row-major)
__device__ __forceinline__ int64_t slice_elem(int64_t s, int k, int lane, int bs)
{
    return s * SLICE * bs + (int64_t)k * SLICE + lane;
}

template <int NV>
__device__ __forceinline__ void slice_partials(const double (&v)[NV], int64_t s, int lane, double *part, int64_t stride)
{
    for (int k = 0; k < NV; ++k) {
        const double t = wave_sum(v[k]);
        if (lane == 0) part[k * stride + s] = t;
    }
}

template <int NV>
__device__ __forceinline__ void group_sum(const double *part, int64_t stride, int64_t s0, int64_t s1, double (&tot)[NV])
{
    __shared__ double sh[NV][FIN / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = 0; k < NV; ++k) {
        double t = 0;
        for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) t += part[k * stride + s];
        t = wave_sum(t);
        if (lane == 0) sh[k][w] = t;
    }
    __syncthreads();
    for (int k = 0; k < NV; ++k) {
        double t = 0;
        for (int i = 0; i < nw; ++i) t += sh[k][i];
        tot[k] = t;
    }
}

template <int BS, typename T>
__global__ __launch_bounds__(WG) void k_g_init(int64_t nslices, const T *__restrict__ dinv, T *__restrict__ x,
                                               const T *__restrict__ r, T *__restrict__ p, double *part,
                                               int64_t stride)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    double v[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        const int64_t e = slice_elem(s, k, lane, BS);
        const T ri = r[e], zi = dinv[e] * ri;
        x[e] = 0;
        p[e] = zi;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    slice_partials<2>(v, s, lane, part, stride);
}

__global__ __launch_bounds__(FIN) void k_g_init_fin(const double *part, int64_t stride, const int64_t *gsp,
                                                    MrScalars *sc, double tol)
{
    const int g = blockIdx.x;
    double tot[2];
    group_sum<2>(part, stride, gsp[g], gsp[g + 1], tot);
    if (threadIdx.x != 0) return;
    sc->rho[g] = tot[0];
    sc->rr[g] = tot[1];
    sc->bb[g] = tot[1];
    sc->tol2[g] = tol * tol * tot[1];
    sc->iter[g] = 0;
    sc->status[g] = FG_OK;
    sc->done[g] = 0;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
        sc->status[g] = FG_ERR_NAN;
        sc->done[g] = 1;
    } else if (tot[1] == 0.0) {
        sc->done[g] = 1;
    } else if (sc->maxit <= 0) {
        sc->status[g] = FG_NOT_CONVERGED;
        sc->done[g] = 1;
    }
}

template <int BS, typename T, typename TV>
__global__ __launch_bounds__(WG) void k_g_spmv(SpmvArgs a, const int32_t *__restrict__ slice_group,
                                               const TV *__restrict__ val, const T *__restrict__ p,
                                               T *__restrict__ q, double *part, int64_t stride, const MrScalars *sc)
{
    extern __shared__ unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T *xs = (T *)smem + (int64_t)wave * a.cap * BS;
    const int64_t s = xcd_block() * (WG / SLICE) + wave;
    const bool live = s < a.nslices && !sc->done[slice_group[s]];
    bool staged = false;
    if (live) staged = stage_halo<BS, T>(s, lane, a.halo_ptr, a.halo, a.cap, p, xs);
    __syncthreads();
    if (!live) return;
    double v[1];
    v[0] = slice_spmv<BS, T, TV>(s, lane, staged, a.slice_ptr, a.col, a.lcol, a.diag_slot, val, p, xs, q);
    slice_partials<1>(v, s, lane, part, stride);
}

__global__ __launch_bounds__(FIN) void k_g_alpha(const double *part, int64_t stride, const int64_t *gsp, MrScalars *sc)
{
    const int g = blockIdx.x;
    if (sc->done[g]) return;
    double tot[1];
    group_sum<1>(part, stride, gsp[g], gsp[g + 1], tot);
    if (threadIdx.x != 0) return;
    const double pq = tot[0];
    sc->pq[g] = pq;
    if (!isfinite(pq)) {
        sc->status[g] = FG_ERR_NAN;
        sc->done[g] = 1;
    } else if (!(pq > 0.0)) {
        sc->status[g] = FG_ERR_BREAKDOWN;
        sc->done[g] = 1;
    } else {
        sc->alpha[g] = sc->rho[g] / pq;
    }
}

template <int BS, typename T>
__global__ __launch_bounds__(WG) void k_g_update(int64_t nslices, const int32_t *__restrict__ slice_group,
                                                 const T *__restrict__ dinv, T *__restrict__ x, T *__restrict__ r,
                                                 const T *__restrict__ p, const T *__restrict__ q, double *part,
                                                 int64_t stride, const MrScalars *sc)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    const int g = slice_group[s];
    if (sc->done[g]) return;
    const T al = (T)sc->alpha[g];
    double v[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        const int64_t e = slice_elem(s, k, lane, BS);
        x[e] += al * p[e];
        const T ri = r[e] - al * q[e];
        r[e] = ri;
        const T zi = dinv[e] * ri;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    slice_partials<2>(v, s, lane, part, stride);
}

__global__ __launch_bounds__(FIN) void k_g_beta(const double *part, int64_t stride, const int64_t *gsp, MrScalars *sc)
{
    const int g = blockIdx.x;
    if (sc->done[g]) return;
    double tot[2];
    group_sum<2>(part, stride, gsp[g], gsp[g + 1], tot);
    if (threadIdx.x != 0) return;
    sc->iter[g] += 1;
    sc->rr[g] = tot[1];
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
        sc->status[g] = FG_ERR_NAN;
        sc->done[g] = 1;
    } else if (tot[1] <= sc->tol2[g]) {
        sc->status[g] = FG_OK;
        sc->done[g] = 1;
    } else if (sc->iter[g] >= sc->maxit) {
        sc->status[g] = FG_NOT_CONVERGED;
        sc->done[g] = 1;
    } else {
        sc->beta[g] = tot[0] / sc->rho[g];
        sc->rho[g] = tot[0];
    }
}

template <int BS, typename T>
__global__ __launch_bounds__(WG) void k_g_pupdate(int64_t nslices, const int32_t *__restrict__ slice_group,
                                                  const T *__restrict__ dinv, const T *__restrict__ r,
                                                  T *__restrict__ p, const MrScalars *sc)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    const int g = slice_group[s];
    if (sc->done[g]) return;
    const T be = (T)sc->beta[g];
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        const int64_t e = slice_elem(s, k, lane, BS);
        p[e] = dinv[e] * r[e] + be * p[e];
    }
}

// Residual replacement of the FP32 grouped CG (reliable updates): per-slice
// partials of r.z and r.r of the new residual; then per group beta against the
// rho the group stopped with (its last direction is kept), the new rho and the
// stop threshold next2[g] (squared; next2[g] <= 0: the group is finished); then
// p = z + beta p on the groups that go on.
template <int BS, typename T>
__global__ __launch_bounds__(WG) void k_g_resume(int64_t nslices, const T *__restrict__ dinv, const T *__restrict__ r,
                                                 double *part, int64_t stride)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    double v[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        const int64_t e = slice_elem(s, k, lane, BS);
        const T ri = r[e], zi = dinv[e] * ri;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    slice_partials<2>(v, s, lane, part, stride);
}

__global__ __launch_bounds__(FIN) void k_g_resume_fin(const double *part, int64_t stride, const int64_t *gsp,
                                                      MrScalars *sc, const double *next2)
{
    const int g = blockIdx.x;
    double tot[2];
    group_sum<2>(part, stride, gsp[g], gsp[g + 1], tot);
    if (threadIdx.x != 0) return;
    sc->status[g] = FG_OK;
    sc->done[g] = 1;
    if (!(next2[g] > 0.0)) return;
    const double beta = tot[0] / sc->rho[g];
    sc->rr[g] = tot[1];
    if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(beta)) {
        sc->status[g] = FG_ERR_NAN;
    } else if (sc->iter[g] >= sc->maxit) {
        sc->status[g] = FG_NOT_CONVERGED;
    } else {
        sc->beta[g] = beta;
        sc->rho[g] = tot[0];
        sc->tol2[g] = next2[g];
        sc->done[g] = 0;
    }
}

template <int BS, typename T>
__global__ __launch_bounds__(WG) void k_g_resume_p(int64_t nslices, const int32_t *__restrict__ slice_group,
                                                   const T *__restrict__ dinv, const T *__restrict__ r,
                                                   T *__restrict__ p, const MrScalars *sc)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    const int g = slice_group[s];
    if (sc->done[g]) return;
    const T be = (T)sc->beta[g];
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        const int64_t e = slice_elem(s, k, lane, BS);
        p[e] = dinv[e] * r[e] + be * p[e];
    }
}

// ---- block-Jacobi preconditioner of the grouped K solve ("k_precond" >= 1) ----
// One thread per row: the lane of a slice's wavefront owns its row's unit (a node,
// or a fault pair when it is the pair's lower row), so the per-slice partials of a
// pair land on its lower row's slice; both lips of a pair belong to one group.
// z = M^-1 r is stored in bj.z (single-vector layout).
// Start (x != nullptr: x = 0, p = z) or resumption after a residual replacement
// (x == nullptr: z only), with the per-slice partials of r.z and r.r.
template <typename T>
__global__ __launch_bounds__(WG) void k_g_init_bj(int64_t nslices, BjCols<T> bj, T *__restrict__ x, const T *__restrict__ r,
                                                  T *__restrict__ p, double *part, int64_t stride)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    const int64_t u = s * SLICE + lane;
    const int ku = bj.fslot[u];
    const int64_t w = ku >= 0 ? bj.fpart[ku] : -1;
    double v[2] = {0, 0};
    if (!(w >= 0 && w < u)) {
        const int nr = w >= 0 ? 2 : 1;
        const int kw = w >= 0 ? bj.fslot[w] : -1;
        T rr[6] = {0, 0, 0, 0, 0, 0};
        for (int m = 0; m < nr; ++m)
            for (int k = 0; k < 3; ++k) {
                rr[3 * m + k] = r[3 * (m == 0 ? u : w) + k];
                v[1] += (double)rr[3 * m + k] * (double)rr[3 * m + k];
            }
        v[0] = bjc_unit_z(bj, u, w, ku, kw, rr, nr, 1, 0);
        if (x)
            for (int m = 0; m < nr; ++m)
                for (int k = 0; k < 3; ++k) {
                    const int64_t i = 3 * (m == 0 ? u : w) + k;
                    x[i] = 0;
                    p[i] = bj.z[i];
                }
    }
    slice_partials<2>(v, s, lane, part, stride);
}

template <typename T>
__global__ __launch_bounds__(WG) void k_g_update_bj(int64_t nslices, const int32_t *__restrict__ slice_group,
                                                    BjCols<T> bj, T *__restrict__ x, T *__restrict__ r,
                                                    const T *__restrict__ p, const T *__restrict__ q, double *part,
                                                    int64_t stride, const MrScalars *sc)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    const int g = slice_group[s];
    if (sc->done[g]) return;
    const T al = (T)sc->alpha[g];
    const int64_t u = s * SLICE + lane;
    const int ku = bj.fslot[u];
    const int64_t w = ku >= 0 ? bj.fpart[ku] : -1;
    double v[2] = {0, 0};
    if (!(w >= 0 && w < u)) {
        const int nr = w >= 0 ? 2 : 1;
        const int kw = w >= 0 ? bj.fslot[w] : -1;
        T rr[6] = {0, 0, 0, 0, 0, 0};
        for (int m = 0; m < nr; ++m)
            for (int k = 0; k < 3; ++k) {
                const int64_t i = 3 * (m == 0 ? u : w) + k;
                x[i] += al * p[i];
                const T ri = r[i] - al * q[i];
                r[i] = ri;
                rr[3 * m + k] = ri;
                v[1] += (double)ri * (double)ri;
            }
        v[0] = bjc_unit_z(bj, u, w, ku, kw, rr, nr, 1, 0);
    }
    slice_partials<2>(v, s, lane, part, stride);
}

// p = z + beta p on the groups that go on (after an update or a residual replacement)
template <typename T>
__global__ __launch_bounds__(WG) void k_g_pupdate_bj(int64_t nslices, const int32_t *__restrict__ slice_group,
                                                     const T *__restrict__ z, T *__restrict__ p, const MrScalars *sc)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    const int g = slice_group[s];
    if (sc->done[g]) return;
    const T be = (T)sc->beta[g];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t e = slice_elem(s, k, lane, 3);
        p[e] = z[e] + be * p[e];
    }
}

// per-group squared norms of a vector (per-slice partials, then k_g_norm_fin)
template <int BS>
__global__ __launch_bounds__(WG) void k_g_sq(int64_t nslices, const double *__restrict__ a, double *part, int64_t stride)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    double v[1] = {0};
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        const double t = a[slice_elem(s, k, lane, BS)];
        v[0] += t * t;
    }
    slice_partials<1>(v, s, lane, part, stride);
}

__global__ __launch_bounds__(FIN) void k_g_norm_fin(const double *part, int64_t stride, const int64_t *gsp, double *res)
{
    double tot[1];
    group_sum<1>(part, stride, gsp[blockIdx.x], gsp[blockIdx.x + 1], tot);
    if (threadIdx.x == 0) res[blockIdx.x] = tot[0];
}

// y = (float)(scale[g] * x) and y64 += scale[g] * x32, group of the element's slice
template <int BS>
__global__ void k_g_to_f32(int64_t nslices, const int32_t *__restrict__ slice_group, const double *__restrict__ sc,
                           const double *__restrict__ x, float *__restrict__ y)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    const double c = sc[slice_group[s]];
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        const int64_t e = slice_elem(s, k, lane, BS);
        y[e] = (float)(c * x[e]);
    }
}

template <int BS>
__global__ void k_g_add_f32(int64_t nslices, const int32_t *__restrict__ slice_group, const double *__restrict__ sc,
                            const float *__restrict__ x, double *__restrict__ y)
{
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;
    const double c = sc[slice_group[s]];
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        const int64_t e = slice_elem(s, k, lane, BS);
        y[e] += c * (double)x[e];
    }
}

// Block-Jacobi data of the grouped CG in precision T (FP32 copies for the FP32 CG).
template <typename T>
inline BjCols<T> g_bj(fg_system *S);
template <>
inline BjCols<double> g_bj<double>(fg_system *S) { return BjCols<double>{S->bjA, S->bjB, S->fslot, S->fpart, S->wz}; }
template <>
inline BjCols<float> g_bj<float>(fg_system *S) { return BjCols<float>{S->bjA32, S->bjB32, S->fslot, S->fpart, S->wz32}; }

}  // namespace

template <int BS, typename T, typename TV>
static void g_launch_batch(fg_system *S, const TV *val, const T *dinv, T *x, T *r, T *p, T *q, int iters,
                           hipStream_t st)
{
    const int64_t gs = grid_xcd((S->nslices + 3) / 4);
    const int G = S->ngroups;
    const int64_t stride = S->nslices;
    for (int it = 0; it < iters; ++it) {
        LAUNCH_SH((k_g_spmv<BS, T, TV>), gs, WG, (spmv_lds<BS, T>(S)), st, spmv_args(S), S->slice_group, val, p, q,
                  S->gpart, stride, S->gsc);
        LAUNCH(k_g_alpha, G, FIN, st, S->gpart, stride, S->group_slice_ptr, S->gsc);
        if constexpr (BS == 3 && std::is_same<T, TV>::value) {
            if (S->k_precond) {
                const BjCols<T> bj = g_bj<T>(S);
                LAUNCH((k_g_update_bj<T>), gs, WG, st, S->nslices, S->slice_group, bj, x, r, p, q, S->gpart, stride,
                       S->gsc);
                LAUNCH(k_g_beta, G, FIN, st, S->gpart, stride, S->group_slice_ptr, S->gsc);
                LAUNCH((k_g_pupdate_bj<T>), gs, WG, st, S->nslices, S->slice_group, (const T *)bj.z, p, S->gsc);
                continue;
            }
        }
        LAUNCH((k_g_update<BS, T>), gs, WG, st, S->nslices, S->slice_group, dinv, x, r, p, q, S->gpart, stride, S->gsc);
        LAUNCH(k_g_beta, G, FIN, st, S->gpart, stride, S->group_slice_ptr, S->gsc);
        LAUNCH((k_g_pupdate<BS, T>), gs, WG, st, S->nslices, S->slice_group, dinv, r, p, S->gsc);
    }
}

template <int BS, typename T, typename TV>
static fg_status g_batch(fg_system *S, const TV *val, const T *dinv, T *x, T *r, T *p, T *q, int iters, int slot,
                         hipStream_t st)
{
    if (!S->use_graphs) {
        g_launch_batch<BS, T, TV>(S, val, dinv, x, r, p, q, iters, st);
        return check_hip("grouped cg batch");
    }
    GraphCache &g = S->g_graph[slot];
    const int key = S->k_precond != 0;
    if (!g.exec || g.iters != iters || g.tile != key) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(S->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return check_hip("grouped cg capture");
        g_launch_batch<BS, T, TV>(S, val, dinv, x, r, p, q, iters, S->cap_stream);
        if (hipStreamEndCapture(S->cap_stream, &graph) != hipSuccess) return check_hip("grouped cg capture end");
        hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g.exec = nullptr;
            return check_hip("grouped cg instantiate");
        }
        g.iters = iters;
        g.tile = key;
    }
    hipGraphLaunch(g.exec, st);
    return check_hip("grouped cg launch");
}

void drop_group_graphs(fg_system *S)
{
    for (GraphCache &g : S->g_graph) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.iters = 0;
    }
}

// Start of the grouped CG on the right-hand side already in S->wr (FP64) or S->fr (FP32).
static fg_status g_init(fg_system *S, int which, bool f32, double tol, int64_t maxit, hipStream_t st)
{
    MrScalars init{};
    init.maxit = maxit;
    init.nrhs = S->ngroups;
    hipMemcpyAsync(S->gsc, &init, sizeof init, hipMemcpyHostToDevice, st);
    const int64_t gs = grid_xcd((S->nslices + 3) / 4), stride = S->nslices;
    if (f32 && !S->k32_valid) refresh_k32(S, st);
    if (which == FG_K && S->k_precond) {
        if (f32) {
            bj_ready32(S, st);
            LAUNCH((k_g_init_bj<float>), gs, WG, st, S->nslices, g_bj<float>(S), S->fx, S->fr, S->fp, S->gpart,
                   stride);
        } else {
            bj_ready(S, st);
            LAUNCH((k_g_init_bj<double>), gs, WG, st, S->nslices, g_bj<double>(S), S->wx, S->wr, S->wp, S->gpart,
                   stride);
        }
        if (S->bj_singular) {
            set_error("fg_pcg_solve: a diagonal or fault-pair block of K is singular (block Jacobi)");
            return FG_ERR_BREAKDOWN;
        }
    } else if (f32) {
        LAUNCH((k_g_init<3, float>), gs, WG, st, S->nslices, S->dinvK32, S->fx, S->fr, S->fp, S->gpart, stride);
    } else if (which == FG_K) {
        LAUNCH((k_g_init<3, double>), gs, WG, st, S->nslices, S->dinvK, S->wx, S->wr, S->wp, S->gpart, stride);
    } else {
        LAUNCH((k_g_init<1, double>), gs, WG, st, S->nslices, S->dinvA, S->wx, S->wr, S->wp, S->gpart, stride);
    }
    LAUNCH(k_g_init_fin, S->ngroups, FIN, st, S->gpart, stride, S->group_slice_ptr, S->gsc, tol);
    return check_hip("grouped cg init");
}

// Batches of iterations until every group is done; per-group results in S->gsc_host.
static fg_status g_loop(fg_system *S, int which, bool f32, int check_every, hipStream_t st)
{
    const int batch = check_every > 0 ? check_every : 32;
    for (;;) {
        hipMemcpyAsync(S->gsc_host, S->gsc, sizeof(MrScalars), hipMemcpyDeviceToHost, st);
        hipStreamSynchronize(st);
        fg_status e = check_hip("grouped cg poll");
        if (e) return e;
        bool all = true;
        for (int g = 0; g < S->ngroups; ++g) all = all && S->gsc_host->done[g];
        if (all) return FG_OK;
        if (f32)
            e = g_batch<3, float, float>(S, S->K32, S->dinvK32, S->fx, S->fr, S->fp, S->fq, batch, 1, st);
        else if (which == FG_K)
            e = g_batch<3, double, double>(S, S->K, S->dinvK, S->wx, S->wr, S->wp, S->wq, batch, 0, st);
        else
            e = g_batch<1, double, double>(S, S->A22, S->dinvA, S->wx, S->wr, S->wp, S->wq, batch, 2, st);
        if (e) return e;
    }
}

fg_status cg_run_grouped(fg_system *S, int which, int precision, double tol, int64_t maxit, int check_every,
                         int64_t *iters, double *relres, hipStream_t st)
{
    const bool f32 = (which == FG_K && precision == FG_F32);
    fg_status e = g_init(S, which, f32, tol, maxit, st);
    if (e) return e;
    e = g_loop(S, which, f32, check_every, st);
    if (e) return e;
    const MrScalars &h = *S->gsc_host;
    fg_status worst = FG_OK;
    int64_t imax = 0;
    double rmax = 0;
    for (int g = 0; g < S->ngroups; ++g) {
        imax = std::max<int64_t>(imax, h.iter[g]);
        const double rel = h.bb[g] > 0 ? std::sqrt(h.rr[g] / h.bb[g]) : 0.0;
        rmax = std::max(rmax, rel);
        S->grp_iters[g] += h.iter[g];
        S->grp_relres[g] = rel;
        S->grp_status[g] = h.status[g];
        if (h.status[g] < 0) worst = std::min(worst, (fg_status)h.status[g]);
        else if (worst >= 0) worst = std::max(worst, (fg_status)h.status[g]);
    }
    *iters = imax;
    *relres = rmax;
    if (worst == FG_ERR_BREAKDOWN) set_error("fg_pcg_solve: CG breakdown in a group (p.Ap <= 0)");
    if (worst == FG_ERR_NAN) set_error("fg_pcg_solve: NaN or Inf in a group");
    return worst;
}

// FG_MIXED K solve of a batched system by reliable updates, group by group: the
// FP32 grouped CG (each group scaled by 1/||b_g||) runs until every group has cut
// its residual by `delta` (or reached 0.5 tol); then each group's FP32 correction
// is added to the FP64 x, the FP64 residual b - K x replaces the FP32 one, and the
// groups above tol go on from their last direction with the threshold
// max(delta rel, 0.5 tol).  rhs, x: internal layout (3 Npad).
fg_status cg_reliable_grouped(fg_system *S, const double *rhs, double *x, double tol, int64_t maxit, int check_every,
                              double delta, int64_t *iters, int64_t *updates, double *worst_rel, hipStream_t st)
{
    const int G = S->ngroups;
    const int64_t n = 3 * S->Npad, gs = grid_xcd((S->nslices + 3) / 4), stride = S->nslices;
    double *r = S->v4, *next2_d = S->gred + MAX_GROUPS;
    std::vector<double> bn(G), rn(G), scale(G), next2(G), rel(G, 0.0);
    if (!S->k32_valid) refresh_k32(S, st);
    group_norms(S, 3, rhs, bn.data(), st);
    for (int g = 0; g < G; ++g) {
        if (!std::isfinite(bn[g])) {
            set_error("fg_pcg_solve: NaN or Inf in a group's right-hand side");
            return FG_ERR_NAN;
        }
        scale[g] = bn[g] > 0 ? 1.0 / bn[g] : 0.0;
    }
    vfill(x, 0.0, n, st);
    group_to_f32(S, scale.data(), rhs, S->fr, st);
    fg_status e = g_init(S, FG_K, true, delta, maxit, st);
    if (e) return e;
    *iters = 0;
    *updates = 0;
    fg_status worst = FG_OK;
    for (;;) {
        e = g_loop(S, FG_K, true, check_every, st);
        if (e) return e;
        const MrScalars &h = *S->gsc_host;
        std::vector<int64_t> it(h.iter, h.iter + G);
        for (int g = 0; g < G; ++g) {
            *iters = std::max<int64_t>(*iters, it[g]);
            if (h.status[g] < 0) {
                set_error(h.status[g] == FG_ERR_NAN ? "fg_pcg_solve: NaN or Inf in a group"
                                                    : "fg_pcg_solve: CG breakdown in a group (p.Ap <= 0)");
                return h.status[g];
            }
        }
        // fold the FP32 corrections into x and replace the residuals by FP64 ones
        group_add_f32(S, bn.data(), S->fx, x, st);
        hipMemsetAsync(S->fx, 0, n * sizeof(float), st);
        spmv(S, FG_K, x, S->wq, st);
        hipMemcpyAsync(r, rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        vaxpby(n, -1.0, S->wq, 1.0, r, st);
        group_norms(S, 3, r, rn.data(), st);
        ++*updates;
        bool any = false;
        *worst_rel = 0;
        for (int g = 0; g < G; ++g) {
            rel[g] = bn[g] > 0 ? rn[g] / bn[g] : 0.0;
            if (!std::isfinite(rel[g])) {
                set_error("fg_pcg_solve: NaN in a group's residual replacement");
                return FG_ERR_NAN;
            }
            *worst_rel = std::max(*worst_rel, rel[g]);
            next2[g] = -1.0;
            if (rel[g] <= tol) continue;
            if (it[g] >= maxit) {
                worst = FG_NOT_CONVERGED;
                continue;
            }
            const double nx = std::max(delta * rel[g], 0.5 * tol);
            next2[g] = nx * nx;
            any = true;
        }
        if (!any) {
            for (int g = 0; g < G; ++g) {
                S->grp_iters[g] += it[g];
                S->grp_relres[g] = rel[g];
                S->grp_status[g] = rel[g] <= tol ? FG_OK : FG_NOT_CONVERGED;
            }
            return worst;
        }
        group_to_f32(S, scale.data(), r, S->fr, st);
        hipMemcpyAsync(next2_d, next2.data(), G * sizeof(double), hipMemcpyHostToDevice, st);
        if (S->k_precond) {
            LAUNCH((k_g_init_bj<float>), gs, WG, st, S->nslices, g_bj<float>(S), (float *)nullptr, S->fr,
                   (float *)nullptr, S->gpart, stride);
            LAUNCH(k_g_resume_fin, G, FIN, st, S->gpart, stride, S->group_slice_ptr, S->gsc, next2_d);
            LAUNCH((k_g_pupdate_bj<float>), gs, WG, st, S->nslices, S->slice_group, (const float *)S->wz32, S->fp,
                   S->gsc);
        } else {
            LAUNCH((k_g_resume<3, float>), gs, WG, st, S->nslices, S->dinvK32, S->fr, S->gpart, stride);
            LAUNCH(k_g_resume_fin, G, FIN, st, S->gpart, stride, S->group_slice_ptr, S->gsc, next2_d);
            LAUNCH((k_g_resume_p<3, float>), gs, WG, st, S->nslices, S->slice_group, S->dinvK32, S->fr, S->fp,
                   S->gsc);
        }
        e = check_hip("grouped cg resume");
        if (e) return e;
    }
}

// Per-group norms of an internal vector with BS values per row.
void group_norms(fg_system *S, int bs, const double *a, double *host, hipStream_t st)
{
    const int64_t gs = grid_xcd((S->nslices + 3) / 4), stride = S->nslices;
    if (bs == 3)
        LAUNCH(k_g_sq<3>, gs, WG, st, S->nslices, a, S->gpart, stride);
    else
        LAUNCH(k_g_sq<1>, gs, WG, st, S->nslices, a, S->gpart, stride);
    LAUNCH(k_g_norm_fin, S->ngroups, FIN, st, S->gpart, stride, S->group_slice_ptr, S->gred);
    hipMemcpyAsync(S->gred_host, S->gred, S->ngroups * sizeof(double), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    for (int g = 0; g < S->ngroups; ++g) host[g] = std::sqrt(S->gred_host[g]);
}

// y32 = scale[group] * x64 and y64 += scale[group] * x32 for K-sized vectors; scale is host data.
void group_to_f32(fg_system *S, const double *scale, const double *x, float *y, hipStream_t st)
{
    hipMemcpyAsync(S->gred, scale, S->ngroups * sizeof(double), hipMemcpyHostToDevice, st);
    LAUNCH(k_g_to_f32<3>, grid_xcd((S->nslices + 3) / 4), WG, st, S->nslices, S->slice_group, S->gred, x, y);
}

void group_add_f32(fg_system *S, const double *scale, const float *x, double *y, hipStream_t st)
{
    hipMemcpyAsync(S->gred, scale, S->ngroups * sizeof(double), hipMemcpyHostToDevice, st);
    LAUNCH(k_g_add_f32<3>, grid_xcd((S->nslices + 3) / 4), WG, st, S->nslices, S->slice_group, S->gred, x, y);
}

}  // namespace fg
