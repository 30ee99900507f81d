// Many right-hand sides on one stiffness: independent point-Jacobi CG per
// column, advanced together so that every iteration streams the matrix once
// per tile of columns instead of once per column.
//
// Vector layout: column-interleaved, element (dof d, column c) at d*nrhs + c, so
// the columns of one DOF are contiguous (one wide load per gathered node).
// Each column has its own alpha, beta, rho and stop flag; a converged column is
// masked out of the vector updates.  nrhs is a power of two <= MR_MAX.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "fg_device.h"
#include "fg_kernels.h"

namespace fg {

namespace {

// per-thread column of an element-wise kernel: the grid size is a multiple of nrhs
__device__ __forceinline__ int elem_col(int nrhs) { return (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) & (nrhs - 1)); }

// Per-column block partials: thread t holds NV sums of column (t mod nrhs); the
// block adds the threads of each column and stores partials[(k*nrhs + c)*stride + block].
template <int NV>
__device__ __forceinline__ void block_partials_cols(const double (&v)[NV], int nrhs, double *partials, int64_t stride)
{
    __shared__ double sh[NV][WG];
    for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    if ((int)threadIdx.x < nrhs)
        for (int k = 0; k < NV; ++k) {
            double s = 0;
            for (int j = threadIdx.x; j < WG; j += nrhs) s += sh[k][j];
            partials[((int64_t)k * nrhs + threadIdx.x) * stride + blockIdx.x] = s;
        }
}

template <int NV>
__device__ __forceinline__ void column_sum(const double *partials, int nrhs, int c, int64_t stride, int64_t nparts,
                                           double (&tot)[NV])
{
    __shared__ double sh[NV][FIN / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = 0; k < NV; ++k) {
        double s = 0;
        for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) s += partials[((int64_t)k * nrhs + c) * stride + i];
        s = wave_sum(s);
        if (lane == 0) sh[k][w] = s;
    }
    __syncthreads();
    for (int k = 0; k < NV; ++k) {
        double s = 0;
        for (int i = 0; i < nw; ++i) s += sh[k][i];
        tot[k] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(WG) void k_mr_init(int64_t n, int nrhs, int lg, const T *__restrict__ dinv, T *__restrict__ x,
                                                const T *__restrict__ r, T *__restrict__ p, double *partials,
                                                int64_t stride)
{
    double v[2] = {0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T ri = r[i], zi = dinv[i >> lg] * ri;
        x[i] = 0;
        p[i] = zi;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    block_partials_cols<2>(v, nrhs, partials, stride);
}

__global__ __launch_bounds__(FIN) void k_mr_init_fin(const double *partials, int nrhs, int64_t stride, int64_t nparts,
                                                     MrScalars *sc, double tol)
{
    const int c = blockIdx.x;
    double tot[2];
    column_sum<2>(partials, nrhs, c, stride, nparts, tot);
    if (threadIdx.x != 0) return;
    sc->rho[c] = tot[0];
    sc->rr[c] = tot[1];
    sc->bb[c] = tot[1];
    sc->tol2[c] = tol * tol * tot[1];
    sc->soft2[c] = sc->overrun2 * sc->tol2[c];
    sc->iter[c] = 0;
    sc->status[c] = FG_OK;
    sc->done[c] = 0;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
        sc->status[c] = FG_ERR_NAN;
        sc->done[c] = 1;
    } else if (tot[1] == 0.0) {
        sc->done[c] = 1;
    } else if (sc->maxit <= 0) {
        sc->status[c] = FG_NOT_CONVERGED;
        sc->done[c] = 1;
    }
    sc->ready[c] = sc->done[c];
}

// Q = K P for the columns [c0, c0 + CT) of one slice per wavefront, with the
// per-column block partials of P.Q.  The 9 values of a slot are loaded once
// and applied to all CT columns; x operands are gathered from global memory.
template <typename T, typename TV, int CT>
__global__ __launch_bounds__(WG) void k_mr_spmm(SpmvArgs a, int nrhs, const TV *__restrict__ val,
                                                const T *__restrict__ p, T *__restrict__ q, double *partials,
                                                int64_t stride, int with_dot)
{
    const int c0 = blockIdx.y * CT;
    const int64_t s = xcd_block() * (WG / SLICE) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double v[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) v[c] = 0;
    if (s < a.nslices) {
        const int64_t base = a.slice_ptr[s];
        const int w = (int)((a.slice_ptr[s + 1] - base) / SLICE);
        const int32_t *cl = a.col + base + lane;
        const TV *vb0 = val + 9 * base + lane;
        T acc[3][CT];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[r][c] = 0;
        for (int j = 0; j < w; ++j) {
            const int64_t cj = cl[(int64_t)j * SLICE];
            const TV *vb = vb0 + (int64_t)9 * j * SLICE;
            T m[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) m[e] = (T)vb[e * SLICE];
            const T *xp = p + 3 * cj * nrhs + c0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    const T xv = xp[k * nrhs + c];
                    acc[0][c] += m[k] * xv;
                    acc[1][c] += m[3 + k] * xv;
                    acc[2][c] += m[6 + k] * xv;
                }
        }
        const int64_t r0 = s * SLICE + lane;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const int64_t i = (3 * r0 + r) * nrhs + c0 + c;
                q[i] = acc[r][c];
                if (with_dot) v[c] += (double)p[i] * (double)acc[r][c];
            }
    }
    if (!with_dot) return;
    // block partials of the CT columns of this tile
    __shared__ double sh[CT][WG / 64];
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const double t = wave_sum(v[c]);
        if (lane == 0) sh[c][wv] = t;
    }
    __syncthreads();
    if (threadIdx.x < CT) {
        double t = 0;
        for (int i = 0; i < WG / 64; ++i) t += sh[threadIdx.x][i];
        partials[(int64_t)(c0 + threadIdx.x) * stride + blockIdx.x] = t;
    }
}

// Q = K P with the columns of a row spread over the lanes: NR/2 lanes per row,
// two adjacent columns per lane, so each gathered node's operands are one
// contiguous run of 3*NR values read by a group of lanes together, and the
// matrix is streamed once for all columns.  One workgroup per slice; its four
// waves take 64/NR*2 rows at a time.  Per-column partials of P.Q go to
// partials[c*stride + block] (P of the row itself comes from the diagonal slot).
template <typename T>
struct Pair;
template <>
struct Pair<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};

// Slots j0 .. j0+U-1 of one row for the row-group product (slots past the
// row's length multiply zeros against the row's own operands).
template <typename T, typename TV, int NR, int U>
__device__ __forceinline__ void mr_rows_slots(int j0, int len, int dj, int64_t r, int gb, int c2,
                                              const int32_t *__restrict__ cl, const TV *__restrict__ vb,
                                              const T *__restrict__ p, typename Pair<T>::type (&acc)[3],
                                              typename Pair<T>::type (&dp)[3])
{
    typedef typename Pair<T>::type T2;
    constexpr int LPR = NR / 2, NL = (9 + LPR - 1) / LPR;
    int64_t cj[U];
    T mv[U][NL];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = j0 + u;
        const bool on = j < len;
        cj[u] = on ? (int64_t)cl[(int64_t)j * SLICE] : r;
#pragma unroll
        for (int w = 0; w < NL; ++w) {
            const int e = w * LPR + c2;
            mv[u][w] = (on && e < 9) ? (T)vb[(int64_t)(9 * j + e) * SLICE] : (T)0;
        }
    }
    T2 xv[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const T2 *xp = (const T2 *)(p + 3 * cj[u] * NR) + c2;
#pragma unroll
        for (int k = 0; k < 3; ++k) xv[u][k] = xp[k * LPR];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        T m[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) m[e] = __shfl(mv[u][e / LPR], gb + e % LPR, 64);
#pragma unroll
        for (int rr = 0; rr < 3; ++rr)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[rr] += m[3 * rr + k] * xv[u][k];
        if (j0 + u == dj)
#pragma unroll
            for (int k = 0; k < 3; ++k) dp[k] = xv[u][k];
    }
}

// Slots of one row for the row-group product, a chunk of NR/2 slots at a time:
// lane c2 of a row group loads the column of slot j0 + c2 once, and the lanes
// take each slot's column from it by a shuffle, so the x gathers of a chunk
// wait on one column load instead of one per slot; the loads of U slots are
// issued before any of them is used.  Every load is unconditional and inside
// the slice: slot indices are clamped to the wave's longest row (at most the
// slice width), padding slots of shorter rows hold zero values against the
// row's own column, and clamped repeats (the chunk's last U-group) are skipped.
// FORM bits: U in 1..4, 8 = nontemporal value and column loads, 16 = every lane
// loads the 9 values of a slot itself (no value broadcast).
template <typename T, typename TV, int NR, int FORM>
__device__ __forceinline__ void mr_rows_chunked(int len_w, int dj, int gb, int c2, const int32_t *__restrict__ cl,
                                                const TV *__restrict__ vb, const T *__restrict__ p,
                                                typename Pair<T>::type (&acc)[3], typename Pair<T>::type (&dp)[3])
{
    typedef typename Pair<T>::type T2;
    constexpr int LPR = NR / 2, NL = (9 + LPR - 1) / LPR, U = FORM & 7;
    constexpr bool NT = (FORM & 8) != 0, VD = (FORM & 16) != 0;
    constexpr int NV = VD ? 9 : NL;
    for (int j0 = 0; j0 < len_w; j0 += LPR) {
        const int cown = ld_val<NT>(cl + (int64_t)min(j0 + c2, len_w - 1) * SLICE);
        const int nj = min(LPR, len_w - j0);
        for (int jj = 0; jj < nj; jj += U) {
            T mv[U][NV];
            T2 xv[U][3];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int js = min(jj + u, nj - 1);
                const int j = j0 + js;
                const int64_t cj = __shfl(cown, gb + js, 64);
#pragma unroll
                for (int w = 0; w < NV; ++w) {
                    const int e = VD ? w : min(w * LPR + c2, 8);
                    mv[u][w] = (T)ld_val<NT>(vb + (int64_t)(9 * j + e) * SLICE);
                }
                const T2 *xp = (const T2 *)(p + 3 * cj * NR) + c2;
#pragma unroll
                for (int k = 0; k < 3; ++k) xv[u][k] = xp[k * LPR];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (jj + u >= nj) break;  // wave-uniform
                T m[9];
#pragma unroll
                for (int e = 0; e < 9; ++e) m[e] = VD ? mv[u][e] : __shfl(mv[u][e / LPR], gb + e % LPR, 64);
#pragma unroll
                for (int rr = 0; rr < 3; ++rr)
#pragma unroll
                    for (int k = 0; k < 3; ++k) acc[rr] += m[3 * rr + k] * xv[u][k];
                if (j0 + jj + u == dj)
#pragma unroll
                    for (int k = 0; k < 3; ++k) dp[k] = xv[u][k];
            }
        }
    }
}

// FORM 0: one column load per slot (mr_rows_slots); else mr_rows_chunked.
template <typename T, typename TV, int NR, int FORM>
__global__ __launch_bounds__(WG) void k_mr_rows(SpmvArgs a, const uint8_t *__restrict__ rowlen,
                                                const TV *__restrict__ val, const T *__restrict__ p,
                                                T *__restrict__ q, double *partials, int64_t stride, int with_dot)
{
    typedef typename Pair<T>::type T2;
    constexpr int LPR = NR / 2, RPW = SLICE / LPR, RPB = (WG / SLICE) * RPW, PASSES = SLICE / RPB;
    constexpr int U = 1;  // deeper unrolling measured no faster: the gathers are bound by the cache, not latency
    const int64_t s = xcd_block();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane / LPR, c2 = lane % LPR;
    double v0 = 0, v1 = 0;
    if (s < a.nslices) {
        const int64_t base = a.slice_ptr[s];
        for (int ps = 0; ps < PASSES; ++ps) {
            const int l = ps * RPB + wave * RPW + g;
            const int64_t r = s * SLICE + l;
            const int len = rowlen[r], dj = a.diag_slot[r];
            const int32_t *cl = a.col + base + l;
            const TV *vb = val + 9 * base + l;
            T2 acc[3], dp[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[k] = T2{0, 0}, dp[k] = T2{0, 0};
            // the 9 values of a slot are loaded once per row group, one per lane, and
            // broadcast to the group's lanes (lane e mod LPR holds value e)
            const int gb = lane - c2;
            int len_w = len;  // the wave's longest row: every lane takes part in the broadcasts
            for (int off = LPR; off < SLICE; off <<= 1) len_w = max(len_w, __shfl_xor(len_w, off, 64));
            if constexpr (FORM == 0) {
                for (int j0 = 0; j0 < len_w; j0 += U) mr_rows_slots<T, TV, NR, U>(j0, len, dj, r, gb, c2, cl, vb, p, acc, dp);
            } else {
                mr_rows_chunked<T, TV, NR, FORM>(__builtin_amdgcn_readfirstlane(len_w), dj, gb, c2, cl, vb, p, acc, dp);
            }
            T2 *qp = (T2 *)(q + 3 * r * NR) + c2;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                qp[k * LPR] = acc[k];
                v0 += (double)dp[k].x * (double)acc[k].x;
                v1 += (double)dp[k].y * (double)acc[k].y;
            }
        }
    }
    if (!with_dot) return;
    // lanes with the same column pair: across the row groups of the wave, then across waves
    for (int off = LPR; off < SLICE; off <<= 1) {
        v0 += __shfl_xor(v0, off, 64);
        v1 += __shfl_xor(v1, off, 64);
    }
    __shared__ double sh[WG / SLICE][NR];
    if (g == 0) sh[wave][2 * c2] = v0, sh[wave][2 * c2 + 1] = v1;
    __syncthreads();
    if ((int)threadIdx.x < NR) {
        double t = 0;
        for (int w = 0; w < WG / SLICE; ++w) t += sh[w][threadIdx.x];
        partials[(int64_t)threadIdx.x * stride + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(FIN) void k_mr_alpha(const double *partials, int nrhs, int64_t stride, int64_t nparts,
                                                  MrScalars *sc)
{
    const int c = blockIdx.x;
    if (sc->done[c]) {
        if (threadIdx.x == 0) sc->upd[c] = 0;
        return;
    }
    double tot[1];
    column_sum<1>(partials, nrhs, c, stride, nparts, tot);
    if (threadIdx.x != 0) return;
    const double pq = tot[0];
    sc->pq[c] = pq;
    sc->upd[c] = 0;
    if (!isfinite(pq)) {
        sc->status[c] = FG_ERR_NAN;
        sc->done[c] = 1;
    } else if (!(pq > 0.0)) {
        sc->status[c] = FG_ERR_BREAKDOWN;
        sc->done[c] = 1;
    } else {
        sc->alpha[c] = sc->rho[c] / pq;
        sc->upd[c] = 1;
    }
}

// r -= alpha q and the per-column partials of r.z and r.r (x += alpha p is
// left to k_mr_pupdate, which reads p anyway).
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_update(int64_t n, int nrhs, int lg, const T *__restrict__ dinv,
                                                  T *__restrict__ r, const T *__restrict__ q, double *partials,
                                                  int64_t stride, const MrScalars *sc)
{
    const int c = elem_col(nrhs);
    double v[2] = {0, 0};
    if (sc->upd[c]) {
        const T al = (T)sc->alpha[c];
#pragma unroll 4
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
            const T ri = r[i] - al * q[i];
            r[i] = ri;
            const T zi = dinv[i >> lg] * ri;
            v[0] += (double)ri * (double)zi;
            v[1] += (double)ri * (double)ri;
        }
    }
    block_partials_cols<2>(v, nrhs, partials, stride);
}

__global__ __launch_bounds__(FIN) void k_mr_beta(const double *partials, int nrhs, int64_t stride, int64_t nparts,
                                                 MrScalars *sc)
{
    const int c = blockIdx.x;
    if (sc->done[c]) return;
    double tot[2];
    column_sum<2>(partials, nrhs, c, stride, nparts, tot);
    if (threadIdx.x != 0) return;
    sc->iter[c] += 1;
    sc->rr[c] = tot[1];
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
        sc->status[c] = FG_ERR_NAN;
        sc->done[c] = 1;
    } else if (tot[1] <= sc->soft2[c]) {
        sc->status[c] = FG_OK;
        sc->done[c] = 1;
        sc->ready[c] = 1;
    } else if (sc->iter[c] >= sc->maxit) {
        sc->status[c] = FG_NOT_CONVERGED;
        sc->done[c] = 1;
    } else {
        if (tot[1] <= sc->tol2[c]) sc->ready[c] = 1;
        sc->beta[c] = tot[0] / sc->rho[c];
        sc->rho[c] = tot[0];
    }
}

// x += alpha p for the columns this iteration advanced, then p = z + beta p for
// those that go on.
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_pupdate(int64_t n, int nrhs, int lg, const T *__restrict__ dinv,
                                                   const T *__restrict__ r, T *__restrict__ x, T *__restrict__ p,
                                                   const MrScalars *sc)
{
    const int c = elem_col(nrhs);
    const bool up = sc->upd[c] != 0, cont = !sc->done[c];
    if (!up) return;  // a column that goes on was advanced
    const T al = (T)sc->alpha[c], be = (T)sc->beta[c];
#pragma unroll 4
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T pi = p[i];
        x[i] += al * pi;
        if (cont) p[i] = dinv[i >> lg] * r[i] + be * pi;
    }
}

// ---- block-Jacobi preconditioner of the block CG ("k_precond" >= 1) ----
// The nodal 3x3 / fault-pair 6x6 inverse blocks of the single-vector solve applied
// to every column: one thread per (unit, column), a unit being a node off the
// interface pairs or a fault pair (taken by its lower row), so each thread owns
// the DOFs of its unit in its column and forms z = M^-1 r from values no other
// thread writes.  z is stored column-interleaved like r.
// Start (x != nullptr: x = 0, p = z) or resumption after a residual replacement
// (x == nullptr: z only), with the per-column partials of r.z and r.r.
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_init_bj(int64_t Npad, int nrhs, int lg, BjCols<T> bj, T *__restrict__ x,
                                                   const T *__restrict__ r, T *__restrict__ p, double *partials,
                                                   int64_t stride)
{
    const int c = elem_col(nrhs);
    double v[2] = {0, 0};
    for (int64_t u = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> lg; u < Npad;
         u += ((int64_t)gridDim.x * blockDim.x) >> lg) {
        const int ku = bj.fslot[u];
        const int64_t w = ku >= 0 ? bj.fpart[ku] : -1;
        if (w >= 0 && w < u) continue;
        const int nr = w >= 0 ? 2 : 1;
        const int kw = w >= 0 ? bj.fslot[w] : -1;
        T rr[6] = {0, 0, 0, 0, 0, 0};
        for (int m = 0; m < nr; ++m)
            for (int k = 0; k < 3; ++k) {
                const int64_t i = (3 * (m == 0 ? u : w) + k) * nrhs + c;
                rr[3 * m + k] = r[i];
                v[1] += (double)rr[3 * m + k] * (double)rr[3 * m + k];
            }
        v[0] += bjc_unit_z(bj, u, w, ku, kw, rr, nr, nrhs, c);
        if (x)
            for (int m = 0; m < nr; ++m)
                for (int k = 0; k < 3; ++k) {
                    const int64_t i = (3 * (m == 0 ? u : w) + k) * nrhs + c;
                    x[i] = 0;
                    p[i] = bj.z[i];
                }
    }
    block_partials_cols<2>(v, nrhs, partials, stride);
}

// r -= alpha q and z = M^-1 r per unit, with the per-column partials of r.z and r.r.
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_update_bj(int64_t Npad, int nrhs, int lg, BjCols<T> bj, T *__restrict__ r,
                                                     const T *__restrict__ q, double *partials, int64_t stride,
                                                     const MrScalars *sc)
{
    const int c = elem_col(nrhs);
    double v[2] = {0, 0};
    if (sc->upd[c]) {
        const T al = (T)sc->alpha[c];
        for (int64_t u = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> lg; u < Npad;
             u += ((int64_t)gridDim.x * blockDim.x) >> lg) {
            const int ku = bj.fslot[u];
            const int64_t w = ku >= 0 ? bj.fpart[ku] : -1;
            if (w >= 0 && w < u) continue;
            const int nr = w >= 0 ? 2 : 1;
            const int kw = w >= 0 ? bj.fslot[w] : -1;
            T rr[6] = {0, 0, 0, 0, 0, 0};
            for (int m = 0; m < nr; ++m)
                for (int k = 0; k < 3; ++k) {
                    const int64_t i = (3 * (m == 0 ? u : w) + k) * nrhs + c;
                    const T ri = r[i] - al * q[i];
                    r[i] = ri;
                    rr[3 * m + k] = ri;
                    v[1] += (double)ri * (double)ri;
                }
            v[0] += bjc_unit_z(bj, u, w, ku, kw, rr, nr, nrhs, c);
        }
    }
    block_partials_cols<2>(v, nrhs, partials, stride);
}

// x += alpha p for the columns this iteration advanced, then p = z + beta p for
// those that go on (z stored by k_mr_update_bj).
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_pupdate_bj(int64_t n, int nrhs, const T *__restrict__ z, T *__restrict__ x,
                                                      T *__restrict__ p, const MrScalars *sc)
{
    const int c = elem_col(nrhs);
    const bool up = sc->upd[c] != 0, cont = !sc->done[c];
    if (!up) return;
    const T al = (T)sc->alpha[c], be = (T)sc->beta[c];
#pragma unroll 4
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T pi = p[i];
        x[i] += al * pi;
        if (cont) p[i] = z[i] + be * pi;
    }
}

// p = z + beta p for the columns that go on after a residual replacement.
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_resume_p_bj(int64_t n, int nrhs, const T *__restrict__ z, T *__restrict__ p,
                                                       const MrScalars *sc)
{
    const int c = elem_col(nrhs);
    if (sc->done[c]) return;
    const T be = (T)sc->beta[c];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + be * p[i];
}

// caller layout (column c of length 3N at c*3N, caller node order) <-> interleaved internal layout
__global__ void k_mr_in(int64_t N, int64_t Npad, int nrhs, const int32_t *__restrict__ perm,
                        const double *__restrict__ b, double *__restrict__ out)
{
    const int64_t n = 3 * Npad * nrhs;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % nrhs);
        const int64_t d = i / nrhs, r = d / 3;
        const int32_t o = perm[r];
        out[i] = o >= 0 ? b[(int64_t)c * 3 * N + 3 * (int64_t)o + (d - 3 * r)] : 0.0;
    }
}

__global__ void k_mr_out(int64_t N, int64_t Npad, int nrhs, const int32_t *__restrict__ perm,
                         const double *__restrict__ in, double *__restrict__ x)
{
    const int64_t n = 3 * Npad * nrhs;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % nrhs);
        const int64_t d = i / nrhs, r = d / 3;
        const int32_t o = perm[r];
        if (o >= 0) x[(int64_t)c * 3 * N + 3 * (int64_t)o + (d - 3 * r)] = in[i];
    }
}

// per-column dot products a_c . b_c (block partials; k_mr_colfin adds them)
__global__ __launch_bounds__(WG) void k_mr_coldot(int64_t n, int nrhs, const double *__restrict__ a,
                                                  const double *__restrict__ b, double *partials, int64_t stride)
{
    double v[1] = {0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[0] += a[i] * b[i];
    block_partials_cols<1>(v, nrhs, partials, stride);
}

__global__ __launch_bounds__(FIN) void k_mr_colfin(const double *partials, int nrhs, int64_t stride, int64_t nparts,
                                                   double *res)
{
    double tot[1];
    column_sum<1>(partials, nrhs, blockIdx.x, stride, nparts, tot);
    if (threadIdx.x == 0) res[blockIdx.x] = tot[0];
}

// y_c = s_c * x_c (per-column scale, FP64 -> FP32 or FP32 -> FP64 accumulate)
__global__ void k_mr_scale_to_f32(int64_t n, int nrhs, const double *__restrict__ s, const double *__restrict__ x,
                                  float *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)(s[i % nrhs] * x[i]);
}

__global__ void k_mr_add_f32(int64_t n, int nrhs, const double *__restrict__ s, const float *__restrict__ x,
                             double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += s[i % nrhs] * (double)x[i];
}

// r = b - q, element-wise
__global__ void k_mr_resid(int64_t n, const double *__restrict__ b, const double *__restrict__ q, double *__restrict__ r)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        r[i] = b[i] - q[i];
}

// Residual replacement of the FP32 block CG (reliable updates): per-column
// partials of r.z and r.r of the new (FP64-derived) residual ...
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_resume(int64_t n, int nrhs, int lg, const T *__restrict__ dinv,
                                                  const T *__restrict__ r, double *partials, int64_t stride)
{
    double v[2] = {0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T ri = r[i], zi = dinv[i >> lg] * ri;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    block_partials_cols<2>(v, nrhs, partials, stride);
}

// Before a residual replacement, a column still iterating (done = 0) holds
// p_{k+1} = z_{k+1} + beta_k p_k and rho_{k+1}; subtracting its recursive z_{k+1}
// leaves beta_k p_k, so that the resume's p = z + (rho_new / rho_{k+1}) p gives
// z + (rho_new / rho_k) p_k, as for a column that stopped at iteration k.
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_strip_z(int64_t n, int nrhs, int lg, const T *__restrict__ dinv,
                                                   const T *__restrict__ r, T *__restrict__ p, const MrScalars *sc)
{
    const int c = elem_col(nrhs);
    if (sc->done[c]) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] -= dinv[i >> lg] * r[i];
}

// The same with the block-Jacobi z stored by the last update.
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_strip_z_bj(int64_t n, int nrhs, const T *__restrict__ z, T *__restrict__ p,
                                                      const MrScalars *sc)
{
    const int c = elem_col(nrhs);
    if (sc->done[c]) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] -= z[i];
}

// ... then, per column, beta against the rho the column stopped with (its last
// direction p is kept; a column still iterating at the replacement was brought to
// that state by k_mr_strip_z), the new rho and stop thresholds from next2[c]
// (squared; a column with next2[c] <= 0 is finished and stays done) ...
__global__ __launch_bounds__(FIN) void k_mr_resume_fin(const double *partials, int nrhs, int64_t stride, int64_t nparts,
                                                       MrScalars *sc, const double *next2)
{
    const int c = blockIdx.x;
    double tot[2];
    column_sum<2>(partials, nrhs, c, stride, nparts, tot);
    if (threadIdx.x != 0) return;
    sc->upd[c] = 0;
    sc->status[c] = FG_OK;
    sc->done[c] = 1;
    sc->ready[c] = 1;
    if (!(next2[c] > 0.0)) return;
    const double beta = tot[0] / sc->rho[c];
    sc->rr[c] = tot[1];
    if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(beta)) {
        sc->status[c] = FG_ERR_NAN;
    } else if (sc->iter[c] >= sc->maxit) {
        sc->status[c] = FG_NOT_CONVERGED;
    } else {
        sc->beta[c] = beta;
        sc->rho[c] = tot[0];
        sc->tol2[c] = next2[c];
        sc->soft2[c] = sc->overrun2 * next2[c];
        sc->done[c] = 0;
        sc->ready[c] = 0;
    }
}

// ... and p = z + beta p for the columns that go on.
template <typename T>
__global__ __launch_bounds__(WG) void k_mr_resume_p(int64_t n, int nrhs, int lg, const T *__restrict__ dinv,
                                                    const T *__restrict__ r, T *__restrict__ p, const MrScalars *sc)
{
    const int c = elem_col(nrhs);
    if (sc->done[c]) return;
    const T be = (T)sc->beta[c];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = dinv[i >> lg] * r[i] + be * p[i];
}

// element-wise grid for column-interleaved vectors; blocks of WG threads make the
// grid a multiple of nrhs, so each thread keeps one column
inline int64_t grid_cols(int64_t n) { return grid_elems(n); }

inline int log2i(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Block-Jacobi data of the block CG in precision T (the FP64 blocks, or their FP32
// copies for the FP32 CG of FG_F32 / FG_MIXED), z in the block workspace.
inline BjCols<double> mr_bj64(fg_system *S) { return BjCols<double>{S->bjA, S->bjB, S->fslot, S->fpart, S->mz}; }
inline BjCols<float> mr_bj32(fg_system *S) { return BjCols<float>{S->bjA32, S->bjB32, S->fslot, S->fpart, S->mfz}; }
template <typename T>
inline BjCols<T> mr_bj(fg_system *S);
template <>
inline BjCols<double> mr_bj<double>(fg_system *S) { return mr_bj64(S); }
template <>
inline BjCols<float> mr_bj<float>(fg_system *S) { return mr_bj32(S); }

}  // namespace

// The row-group product in the slot-loop form that fg_tune "mr_form" selects.
template <typename T, typename TV, int NR>
static void mr_rows_launch(int form, int64_t gr, hipStream_t st, const SpmvArgs &a, fg_system *S, const TV *val,
                           const T *p, T *q, int with_dot)
{
#define MR_FORM(F)                                                                                                  \
    case F:                                                                                                         \
        LAUNCH((k_mr_rows<T, TV, NR, F>), gr, WG, st, a, S->rowlen, val, p, q, S->mpart, S->mpart_stride, with_dot); \
        break;
    switch (form) {
        MR_FORM(1)
        MR_FORM(2)
        MR_FORM(4)
        MR_FORM(9)
        MR_FORM(10)
        MR_FORM(12)
        MR_FORM(17)
        MR_FORM(18)
        MR_FORM(25)
        MR_FORM(26)
    default:
        MR_FORM(0)
    }
#undef MR_FORM
}

// Q = K P for all columns; returns the number of per-column partials written.
// rhs_tile 0 (default): the row-group kernel for nrhs >= 8; otherwise the
// column-tile kernel with rhs_tile columns per pass.
template <typename T, typename TV>
static int64_t mr_launch_spmm(fg_system *S, int nrhs, const TV *val, const T *p, T *q, int with_dot, hipStream_t st)
{
    const SpmvArgs a = spmv_args(S);
    if (S->mr_tile == 0 && nrhs >= 8) {
        const int64_t gr = grid_xcd(S->nslices);
        switch (nrhs) {
        case 8:
            mr_rows_launch<T, TV, 8>(S->mr_form, gr, st, a, S, val, p, q, with_dot);
            break;
        case 16:
            mr_rows_launch<T, TV, 16>(S->mr_form, gr, st, a, S, val, p, q, with_dot);
            break;
        case 32:
            mr_rows_launch<T, TV, 32>(S->mr_form, gr, st, a, S, val, p, q, with_dot);
            break;
        default:
            mr_rows_launch<T, TV, 64>(S->mr_form, gr, st, a, S, val, p, q, with_dot);
            break;
        }
        return gr;
    }
    const int64_t gx = grid_xcd((S->nslices + 3) / 4);
    const int ct = S->mr_tile == 0 ? std::min(8, nrhs) : std::min(S->mr_tile, nrhs);
    switch (ct) {
    case 1:
        hipLaunchKernelGGL((k_mr_spmm<T, TV, 1>), dim3(gx, nrhs / 1), dim3(WG), 0, st, a, nrhs, val, p, q, S->mpart,
                           S->mpart_stride, with_dot);
        break;
    case 2:
        hipLaunchKernelGGL((k_mr_spmm<T, TV, 2>), dim3(gx, nrhs / 2), dim3(WG), 0, st, a, nrhs, val, p, q, S->mpart,
                           S->mpart_stride, with_dot);
        break;
    case 4:
        hipLaunchKernelGGL((k_mr_spmm<T, TV, 4>), dim3(gx, nrhs / 4), dim3(WG), 0, st, a, nrhs, val, p, q, S->mpart,
                           S->mpart_stride, with_dot);
        break;
    case 8:
        hipLaunchKernelGGL((k_mr_spmm<T, TV, 8>), dim3(gx, nrhs / 8), dim3(WG), 0, st, a, nrhs, val, p, q, S->mpart,
                           S->mpart_stride, with_dot);
        break;
    default:
        hipLaunchKernelGGL((k_mr_spmm<T, TV, 16>), dim3(gx, nrhs / 16), dim3(WG), 0, st, a, nrhs, val, p, q, S->mpart,
                           S->mpart_stride, with_dot);
        break;
    }
    return gx;
}

template <typename T, typename TV>
static void mr_launch_batch(fg_system *S, int nrhs, const TV *val, const T *dinv, T *x, T *r, T *p, T *q, int iters,
                            hipStream_t st)
{
    const int64_t n = 3 * S->Npad * nrhs;
    const int64_t ge = grid_cols(n);
    const bool bj = S->k_precond != 0;
    for (int it = 0; it < iters; ++it) {
        const int64_t gx = mr_launch_spmm<T, TV>(S, nrhs, val, p, q, 1, st);
        hipLaunchKernelGGL(k_mr_alpha, dim3(nrhs), dim3(FIN), 0, st, S->mpart, nrhs, S->mpart_stride, gx, S->msc);
        if (bj) {
            const BjCols<T> m = mr_bj<T>(S);
            hipLaunchKernelGGL((k_mr_update_bj<T>), dim3(ge), dim3(WG), 0, st, S->Npad, nrhs, log2i(nrhs), m, r, q,
                               S->mpart, S->mpart_stride, S->msc);
            hipLaunchKernelGGL(k_mr_beta, dim3(nrhs), dim3(FIN), 0, st, S->mpart, nrhs, S->mpart_stride, ge, S->msc);
            hipLaunchKernelGGL((k_mr_pupdate_bj<T>), dim3(ge), dim3(WG), 0, st, n, nrhs, (const T *)m.z, x, p, S->msc);
            continue;
        }
        hipLaunchKernelGGL((k_mr_update<T>), dim3(ge), dim3(WG), 0, st, n, nrhs, log2i(nrhs), dinv, r, q, S->mpart,
                           S->mpart_stride, S->msc);
        hipLaunchKernelGGL(k_mr_beta, dim3(nrhs), dim3(FIN), 0, st, S->mpart, nrhs, S->mpart_stride, ge, S->msc);
        hipLaunchKernelGGL((k_mr_pupdate<T>), dim3(ge), dim3(WG), 0, st, n, nrhs, log2i(nrhs), dinv, r, x, p, S->msc);
    }
}

// Allocate the block workspaces for nrhs columns (grown on demand).
fg_status mr_reserve(fg_system *S, int nrhs)
{
    if (nrhs <= S->mr_cap) return FG_OK;
    double **d[] = {&S->mx, &S->mr, &S->mp, &S->mq, &S->mb, &S->mx64, &S->mr64, &S->mz};
    float **f[] = {&S->mfx, &S->mfr, &S->mfp, &S->mfq, &S->mfz};
    for (double **p : d) {
        if (*p) hipFree(*p);
        *p = nullptr;
    }
    for (float **p : f) {
        if (*p) hipFree(*p);
        *p = nullptr;
    }
    drop_mr_graphs(S);
    const size_t n = (size_t)3 * S->Npad * nrhs;
    for (double **p : d)
        if (hipMalloc((void **)p, n * sizeof(double)) != hipSuccess) {
            hipGetLastError();
            set_error("fg_pcg_solve: device allocation for the block solve failed");
            return FG_ERR_OOM;
        }
    for (float **p : f)
        if (hipMalloc((void **)p, n * sizeof(float)) != hipSuccess) {
            hipGetLastError();
            set_error("fg_pcg_solve: device allocation for the block solve failed");
            return FG_ERR_OOM;
        }
    S->mr_cap = nrhs;
    return FG_OK;
}

void drop_mr_graphs(fg_system *S)
{
    for (GraphCache &g : S->mr_graph) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.iters = 0;
    }
}

// Start of a block CG on the interleaved right-hand sides already in S->mr (FP64)
// or S->mfr (FP32): x = 0, p = z, per-column rho, thresholds and flags.
static fg_status mr_cg_init(fg_system *S, int nrhs, bool f32, double tol, int64_t maxit, double overrun2,
                            hipStream_t st)
{
    const int64_t n = 3 * S->Npad * nrhs;
    MrScalars init{};
    init.maxit = maxit;
    init.overrun2 = overrun2;
    init.nrhs = nrhs;
    hipMemcpyAsync(S->msc, &init, sizeof init, hipMemcpyHostToDevice, st);
    const int64_t ge = grid_cols(n);
    if (f32 && !S->k32_valid) refresh_k32(S, st);
    if (S->k_precond) {
        if (f32) {
            bj_ready32(S, st);
            hipLaunchKernelGGL((k_mr_init_bj<float>), dim3(ge), dim3(WG), 0, st, S->Npad, nrhs, log2i(nrhs),
                               mr_bj32(S), S->mfx, S->mfr, S->mfp, S->mpart, S->mpart_stride);
        } else {
            bj_ready(S, st);
            hipLaunchKernelGGL((k_mr_init_bj<double>), dim3(ge), dim3(WG), 0, st, S->Npad, nrhs, log2i(nrhs),
                               mr_bj64(S), S->mx, S->mr, S->mp, S->mpart, S->mpart_stride);
        }
        if (S->bj_singular) {
            set_error("fg_pcg_solve: a diagonal or fault-pair block of K is singular (block Jacobi)");
            return FG_ERR_BREAKDOWN;
        }
    } else if (f32) {
        hipLaunchKernelGGL((k_mr_init<float>), dim3(ge), dim3(WG), 0, st, n, nrhs, log2i(nrhs), S->dinvK32, S->mfx, S->mfr, S->mfp,
                           S->mpart, S->mpart_stride);
    } else {
        hipLaunchKernelGGL((k_mr_init<double>), dim3(ge), dim3(WG), 0, st, n, nrhs, log2i(nrhs), S->dinvK, S->mx, S->mr, S->mp,
                           S->mpart, S->mpart_stride);
    }
    hipLaunchKernelGGL(k_mr_init_fin, dim3(nrhs), dim3(FIN), 0, st, S->mpart, nrhs, S->mpart_stride, ge, S->msc, tol);
    return check_hip("block cg init");
}

// Iterations until every column is done (batches of check_every, replayed as
// HIP graphs); solutions in S->mx / S->mfx, per-column results in S->msc_host.
static fg_status mr_cg_loop(fg_system *S, int nrhs, bool f32, int check_every, hipStream_t st)
{
    fg_status e = FG_OK;
    const int batch = check_every > 0 ? check_every : 32;
    GraphCache &g = S->mr_graph[f32 ? 1 : 0];
    for (;;) {
        hipMemcpyAsync(S->msc_host, S->msc, sizeof(MrScalars), hipMemcpyDeviceToHost, st);
        hipStreamSynchronize(st);
        e = check_hip("block cg poll");
        if (e) return e;
        bool all = true;
        for (int c = 0; c < nrhs; ++c) all = all && (S->msc_host->done[c] || S->msc_host->ready[c]);
        if (all) break;
        if (!S->use_graphs) {
            if (f32)
                mr_launch_batch<float, float>(S, nrhs, S->K32, S->dinvK32, S->mfx, S->mfr, S->mfp, S->mfq, batch, st);
            else
                mr_launch_batch<double, double>(S, nrhs, S->K, S->dinvK, S->mx, S->mr, S->mp, S->mq, batch, st);
        } else {
            const int key = S->mr_tile + 256 * S->mr_form + 65536 * (S->k_precond != 0);
            if (!g.exec || g.iters != batch || g.nrhs != nrhs || g.tile != key) {
                if (g.exec) hipGraphExecDestroy(g.exec);
                g.exec = nullptr;
                hipGraph_t graph = nullptr;
                if (hipStreamBeginCapture(S->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                    return check_hip("block cg capture");
                if (f32)
                    mr_launch_batch<float, float>(S, nrhs, S->K32, S->dinvK32, S->mfx, S->mfr, S->mfp, S->mfq, batch,
                                                  S->cap_stream);
                else
                    mr_launch_batch<double, double>(S, nrhs, S->K, S->dinvK, S->mx, S->mr, S->mp, S->mq, batch,
                                                    S->cap_stream);
                if (hipStreamEndCapture(S->cap_stream, &graph) != hipSuccess) return check_hip("block cg capture end");
                hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
                hipGraphDestroy(graph);
                if (ie != hipSuccess) {
                    g.exec = nullptr;
                    return check_hip("block cg instantiate");
                }
                g.iters = batch;
                g.nrhs = nrhs;
                g.tile = key;
            }
            hipGraphLaunch(g.exec, st);
        }
        e = check_hip("block cg batch");
        if (e) return e;
    }
    return FG_OK;
}

static fg_status mr_cg(fg_system *S, int nrhs, bool f32, double tol, int64_t maxit, int check_every, hipStream_t st)
{
    fg_status e = mr_cg_init(S, nrhs, f32, tol, maxit, 1.0, st);
    return e ? e : mr_cg_loop(S, nrhs, f32, check_every, st);
}

static void mr_colnorms(fg_system *S, int nrhs, const double *a, double *host, hipStream_t st)
{
    const int64_t n = 3 * S->Npad * nrhs, ge = grid_cols(n);
    hipLaunchKernelGGL(k_mr_coldot, dim3(ge), dim3(WG), 0, st, n, nrhs, a, a, S->mpart, S->mpart_stride);
    hipLaunchKernelGGL(k_mr_colfin, dim3(nrhs), dim3(FIN), 0, st, S->mpart, nrhs, S->mpart_stride, ge, S->mred);
    hipMemcpyAsync(S->mred_host, S->mred, nrhs * sizeof(double), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    for (int c = 0; c < nrhs; ++c) host[c] = std::sqrt(S->mred_host[c]);
}

// FG_MIXED block solve by reliable updates: one FP32 block CG on K32, each column
// scaled by 1/||b_c||, runs until every column has cut its residual by `delta`
// (or reached 0.5 tol); then every column's FP32 correction is added to the FP64
// x, the FP64 residual b - K x replaces the FP32 one, and the columns above tol
// go on from their last direction with the next threshold max(delta rel, 0.5 tol).
// Extra reduction (squared) a column may make past its replacement threshold
// while it waits for the others: a factor 10 in norm.  The recursive residual must
// stay well above its rounding gap to the true one (about the FP32 unit roundoff
// times the residual at the last replacement, times a growth factor): a column
// let run 1e3 past a 1e-2 threshold has diverged after the replacement.
constexpr double MR_OVERRUN2 = 1e-2;

static fg_status mr_reliable(fg_system *S, int nrhs, double tol, int64_t maxit, int check_every, double delta,
                             int64_t *iters, int64_t *updates, double *worst_rel, fg_status *worst, hipStream_t st)
{
    const int64_t n = 3 * S->Npad * nrhs, ge = grid_cols(n);
    const int lg = log2i(nrhs);
    if (!S->k32_valid) refresh_k32(S, st);
    std::vector<double> bn(nrhs), rn(nrhs), scale(nrhs), fold(nrhs), next2(nrhs);
    mr_colnorms(S, nrhs, S->mb, bn.data(), st);
    for (int c = 0; c < nrhs; ++c) {
        if (!std::isfinite(bn[c])) {
            set_error("fg_pcg_solve: NaN or Inf in a right-hand side");
            return FG_ERR_NAN;
        }
        scale[c] = bn[c] > 0 ? 1.0 / bn[c] : 0.0;
        fold[c] = bn[c];
    }
    double *next2_d = S->mred + MR_MAX;
    hipMemcpyAsync(S->mred, scale.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st);
    hipLaunchKernelGGL(k_mr_scale_to_f32, dim3(ge), dim3(WG), 0, st, n, nrhs, S->mred, S->mb, S->mfr);
    hipMemsetAsync(S->mx64, 0, n * sizeof(double), st);
    fg_status e = mr_cg_init(S, nrhs, true, delta, maxit, MR_OVERRUN2, st);
    if (e) return e;
    *iters = 0;
    *updates = 0;
    *worst = FG_OK;
    for (;;) {
        e = mr_cg_loop(S, nrhs, true, check_every, st);
        if (e) return e;
        const MrScalars &h = *S->msc_host;
        for (int c = 0; c < nrhs; ++c) {
            *iters = std::max<int64_t>(*iters, h.iter[c]);
            if (h.status[c] < 0) {
                char msg[256];
                std::snprintf(msg, sizeof msg,
                              "fg_pcg_solve: %s in column %d at FP32 iteration %lld after %lld residual replacements "
                              "(rho %.3e, p.Ap %.3e, r.r %.3e, beta %.3e)",
                              h.status[c] == FG_ERR_NAN ? "NaN or Inf" : "CG breakdown (p.Ap <= 0)", c,
                              (long long)h.iter[c], (long long)*updates, h.rho[c], h.pq[c], h.rr[c], h.beta[c]);
                set_error(msg);
                return h.status[c];
            }
        }
        std::vector<int64_t> it(h.iter, h.iter + nrhs);
        // columns still iterating: back to the state of a column that stopped
        if (S->k_precond)
            hipLaunchKernelGGL((k_mr_strip_z_bj<float>), dim3(ge), dim3(WG), 0, st, n, nrhs, (const float *)S->mfz,
                               S->mfp, S->msc);
        else
            hipLaunchKernelGGL((k_mr_strip_z<float>), dim3(ge), dim3(WG), 0, st, n, nrhs, lg, S->dinvK32, S->mfr,
                               S->mfp, S->msc);
        // fold the FP32 corrections into x and replace the residuals by FP64 ones
        hipMemcpyAsync(S->mred, fold.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st);
        hipLaunchKernelGGL(k_mr_add_f32, dim3(ge), dim3(WG), 0, st, n, nrhs, S->mred, S->mfx, S->mx64);
        hipMemsetAsync(S->mfx, 0, n * sizeof(float), st);
        mr_launch_spmm<double, double>(S, nrhs, S->K, S->mx64, S->mq, 0, st);
        hipLaunchKernelGGL(k_mr_resid, dim3(ge), dim3(WG), 0, st, n, S->mb, S->mq, S->mr64);
        mr_colnorms(S, nrhs, S->mr64, rn.data(), st);
        ++*updates;
        bool any = false;
        *worst_rel = 0;
        for (int c = 0; c < nrhs; ++c) {
            const double rel = bn[c] > 0 ? rn[c] / bn[c] : 0.0;
            if (!std::isfinite(rel)) {
                set_error("fg_pcg_solve: NaN in a block residual replacement");
                return FG_ERR_NAN;
            }
            *worst_rel = std::max(*worst_rel, rel);
            next2[c] = -1.0;
            if (rel <= tol) continue;
            if (it[c] >= maxit) {
                *worst = FG_NOT_CONVERGED;
                continue;
            }
            const double nx = std::max(delta * rel, 0.5 * tol);
            next2[c] = nx * nx;
            any = true;
        }
        if (!any) return FG_OK;
        hipMemcpyAsync(S->mred, scale.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st);
        hipLaunchKernelGGL(k_mr_scale_to_f32, dim3(ge), dim3(WG), 0, st, n, nrhs, S->mred, S->mr64, S->mfr);
        hipMemcpyAsync(next2_d, next2.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st);
        if (S->k_precond) {
            hipLaunchKernelGGL((k_mr_init_bj<float>), dim3(ge), dim3(WG), 0, st, S->Npad, nrhs, lg, mr_bj32(S),
                               (float *)nullptr, S->mfr, (float *)nullptr, S->mpart, S->mpart_stride);
            hipLaunchKernelGGL(k_mr_resume_fin, dim3(nrhs), dim3(FIN), 0, st, S->mpart, nrhs, S->mpart_stride, ge,
                               S->msc, next2_d);
            hipLaunchKernelGGL((k_mr_resume_p_bj<float>), dim3(ge), dim3(WG), 0, st, n, nrhs, (const float *)S->mfz,
                               S->mfp, S->msc);
        } else {
            hipLaunchKernelGGL((k_mr_resume<float>), dim3(ge), dim3(WG), 0, st, n, nrhs, lg, S->dinvK32, S->mfr,
                               S->mpart, S->mpart_stride);
            hipLaunchKernelGGL(k_mr_resume_fin, dim3(nrhs), dim3(FIN), 0, st, S->mpart, nrhs, S->mpart_stride, ge,
                               S->msc, next2_d);
            hipLaunchKernelGGL((k_mr_resume_p<float>), dim3(ge), dim3(WG), 0, st, n, nrhs, lg, S->dinvK32, S->mfr,
                               S->mfp, S->msc);
        }
        e = check_hip("block cg resume");
        if (e) return e;
    }
}

// Multi-right-hand-side K solve: b, x in the caller layout (column c at c*3N).
fg_status block_solve(fg_system *S, int nrhs, const double *b, double *x, int precision, double tol, int64_t maxit,
                      int check_every, fg_pcg_info *info, hipStream_t st)
{
    if (nrhs > MR_MAX || (nrhs & (nrhs - 1))) {
        set_error("fg_pcg_solve: the block solve takes a power-of-two number of right-hand sides up to 64");
        return FG_ERR_ARG;
    }
    fg_status e = mr_reserve(S, nrhs);
    if (e) return e;
    const int64_t n = 3 * S->Npad * nrhs, ge = grid_cols(n);
    hipLaunchKernelGGL(k_mr_in, dim3(ge), dim3(WG), 0, st, S->N, S->Npad, nrhs, S->perm, b, S->mb);
    fg_status worst = FG_OK;
    int64_t max_iters = 0, cycles = 0;
    double worst_rel = 0;
    if (precision == FG_F64 || precision == FG_F32) {
        const bool f32 = precision == FG_F32;
        if (f32) {
            std::vector<double> ones(nrhs, 1.0);
            hipMemcpyAsync(S->mred, ones.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st);
            hipLaunchKernelGGL(k_mr_scale_to_f32, dim3(ge), dim3(WG), 0, st, n, nrhs, S->mred, S->mb, S->mfr);
        } else {
            hipMemcpyAsync(S->mr, S->mb, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        }
        e = mr_cg(S, nrhs, f32, tol, maxit, check_every, st);
        if (e) return e;
        if (f32) {
            hipMemsetAsync(S->mx64, 0, n * sizeof(double), st);
            std::vector<double> ones(nrhs, 1.0);
            hipMemcpyAsync(S->mred, ones.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st);
            hipLaunchKernelGGL(k_mr_add_f32, dim3(ge), dim3(WG), 0, st, n, nrhs, S->mred, S->mfx, S->mx64);
            hipLaunchKernelGGL(k_mr_out, dim3(ge), dim3(WG), 0, st, S->N, S->Npad, nrhs, S->perm, S->mx64, x);
        } else {
            hipLaunchKernelGGL(k_mr_out, dim3(ge), dim3(WG), 0, st, S->N, S->Npad, nrhs, S->perm, S->mx, x);
        }
        const MrScalars &h = *S->msc_host;
        for (int c = 0; c < nrhs; ++c) {
            max_iters = std::max<int64_t>(max_iters, h.iter[c]);
            worst_rel = std::max(worst_rel, h.bb[c] > 0 ? std::sqrt(h.rr[c] / h.bb[c]) : 0.0);
            if (h.status[c] < 0) worst = h.status[c] < worst ? h.status[c] : worst;
            else if (worst >= 0 && h.status[c] > worst) worst = h.status[c];
        }
        cycles = 1;
    } else {
        // FP32 block CG with FP64 residual replacement per column
        e = mr_reliable(S, nrhs, tol, maxit, check_every, 1.0 / S->mixed_update, &max_iters, &cycles, &worst_rel, &worst,
                        st);
        if (e) return e;
        hipLaunchKernelGGL(k_mr_out, dim3(ge), dim3(WG), 0, st, S->N, S->Npad, nrhs, S->perm, S->mx64, x);
    }
    hipStreamSynchronize(st);
    if (info) {
        info->iters = max_iters;
        info->cycles = cycles;
        info->relres = worst_rel;
        info->status = worst;
    }
    if (worst == FG_ERR_BREAKDOWN) set_error("fg_pcg_solve: CG breakdown in a column (p.Ap <= 0)");
    if (worst == FG_ERR_NAN) set_error("fg_pcg_solve: NaN or Inf in a column");
    e = check_hip("fg_pcg_solve (block)");
    return e ? e : worst;
}

}  // namespace fg
