// Device helpers shared by the libfg kernel sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fg_internal.h"

namespace fg {

namespace {

__device__ __forceinline__ double wave_sum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
}

// Grid-wide sums without device-scope fences: every block stores its partial
// sums with plain stores and a one-block finalize kernel adds them in a fixed
// order after the kernel boundary (which makes the stores visible across XCDs).
// Per-block fences would write back L2 once per block on this multi-XCD part.
template <int NV>
__device__ __forceinline__ void block_partials(const double (&v)[NV], double *partials, int64_t stride)
{
    __shared__ double sh[NV][WG / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) sh[k][w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) {
            double s = 0;
            for (int i = 0; i < nw; ++i) s += sh[k][i];
            partials[k * stride + blockIdx.x] = s;
        }
}

// Sum of nparts partials per value, in a fixed order; result valid in every thread.
constexpr int FIN = 1024;  // threads of the one-block finalize kernels

template <int NV>
__device__ __forceinline__ void finalize_sum(const double *partials, int64_t stride, int64_t nparts, double (&tot)[NV])
{
    __shared__ double sh[NV][FIN / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = 0; k < NV; ++k) {
        double s = 0;
        for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) s += partials[k * stride + i];
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

// Workgroups are dispatched round-robin over the 8 XCDs; hand each XCD a
// contiguous range of work so that its L2 sees neighbouring slices.  The grid
// is a multiple of 8.
__device__ __forceinline__ int64_t xcd_block()
{
    const int64_t per = gridDim.x / 8;
    return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

inline int64_t grid_xcd(int64_t nblocks) { return ((nblocks + 7) / 8) * 8; }

inline int64_t grid_elems(int64_t n)
{
    int64_t g = (n + WG - 1) / WG;
    return g < 2048 ? (g < 1 ? 1 : g) : 2048;
}

// Grid of the CG vector kernels that also add the previous kernel's partial sums
// in every block: fewer, longer-running blocks keep that redundant sum small.
inline int64_t grid_vec(int64_t n)
{
    int64_t g = (n + WG - 1) / WG;
    return g < 512 ? (g < 1 ? 1 : g) : 512;
}

// Load of data streamed once per product (nontemporal hint when NT).
template <bool NT, typename TV>
__device__ __forceinline__ TV ld_val(const TV *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Block-Jacobi preconditioner of K (nodal 3x3 inverse blocks, 6x6 over the two
// lips' nodes of a fault pair) on column-interleaved vectors: element (DOF d,
// column c) at d*nrhs + c (nrhs = 1: one vector).  A unit is a node off the
// interface pairs or a fault pair, owned by its lower row.
template <typename T>
struct BjCols {
    const T *A;            // [Npad*6] symmetric inverse blocks, xx yy zz yz xz xy
    const T *B;            // [nfr*9] pair coupling blocks of the inverse, row-major
    const int32_t *fslot;  // [Npad] index into the fault rows, -1 off the interface
    const int32_t *fpart;  // [nfr] partner row, -1 if none
    T *z;                  // [3*Npad*nrhs], column-interleaved like r
};

template <typename T>
__device__ __forceinline__ T bjc_sym(const T *d, int r, int c)
{
    if (r == c) return d[r];
    const int s = r + c;  // 1: xy, 2: xz, 3: yz
    return s == 3 ? d[3] : (s == 2 ? d[4] : d[5]);
}

// z = M^-1 r of unit (u, w) in column c (r of the unit in rr); returns r.z of the unit.
template <typename T>
__device__ __forceinline__ double bjc_unit_z(const BjCols<T> &bj, int64_t u, int64_t w, int ku, int kw,
                                            const T (&rr)[6], int nr, int nrhs, int c)
{
    double rz = 0;
    for (int m = 0; m < nr; ++m) {
        const int64_t row = m == 0 ? u : w;
        const int kk = m == 0 ? ku : kw;
        const T *a = bj.A + 6 * row;
        const T *ro = rr + 3 * m, *rp = rr + 3 * (1 - m);
        for (int k = 0; k < 3; ++k) {
            T z = bjc_sym(a, k, 0) * ro[0] + bjc_sym(a, k, 1) * ro[1] + bjc_sym(a, k, 2) * ro[2];
            if (nr == 2) {
                const T *b = bj.B + 9 * kk + 3 * k;
                z += b[0] * rp[0] + b[1] * rp[1] + b[2] * rp[2];
            }
            bj.z[(3 * row + k) * nrhs + c] = z;
            rz += (double)ro[k] * (double)z;
        }
    }
    return rz;
}

struct SpmvArgs {
    int64_t nslices;
    const int64_t *slice_ptr;
    const int32_t *col;
    const uint16_t *lcol;
    const int32_t *diag_slot;
    const int64_t *halo_ptr;
    const int32_t *halo;
    int cap;
};

// Each wavefront owns one slice.  It first copies x of the slice's halo (the
// sorted distinct columns of its 64 rows) into its own LDS window, then walks
// the slots: the 9 (or 1) values of a slot are 64-wide coalesced loads and the
// x operands come from LDS through 16-bit local column indices.  A slice whose
// halo exceeds the LDS window (irregular meshes) gathers x from global memory.
template <int BS, typename T, bool NT = true>
__device__ __forceinline__ bool stage_halo(int64_t s, int lane, const int64_t *__restrict__ halo_ptr,
                                           const int32_t *__restrict__ halo, int cap, const T *__restrict__ x, T *xs)
{
    const int64_t h0 = halo_ptr[s];
    const int hn = (int)(halo_ptr[s + 1] - h0);
    if (hn > cap) return false;
    for (int i = lane; i < hn; i += SLICE) {
        const int64_t node = ld_val<NT>(halo + h0 + i);
#pragma unroll
        for (int k = 0; k < BS; ++k) xs[BS * i + k] = x[BS * node + k];
    }
    return true;
}

// y = A x for one row (lane) of a slice; IDX is uint16_t (halo-local, xs in LDS)
// or int32_t (global, xs = x).  dj: slot of the row's diagonal, whose x is
// returned in d0..d2 (for p.Ap).  UNR slots are unrolled per step.
template <int BS, typename T, typename TV, typename IDX, int UNR = 2, int NT = 3>
__device__ __forceinline__ void slice_row(int64_t base, int w, int lane, int dj, const IDX *__restrict__ idx,
                                          const TV *__restrict__ val, const T *xs, T (&y)[BS], T (&d)[BS])
{
    const IDX *c = idx + base + lane;
    const TV *v = val + BS * BS * base + lane;
#pragma unroll
    for (int r = 0; r < BS; ++r) y[r] = 0, d[r] = 0;
#pragma unroll UNR
    for (int j = 0; j < w; ++j) {
        const int64_t cj = ld_val<(NT & 2) != 0>(c + (int64_t)j * SLICE);
        T xv[BS];
#pragma unroll
        for (int k = 0; k < BS; ++k) xv[k] = xs[BS * cj + k];
        const TV *vb = v + (int64_t)BS * BS * j * SLICE;
#pragma unroll
        for (int r = 0; r < BS; ++r)
#pragma unroll
            for (int k = 0; k < BS; ++k) y[r] += (T)ld_val<(NT & 1) != 0>(vb + (BS * r + k) * SLICE) * xv[k];
        if (j == dj)
#pragma unroll
            for (int k = 0; k < BS; ++k) d[k] = xv[k];
    }
}

// The LDS-staged row product with its memory accesses software-pipelined: the
// column indices and values of the next group of UNR slots are loaded into a
// second register buffer before the current group is used, so every wave keeps
// a group of loads in flight while it computes instead of draining its loads
// group by group.  The steady-state loop runs over whole groups only and its
// loads are unconditional (a load under a branch makes the compiler wait for all
// outstanding loads at the join); the slice width is made wave-uniform for the
// same reason.  Same arithmetic, in the same order, as slice_row.
template <int BS, typename T, typename TV, int UNR, int NT>
__device__ __forceinline__ void slice_row_pipe(int64_t base, int w_lane, int lane, int dj,
                                               const uint16_t *__restrict__ idx, const TV *__restrict__ val,
                                               const T *xs, T (&y)[BS], T (&d)[BS])
{
    const int w = __builtin_amdgcn_readfirstlane(w_lane);
    const uint16_t *c = idx + base + lane;
    const TV *v = val + BS * BS * base + lane;
#pragma unroll
    for (int r = 0; r < BS; ++r) y[r] = 0, d[r] = 0;
    auto slot = [&](int j, int cj, const TV *vv) {
        T xv[BS];
#pragma unroll
        for (int k = 0; k < BS; ++k) xv[k] = xs[BS * cj + k];
#pragma unroll
        for (int r = 0; r < BS; ++r)
#pragma unroll
            for (int k = 0; k < BS; ++k) y[r] += (T)vv[BS * r + k] * xv[k];
        if (j == dj)
#pragma unroll
            for (int k = 0; k < BS; ++k) d[k] = xv[k];
    };
    auto load = [&](int j0, uint16_t(&cc)[UNR], TV(&vv)[UNR][BS * BS]) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            cc[u] = ld_val<(NT & 2) != 0>(c + (int64_t)(j0 + u) * SLICE);
#pragma unroll
            for (int e = 0; e < BS * BS; ++e)
                vv[u][e] = ld_val<(NT & 1) != 0>(v + (int64_t)(BS * BS * (j0 + u) + e) * SLICE);
        }
    };
    auto use = [&](int j0, const uint16_t(&cc)[UNR], const TV(&vv)[UNR][BS * BS]) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) slot(j0 + u, cc[u], vv[u]);
    };
    const int ng = w / UNR;  // whole groups
    uint16_t ca[UNR], cb[UNR];
    TV va[UNR][BS * BS], vb[UNR][BS * BS];
    int g = 0;
    if (ng > 0) {
        load(0, ca, va);
        for (; g + 2 < ng; g += 2) {
            load((g + 1) * UNR, cb, vb);
            use(g * UNR, ca, va);
            load((g + 2) * UNR, ca, va);
            use((g + 1) * UNR, cb, vb);
        }
        if (g + 1 < ng) {
            load((g + 1) * UNR, cb, vb);
            use(g * UNR, ca, va);
            use((g + 1) * UNR, cb, vb);
        } else {
            use(g * UNR, ca, va);
        }
    }
    for (int j = ng * UNR; j < w; ++j) {  // the last w mod UNR slots
        TV vv[BS * BS];
        const int cj = ld_val<(NT & 2) != 0>(c + (int64_t)j * SLICE);
#pragma unroll
        for (int e = 0; e < BS * BS; ++e) vv[e] = ld_val<(NT & 1) != 0>(v + (int64_t)(BS * BS * j + e) * SLICE);
        slot(j, cj, vv);
    }
}

// q = A p for the rows of one slice; returns p.q of the lane's row.
// NT bit mask: nontemporal accesses (1 matrix values, 2 column indices, 8 the
// stores of y) and 16 the software-pipelined staged row product.
template <int BS, typename T, typename TV, int UNR = 2, int NT = 3>
__device__ __forceinline__ double slice_spmv(int64_t s, int lane, bool staged, const int64_t *__restrict__ slice_ptr,
                                             const int32_t *__restrict__ col, const uint16_t *__restrict__ lcol,
                                             const int32_t *__restrict__ diag_slot, const TV *__restrict__ val,
                                             const T *__restrict__ x, const T *xs, T *__restrict__ y)
{
    const int64_t base = slice_ptr[s];
    const int w = (int)((slice_ptr[s + 1] - base) / SLICE);
    const int64_t r = s * SLICE + lane;
    const int dj = diag_slot[r];
    T yv[BS], d[BS];
    if (staged) {
        if constexpr ((NT & 16) != 0)
            slice_row_pipe<BS, T, TV, UNR, NT>(base, w, lane, dj, lcol, val, xs, yv, d);
        else
            slice_row<BS, T, TV, uint16_t, UNR, NT>(base, w, lane, dj, lcol, val, xs, yv, d);
    } else
        slice_row<BS, T, TV, int32_t, UNR, NT>(base, w, lane, dj, col, val, x, yv, d);
    double pq = 0;
#pragma unroll
    for (int k = 0; k < BS; ++k) {
        if constexpr ((NT & 8) != 0)
            __builtin_nontemporal_store(yv[k], y + BS * r + k);
        else
            y[BS * r + k] = yv[k];
        pq += (double)d[k] * (double)yv[k];
    }
    return pq;
}


}  // namespace

#define LAUNCH(kern, grid, block, st, ...) hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, __VA_ARGS__)
#define LAUNCH_SH(kern, grid, block, sh, st, ...) \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), sh, st, __VA_ARGS__)

inline SpmvArgs spmv_args(const fg_system *S)
{
    return SpmvArgs{S->nslices, S->slice_ptr, S->col, S->lcol, S->diag_slot, S->halo_ptr, S->halo, S->halo_cap};
}

template <int BS, typename T>
inline size_t spmv_lds(const fg_system *S)
{
    return (size_t)(WG / SLICE) * S->halo_cap * BS * sizeof(T);
}


}  // namespace fg
