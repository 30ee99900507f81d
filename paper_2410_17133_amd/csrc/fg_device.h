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
