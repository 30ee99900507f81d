// Smoothed-aggregation AMG preconditioner of K (fg_tune "k_precond" 3): the third
// stage of the stronger preconditioner, after block Jacobi and Chebyshev.
//
// Smoothed aggregation (Vanek, Mandel and Brezina, Computing 56, 1996) with the six
// rigid-body modes as near-null space:
//  - aggregates: three passes over the node graph of each level in increasing node
//    order (level 0 in the caller's numbering; the two lips of a fault pair count as
//    one node): (1) a node whose neighbours are all free starts an aggregate with
//    them; (2) a free node joins the aggregate of its lowest-numbered neighbour
//    aggregated in pass 1; (3) a node still free starts one with its free neighbours;
//  - tentative prolongator: per aggregate the near-null-space rows of its nodes
//    (level 0: translations and rotations about the aggregate's centroid, zero on
//    held DOFs; below: the R factor of the node's aggregate), orthonormalised by
//    modified Gram-Schmidt, a vanishing column dropped;
//  - P = (I - w D^-1 A) Ptent with D the block diagonal, w = 4 / (3 rho), rho the
//    Gershgorin bound of D^-1 A; Galerkin A_c = P^T A P; a coarse DOF with an empty
//    row gets a unit diagonal; at most 6 levels, the last solved by its dense inverse;
//  - V-cycle: pre- and post-smoothing by the degree-2 Chebyshev polynomial over
//    block Jacobi (level 0: the nodal / fault-pair blocks of "k_precond" 1 on
//    [hi/30, hi], hi the Chebyshev preconditioner's upper end; below: 6x6 diagonal
//    blocks on [rho/30, rho]).
// The patterns (aggregates, P, W = A P, A_c) are symbolic and built on the host once
// per mesh; every numeric step (diagonal blocks, Gershgorin bounds, P, W, A_c, the
// cycle) runs on the GPU when K changes.  Only the coarsest matrix (a few hundred
// unknowns) is inverted on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <thread>
#include <vector>

#include "fg_device.h"
#include "fg_kernels.h"

namespace fg {

constexpr int AMG_MAXLEV = 6;

struct AmgLevel {
    int bs = 3;
    int64_t nn = 0, nc = 0;            // nodes (level 0: Npad internal rows), aggregates
    int64_t nnzb = 0, npz = 0, nwz = 0, nrz = 0;
    int64_t *arow = nullptr;           // block CSR of A (level 0: K's slots, internal order)
    int32_t *acol = nullptr;
    int32_t *arid = nullptr;           // coarse levels: row of each block
    double *aval = nullptr;            // [nnzb bs bs]
    int32_t *agg = nullptr;            // [nn] aggregate of each node (-1: padding row)
    double *q = nullptr;               // [nn bs 6] tentative prolongator rows
    int64_t *prow = nullptr;           // P: per node, sorted aggregates
    int32_t *pcol = nullptr;
    double *pval = nullptr;            // [npz bs 6]
    int64_t *wrow = nullptr;           // W = A P
    int32_t *wcol = nullptr;
    double *wval = nullptr;            // [nwz bs 6]
    int64_t *rrow = nullptr;           // P^T: per aggregate, (node, P entry) in increasing node order
    int32_t *rnode = nullptr;
    int64_t *rent = nullptr;
    double *rval = nullptr;            // [nrz bs 6] the P entries in P^T order (restriction)
    double *dinv = nullptr;            // [nn bs bs]
    double rho = 0;
    // cycle vectors of the level: x, b (coarse levels), r (A x, then the residual), and
    // the smoother's d and t = A d
    double *x = nullptr, *b = nullptr, *r = nullptr, *t = nullptr, *d = nullptr;
    // FP32 copies for the mixed-precision cycle (allocated on its first use): A and
    // dinv (coarse levels), P (every level but the coarsest), the cycle vectors
    float *aval32 = nullptr, *dinv32 = nullptr, *pval32 = nullptr, *rval32 = nullptr;
    float *x32 = nullptr, *b32 = nullptr, *r32 = nullptr, *t32 = nullptr, *d32 = nullptr;
};

struct AmgData {
    int nlev = 0;
    AmgLevel L[AMG_MAXLEV];
    int64_t nco = 0;                   // coarsest unknowns
    double *cinv = nullptr;            // [nco nco] inverse of the coarsest matrix
    double *part = nullptr;            // reduction partials
    // the PCG's r, z, p, q (3 Npad each): its own, since callers of the K solve pass
    // the system's shared work vectors as right-hand side and solution
    double *cr = nullptr, *cz = nullptr, *cp = nullptr, *cq = nullptr;
    int64_t epoch = -1;                // bj_epoch of the numeric set-up
    // mixed precision: FP32 coarsest inverse, the cycle's FP32 right-hand side and
    // result, the previous preconditioned residual of the flexible CG
    float *cinv32 = nullptr, *cr32 = nullptr, *cz32 = nullptr;
    double *cz0 = nullptr;
    double *sc32 = nullptr;            // [2] the device-side scale of amg_apply32 and its inverse
    int64_t epoch32 = -1;              // bj_epoch of the FP32 copies
    int64_t coarse_nodes = 64;
};

namespace {

// ------------------------------------------------------------ host symbolic set-up
typedef std::vector<std::vector<int32_t>> Lists;

// f(begin, end) over [0, n) split in contiguous ranges across up to 16 host threads
// (one range below 4096 items); f writes only what its own items own.
template <typename F>
void par_for(int64_t n, F &&f)
{
    const unsigned hw = std::max(1u, std::min(std::thread::hardware_concurrency(), 16u));
    const int64_t nt = std::min<int64_t>((int64_t)hw, (n + 4095) / 4096);
    if (nt <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    th.reserve((size_t)nt);
    int64_t t = 0;
    try {
        for (; t < nt; ++t) th.emplace_back([&f, n, nt, t] { f(n * t / nt, n * (t + 1) / nt); });
    } catch (...) {   // no thread to be had: the remaining ranges on this one
        for (; t < nt; ++t) f(n * t / nt, n * (t + 1) / nt);
    }
    for (std::thread &x : th) x.join();
}

// The three aggregation passes (see the file comment); twin[i] the other lip of a
// fault pair or -1 (level 0 only).  Returns the number of aggregates.
int64_t aggregate(int64_t nn, const Lists &adj, const std::vector<int32_t> *twin, std::vector<int32_t> &agg)
{
    agg.assign(nn, -1);
    auto members = [&](int64_t i, int32_t (&mem)[2]) {
        mem[0] = (int32_t)i;
        mem[1] = -1;
        int nm = 1;
        if (twin && (*twin)[i] >= 0) mem[nm++] = (*twin)[i];
        return nm;
    };
    auto led_by_other = [&](int64_t i) { return twin && (*twin)[i] >= 0 && (*twin)[i] < i; };
    int64_t na = 0;
    for (int64_t i = 0; i < nn; ++i) {
        if (led_by_other(i) || agg[i] >= 0) continue;
        int32_t mem[2];
        const int nm = members(i, mem);
        bool free_all = true;
        for (int u = 0; u < nm && free_all; ++u)
            for (int32_t j : adj[mem[u]])
                if (agg[j] >= 0) {
                    free_all = false;
                    break;
                }
        if (!free_all) continue;
        for (int u = 0; u < nm; ++u) {
            agg[mem[u]] = (int32_t)na;
            for (int32_t j : adj[mem[u]]) {
                agg[j] = (int32_t)na;
                if (twin && (*twin)[j] >= 0) agg[(*twin)[j]] = (int32_t)na;
            }
        }
        ++na;
    }
    const std::vector<int32_t> agg1 = agg;
    for (int64_t i = 0; i < nn; ++i) {
        if (led_by_other(i) || agg[i] >= 0) continue;
        int32_t mem[2];
        const int nm = members(i, mem);
        int32_t best = -1, bestj = INT32_MAX;
        for (int u = 0; u < nm; ++u)
            for (int32_t j : adj[mem[u]])
                if (agg1[j] >= 0 && j < bestj) {
                    bestj = j;
                    best = agg1[j];
                }
        if (best >= 0)
            for (int u = 0; u < nm; ++u) agg[mem[u]] = best;
    }
    for (int64_t i = 0; i < nn; ++i) {
        if (led_by_other(i) || agg[i] >= 0) continue;
        int32_t mem[2];
        const int nm = members(i, mem);
        for (int u = 0; u < nm; ++u) {
            agg[mem[u]] = (int32_t)na;
            for (int32_t j : adj[mem[u]])
                if (agg[j] < 0) {
                    agg[j] = (int32_t)na;
                    if (twin && (*twin)[j] >= 0) agg[(*twin)[j]] = (int32_t)na;
                }
        }
        ++na;
    }
    return na;
}

// Tentative prolongator rows Q [nn bs 6] and the coarse near-null space Bc
// [na 6 6] from the near-null-space rows B [nn bs 6] (modified Gram-Schmidt per
// aggregate over its nodes in increasing order).
void tentative(int bs, int64_t nn, int64_t na, const std::vector<int32_t> &agg, const std::vector<double> &B,
               std::vector<double> &Q, std::vector<double> &Bc)
{
    std::vector<std::vector<int32_t>> mem(na);
    for (int64_t i = 0; i < nn; ++i) mem[agg[i]].push_back((int32_t)i);
    Q.assign(nn * bs * 6, 0.0);
    Bc.assign(na * 36, 0.0);
    par_for(na, [&](int64_t a0, int64_t a1) {
    for (int64_t a = a0; a < a1; ++a) {
        const int64_t rows = (int64_t)mem[a].size() * bs;
        std::vector<double> M(rows * 6);
        for (size_t t = 0; t < mem[a].size(); ++t)
            for (int r = 0; r < bs; ++r)
                for (int k = 0; k < 6; ++k) M[(t * bs + r) * 6 + k] = B[((int64_t)mem[a][t] * bs + r) * 6 + k];
        double R[36] = {0};
        for (int k = 0; k < 6; ++k) {
            double n0 = 0;
            for (int64_t q = 0; q < rows; ++q) n0 += M[q * 6 + k] * M[q * 6 + k];
            n0 = std::sqrt(n0);
            for (int j = 0; j < k; ++j) {
                double d = 0;
                for (int64_t q = 0; q < rows; ++q) d += M[q * 6 + j] * M[q * 6 + k];
                R[6 * j + k] = d;
                for (int64_t q = 0; q < rows; ++q) M[q * 6 + k] -= d * M[q * 6 + j];
            }
            double nk = 0;
            for (int64_t q = 0; q < rows; ++q) nk += M[q * 6 + k] * M[q * 6 + k];
            nk = std::sqrt(nk);
            if (!(nk > 1e-10 * n0) || nk == 0.0) {
                for (int64_t q = 0; q < rows; ++q) M[q * 6 + k] = 0;
                for (int j = 0; j < k; ++j) R[6 * j + k] = 0;
                R[6 * k + k] = 0;
            } else {
                for (int64_t q = 0; q < rows; ++q) M[q * 6 + k] /= nk;
                R[6 * k + k] = nk;
            }
        }
        for (size_t t = 0; t < mem[a].size(); ++t)
            for (int r = 0; r < bs; ++r)
                for (int k = 0; k < 6; ++k) Q[((int64_t)mem[a][t] * bs + r) * 6 + k] = M[(t * bs + r) * 6 + k];
        std::memcpy(&Bc[a * 36], R, sizeof R);
    }
    });
}

void sorted_union(std::vector<int32_t> &v)
{
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
}

template <typename T>
fg_status up(T **p, const std::vector<T> &v)
{
    const size_t n = std::max<size_t>(v.size(), 1);
    if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess) {
        hipGetLastError();
        return FG_ERR_OOM;
    }
    if (!v.empty()) hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return FG_OK;
}

template <typename T>
fg_status dmal(T **p, int64_t n)
{
    if (hipMalloc((void **)p, std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess) {
        hipGetLastError();
        return FG_ERR_OOM;
    }
    return FG_OK;
}

// CSR of per-row sorted lists; row r is list perm[r] (empty where perm[r] < 0), or
// list r without perm.
void to_csr(const Lists &l, std::vector<int64_t> &row, std::vector<int32_t> &col, int64_t nrows = -1,
            const int32_t *perm = nullptr)
{
    if (nrows < 0) nrows = (int64_t)l.size();
    auto src = [&](int64_t r) { return perm ? perm[r] : (int32_t)r; };
    row.assign(nrows + 1, 0);
    for (int64_t r = 0; r < nrows; ++r) row[r + 1] = row[r] + (src(r) >= 0 ? (int64_t)l[src(r)].size() : 0);
    col.resize((size_t)row.back());
    par_for(nrows, [&](int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r)
            if (src(r) >= 0) std::copy(l[src(r)].begin(), l[src(r)].end(), col.begin() + row[r]);
    });
}

// ------------------------------------------------------------ numeric kernels
// A entry (row, k) of level 0 = K's slots (block CSR copy).
__global__ void k_amg_copy_k(int64_t Npad, const int64_t *__restrict__ slice_ptr, const uint8_t *__restrict__ rowlen,
                             const int32_t *__restrict__ col, const double *__restrict__ K,
                             const int64_t *__restrict__ arow, int32_t *acol, double *aval)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= Npad) return;
    const int64_t base = slice_ptr[r / SLICE], l = r % SLICE;
    const int len = rowlen[r];
    for (int j = 0; j < len; ++j) {
        const int64_t o = arow[r] + j;
        acol[o] = col[base + (int64_t)j * SLICE + l];
        for (int e = 0; e < 9; ++e) aval[9 * o + e] = K[9 * base + (int64_t)(9 * j + e) * SLICE + l];
    }
}

// In-place Gauss-Jordan inverse with partial pivoting of an n x n block (n <= 6).
__device__ bool amg_inverse(int n, double *a, double *inv)
{
    for (int i = 0; i < n * n; ++i) inv[i] = (i / n == i % n) ? 1.0 : 0.0;
    for (int c = 0; c < n; ++c) {
        int pr = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[n * r + c]) > fabs(a[n * pr + c])) pr = r;
        if (!(fabs(a[n * pr + c]) > 0.0)) return false;
        if (pr != c)
            for (int k = 0; k < n; ++k) {
                double t = a[n * c + k];
                a[n * c + k] = a[n * pr + k];
                a[n * pr + k] = t;
                t = inv[n * c + k];
                inv[n * c + k] = inv[n * pr + k];
                inv[n * pr + k] = t;
            }
        const double p = 1.0 / a[n * c + c];
        for (int k = 0; k < n; ++k) {
            a[n * c + k] *= p;
            inv[n * c + k] *= p;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = a[n * r + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                a[n * r + k] -= f * a[n * c + k];
                inv[n * r + k] -= f * inv[n * c + k];
            }
        }
    }
    return true;
}

// Inverse diagonal blocks and the per-node maximum scalar-row sum of |D^-1 A|
// (one partial per block; the host takes the maximum).
template <int BS>
__global__ void k_amg_diag(int64_t nn, const int64_t *__restrict__ arow, const int32_t *__restrict__ acol,
                           const double *__restrict__ aval, double *dinv, double *part, int *bad)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double mx = 0;
    if (i < nn && arow[i + 1] > arow[i]) {
        double a[BS * BS], inv[BS * BS];
        int64_t dslot = -1;
        for (int64_t o = arow[i]; o < arow[i + 1]; ++o)
            if (acol[o] == i) dslot = o;
        if (dslot < 0) {
            *bad = 1;
        } else {
            for (int e = 0; e < BS * BS; ++e) a[e] = aval[BS * BS * dslot + e];
            if (!amg_inverse(BS, a, inv)) *bad = 1;
            for (int e = 0; e < BS * BS; ++e) dinv[BS * BS * i + e] = inv[e];
            double s[BS];
            for (int r = 0; r < BS; ++r) s[r] = 0;
            for (int64_t o = arow[i]; o < arow[i + 1]; ++o) {
                const double *m = aval + BS * BS * o;
                for (int r = 0; r < BS; ++r)
                    for (int c = 0; c < BS; ++c) {
                        double v = 0;
                        for (int k = 0; k < BS; ++k) v += inv[BS * r + k] * m[BS * k + c];
                        s[r] += fabs(v);
                    }
            }
            for (int r = 0; r < BS; ++r) mx = fmax(mx, s[r]);
        }
    }
    __shared__ double sh[WG];
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Position of aggregate c in the sorted list col[lo, hi), -1 if absent.
__device__ __forceinline__ int64_t amg_find(const int32_t *__restrict__ col, int64_t lo, int64_t hi, int32_t c)
{
    const int64_t end = hi;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && col[lo] == c) ? lo : -1;
}

// P entry (i, a) = [i in a] Q_i - w D_i^-1 sum_{j in row i, agg(j) = a} A_ij Q_j.
template <int BS>
__global__ void k_amg_prolong(int64_t nn, const int64_t *__restrict__ arow, const int32_t *__restrict__ acol,
                              const double *__restrict__ aval, const int32_t *__restrict__ agg,
                              const double *__restrict__ q, const double *__restrict__ dinv,
                              const int64_t *__restrict__ prow, const int32_t *__restrict__ pcol, double w,
                              double *pval)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nn) return;
    for (int64_t e = prow[i]; e < prow[i + 1]; ++e) {
        const int32_t a = pcol[e];
        double acc[BS * 6];
        for (int k = 0; k < BS * 6; ++k) acc[k] = 0;
        for (int64_t o = arow[i]; o < arow[i + 1]; ++o) {
            const int32_t j = acol[o];
            if (agg[j] != a) continue;
            const double *m = aval + BS * BS * o, *qj = q + (int64_t)BS * 6 * j;
            for (int r = 0; r < BS; ++r)
                for (int k = 0; k < BS; ++k) {
                    const double mv = m[BS * r + k];
                    for (int c = 0; c < 6; ++c) acc[6 * r + c] += mv * qj[6 * k + c];
                }
        }
        const double *di = dinv + BS * BS * i;
        const bool own = agg[i] == a;
        for (int r = 0; r < BS; ++r)
            for (int c = 0; c < 6; ++c) {
                double v = 0;
                for (int k = 0; k < BS; ++k) v += di[BS * r + k] * acc[6 * k + c];
                pval[BS * 6 * e + 6 * r + c] = (own ? q[(int64_t)BS * 6 * i + 6 * r + c] : 0.0) - w * v;
            }
    }
}

// W entry (i, J) = sum_{j in row i} A_ij P(j, J).
template <int BS>
__global__ void k_amg_ap(int64_t nn, const int64_t *__restrict__ arow, const int32_t *__restrict__ acol,
                         const double *__restrict__ aval, const int64_t *__restrict__ prow,
                         const int32_t *__restrict__ pcol, const double *__restrict__ pval,
                         const int64_t *__restrict__ wrow, const int32_t *__restrict__ wcol, double *wval)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nn) return;
    for (int64_t e = wrow[i]; e < wrow[i + 1]; ++e) {
        const int32_t J = wcol[e];
        double acc[BS * 6];
        for (int k = 0; k < BS * 6; ++k) acc[k] = 0;
        for (int64_t o = arow[i]; o < arow[i + 1]; ++o) {
            const int32_t j = acol[o];
            const int64_t f = amg_find(pcol, prow[j], prow[j + 1], J);
            if (f < 0) continue;
            const double *m = aval + BS * BS * o, *pj = pval + BS * 6 * f;
            for (int r = 0; r < BS; ++r)
                for (int k = 0; k < BS; ++k) {
                    const double mv = m[BS * r + k];
                    for (int c = 0; c < 6; ++c) acc[6 * r + c] += mv * pj[6 * k + c];
                }
        }
        for (int k = 0; k < BS * 6; ++k) wval[BS * 6 * e + k] = acc[k];
    }
}

// A_c entry (I, J) = sum_{(i, e) in P^T row I} P_e^T W(i, J): one thread per coarse block.
template <int BS>
__global__ void k_amg_rap(int64_t nnzc, const int32_t *__restrict__ crid, const int32_t *__restrict__ ccol,
                          const int64_t *__restrict__ rrow, const int32_t *__restrict__ rnode,
                          const int64_t *__restrict__ rent, const double *__restrict__ pval,
                          const int64_t *__restrict__ wrow, const int32_t *__restrict__ wcol,
                          const double *__restrict__ wval, double *cval)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nnzc) return;
    const int32_t I = crid[e], J = ccol[e];
    double acc[36];
    for (int k = 0; k < 36; ++k) acc[k] = 0;
    for (int64_t t = rrow[I]; t < rrow[I + 1]; ++t) {
        const int32_t i = rnode[t];
        const int64_t f = amg_find(wcol, wrow[i], wrow[i + 1], J);
        if (f < 0) continue;
        const double *p = pval + BS * 6 * rent[t], *wv = wval + BS * 6 * f;
        for (int k = 0; k < BS; ++k)
            for (int r = 0; r < 6; ++r) {
                const double pv = p[6 * k + r];
                for (int c = 0; c < 6; ++c) acc[6 * r + c] += pv * wv[6 * k + c];
            }
    }
    for (int k = 0; k < 36; ++k) cval[36 * e + k] = acc[k];
}

// A coarse DOF whose row of A_c is empty (its prolongator column vanished) gets a
// unit diagonal, so the coarse matrix stays invertible.
__global__ void k_amg_unit_empty(int64_t nc, const int64_t *__restrict__ crow, const int32_t *__restrict__ ccol,
                                 double *cval)
{
    const int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (I >= nc) return;
    double rs[6] = {0, 0, 0, 0, 0, 0};
    int64_t dslot = -1;
    for (int64_t e = crow[I]; e < crow[I + 1]; ++e) {
        if (ccol[e] == I) dslot = e;
        for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) rs[r] += fabs(cval[36 * e + 6 * r + c]);
    }
    if (dslot >= 0)
        for (int r = 0; r < 6; ++r)
            if (rs[r] == 0.0) cval[36 * dslot + 7 * r] = 1.0;
}

// ------------------------------------------------------------ cycle kernels
// T: double for the FP64 cycle, float for the FP32 cycle of the mixed-precision solve.
//
// y = A x with 6x6 blocks (the coarse levels): 8 H lanes per block row, lane group q
// (H lanes) taking the row's blocks q, q + 8, ... (each block's 36 values contiguous,
// so a group reads 8 consecutive blocks at once), lane h of the group rows 6h/H to
// 6(h+1)/H - 1 of each (H = 2 for FP64 keeps a lane's share of a block in registers);
// then a fixed-order xor reduction over the groups.
template <typename T, int H>
__global__ __launch_bounds__(WG) void k_amg_spmv6(int64_t nn, const int64_t *__restrict__ arow,
                                                  const int32_t *__restrict__ acol, const T *__restrict__ aval,
                                                  const T *__restrict__ x, T *__restrict__ y)
{
    constexpr int G = 8 * H, RL = 6 / H;
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;   // uniform per G lanes
    const int j = threadIdx.x & (G - 1);
    const int h = j % H, q = j / H;
    if (i >= nn) return;
    T s[RL];
    for (int r = 0; r < RL; ++r) s[r] = 0;
    const int64_t o1 = arow[i + 1];
    for (int64_t o = arow[i] + q; o < o1; o += 8) {
        const T *m = aval + 36 * o + 6 * RL * h;
        const T *xj = x + 6 * (int64_t)acol[o];
        T xv[6];
        for (int k = 0; k < 6; ++k) xv[k] = xj[k];
        for (int r = 0; r < RL; ++r)
            for (int k = 0; k < 6; ++k) s[r] += m[6 * r + k] * xv[k];
    }
    T out = 0;
    for (int r = 0; r < RL; ++r) {
        for (int d = G / 2; d >= H; d >>= 1) s[r] += __shfl_xor(s[r], d, G);
        if (r == q) out = s[r];
    }
    if (q < RL) y[6 * i + RL * h + q] = out;
}

// Degree-2 Chebyshev smoothing over the 6x6 diagonal blocks of a coarse level, one
// kernel per step, a thread per scalar row.  step 0: d = D^-1 b / theta, then x = d
// (acc: x += d).  step 1, on kd = A d: x += c2 D^-1 (b - kd) + c1 d.
template <typename T>
__global__ void k_amg_dsmooth(int64_t nn, int step, int acc, const T *__restrict__ dinv, T inv_theta, T c1, T c2,
                              const T *__restrict__ b, const T *__restrict__ kd, T *__restrict__ d, T *__restrict__ x)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= nn * 6) return;
    const int64_t i = g / 6;
    const int r = (int)(g - i * 6);
    T w = 0;
    for (int k = 0; k < 6; ++k) {
        const T sk = step ? b[6 * i + k] - kd[6 * i + k] : b[6 * i + k];
        w += dinv[36 * i + 6 * r + k] * sk;
    }
    if (step == 0) {
        const T di = w * inv_theta;
        d[g] = di;
        x[g] = acc ? x[g] + di : di;
    } else {
        x[g] += c2 * w + c1 * d[g];
    }
}

// The P entries in P^T order: rval(t) = pval(rent(t)), after every change of P.
template <int BS>
__global__ void k_amg_rfill(int64_t nrz, const int64_t *__restrict__ rent, const double *__restrict__ pval,
                            double *__restrict__ rval)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= nrz * BS * 6) return;
    const int64_t t = g / (BS * 6);
    rval[g] = pval[BS * 6 * rent[t] + (g - t * BS * 6)];
}

// bc(I) = sum_{(i, e)} P_e^T r_i with the residual r = b - ax formed on the fly: LN
// lanes per aggregate taking every LN-th entry of its P^T list (values stored in that
// order, so the lanes read consecutive entries), then a fixed-order xor reduction;
// lane c < 6 writes coarse DOF c.  A wavefront per aggregate (LN = 64): on level 0
// (about 100 entries per aggregate) 16 lanes measured slower, each lane's entries
// then being a dependent chain.
template <int BS, typename T, int LN>
__global__ __launch_bounds__(WG) void k_amg_restrict(int64_t nc, const int64_t *__restrict__ rrow,
                                                     const int32_t *__restrict__ rnode, const T *__restrict__ rval,
                                                     const T *__restrict__ b, const T *__restrict__ ax, T *bc)
{
    const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / LN;   // uniform per LN lanes
    const int lane = threadIdx.x & (LN - 1);
    if (I >= nc) return;
    T s[6] = {0, 0, 0, 0, 0, 0};
    const int64_t t1 = rrow[I + 1];
    for (int64_t t = rrow[I] + lane; t < t1; t += LN) {
        const T *p = rval + BS * 6 * t;
        const T *bi = b + (int64_t)BS * rnode[t], *ai = ax + (int64_t)BS * rnode[t];
        for (int k = 0; k < BS; ++k) {
            const T rk = bi[k] - ai[k];
            for (int c = 0; c < 6; ++c) s[c] += p[6 * k + c] * rk;
        }
    }
    T out = 0;
    for (int c = 0; c < 6; ++c) {
        for (int o = LN / 2; o > 0; o >>= 1) s[c] += __shfl_xor(s[c], o, LN);
        if (c == lane) out = s[c];
    }
    if (lane < 6) bc[6 * I + lane] = out;
}

// x_i += sum_{e in P row i} P_e xc(agg) on level 0 (3 rows per node): 4 lanes per node
// taking every 4th entry of its P row (the node's entries contiguous, so the lanes
// read consecutive entries), a fixed-order xor reduction, lane r < 3 updates row r.
template <typename T>
__global__ __launch_bounds__(WG) void k_amg_prolong_add3(int64_t nn, const int64_t *__restrict__ prow,
                                                         const int32_t *__restrict__ pcol, const T *__restrict__ pval,
                                                         const T *__restrict__ xc, T *x)
{
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 2;   // uniform per 4 lanes
    const int q = threadIdx.x & 3;
    if (i >= nn) return;
    T s[3] = {0, 0, 0};
    const int64_t e1 = prow[i + 1];
    for (int64_t e = prow[i] + q; e < e1; e += 4) {
        const T *p = pval + 18 * e;
        const T *xa = xc + 6 * (int64_t)pcol[e];
        T xv[6];
        for (int c = 0; c < 6; ++c) xv[c] = xa[c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 6; ++c) s[r] += p[6 * r + c] * xv[c];
    }
    T out = 0;
    for (int r = 0; r < 3; ++r) {
        s[r] += __shfl_xor(s[r], 2, 4);
        s[r] += __shfl_xor(s[r], 1, 4);
        if (r == q) out = s[r];
    }
    if (q < 3) x[3 * i + q] += out;
}

// x_i += sum_{e in P row i} P_e xc(agg) on the coarse levels (6 rows per node): a
// thread per scalar row.
template <typename T>
__global__ void k_amg_prolong_add6(int64_t nn, const int64_t *__restrict__ prow, const int32_t *__restrict__ pcol,
                                   const T *__restrict__ pval, const T *__restrict__ xc, T *x)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= nn * 6) return;
    const int64_t i = g / 6;
    const int r = (int)(g - i * 6);
    T s = 0;
    for (int64_t e = prow[i]; e < prow[i + 1]; ++e) {
        const T *p = pval + 36 * e + 6 * r;
        const T *xa = xc + 6 * (int64_t)pcol[e];
        for (int c = 0; c < 6; ++c) s += p[c] * xa[c];
    }
    x[g] += s;
}

// y = Ainv x for the coarsest level: one wavefront per row.
template <typename T>
__global__ __launch_bounds__(WG) void k_amg_dense(int64_t n, const T *__restrict__ Ainv, const T *__restrict__ x, T *y)
{
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    T s = 0;
    for (int64_t k = lane; k < n; k += 64) s += Ainv[i * n + k] * x[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) y[i] = s;
}

// FP32 vector helpers of the mixed cycle (the FP64 cycle uses the library's).
__global__ void k_amg_axpby32(int64_t n, float a, const float *__restrict__ x, float b, float *__restrict__ y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}

// Per-block max |x| (the scale of the FP32 cycle inside BiCGStab, formed on the device).
__global__ __launch_bounds__(WG) void k_amg_absmax(int64_t n, const double *__restrict__ x, double *part)
{
    __shared__ double sh[WG];
    double m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, fabs(x[i]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = WG / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// sc[0] = 2^-e with 2^e <= max |x| < 2^(e+1) (1 for a zero, tiny or non-finite x), sc[1] = 1 / sc[0]:
// powers of two, so scaling by them rounds nothing.
__global__ void k_amg_scale_fin(int nparts, const double *__restrict__ part, double *sc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double m = 0;
    for (int i = 0; i < nparts; ++i) m = fmax(m, part[i]);
    const bool ok = m > 0x1p-1000 && isfinite(m);
    sc[0] = ok ? ldexp(1.0, -ilogb(m)) : 1.0;
    sc[1] = ok ? ldexp(1.0, ilogb(m)) : 1.0;
}

__global__ void k_amg_narrow_sc(int64_t n, const double *__restrict__ sc, const double *__restrict__ x,
                                float *__restrict__ y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)(sc[0] * x[i]);
}

__global__ void k_amg_widen_sc(int64_t n, const double *__restrict__ sc, const float *__restrict__ x,
                               double *__restrict__ y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = sc[1] * (double)x[i];
}

// y = s x, FP32 to FP64 (the preconditioned residual of the mixed cycle).
__global__ void k_amg_widen(int64_t n, double s, const float *__restrict__ x, double *__restrict__ y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = s * (double)x[i];
}

inline int64_t nb(int64_t n) { return std::max<int64_t>((n + WG - 1) / WG, 1); }

void free_level(AmgLevel &L)
{
    void *p[] = {L.arow, L.acol, L.arid, L.aval, L.agg, L.q, L.prow, L.pcol, L.pval, L.wrow, L.wcol, L.wval,
                 L.rrow, L.rnode, L.rent, L.rval, L.dinv, L.x, L.b, L.r, L.t, L.d,
                 L.aval32, L.dinv32, L.pval32, L.rval32, L.x32, L.b32, L.r32, L.t32, L.d32};
    for (void *v : p)
        if (v) hipFree(v);
    L = AmgLevel{};
}

}  // namespace

void amg_destroy(fg_system *S)
{
    if (!S->amg) return;
    for (AmgLevel &L : S->amg->L) free_level(L);
    if (S->amg->cinv) hipFree(S->amg->cinv);
    if (S->amg->part) hipFree(S->amg->part);
    for (double *v : {S->amg->cr, S->amg->cz, S->amg->cp, S->amg->cq, S->amg->cz0, S->amg->sc32})
        if (v) hipFree(v);
    for (float *v : {S->amg->cinv32, S->amg->cr32, S->amg->cz32})
        if (v) hipFree(v);
    delete S->amg;
    S->amg = nullptr;
}

// ------------------------------------------------------------ symbolic set-up (host, once per mesh)
static fg_status amg_plan(fg_system *S)
{
    const Plan &P = S->plan;
    const int64_t N = S->N, Npad = S->Npad;
    AmgData *G = new AmgData();
    G->coarse_nodes = S->amg_coarse;
    S->amg = G;
    // level 0 in the caller's numbering: node graph, fault twins, coordinates, held DOFs
    Lists adj(N);
    std::vector<int32_t> twin(N, -1);
    std::vector<double> xyz(3 * N);
    std::vector<uint8_t> held(3 * N);
    par_for(Npad, [&](int64_t r0, int64_t r1) {   // row r fills node perm[r] only
        for (int64_t r = r0; r < r1; ++r) {
            const int32_t i = P.perm[r];
            if (i < 0) continue;
            const int64_t base = P.slice_ptr[r / SLICE] + r % SLICE;
            for (int j = 0; j < P.rowlen[r]; ++j) {
                const int32_t c = P.perm[P.col[base + (int64_t)j * SLICE]];
                if (c != i && c >= 0) adj[i].push_back(c);
            }
            sorted_union(adj[i]);
            const int32_t k = P.fslot.empty() ? -1 : P.fslot[r];
            if (k >= 0 && P.fpart[k] >= 0) twin[i] = P.perm[P.fpart[k]];
            for (int c = 0; c < 3; ++c) {
                xyz[3 * i + c] = P.xyz[3 * r + c];
                held[3 * i + c] = P.dir_u[3 * r + c];
            }
        }
    });
    for (int64_t i = 0; i < N; ++i)
        if (twin[i] >= 0 && twin[twin[i]] != i) twin[i] = -1;
    std::vector<double> B(N * 18, 0.0);
    int64_t nn = N;
    int bs = 3;
    Lists A_pat(N);   // per node, neighbours and itself, sorted
    par_for(N, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            A_pat[i] = adj[i];
            A_pat[i].insert(std::lower_bound(A_pat[i].begin(), A_pat[i].end(), (int32_t)i), (int32_t)i);
        }
    });
    fg_status st = FG_OK;
#define AMG_CK(x)                         \
    do {                                  \
        if ((st = (x)) != FG_OK) {        \
            amg_destroy(S);               \
            set_error("AMG set-up: device allocation failed"); \
            return st;                    \
        }                                 \
    } while (0)
    for (int l = 0; l < AMG_MAXLEV; ++l) {
        AmgLevel &L = G->L[l];
        L.bs = bs;
        G->nlev = l + 1;
        // this level's matrix pattern on the device (level 0: rows in internal order)
        const int64_t rows = l == 0 ? Npad : nn;
        if (l == 0) {
            std::vector<int64_t> arow(Npad + 1, 0);
            for (int64_t r = 0; r < Npad; ++r) arow[r + 1] = arow[r] + P.rowlen[r];
            L.nnzb = arow.back();
            AMG_CK(up(&L.arow, arow));
            AMG_CK(up(&L.acol, std::vector<int32_t>((size_t)L.nnzb)));
        } else {
            std::vector<int64_t> arow;
            std::vector<int32_t> acol;
            to_csr(A_pat, arow, acol);
            L.nnzb = arow.back();
            std::vector<int32_t> arid((size_t)L.nnzb);
            for (int64_t i = 0; i < nn; ++i)
                for (int64_t o = arow[i]; o < arow[i + 1]; ++o) arid[o] = (int32_t)i;
            AMG_CK(up(&L.arow, arow));
            AMG_CK(up(&L.acol, acol));
            AMG_CK(up(&L.arid, arid));
        }
        L.nn = rows;
        AMG_CK(dmal(&L.aval, L.nnzb * bs * bs));
        AMG_CK(dmal(&L.dinv, rows * bs * bs));
        double **vec[] = {&L.x, &L.b, &L.r, &L.t, &L.d};
        for (double **v : vec) AMG_CK(dmal(v, rows * bs));
        if (nn <= G->coarse_nodes || l == AMG_MAXLEV - 1) break;
        // aggregation on the level's node graph (level 0: adj, the neighbours without self)
        Lists nb_l(l == 0 ? 0 : nn);
        if (l > 0)
            par_for(nn, [&](int64_t i0, int64_t i1) {
                for (int64_t i = i0; i < i1; ++i)
                    for (int32_t j : A_pat[i])
                        if (j != i) nb_l[i].push_back(j);
            });
        std::vector<int32_t> agg;
        const int64_t na = aggregate(nn, l == 0 ? adj : nb_l, l == 0 ? &twin : nullptr, agg);
        L.nc = na;
        if (l == 0) {
            std::vector<double> cen(3 * na, 0.0);
            std::vector<int64_t> cnt(na, 0);
            for (int64_t i = 0; i < N; ++i) {
                for (int c = 0; c < 3; ++c) cen[3 * agg[i] + c] += xyz[3 * i + c];
                cnt[agg[i]]++;
            }
            for (int64_t a = 0; a < na; ++a)
                for (int c = 0; c < 3; ++c) cen[3 * a + c] /= (double)cnt[a];
            for (int64_t i = 0; i < N; ++i) {
                const double *c0 = &cen[3 * agg[i]];
                const double dx = xyz[3 * i] - c0[0], dy = xyz[3 * i + 1] - c0[1], dz = xyz[3 * i + 2] - c0[2];
                const double rw[3][6] = {{1, 0, 0, 0, dz, -dy}, {0, 1, 0, -dz, 0, dx}, {0, 0, 1, dy, -dx, 0}};
                for (int r = 0; r < 3; ++r)
                    for (int k = 0; k < 6; ++k) B[(3 * i + r) * 6 + k] = held[3 * i + r] ? 0.0 : rw[r][k];
            }
        }
        std::vector<double> Q, Bc;
        tentative(bs, nn, na, agg, B, Q, Bc);
        // patterns of P, W = A P and A_c = P^T W (entries touched by the products): sorted
        // unions, W's and A_c's by a per-thread marker over the aggregates
        Lists Pp(nn), Wp(nn), Cp(na);
        par_for(nn, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                for (int32_t j : A_pat[i]) Pp[i].push_back(agg[j]);
                sorted_union(Pp[i]);
            }
        });
        par_for(nn, [&](int64_t i0, int64_t i1) {
            std::vector<int32_t> mark((size_t)na, -1);
            for (int64_t i = i0; i < i1; ++i) {
                for (int32_t j : A_pat[i])
                    for (int32_t a : Pp[j])
                        if (mark[a] != (int32_t)i) {
                            mark[a] = (int32_t)i;
                            Wp[i].push_back(a);
                        }
                std::sort(Wp[i].begin(), Wp[i].end());
            }
        });
        std::vector<std::vector<std::pair<int32_t, int64_t>>> Rl(na);   // (node, P entry), increasing node
        std::vector<int64_t> prow_c(nn + 1, 0);
        for (int64_t i = 0; i < nn; ++i) prow_c[i + 1] = prow_c[i] + (int64_t)Pp[i].size();
        for (int64_t i = 0; i < nn; ++i)
            for (size_t t = 0; t < Pp[i].size(); ++t) Rl[Pp[i][t]].push_back({(int32_t)i, prow_c[i] + (int64_t)t});
        par_for(na, [&](int64_t a0, int64_t a1) {
            std::vector<int32_t> mark((size_t)na, -1);
            for (int64_t a = a0; a < a1; ++a) {
                for (const auto &pr : Rl[a])
                    for (int32_t c : Wp[pr.first])
                        if (mark[c] != (int32_t)a) {
                            mark[c] = (int32_t)a;
                            Cp[a].push_back(c);
                        }
                std::sort(Cp[a].begin(), Cp[a].end());
            }
        });
        // to the device; level 0 rows go to internal order
        std::vector<int64_t> prow, wrow, rrow(na + 1, 0), rent;
        std::vector<int32_t> pcol, wcol, rnode, aggd;
        std::vector<double> qd;
        if (l == 0) {
            std::vector<int32_t> ag(Npad, -1);
            qd.assign(Npad * 18, 0.0);
            for (int64_t r = 0; r < Npad; ++r) {
                const int32_t i = P.perm[r];
                if (i < 0) continue;
                ag[r] = agg[i];
                std::memcpy(&qd[r * 18], &Q[(int64_t)i * 18], 18 * sizeof(double));
            }
            to_csr(Pp, prow, pcol, Npad, P.perm.data());
            to_csr(Wp, wrow, wcol, Npad, P.perm.data());
            aggd = ag;
            // P^T lists: internal row and internal P entry, in increasing caller node order
            for (int64_t a = 0; a < na; ++a) {
                rrow[a + 1] = rrow[a] + (int64_t)Rl[a].size();
                for (auto &pr : Rl[a]) {
                    const int32_t r = P.iperm[pr.first];
                    const int64_t t = pr.second - prow_c[pr.first];
                    rnode.push_back(r);
                    rent.push_back(prow[r] + t);
                }
            }
        } else {
            to_csr(Pp, prow, pcol);
            to_csr(Wp, wrow, wcol);
            aggd = agg;
            qd = Q;
            for (int64_t a = 0; a < na; ++a) {
                rrow[a + 1] = rrow[a] + (int64_t)Rl[a].size();
                for (auto &pr : Rl[a]) {
                    rnode.push_back(pr.first);
                    rent.push_back(pr.second);
                }
            }
        }
        L.npz = (int64_t)pcol.size();
        L.nwz = (int64_t)wcol.size();
        L.nrz = (int64_t)rnode.size();
        AMG_CK(up(&L.agg, aggd));
        AMG_CK(up(&L.q, qd));
        AMG_CK(up(&L.prow, prow));
        AMG_CK(up(&L.pcol, pcol));
        AMG_CK(dmal(&L.pval, L.npz * bs * 6));
        AMG_CK(up(&L.wrow, wrow));
        AMG_CK(up(&L.wcol, wcol));
        AMG_CK(dmal(&L.wval, L.nwz * bs * 6));
        AMG_CK(up(&L.rrow, rrow));
        AMG_CK(up(&L.rnode, rnode));
        AMG_CK(up(&L.rent, rent));
        AMG_CK(dmal(&L.rval, L.nrz * bs * 6));
        // next level
        A_pat.swap(Cp);
        for (int64_t a = 0; a < na; ++a) {
            bool self = std::binary_search(A_pat[a].begin(), A_pat[a].end(), (int32_t)a);
            if (!self) {
                A_pat[a].push_back((int32_t)a);
                sorted_union(A_pat[a]);
            }
        }
        B.assign(na * 36, 0.0);
        for (int64_t a = 0; a < na; ++a)
            for (int k = 0; k < 36; ++k) B[a * 36 + k] = Bc[a * 36 + k];
        nn = na;
        bs = 6;
    }
#undef AMG_CK
    const AmgLevel &C = G->L[G->nlev - 1];
    G->nco = C.nn * C.bs;
    const bool too_big = G->nco > 8192;
    if (too_big || dmal(&G->cinv, G->nco * G->nco) || dmal(&G->part, 1 << 16) || dmal(&G->cr, 3 * Npad) ||
        dmal(&G->cz, 3 * Npad) || dmal(&G->cp, 3 * Npad) || dmal(&G->cq, 3 * Npad)) {
        amg_destroy(S);   // frees G
        set_error(too_big ? "AMG set-up: the coarsest level stays above 8192 unknowns"
                          : "AMG set-up: device allocation failed");
        return too_big ? FG_ERR_ARG : FG_ERR_OOM;
    }
    return FG_OK;
}

// ------------------------------------------------------------ numeric set-up (GPU, per K)
static fg_status amg_diag_level(fg_system *S, AmgLevel &L, hipStream_t st)
{
    AmgData *G = S->amg;
    int *bad = (int *)S->red_counter + 3;
    hipMemsetAsync(bad, 0, sizeof(int), st);
    const int64_t blocks = nb(L.nn);
    if (blocks > (1 << 16)) {
        set_error("AMG set-up: level too large for the reduction workspace");
        return FG_ERR_ARG;
    }
    if (L.bs == 3)
        LAUNCH((k_amg_diag<3>), blocks, WG, st, L.nn, L.arow, L.acol, L.aval, L.dinv, G->part, bad);
    else
        LAUNCH((k_amg_diag<6>), blocks, WG, st, L.nn, L.arow, L.acol, L.aval, L.dinv, G->part, bad);
    std::vector<double> part(blocks);
    int h = 0;
    hipMemcpyAsync(part.data(), G->part, blocks * sizeof(double), hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    L.rho = 0;
    for (double v : part) L.rho = std::max(L.rho, v);
    if (h || !(L.rho > 0) || !std::isfinite(L.rho)) {
        set_error("AMG set-up: a diagonal block is singular");
        return FG_ERR_BREAKDOWN;
    }
    return check_hip("AMG diagonal blocks");
}

static fg_status amg_numeric(fg_system *S, hipStream_t st)
{
    AmgData *G = S->amg;
    bj_ready(S, st);
    if (S->bj_singular) {
        set_error("AMG set-up: a diagonal or fault-pair block of K is singular");
        return FG_ERR_BREAKDOWN;
    }
    fg_status e = cheb_interval_ready(S, st);   // the level-0 smoother's interval
    if (e) return e;
    LAUNCH(k_amg_copy_k, nb(S->Npad), WG, st, S->Npad, S->slice_ptr, S->rowlen, S->col, S->K, G->L[0].arow,
           G->L[0].acol, G->L[0].aval);
    for (int l = 0; l < G->nlev; ++l) {
        AmgLevel &L = G->L[l];
        e = amg_diag_level(S, L, st);
        if (e) return e;
        if (l == G->nlev - 1) break;
        AmgLevel &C = G->L[l + 1];
        const double w = 4.0 / (3.0 * L.rho);
        if (L.bs == 3) {
            LAUNCH((k_amg_prolong<3>), nb(L.nn), WG, st, L.nn, L.arow, L.acol, L.aval, L.agg, L.q, L.dinv, L.prow,
                   L.pcol, w, L.pval);
            LAUNCH((k_amg_rfill<3>), nb(18 * L.nrz), WG, st, L.nrz, L.rent, L.pval, L.rval);
            LAUNCH((k_amg_ap<3>), nb(L.nn), WG, st, L.nn, L.arow, L.acol, L.aval, L.prow, L.pcol, L.pval, L.wrow,
                   L.wcol, L.wval);
            LAUNCH((k_amg_rap<3>), nb(C.nnzb), WG, st, C.nnzb, C.arid, C.acol, L.rrow, L.rnode, L.rent, L.pval,
                   L.wrow, L.wcol, L.wval, C.aval);
        } else {
            LAUNCH((k_amg_prolong<6>), nb(L.nn), WG, st, L.nn, L.arow, L.acol, L.aval, L.agg, L.q, L.dinv, L.prow,
                   L.pcol, w, L.pval);
            LAUNCH((k_amg_rfill<6>), nb(36 * L.nrz), WG, st, L.nrz, L.rent, L.pval, L.rval);
            LAUNCH((k_amg_ap<6>), nb(L.nn), WG, st, L.nn, L.arow, L.acol, L.aval, L.prow, L.pcol, L.pval, L.wrow,
                   L.wcol, L.wval);
            LAUNCH((k_amg_rap<6>), nb(C.nnzb), WG, st, C.nnzb, C.arid, C.acol, L.rrow, L.rnode, L.rent, L.pval,
                   L.wrow, L.wcol, L.wval, C.aval);
        }
        LAUNCH(k_amg_unit_empty, nb(L.nc), WG, st, L.nc, C.arow, C.acol, C.aval);
        e = check_hip("AMG prolongator and coarse operator");
        if (e) return e;
    }
    // the coarsest matrix: dense inverse on the host (Cholesky, then columns of the inverse)
    const AmgLevel &C = G->L[G->nlev - 1];
    const int64_t n = G->nco;
    std::vector<int64_t> arow(C.nn + 1);
    std::vector<int32_t> acol(C.nnzb);
    std::vector<double> aval(C.nnzb * C.bs * C.bs);
    hipMemcpyAsync(arow.data(), C.arow, arow.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(acol.data(), C.acol, acol.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    hipMemcpyAsync(aval.data(), C.aval, aval.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    const int bs = C.bs;
    std::vector<double> L(n * n, 0.0), inv(n * n, 0.0);
    for (int64_t i = 0; i < C.nn; ++i)
        for (int64_t o = arow[i]; o < arow[i + 1]; ++o)
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < bs; ++c) L[(bs * i + r) * n + bs * (int64_t)acol[o] + c] = aval[bs * bs * o + bs * r + c];
    // rows without entries (the slices' padding rows when the whole mesh is the coarsest
    // level) are decoupled: a unit diagonal keeps the matrix invertible, and their
    // right-hand sides are zero, so the other unknowns do not change
    for (int64_t j = 0; j < n; ++j) {
        bool empty = true;
        for (int64_t k = 0; k < n && empty; ++k) empty = L[j * n + k] == 0.0;
        if (empty) L[j * n + j] = 1.0;
    }
    for (int64_t j = 0; j < n; ++j) {
        double d = L[j * n + j];
        for (int64_t k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0)) {
            set_error("AMG set-up: the coarsest matrix is not positive definite");
            return FG_ERR_BREAKDOWN;
        }
        d = std::sqrt(d);
        L[j * n + j] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = L[i * n + j];
            for (int64_t k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / d;
        }
    }
    std::vector<double> col(n);
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = 0; i < n; ++i) {
            double s = i == c ? 1.0 : 0.0;
            for (int64_t k = 0; k < i; ++k) s -= L[i * n + k] * col[k];
            col[i] = s / L[i * n + i];
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = col[i];
            for (int64_t k = i + 1; k < n; ++k) s -= L[k * n + i] * col[k];
            col[i] = s / L[i * n + i];
        }
        for (int64_t i = 0; i < n; ++i) inv[i * n + c] = col[i];
    }
    hipMemcpyAsync(G->cinv, inv.data(), n * n * sizeof(double), hipMemcpyHostToDevice, st);
    hipStreamSynchronize(st);
    G->epoch = S->bj_epoch;
    return check_hip("AMG coarsest inverse");
}

fg_status amg_ready(fg_system *S, hipStream_t st)
{
    if (S->ngroups > 1) {
        set_error("AMG: batched systems are not supported");
        return FG_ERR_ARG;
    }
    if (!S->amg) {
        fg_status e = amg_plan(S);
        if (e) return e;
    }
    bj_ready(S, st);
    if (S->amg->epoch == S->bj_epoch) return FG_OK;
    return amg_numeric(S, st);
}

// ------------------------------------------------------------ FP32 copies (mixed precision)
static void free32(AmgData *G)
{
    for (AmgLevel &L : G->L) {
        float **p[] = {&L.aval32, &L.dinv32, &L.pval32, &L.rval32, &L.x32, &L.b32, &L.r32, &L.t32, &L.d32};
        for (float **v : p) {
            if (*v) hipFree(*v);
            *v = nullptr;
        }
    }
    for (float **v : {&G->cinv32, &G->cr32, &G->cz32}) {
        if (*v) hipFree(*v);
        *v = nullptr;
    }
    for (double **v : {&G->cz0, &G->sc32}) {
        if (*v) hipFree(*v);
        *v = nullptr;
    }
    G->epoch32 = -1;
}

// The hierarchy's values in FP32 for the current K (after amg_ready): every level's
// matrix (level 0: K's own FP32 copy), block-Jacobi inverses, prolongator and the
// coarsest inverse, rounded from the FP64 set-up.
static fg_status amg_ready32(fg_system *S, hipStream_t st)
{
    AmgData *G = S->amg;
    if (!G->cr32) {
        bool ok = true;
        for (int l = 0; l < G->nlev && ok; ++l) {
            AmgLevel &L = G->L[l];
            const int64_t n = L.nn * L.bs;
            if (l > 0) ok = ok && !dmal(&L.aval32, L.nnzb * L.bs * L.bs) && !dmal(&L.dinv32, n * L.bs);
            if (l < G->nlev - 1)
                ok = ok && !dmal(&L.pval32, L.npz * L.bs * 6) && !dmal(&L.rval32, L.nrz * L.bs * 6);
            float **vec[] = {&L.x32, &L.b32, &L.r32, &L.t32, &L.d32};
            for (float **v : vec) ok = ok && !dmal(v, n);
        }
        const int64_t n0 = 3 * S->Npad;
        ok = ok && !dmal(&G->cinv32, G->nco * G->nco) && !dmal(&G->cr32, n0) && !dmal(&G->cz32, n0) &&
             !dmal(&G->cz0, n0) && !dmal(&G->sc32, 2);
        if (!ok) {
            free32(G);
            set_error("AMG: device allocation for the FP32 cycle failed");
            return FG_ERR_OOM;
        }
    }
    if (!S->k32_valid) refresh_k32(S, st);
    bj_ready32(S, st);
    if (G->epoch32 == G->epoch) return FG_OK;
    for (int l = 0; l < G->nlev; ++l) {
        AmgLevel &L = G->L[l];
        if (l > 0) {
            to_f32(L.nnzb * L.bs * L.bs, 1.0, L.aval, L.aval32, st);
            to_f32(L.nn * L.bs * L.bs, 1.0, L.dinv, L.dinv32, st);
        }
        if (l < G->nlev - 1) {
            to_f32(L.npz * L.bs * 6, 1.0, L.pval, L.pval32, st);
            to_f32(L.nrz * L.bs * 6, 1.0, L.rval, L.rval32, st);
        }
    }
    to_f32(G->nco * G->nco, 1.0, G->cinv, G->cinv32, st);
    G->epoch32 = G->epoch;
    return check_hip("AMG FP32 copies");
}

// ------------------------------------------------------------ the V-cycle
// One level's cycle arrays in the cycle's precision.
template <typename T>
struct Lv {
    const T *aval, *dinv, *pval, *rval;
    T *x, *b, *r, *t, *d;
};
static Lv<double> lv(const AmgLevel &L, double)
{
    return {L.aval, L.dinv, L.pval, L.rval, L.x, L.b, L.r, L.t, L.d};
}
static Lv<float> lv(const AmgLevel &L, float)
{
    return {L.aval32, L.dinv32, L.pval32, L.rval32, L.x32, L.b32, L.r32, L.t32, L.d32};
}
static const double *cinv_of(const AmgData *G, double) { return G->cinv; }
static const float *cinv_of(const AmgData *G, float) { return G->cinv32; }

// Level 0 works on K itself: the library's product and block-Jacobi smoothing.
static void l0_mul(fg_system *S, const double *x, double *y, hipStream_t st) { spmv(S, FG_K, x, y, st); }
static void l0_mul(fg_system *S, const float *x, float *y, hipStream_t st) { spmv_k32(S, x, y, st); }
static void axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t st)
{
    vaxpby(n, a, x, b, y, st);
}
static void axpby(int64_t n, double a, const float *x, double b, float *y, hipStream_t st)
{
    LAUNCH(k_amg_axpby32, nb(n), WG, st, n, (float)a, x, (float)b, y);
}

// y = A_l x on level l.
template <typename T>
static void amg_mul(fg_system *S, int l, const T *x, T *y, hipStream_t st)
{
    const AmgLevel &L = S->amg->L[l];
    if (l == 0)
        l0_mul(S, x, y, st);
    else
        LAUNCH((k_amg_spmv6<T, sizeof(T) == 8 ? 2 : 1>), nb((sizeof(T) == 8 ? 16 : 8) * L.nn), WG, st, L.nn, L.arow,
               L.acol, lv(L, T()).aval, x, y);
}

// x = p(M^-1 A) M^-1 b (acc: x += p(M^-1 A) M^-1 b), degree-2 Chebyshev over the level's
// block Jacobi on [hi/30, hi]: d0 = M^-1 b / theta, d1 = c1 d0 + c2 M^-1 (b - A d0),
// x = d0 + d1 (level 0: the blocks of "k_precond" 1, hi as for the Chebyshev
// preconditioner; below: 6x6 diagonal blocks, hi their Gershgorin bound).
template <typename T>
static void amg_smooth(fg_system *S, int l, const T *b, T *x, int acc, hipStream_t st)
{
    AmgData *G = S->amg;
    AmgLevel &L = G->L[l];
    const Lv<T> v = lv(L, T());
    const int64_t n = L.nn * L.bs;
    const double hi = l == 0 ? S->cheb_hi : L.rho, lo = hi / 30.0;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    const double rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
    const double c1 = rho1 * rho0, c2 = 2.0 * rho1 / delta;
    auto step = [&](int k) {
        if (l == 0)
            bj_smooth(S, k, acc, 1.0 / theta, c1, c2, b, v.t, v.d, x, st);
        else
            LAUNCH((k_amg_dsmooth<T>), nb(n), WG, st, L.nn, k, acc, v.dinv, (T)(1.0 / theta), (T)c1, (T)c2, b, v.t,
                   v.d, x);
    };
    step(0);
    amg_mul(S, l, (const T *)v.d, v.t, st);
    step(1);
}

template <typename T>
static void amg_vcycle(fg_system *S, int l, const T *b, T *x, hipStream_t st)
{
    AmgData *G = S->amg;
    AmgLevel &L = G->L[l];
    const Lv<T> v = lv(L, T());
    const int64_t n = L.nn * L.bs;
    if (l == G->nlev - 1) {
        LAUNCH((k_amg_dense<T>), nb(64 * n), WG, st, n, cinv_of(G, T()), b, x);
        return;
    }
    const Lv<T> c = lv(G->L[l + 1], T());
    amg_smooth(S, l, b, x, 0, st);                    // pre-smoothing from zero
    amg_mul(S, l, (const T *)x, v.r, st);             // restriction of b - A x
    if (L.bs == 3)
        LAUNCH((k_amg_restrict<3, T, 64>), nb(64 * L.nc), WG, st, L.nc, L.rrow, L.rnode, v.rval, b, v.r, c.b);
    else
        LAUNCH((k_amg_restrict<6, T, 64>), nb(64 * L.nc), WG, st, L.nc, L.rrow, L.rnode, v.rval, b, v.r, c.b);
    amg_vcycle(S, l + 1, (const T *)c.b, c.x, st);
    if (L.bs == 3)
        LAUNCH((k_amg_prolong_add3<T>), nb(4 * L.nn), WG, st, L.nn, L.prow, L.pcol, v.pval, c.x, x);
    else
        LAUNCH((k_amg_prolong_add6<T>), nb(n), WG, st, L.nn, L.prow, L.pcol, v.pval, c.x, x);
    amg_mul(S, l, (const T *)x, v.r, st);
    axpby(n, 1.0, b, -1.0, v.r, st);                  // r = b - A x
    amg_smooth(S, l, (const T *)v.r, x, 1, st);       // post-smoothing on the residual, added to x
}

// z = B r, one FP64 V-cycle on the hierarchy of the current K (after amg_ready); the
// preconditioner of the exact-tangent BiCGStab (r, z internal vectors, not the AMG's).
void amg_apply(fg_system *S, const double *r, double *z, hipStream_t st) { amg_vcycle(S, 0, r, z, st); }

// The same with the V-cycle in FP32 (after amg_ready_f32): r scaled on the device by the
// power of two below max |r| (no host synchronisation), the result scaled back.
void amg_apply32(fg_system *S, const double *r, double *z, hipStream_t st)
{
    AmgData *G = S->amg;
    const int64_t n = 3 * S->Npad;
    const int nparts = (int)std::min<int64_t>(nb(n), 1024);
    LAUNCH(k_amg_absmax, nparts, WG, st, n, r, G->part);
    LAUNCH(k_amg_scale_fin, 1, 64, st, nparts, (const double *)G->part, G->sc32);
    LAUNCH(k_amg_narrow_sc, nb(n), WG, st, n, (const double *)G->sc32, r, G->cr32);
    amg_vcycle(S, 0, (const float *)G->cr32, G->cz32, st);
    LAUNCH(k_amg_widen_sc, nb(n), WG, st, n, (const double *)G->sc32, (const float *)G->cz32, z);
}

fg_status amg_ready_f32(fg_system *S, hipStream_t st)
{
    const fg_status e = amg_ready(S, st);
    return e ? e : amg_ready32(S, st);
}

fg_status amg_aggregates(const fg_system *S, int level, int32_t *out)
{
    const AmgData *G = S->amg;
    if (!G || level < 0 || level >= G->nlev - 1) {
        set_error("fg_amg_aggregates: level must be below the coarsest level of the hierarchy");
        return FG_ERR_ARG;
    }
    const AmgLevel &L = G->L[level];
    std::vector<int32_t> a((size_t)L.nn);
    if (hipMemcpy(a.data(), L.agg, a.size() * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return check_hip("fg_amg_aggregates");
    if (level == 0)   // internal rows to the caller's node numbering
        for (int64_t i = 0; i < S->N; ++i) out[i] = a[(size_t)S->plan.iperm[i]];
    else
        std::memcpy(out, a.data(), a.size() * sizeof(int32_t));
    return FG_OK;
}

void amg_levels(const fg_system *S, int *nlev, int64_t *nodes)
{
    *nlev = S->amg ? S->amg->nlev : 0;
    for (int l = 0; l < AMG_MAXLEV; ++l)
        nodes[l] = (S->amg && l < S->amg->nlev) ? (l == 0 ? S->N : S->amg->L[l].nn) : 0;
}

// PCG on K with the V-cycle (internal vectors; same recurrence and stop test as cg_run).
// f32: the cycle runs in FP32 on r scaled to unit norm by the last residual norm, and
// its result is scaled back; the CG stays FP64 and, since rounding makes that cycle
// slightly non-symmetric, takes beta in the flexible form
// r_{k+1}.(z_{k+1} - z_k) / r_k.z_k (Golub and Ye, SIAM J. Sci. Comput. 21, 1999).
fg_status amg_pcg(fg_system *S, const double *b, double *x, double tol, int64_t maxit, bool f32, int64_t *iters,
                  double *relres, hipStream_t st)
{
    *iters = 0;
    *relres = 0;
    fg_status e = amg_ready(S, st);
    if (e) return e;
    if (f32) {
        e = amg_ready32(S, st);
        if (e) return e;
    }
    AmgData *G = S->amg;
    const int64_t n = 3 * S->Npad;
    double *r = G->cr, *z = G->cz, *p = G->cp, *q = G->cq, *z0 = G->cz0;
    auto precond = [&](double rn) {
        if (!f32) {
            amg_vcycle(S, 0, (const double *)r, z, st);
            return;
        }
        to_f32(n, 1.0 / rn, r, G->cr32, st);
        amg_vcycle(S, 0, (const float *)G->cr32, G->cz32, st);
        LAUNCH(k_amg_widen, nb(n), WG, st, n, rn, G->cz32, z);
    };
    vfill(x, 0.0, n, st);
    hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    double bn, rho;
    if (f32) {
        const double *A[1] = {b};
        vdots(S, n, 1, A, A, &bn, st);
        bn = std::sqrt(bn);
        if (!(bn > 0)) return std::isfinite(bn) ? FG_OK : FG_ERR_NAN;
        precond(bn);
        const double *R[1] = {r}, *Z[1] = {z};
        vdots(S, n, 1, R, Z, &rho, st);
    } else {
        precond(1.0);
        double d2[2];
        const double *A[2] = {b, r}, *B2[2] = {b, z};
        vdots(S, n, 2, A, B2, d2, st);
        bn = std::sqrt(d2[0]);
        rho = d2[1];
        if (!(bn > 0)) return std::isfinite(bn) ? FG_OK : FG_ERR_NAN;
    }
    hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    double rr;   // r.r, taken in the same reduction as r.z after every update
    {
        const double *A[1] = {r};
        vdots(S, n, 1, A, A, &rr, st);
    }
    int64_t it = 0;
    for (;;) {
        const double rel = std::sqrt(rr) / bn;
        *relres = rel;
        if (!std::isfinite(rel)) {
            set_error("fg_pcg_solve: NaN in the AMG-preconditioned CG");
            return FG_ERR_NAN;
        }
        if (rel <= tol) break;
        if (it >= maxit) {
            *iters = it;
            return FG_NOT_CONVERGED;
        }
        spmv(S, FG_K, p, q, st);
        double pq;
        {
            const double *A[1] = {p}, *B1[1] = {q};
            vdots(S, n, 1, A, B1, &pq, st);
        }
        if (!(pq > 0.0)) {
            set_error("fg_pcg_solve: CG breakdown (p.Ap <= 0) with the AMG preconditioner");
            *iters = it;
            return FG_ERR_BREAKDOWN;
        }
        const double al = rho / pq;
        vaxpby(n, al, p, 1.0, x, st);
        vaxpby(n, -al, q, 1.0, r, st);
        if (f32) std::swap(z, z0);   // z0: the last preconditioned residual
        precond(std::sqrt(rr));
        double rho2, rz0 = 0.0;
        if (f32) {
            double d3[3];
            const double *A[3] = {r, r, r}, *B3[3] = {z, r, z0};
            vdots(S, n, 3, A, B3, d3, st);
            rho2 = d3[0];
            rr = d3[1];
            rz0 = d3[2];
        } else {
            double d2[2];
            const double *A[2] = {r, r}, *B2[2] = {z, r};
            vdots(S, n, 2, A, B2, d2, st);
            rho2 = d2[0];
            rr = d2[1];
        }
        const double be = (rho2 - rz0) / rho;
        rho = rho2;
        vaxpby(n, 1.0, z, be, p, st);
        ++it;
    }
    *iters = it;
    return check_hip("AMG PCG");
}

}  // namespace fg
