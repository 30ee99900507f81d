// Chebyshev polynomial preconditioner over block Jacobi for the FP64 K solve.
//
// The inner K solves of the partitioned iteration (Sec. 3.3.2) are preconditioned
// by z = p(M^-1 K) M^-1 r, where M is the nodal / fault-pair block Jacobi of K and
// p makes 1 - t p(t) the scaled Chebyshev polynomial T_m((hi + lo - 2t)/(hi - lo)) /
// T_m((hi + lo)/(hi - lo)) of degree m on an interval [lo, hi] of the spectrum of
// M^-1 K: m steps of the Chebyshev iteration (Saad, Iterative Methods for Sparse
// Linear Systems, Sec. 12.3) from z = 0, m - 1 products with K.  p(t) t > 0 on
// (0, hi + lo), so the preconditioner is SPD and plain CG applies.
//
// hi is 1.1 times the largest Ritz value of a short block-Jacobi CG on a fixed
// probe vector (the CG coefficients give the Lanczos matrix, Saad Sec. 6.7.3),
// estimated once per K; lo = hi / ratio.  The probe is SplitMix64 (Steele, Lea
// and Flood 2014) of the caller-order DOF index, zero on Dirichlet DOFs.
//
// Each Chebyshev step is one K product (the CG product kernel) and one vector
// kernel whose threads own whole preconditioner units (a node, or both nodes of a
// fault pair, taken by the lower row), so s -= K d, w = M^-1 s, d = c1 d + c2 w and
// z += d need no other thread's values and no global reduction.  A CG iteration
// therefore reduces twice per m products instead of twice per product.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "fg_device.h"
#include "fg_kernels.h"

namespace fg {

namespace {

template <typename T>
struct BjViewT {
    const T *A;            // [Npad*6] symmetric 3x3 blocks of M^-1: xx yy zz yz xz xy
    const T *B;            // [nfr*9] pair coupling blocks of M^-1, row-major
    const int32_t *fslot;  // [Npad] fault-row index, -1 off the interface
    const int32_t *fpart;  // [nfr] partner row, -1 if none
};
typedef BjViewT<double> BjView;

template <typename T>
__device__ __forceinline__ T sym6(const T *a, int r, int c)
{
    if (r == c) return a[r];
    const int s = r + c;  // 1: xy, 2: xz, 3: yz
    return s == 3 ? a[3] : (s == 2 ? a[4] : a[5]);
}

// w = M^-1 s on one unit: row u alone (nr = 1) or rows u, v of a pair (nr = 2).
template <typename T>
__device__ __forceinline__ void unit_apply(const BjViewT<T> &m, int64_t u, int64_t v, int ku, int kv, const T (&s)[6],
                                           int nr, T (&w)[6])
{
    for (int h = 0; h < nr; ++h) {
        const int64_t row = h == 0 ? u : v;
        const int kk = h == 0 ? ku : kv;
        const T *a = m.A + 6 * row;
        const T *so = s + 3 * h, *sp = s + 3 * (1 - h);
        for (int c = 0; c < 3; ++c) {
            T z = sym6(a, c, 0) * so[0] + sym6(a, c, 1) * so[1] + sym6(a, c, 2) * so[2];
            if (nr == 2) {
                const T *b = m.B + 9 * kk + 3 * c;
                z += b[0] * sp[0] + b[1] * sp[1] + b[2] * sp[2];
            }
            w[3 * h + c] = z;
        }
    }
}

// Unit of row u: false if u is the upper row of a pair (its lower row owns it).
template <typename T>
__device__ __forceinline__ bool unit_of(const BjViewT<T> &m, int64_t u, int64_t &v, int &ku, int &kv, int &nr)
{
    ku = m.fslot[u];
    v = ku >= 0 ? m.fpart[ku] : -1;
    if (v >= 0 && v < u) return false;
    nr = v >= 0 ? 2 : 1;
    kv = v >= 0 ? m.fslot[v] : -1;
    return true;
}

__device__ __forceinline__ int64_t unit_dof(int64_t u, int64_t v, int e) { return 3 * (e < 3 ? u : v) + e % 3; }

// out = M^-1 in (the Lanczos estimate).
template <typename T>
__global__ __launch_bounds__(WG) void k_ch_bj(int64_t Npad, BjViewT<T> m, const T *__restrict__ in,
                                              T *__restrict__ out)
{
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < Npad; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t v;
        int ku, kv, nr;
        if (!unit_of(m, u, v, ku, kv, nr)) continue;
        T s[6] = {0, 0, 0, 0, 0, 0}, w[6];
        for (int e = 0; e < 3 * nr; ++e) s[e] = in[unit_dof(u, v, e)];
        unit_apply(m, u, v, ku, kv, s, nr, w);
        for (int e = 0; e < 3 * nr; ++e) out[unit_dof(u, v, e)] = w[e];
    }
}

// Degree-2 Chebyshev smoothing over block Jacobi, one kernel per step (level 0 of the
// AMG cycle, FP64 or FP32).  step 0: d = M^-1 b / theta, then x = d (acc: x += d).
// step 1, on kd = K d: x += c2 M^-1 (b - kd) + c1 d.  Each thread owns whole units.
template <typename T>
__global__ __launch_bounds__(WG) void k_bj_smooth(int64_t Npad, int step, int acc, BjViewT<T> m, T inv_theta, T c1,
                                                  T c2, const T *__restrict__ b, const T *__restrict__ kd,
                                                  T *__restrict__ d, T *__restrict__ x)
{
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < Npad; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t v;
        int ku, kv, nr;
        if (!unit_of(m, u, v, ku, kv, nr)) continue;
        T s[6] = {0, 0, 0, 0, 0, 0}, w[6];
        for (int e = 0; e < 3 * nr; ++e) {
            const int64_t i = unit_dof(u, v, e);
            s[e] = step ? b[i] - kd[i] : b[i];
        }
        unit_apply(m, u, v, ku, kv, s, nr, w);
        for (int e = 0; e < 3 * nr; ++e) {
            const int64_t i = unit_dof(u, v, e);
            if (step == 0) {
                const T di = w[e] * inv_theta;
                d[i] = di;
                x[i] = acc ? x[i] + di : di;
            } else {
                x[i] += c2 * w[e] + c1 * d[i];
            }
        }
    }
}

// Probe vector in caller order: SplitMix64 of the DOF index mapped to [-1/2, 1/2).
__global__ void k_ch_probe(int64_t n, double *v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = ((uint64_t)i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

// CG update and first Chebyshev step.  first: x = 0 and r already holds b.
// Otherwise alpha = rho / (p.q) from the product's partials (every block sums
// them in the same order), x += alpha p, r -= alpha q.  Then, per unit,
// d = M^-1 r / theta (z = d when the degree is 1, else the next step forms z and
// s from d and r), and the partials of r.d and r.r (rows 2, 3).
__global__ __launch_bounds__(WG) void k_ch_update(int64_t Npad, int par, int first, int write_z, BjView m,
                                                  double inv_theta, double *__restrict__ x, double *__restrict__ r,
                                                  const double *__restrict__ p, const double *__restrict__ q,
                                                  double *__restrict__ d, double *__restrict__ z, double *partials,
                                                  int64_t stride, int64_t nparts, CgScalars *sc)
{
    if (__syncthreads_or(sc->done)) return;
    double alpha = 0;
    if (!first) {
        double tot[1];
        finalize_sum<1>(partials, stride, nparts, tot);
        const double pq = tot[0];
        alpha = sc->rho[par] / pq;
        const bool ok = isfinite(pq) && pq > 0.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->pq = pq;
            if (!isfinite(pq)) {
                sc->status = FG_ERR_NAN;
                sc->done = 1;
            } else if (!(pq > 0.0)) {
                sc->status = FG_ERR_BREAKDOWN;
                sc->done = 1;
            } else {
                sc->alpha = alpha;
            }
        }
        if (!ok) return;
    }
    double acc[2] = {0, 0};
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < Npad; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t v;
        int ku, kv, nr;
        if (!unit_of(m, u, v, ku, kv, nr)) continue;
        double rr[6] = {0, 0, 0, 0, 0, 0}, w[6];
        for (int e = 0; e < 3 * nr; ++e) {
            const int64_t i = unit_dof(u, v, e);
            double ri = r[i];
            if (first) {
                x[i] = 0.0;
            } else {
                x[i] += alpha * p[i];
                ri -= alpha * q[i];
                r[i] = ri;
            }
            rr[e] = ri;
            acc[1] += ri * ri;
        }
        unit_apply(m, u, v, ku, kv, rr, nr, w);
        for (int e = 0; e < 3 * nr; ++e) {
            const int64_t i = unit_dof(u, v, e);
            const double di = w[e] * inv_theta;
            d[i] = di;
            if (write_z) z[i] = di;
            acc[0] += rr[e] * di;
        }
    }
    block_partials<2>(acc, partials + 2 * stride, stride);
}

// One further Chebyshev step on the product kd = K d: s -= kd, d = c1 d + c2 M^-1 s,
// z += d.  The first of these steps starts from s = r and z = d; the last one
// stores only z and forms the partials of r.z (row 2).
__global__ __launch_bounds__(WG) void k_ch_step(int64_t Npad, int first, int last, BjView m, double c1, double c2,
                                                const double *__restrict__ r, const double *__restrict__ kd,
                                                double *__restrict__ d, double *__restrict__ s,
                                                double *__restrict__ z, double *partials, int64_t stride,
                                                const CgScalars *sc)
{
    if (__syncthreads_or(sc->done)) return;
    double acc[1] = {0};
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < Npad; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t v;
        int ku, kv, nr;
        if (!unit_of(m, u, v, ku, kv, nr)) continue;
        double sv[6] = {0, 0, 0, 0, 0, 0}, w[6];
        for (int e = 0; e < 3 * nr; ++e) {
            const int64_t i = unit_dof(u, v, e);
            const double si = (first ? r[i] : s[i]) - kd[i];
            if (!last) s[i] = si;
            sv[e] = si;
        }
        unit_apply(m, u, v, ku, kv, sv, nr, w);
        for (int e = 0; e < 3 * nr; ++e) {
            const int64_t i = unit_dof(u, v, e);
            const double dold = d[i];
            const double di = c1 * dold + c2 * w[e];
            if (!last) d[i] = di;
            const double zi = (first ? dold : z[i]) + di;
            z[i] = zi;
            if (last) acc[0] += r[i] * zi;
        }
    }
    if (last) block_partials<1>(acc, partials + 2 * stride, stride);
}

// End of an iteration (or of the start when init): rho' = r.z, r.r from rows 2, 3;
// stop test on ||r|| <= tol ||b||; beta = rho' / rho; p = z + beta p.
__global__ __launch_bounds__(WG) void k_ch_pupdate(int64_t n, int par, int init, double tol, const double *__restrict__ z,
                                                   double *__restrict__ p, const double *partials, int64_t stride,
                                                   int64_t nparts, CgScalars *sc)
{
    if (__syncthreads_or(sc->done)) return;
    double tot[2];
    finalize_sum<2>(partials + 2 * stride, stride, nparts, tot);
    const bool finite = isfinite(tot[0]) && isfinite(tot[1]);
    const int64_t it = init ? 0 : sc->iter[par] + 1;
    const double tol2 = init ? tol * tol * tot[1] : sc->tol2;
    const bool conv = init ? !(tot[1] > 0.0) : tot[1] <= tol2;
    const bool stop = !finite || conv || (!init && it >= sc->maxit);
    const double beta = init ? 0.0 : tot[0] / sc->rho[par];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int nxt = init ? 0 : par ^ 1;
        if (init) {
            sc->bb = tot[1];
            sc->tol2 = tol2;
        }
        sc->iter[nxt] = it;
        sc->iters = it;
        sc->rr = tot[1];
        sc->rho[nxt] = tot[0];
        sc->rho_cur = tot[0];
        if (!finite) {
            sc->status = FG_ERR_NAN;
            sc->done = 1;
        } else if (conv) {
            sc->status = FG_OK;
            sc->done = 1;
        } else if (stop) {
            sc->status = FG_NOT_CONVERGED;
            sc->done = 1;
        } else {
            sc->beta = beta;
        }
    }
    if (stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
}

BjView bj_view(const fg_system *S) { return BjView{S->bjA, S->bjB, S->fslot, S->fpart}; }

// Smallest (lowest = true) or largest eigenvalue of the symmetric tridiagonal
// matrix (diag a, off-diagonal b) by bisection on the Sturm count (number of
// eigenvalues below x from the signs of the LDL^T pivots of T - x I).
double tridiag_extreme_eig(const std::vector<double> &a, const std::vector<double> &b, bool lowest)
{
    const size_t m = a.size();
    double lo = a[0], hi = a[0];
    for (size_t j = 0; j < m; ++j) {
        const double rad = (j > 0 ? std::fabs(b[j - 1]) : 0.0) + (j + 1 < m ? std::fabs(b[j]) : 0.0);
        lo = std::min(lo, a[j] - rad);
        hi = std::max(hi, a[j] + rad);
    }
    auto below = [&](double x) {
        size_t cnt = 0;
        double dj = a[0] - x;
        for (size_t j = 0;;) {
            if (dj == 0.0) dj = -1e-300;
            if (dj < 0.0) ++cnt;
            if (++j == m) break;
            dj = a[j] - x - b[j - 1] * b[j - 1] / dj;
        }
        return cnt;
    };
    const size_t target = lowest ? 1 : m;  // x is above the eigenvalue once below(x) reaches this count
    for (int k = 0; k < 200 && hi - lo > 1e-15 * std::max(std::fabs(hi), std::fabs(lo)); ++k) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) >= target)
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b)
{
    return tridiag_extreme_eig(a, b, false);
}

// Lanczos matrix (diagonal a, off-diagonal b) of `steps` block-Jacobi CG steps on
// the probe vector for the current K (Saad, Sec. 6.7.3).  Uses the Chebyshev work
// vectors and wz; fewer steps if r.z vanishes first.
fg_status bj_lanczos(fg_system *S, int steps, std::vector<double> &a, std::vector<double> &b, hipStream_t st)
{
    const int64_t n = 3 * S->Npad;
    double *r = S->chd, *z = S->chs, *q = S->chq, *p = S->wz;
    const BjView m = bj_view(S);
    LAUNCH(k_ch_probe, (3 * S->N + WG - 1) / WG, WG, st, 3 * S->N, q);
    perm_in(S, 3, q, r, st);
    vmask(n, S->dir_u, r, st);
    LAUNCH(k_ch_bj<double>, grid_elems(S->Npad), WG, st, S->Npad, m, r, z);
    hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    double rho = 0;
    {
        const double *A[1] = {r}, *B[1] = {z};
        vdots(S, n, 1, A, B, &rho, st);
    }
    std::vector<double> al, be;
    for (int j = 0; j < steps && rho > 0.0; ++j) {
        spmv(S, FG_K, p, q, st);
        double pq = 0;
        {
            const double *A[1] = {p}, *B[1] = {q};
            vdots(S, n, 1, A, B, &pq, st);
        }
        if (!(std::isfinite(pq) && pq > 0.0)) {
            set_error("fg_pcg_solve: K is not SPD (p.Kp <= 0 in the spectrum estimate of the Chebyshev preconditioner)");
            return FG_ERR_BREAKDOWN;
        }
        const double alpha = rho / pq;
        vaxpby(n, -alpha, q, 1.0, r, st);
        LAUNCH(k_ch_bj<double>, grid_elems(S->Npad), WG, st, S->Npad, m, r, z);
        double rho2 = 0;
        {
            const double *A[1] = {r}, *B[1] = {z};
            vdots(S, n, 1, A, B, &rho2, st);
        }
        al.push_back(alpha);
        be.push_back(rho2 / rho);
        rho = rho2;
        vaxpby(n, 1.0, z, be.back(), p, st);
    }
    fg_status e = check_hip("chebyshev estimate");
    if (e) return e;
    if (al.empty()) {
        set_error("fg_pcg_solve: the probe vector of the Chebyshev spectrum estimate vanished (all DOFs fixed?)");
        return FG_ERR_BREAKDOWN;
    }
    a.assign(al.size(), 0.0);
    b.assign(al.size(), 0.0);
    for (size_t j = 0; j < al.size(); ++j) {
        a[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
        b[j] = std::sqrt(be[j]) / al[j];
    }
    return FG_OK;
}

// Interval [lo, hi] for the current K from cheb_lanczos block-Jacobi CG steps on
// the probe vector.
fg_status cheb_estimate(fg_system *S, hipStream_t st)
{
    std::vector<double> a, b;
    fg_status e = bj_lanczos(S, S->cheb_lanczos, a, b, st);
    if (e) return e;
    const double top = tridiag_max_eig(a, b);
    if (!(std::isfinite(top) && top > 0.0)) {
        set_error("fg_pcg_solve: the Chebyshev spectrum estimate is not positive and finite");
        return FG_ERR_NAN;
    }
    S->cheb_hi = 1.1 * top;
    S->cheb_lo = S->cheb_hi / S->cheb_ratio;
    S->cheb_epoch = S->bj_epoch;
    return FG_OK;
}

}  // namespace

void bj_apply(fg_system *S, const double *in, double *out, hipStream_t st)
{
    LAUNCH(k_ch_bj<double>, grid_elems(S->Npad), WG, st, S->Npad, bj_view(S), in, out);
}

void bj_smooth(fg_system *S, int step, int acc, double inv_theta, double c1, double c2, const double *b,
               const double *kd, double *d, double *x, hipStream_t st)
{
    LAUNCH(k_bj_smooth<double>, grid_elems(S->Npad), WG, st, S->Npad, step, acc, bj_view(S), inv_theta, c1, c2, b, kd,
           d, x);
}

void bj_smooth(fg_system *S, int step, int acc, double inv_theta, double c1, double c2, const float *b,
               const float *kd, float *d, float *x, hipStream_t st)
{
    const BjViewT<float> m{S->bjA32, S->bjB32, S->fslot, S->fpart};
    LAUNCH(k_bj_smooth<float>, grid_elems(S->Npad), WG, st, S->Npad, step, acc, m, (float)inv_theta, (float)c1,
           (float)c2, b, kd, d, x);
}

fg_status cheb_interval_ready(fg_system *S, hipStream_t st)
{
    bj_ready(S, st);
    if (S->bj_singular) {
        set_error("fg_pcg_solve: a diagonal or fault-pair block of K is singular (block Jacobi)");
        return FG_ERR_BREAKDOWN;
    }
    if (S->cheb_epoch == S->bj_epoch) return FG_OK;
    return cheb_estimate(S, st);
}

fg_status lanczos_bounds(fg_system *S, int steps, double *lo, double *hi, hipStream_t st)
{
    bj_ready(S, st);
    if (S->bj_singular) {
        set_error("fg_lanczos_bounds: a diagonal or fault-pair block of K is singular (block Jacobi)");
        return FG_ERR_BREAKDOWN;
    }
    std::vector<double> a, b;
    fg_status e = bj_lanczos(S, steps, a, b, st);
    if (e) return e;
    *lo = tridiag_extreme_eig(a, b, true);
    *hi = tridiag_extreme_eig(a, b, false);
    if (!(std::isfinite(*lo) && std::isfinite(*hi) && *hi > 0.0)) {
        set_error("fg_lanczos_bounds: the Ritz values are not finite and positive");
        return FG_ERR_NAN;
    }
    return FG_OK;
}

fg_status cheb_cg(fg_system *S, const double *b, double *x, double tol, int64_t maxit, int check_every, int64_t *iters,
                  double *relres, hipStream_t st)
{
    *iters = 0;
    *relres = 0;
    fg_status e = cheb_interval_ready(S, st);
    if (e) return e;
    const int64_t n = 3 * S->Npad;
    const BjView m = bj_view(S);
    const double theta = 0.5 * (S->cheb_hi + S->cheb_lo), delta = 0.5 * (S->cheb_hi - S->cheb_lo);
    const double sigma = theta / delta;
    // Chebyshev step coefficients: rho_k = 1/(2 sigma - rho_{k-1}), c1 = rho_k rho_{k-1}, c2 = 2 rho_k / delta
    std::vector<double> c1, c2;
    {
        double rho = 1.0 / sigma;
        for (int k = 1; k < S->cheb_degree; ++k) {
            const double rho1 = 1.0 / (2.0 * sigma - rho);
            c1.push_back(rho1 * rho);
            c2.push_back(2.0 * rho1 / delta);
            rho = rho1;
        }
    }
    CgScalars init{};
    init.maxit = maxit;
    hipMemcpyAsync(S->sc, &init, sizeof init, hipMemcpyHostToDevice, st);
    hipMemcpyAsync(S->wr, b, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    const int64_t gu = grid_vec(S->Npad);
    int64_t gs = 0;
    auto precond = [&](int par, int first) {
        LAUNCH(k_ch_update, gu, WG, st, S->Npad, par, first, (int)c1.empty(), m, 1.0 / theta, S->wx, S->wr, S->wp,
               S->wq, S->chd, S->wz, S->partials, S->npartials, gs, S->sc);
        for (size_t k = 0; k < c1.size(); ++k) {
            cg_spmv_k(S, S->chd, S->chq, st);
            LAUNCH(k_ch_step, gu, WG, st, S->Npad, (int)(k == 0), (int)(k + 1 == c1.size()), m, c1[k], c2[k], S->wr,
                   S->chq, S->chd, S->chs, S->wz, S->partials, S->npartials, S->sc);
        }
    };
    precond(0, 1);
    LAUNCH(k_ch_pupdate, grid_vec(n), WG, st, n, 0, 1, tol, S->wz, S->wp, S->partials, S->npartials, gu, S->sc);
    e = check_hip("chebyshev cg init");
    if (e) return e;
    const int batch = check_every > 0 ? (check_every + 1) / 2 * 2 : 32;
    for (;;) {
        hipMemcpyAsync(S->sc_host, S->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, st);
        hipStreamSynchronize(st);
        e = check_hip("chebyshev cg poll");
        if (e) return e;
        if (S->sc_host->done) break;
        for (int it = 0; it < batch; ++it) {
            const int par = it & 1;  // batches have an even length: iteration k has parity k & 1
            gs = cg_spmv_k(S, S->wp, S->wq, st);
            precond(par, 0);
            LAUNCH(k_ch_pupdate, grid_vec(n), WG, st, n, par, 0, tol, S->wz, S->wp, S->partials, S->npartials, gu,
                   S->sc);
        }
    }
    hipMemcpyAsync(x, S->wx, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    const CgScalars &h = *S->sc_host;
    *iters = h.iters;
    *relres = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    if (h.status == FG_ERR_BREAKDOWN) set_error("fg_pcg_solve: CG breakdown (p.Ap <= 0): operator not SPD");
    if (h.status == FG_ERR_NAN) set_error("fg_pcg_solve: NaN or Inf in the CG iteration");
    return h.status;
}

}  // namespace fg
