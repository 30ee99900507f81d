// The exact interface tangent K_t + N and a Krylov solver for it.
//
// The Newton tangent K_t keeps the symmetric part of the slip tangent; at a slip
// point the return map of Sec. 2.2.1 also makes the shear traction's magnitude
// f t'_n follow the normal opening, d t_s / d delta_n = -f k_n tau, a term that is
// not symmetric.  Its global form N (nonzero on the fault rows only) is
//   (N x)_a = +-sum_q w N_a(q) (-f k_n tau_q) (n . jump(x)(q))  on the + / - lip,
// the transpose of the N^T product of the adjoint.  K_t + N is solved by BiCGStab
// (van der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992) with the K_t preconditioner
// (point or block Jacobi, or a V-cycle of the AMG hierarchy of K_t) applied on the
// right.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fg_device.h"
#include "fg_kernels.h"

namespace fg {

namespace {

// barycentric weight of vertex a at interior Gauss point q
__device__ __forceinline__ double bary(int q, int a) { return q == a ? 2.0 / 3.0 : 1.0 / 6.0; }

// N x, step 1: per point s_q = n . jump(x)(q), held DOFs read as zero.
__global__ void k_n_qp(int64_t nq, const int32_t *__restrict__ coh, const double *__restrict__ geo,
                       const double *__restrict__ x, const uint8_t *__restrict__ dir_u, double *qpS)
{
    const int64_t iq = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (iq >= nq) return;
    const int64_t t = iq / 3;
    const int q = (int)(iq - 3 * t);
    const int32_t *c = coh + 6 * t;
    const double *nv = geo + 10 * t + 1;
    double s = 0;
    for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r) {
            const int64_t ip = 3 * (int64_t)c[a] + r, im = 3 * (int64_t)c[3 + a] + r;
            s += nv[r] * bary(q, a) * ((dir_u[ip] ? 0.0 : x[ip]) - (dir_u[im] ? 0.0 : x[im]));
        }
    qpS[iq] = s;
}

// N x, step 2: per fault row, y += +-sum over incident elements and points of
// w N_a(q) s_q (-f k_n tau_q); held DOFs unchanged.
__global__ void k_n_rows(int64_t nfr, const int32_t *__restrict__ frows, const int32_t *__restrict__ fadj_ptr,
                         const int32_t *__restrict__ fadj, const double *__restrict__ geo,
                         const double *__restrict__ qpS, const double *__restrict__ qpNs,
                         const uint8_t *__restrict__ dir_u, double *y)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nfr) return;
    const int64_t row = frows[k];
    double acc[3] = {0, 0, 0};
    for (int m = fadj_ptr[k]; m < fadj_ptr[k + 1]; ++m) {
        const int64_t t = fadj[m] / 6;
        const int la = fadj[m] % 6, va = la % 3;
        const double w = (la < 3 ? 1.0 : -1.0) * geo[10 * t] / 3.0;
        for (int q = 0; q < 3; ++q) {
            const int64_t iq = 3 * t + q;
            const double cq = w * bary(q, va) * qpS[iq];
            for (int r = 0; r < 3; ++r) acc[r] += cq * qpNs[3 * iq + r];
        }
    }
    for (int r = 0; r < 3; ++r)
        if (!dir_u[3 * row + r]) y[3 * row + r] += acc[r];
}

// N^T x, step 1: per point s_q = (-f k_n tau_q) . jump(x)(q), held DOFs read as zero.
__global__ void k_nt_jump(int64_t nq, const int32_t *__restrict__ coh, const double *__restrict__ qpNs,
                          const double *__restrict__ x, const uint8_t *__restrict__ dir_u, double *qpS)
{
    const int64_t iq = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (iq >= nq) return;
    const int64_t t = iq / 3;
    const int q = (int)(iq - 3 * t);
    const int32_t *c = coh + 6 * t;
    double s = 0;
    for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r) {
            const int64_t ip = 3 * (int64_t)c[a] + r, im = 3 * (int64_t)c[3 + a] + r;
            s += qpNs[3 * iq + r] * bary(q, a) * ((dir_u[ip] ? 0.0 : x[ip]) - (dir_u[im] ? 0.0 : x[im]));
        }
    qpS[iq] = s;
}

// N^T x, step 2: per fault row, y += +-sum over incident elements and points of
// w N_a(q) s_q n; held DOFs unchanged.
__global__ void k_nt_rows_add(int64_t nfr, const int32_t *__restrict__ frows, const int32_t *__restrict__ fadj_ptr,
                              const int32_t *__restrict__ fadj, const double *__restrict__ geo,
                              const double *__restrict__ qpS, const uint8_t *__restrict__ dir_u, double *y)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nfr) return;
    const int64_t row = frows[k];
    double acc[3] = {0, 0, 0};
    for (int m = fadj_ptr[k]; m < fadj_ptr[k + 1]; ++m) {
        const int64_t t = fadj[m] / 6;
        const int la = fadj[m] % 6, va = la % 3;
        const double w = (la < 3 ? 1.0 : -1.0) * geo[10 * t] / 3.0;
        double sw = 0;
        for (int q = 0; q < 3; ++q) sw += w * bary(q, va) * qpS[3 * t + q];
        for (int r = 0; r < 3; ++r) acc[r] += sw * geo[10 * t + 1 + r];
    }
    for (int r = 0; r < 3; ++r)
        if (!dir_u[3 * row + r]) y[3 * row + r] += acc[r];
}

// Device-resident scalars of one BiCGStab solve, kept after the work vectors in
// S->bx.  rho (rh.r) is kept per iteration parity: the kernel that forms the new
// value reads the current slot and writes the other.
struct BiScalars {
    double rho[2];
    double alpha, omega;
    double rr, bb, tol2;
    int64_t iters, maxit;
    int32_t done, status;
};
static_assert(sizeof(BiScalars) <= BX_TAIL * sizeof(double), "BiCGStab scalars exceed their room");

// x = 0, r = rh = b, p = v = 0; partials of rh.r and r.r (rows 2, 3); scalars reset.
__global__ __launch_bounds__(WG) void k_bi_init(int64_t n, int64_t maxit, const double *__restrict__ b,
                                                double *__restrict__ x, double *__restrict__ r,
                                                double *__restrict__ rh, double *__restrict__ p,
                                                double *__restrict__ v, double *partials, int64_t stride,
                                                BiScalars *sc)
{
    double acc[2] = {0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double bi = b[i];
        x[i] = 0.0;
        r[i] = bi;
        rh[i] = bi;
        p[i] = 0.0;
        v[i] = 0.0;
        acc[0] += bi * bi;
    }
    acc[1] = acc[0];
    block_partials<2>(acc, partials + 2 * stride, stride);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rho[0] = sc->rho[1] = 1.0;
        sc->alpha = sc->omega = 1.0;
        sc->rr = sc->bb = sc->tol2 = 0.0;
        sc->iters = 0;
        sc->maxit = maxit;
        sc->done = 0;
        sc->status = FG_OK;
    }
}

// Top of an iteration: rho' = rh.r and r.r from rows 2, 3; the stop tests in the
// order NaN, ||r|| <= tol ||b||, iteration cap, breakdown (rho' or omega zero);
// beta = (rho'/rho)(alpha/omega), p = r + beta (p - omega v).
__global__ __launch_bounds__(WG) void k_bi_p(int64_t n, int par, int first, double tol, const double *__restrict__ r,
                                             double *__restrict__ p, const double *__restrict__ v,
                                             const double *partials, int64_t stride, int64_t nparts, BiScalars *sc)
{
    if (__syncthreads_or(sc->done)) return;
    double tot[2];
    finalize_sum<2>(partials + 2 * stride, stride, nparts, tot);
    const double rho1 = tot[0], rr = tot[1];
    const double tol2 = first ? tol * tol * rr : sc->tol2;
    const double omega = sc->omega;
    const bool finite = isfinite(rho1) && isfinite(rr);
    const bool conv = rr <= tol2;
    const bool capped = sc->iters >= sc->maxit;
    const bool broken = rho1 == 0.0 || omega == 0.0;
    const bool stop = !finite || conv || capped || broken;
    const double beta = (rho1 / sc->rho[par]) * (sc->alpha / omega);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (first) {
            sc->bb = rr;
            sc->tol2 = tol2;
        }
        sc->rr = rr;
        sc->rho[par ^ 1] = rho1;
        if (stop) {
            sc->status = !finite ? FG_ERR_NAN : conv ? FG_OK : capped ? FG_NOT_CONVERGED : FG_ERR_BREAKDOWN;
            sc->done = 1;
        }
    }
    if (stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// Partials of a.b (row 0).
__global__ __launch_bounds__(WG) void k_bi_dot(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                                               double *partials, int64_t stride)
{
    double acc[1] = {0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc[0] += a[i] * b[i];
    block_partials<1>(acc, partials, stride);
}

// alpha = rho' / (rh.v) from row 0; s = r - alpha v.
__global__ __launch_bounds__(WG) void k_bi_s(int64_t n, int par, const double *__restrict__ r,
                                             const double *__restrict__ v, double *__restrict__ s,
                                             const double *partials, int64_t stride, int64_t nparts, BiScalars *sc)
{
    if (__syncthreads_or(sc->done)) return;
    double tot[1];
    finalize_sum<1>(partials, stride, nparts, tot);
    const double rv = tot[0];
    const bool ok = isfinite(rv) && rv != 0.0;
    const double alpha = sc->rho[par ^ 1] / rv;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (ok) {
            sc->alpha = alpha;
        } else {
            sc->status = isfinite(rv) ? FG_ERR_BREAKDOWN : FG_ERR_NAN;
            sc->done = 1;
        }
    }
    if (!ok) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s[i] = r[i] - alpha * v[i];
}

// Partials of t.s and t.t (rows 0, 1).
__global__ __launch_bounds__(WG) void k_bi_dot2(int64_t n, const double *__restrict__ t, const double *__restrict__ s,
                                                double *partials, int64_t stride)
{
    double acc[2] = {0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ti = t[i];
        acc[0] += ti * s[i];
        acc[1] += ti * ti;
    }
    block_partials<2>(acc, partials, stride);
}

// omega = (t.s)/(t.t) from rows 0, 1; x += alpha ph + omega sh, r = s - omega t;
// partials of rh.r and r.r for the next iteration (rows 2, 3).
__global__ __launch_bounds__(WG) void k_bi_xr(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                              const double *__restrict__ ph, const double *__restrict__ sh,
                                              const double *__restrict__ s, const double *__restrict__ t,
                                              const double *__restrict__ rh, double *partials, int64_t stride,
                                              int64_t nparts, BiScalars *sc)
{
    if (__syncthreads_or(sc->done)) return;
    double tot[2];
    finalize_sum<2>(partials, stride, nparts, tot);
    const bool ok = isfinite(tot[0]) && isfinite(tot[1]) && tot[1] != 0.0;
    const double omega = tot[0] / tot[1], alpha = sc->alpha;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (ok) {
            sc->omega = omega;
            sc->iters += 1;
        } else {
            sc->status = (isfinite(tot[0]) && isfinite(tot[1])) ? FG_ERR_BREAKDOWN : FG_ERR_NAN;
            sc->done = 1;
        }
    }
    if (!ok) return;
    double acc[2] = {0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * ph[i] + omega * sh[i];
        const double ri = s[i] - omega * t[i];
        r[i] = ri;
        acc[0] += rh[i] * ri;
        acc[1] += ri * ri;
    }
    block_partials<2>(acc, partials + 2 * stride, stride);
}

__global__ void k_dmul(int64_t n, const double *__restrict__ d, const double *__restrict__ x, double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = d[i] * x[i];
}

// y = M^-1 x with the K_t preconditioner of the single-vector solves (f32: the V-cycle
// in FP32).
void precond(fg_system *S, const double *x, double *y, bool f32, hipStream_t st)
{
    const int64_t n = 3 * S->Npad;
    if (S->k_precond == 3 && f32)
        amg_apply32(S, x, y, st);
    else if (S->k_precond == 3)
        amg_apply(S, x, y, st);
    else if (S->k_precond)
        bj_apply(S, x, y, st);
    else
        LAUNCH(k_dmul, grid_elems(n), WG, st, n, S->dinvK, x, y);
}

}  // namespace

void apply_N_add(fg_system *S, const double *x, double *y, hipStream_t st)
{
    if (S->nq == 0) return;
    LAUNCH(k_n_qp, (S->nq + WG - 1) / WG, WG, st, S->nq, S->coh, S->tri_geo, x, S->dir_u, S->qpS);
    LAUNCH(k_n_rows, (S->nfr + WG - 1) / WG, WG, st, S->nfr, S->frows, S->fadj_ptr, S->fadj, S->tri_geo, S->qpS,
           S->qpNs, S->dir_u, y);
}

void apply_NT_add(fg_system *S, const double *x, double *y, hipStream_t st)
{
    if (S->nq == 0) return;
    LAUNCH(k_nt_jump, (S->nq + WG - 1) / WG, WG, st, S->nq, S->coh, S->qpNs, x, S->dir_u, S->qpS);
    LAUNCH(k_nt_rows_add, (S->nfr + WG - 1) / WG, WG, st, S->nfr, S->frows, S->fadj_ptr, S->fadj, S->tri_geo, S->qpS,
           S->dir_u, y);
}

void spmv_exact(fg_system *S, const double *x, double *y, bool transposed, hipStream_t st)
{
    spmv(S, FG_K, x, y, st);
    if (transposed)
        apply_NT_add(S, x, y, st);
    else
        apply_N_add(S, x, y, st);
}

fg_status bicgstab_exact(fg_system *S, const double *b, double *x, double tol, int64_t maxit, bool transposed,
                         int64_t *iters, double *relres, hipStream_t st, bool f32)
{
    const int64_t n = 3 * S->Npad;
    *iters = 0;
    *relres = 0;
    if (S->k_precond == 3) {   // the V-cycle of the symmetric tangent (amg_ready checks the blocks)
        const fg_status e = f32 ? amg_ready_f32(S, st) : amg_ready(S, st);
        if (e) return e;
    } else if (S->k_precond) {
        bj_ready(S, st);
        if (S->bj_singular) {
            set_error("fg_exact_solve: a diagonal or fault-pair block of K is singular (block Jacobi)");
            return FG_ERR_BREAKDOWN;
        }
    }
    if (!S->bx) {
        set_error("fg_exact_solve: BiCGStab work vectors not allocated");
        return FG_ERR_STATE;
    }
    // r, p, v share CG's work vectors; the caller's b and x are none of these
    double *r = S->wr, *p = S->wp, *v = S->wq;
    double *rh = S->bx, *ph = S->bx + n, *s = S->bx + 2 * n, *sh = S->bx + 3 * n, *t = S->bx + 4 * n;
    BiScalars *sc = (BiScalars *)(S->bx + 5 * n);
    double *part = S->partials;
    const int64_t stride = S->npartials, gv = grid_vec(n);
    LAUNCH(k_bi_init, gv, WG, st, n, maxit, b, x, r, rh, p, v, part, stride, sc);
    fg_status e = check_hip("fg_exact_solve init");
    if (e) return e;
    BiScalars h{};
    // the kernels stop at the device's flag, the preconditioner does not: with the
    // V-cycle (two per iteration) the flag is read after every iteration
    const int batch = S->k_precond == 3 ? 1 : 16;
    for (int64_t k = 0;;) {
        for (int j = 0; j < batch; ++j, ++k) {
            const int par = (int)(k & 1);
            LAUNCH(k_bi_p, gv, WG, st, n, par, (int)(k == 0), tol, r, p, v, part, stride, gv, sc);
            precond(S, p, ph, f32, st);
            spmv_exact(S, ph, v, transposed, st);
            LAUNCH(k_bi_dot, gv, WG, st, n, rh, v, part, stride);
            LAUNCH(k_bi_s, gv, WG, st, n, par, r, v, s, part, stride, gv, sc);
            precond(S, s, sh, f32, st);
            spmv_exact(S, sh, t, transposed, st);
            LAUNCH(k_bi_dot2, gv, WG, st, n, t, s, part, stride);
            LAUNCH(k_bi_xr, gv, WG, st, n, x, r, ph, sh, s, t, rh, part, stride, gv, sc);
        }
        hipMemcpyAsync(&h, sc, sizeof h, hipMemcpyDeviceToHost, st);
        hipStreamSynchronize(st);
        e = check_hip("fg_exact_solve poll");
        if (e) return e;
        if (h.done) break;
    }
    *iters = h.iters;
    *relres = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    if (h.status == FG_ERR_NAN) set_error("fg_exact_solve: NaN or Inf in the BiCGStab iteration");
    if (h.status == FG_ERR_BREAKDOWN) set_error("fg_exact_solve: BiCGStab breakdown (rh.r, rh.v, t.t or omega vanished)");
    return h.status;
}

}  // namespace fg
