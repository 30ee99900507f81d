// The exact interface tangent K_t + N and a Krylov solver for it.
//
// The Newton tangent K_t keeps the symmetric part of the slip tangent; at a slip
// point the return map of Sec. 2.2.1 also makes the shear traction's magnitude
// f t'_n follow the normal opening, d t_s / d delta_n = -f k_n tau, a term that is
// not symmetric.  Its global form N (nonzero on the fault rows only) is
//   (N x)_a = +-sum_q w N_a(q) (-f k_n tau_q) (n . jump(x)(q))  on the + / - lip,
// the transpose of the N^T product of the adjoint.  K_t + N is solved by BiCGStab
// (van der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992) with the K_t preconditioner
// (point or block Jacobi) applied on the right.
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

__global__ void k_dmul(int64_t n, const double *__restrict__ d, const double *__restrict__ x, double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = d[i] * x[i];
}

// y = M^-1 x with the K_t preconditioner of the single-vector solves.
void precond(fg_system *S, const double *x, double *y, hipStream_t st)
{
    const int64_t n = 3 * S->Npad;
    if (S->k_precond)
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

void spmv_exact(fg_system *S, const double *x, double *y, hipStream_t st)
{
    spmv(S, FG_K, x, y, st);
    apply_N_add(S, x, y, st);
}

fg_status bicgstab_exact(fg_system *S, const double *b, double *x, double tol, int64_t maxit, int64_t *iters,
                         double *relres, hipStream_t st)
{
    const int64_t n = 3 * S->Npad;
    *iters = 0;
    *relres = 0;
    if (S->k_precond) {
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
    auto dots2 = [&](const double *a0, const double *b0, const double *a1, const double *b1, double *h) {
        const double *A[2] = {a0, a1}, *B[2] = {b0, b1};
        vdots(S, n, 2, A, B, h, st);
    };
    vfill(x, 0.0, n, st);
    vfill(p, 0.0, n, st);
    vfill(v, 0.0, n, st);
    hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    hipMemcpyAsync(rh, b, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    double h[2];
    dots2(b, b, b, b, h);
    const double bn = std::sqrt(h[0]);
    if (!std::isfinite(bn)) {
        set_error("fg_exact_solve: NaN or Inf in the right-hand side");
        return FG_ERR_NAN;
    }
    if (bn == 0.0) return check_hip("fg_exact_solve");
    double rho = 1, alpha = 1, omega = 1;
    int64_t it = 0;
    fg_status status = FG_OK;
    for (;;) {
        dots2(rh, r, r, r, h);
        const double rho1 = h[0], rel = std::sqrt(h[1]) / bn;
        *relres = rel;
        if (!std::isfinite(rho1) || !std::isfinite(rel)) {
            set_error("fg_exact_solve: NaN or Inf in the BiCGStab iteration");
            status = FG_ERR_NAN;
            break;
        }
        if (rel <= tol) break;
        if (it >= maxit) {
            status = FG_NOT_CONVERGED;
            break;
        }
        if (rho1 == 0.0 || omega == 0.0) {
            set_error("fg_exact_solve: BiCGStab breakdown (rho or omega vanished)");
            status = FG_ERR_BREAKDOWN;
            break;
        }
        const double beta = (rho1 / rho) * (alpha / omega);
        vaxpby(n, -omega, v, 1.0, p, st);  // p = r + beta (p - omega v)
        vaxpby(n, 1.0, r, beta, p, st);
        precond(S, p, ph, st);
        spmv_exact(S, ph, v, st);
        dots2(rh, v, rh, v, h);
        if (!std::isfinite(h[0]) || h[0] == 0.0) {
            set_error("fg_exact_solve: BiCGStab breakdown (rh.v vanished or is not finite)");
            status = std::isfinite(h[0]) ? FG_ERR_BREAKDOWN : FG_ERR_NAN;
            break;
        }
        alpha = rho1 / h[0];
        hipMemcpyAsync(s, r, n * sizeof(double), hipMemcpyDeviceToDevice, st);  // s = r - alpha v
        vaxpby(n, -alpha, v, 1.0, s, st);
        precond(S, s, sh, st);
        spmv_exact(S, sh, t, st);
        dots2(t, s, t, t, h);
        if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || h[1] == 0.0) {
            set_error("fg_exact_solve: BiCGStab breakdown (t.t vanished or is not finite)");
            status = (std::isfinite(h[0]) && std::isfinite(h[1])) ? FG_ERR_BREAKDOWN : FG_ERR_NAN;
            break;
        }
        omega = h[0] / h[1];
        vaxpby(n, alpha, ph, 1.0, x, st);  // x += alpha ph + omega sh
        vaxpby(n, omega, sh, 1.0, x, st);
        hipMemcpyAsync(r, s, n * sizeof(double), hipMemcpyDeviceToDevice, st);  // r = s - omega t
        vaxpby(n, -omega, t, 1.0, r, st);
        rho = rho1;
        ++it;
    }
    *iters = it;
    fg_status e = check_hip("fg_exact_solve");
    return e ? e : status;
}

}  // namespace fg
