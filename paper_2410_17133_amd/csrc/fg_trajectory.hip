// Adjoint through the inelastic slip carried from step to step of a time loop.
//
// Each implicit step maps the start-of-step slip die_old to die_new = Phi(U, die_old)
// by the return map of Sec. 2.2.1 (eq. plastic_slip_increment, eq. corrector) at every
// interface point, and its interface force reads die_old through the trial traction.
// A reverse sweep over the steps therefore needs, per point, the transposed
// derivatives of Phi and of the force with respect to die_old:
//   gU    = (dPhi/dU)^T a_new                         (joins the step's dJ/dU)
//   a_old = (dPhi/ddie_old)^T a_new - (df_coh/ddie_old)^T lam_u
// a_new is the adjoint of the slip the step produced, lam_u the step's displacement
// multipliers.  In the point frame (n, t1, t2), with opening d = (d_n, d_s), trial
// traction t_tr = k_s (t'_s0/k_s + d_s - die_old), t'_n = k_n max(-(d_n - t'_n0/k_n), 0),
// c = f t'_n / |t_tr| and P = I - tau tau^T (tau = t_tr / |t_tr|):
//   stick:  ddie/ddie_old = I,     ddie/dd_s = 0,         ddie/dd_n = 0,
//           dt_s/ddie_old = -k_s I
//   slip:   ddie/ddie_old = c P,   ddie/dd_s = I - c P,   ddie/dd_n = -(f/k_s) tau dt'_n/dd_n,
//           dt_s/ddie_old = -k_s c P
// (open points take the slip branch with t'_n = 0).
#include <hip/hip_runtime.h>

#include <cmath>

#include "fg_device.h"
#include "fg_kernels.h"

namespace fg {

namespace {

// barycentric weight of vertex a at interior Gauss point q (2/3 on the diagonal)
__device__ __forceinline__ double bary(int q, int a) { return q == a ? 2.0 / 3.0 : 1.0 / 6.0; }

// Per point: the global vector (dPhi/d jump)^T a_new (scattered by the row kernel)
// and a_old.  geo per triangle: area, n, t1, t2.
__global__ void k_slip_adj_qp(int64_t nq, const int32_t *__restrict__ coh, const double *__restrict__ geo,
                              const double *__restrict__ U, const double *__restrict__ die_old,
                              const double *__restrict__ t0, const fg_params *__restrict__ gprm,
                              const int32_t *__restrict__ sgrp, const double *__restrict__ a_new,
                              const double *__restrict__ lam, const uint8_t *__restrict__ dir_u, double *qpG,
                              double *a_old)
{
    const int64_t iq = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (iq >= nq) return;
    const int64_t t = iq / 3;
    const int q = (int)(iq - 3 * t);
    const int32_t *c = coh + 6 * t;
    const double *g = geo + 10 * t;
    const fg_params &prm = gprm[sgrp[c[0] / SLICE]];
    const double kn = prm.k_n, ks = prm.k_s, fr = prm.friction;
    double jmp[3] = {0, 0, 0}, lj[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        const double w = bary(q, a);
        for (int r = 0; r < 3; ++r) {
            const int64_t ip = 3 * (int64_t)c[a] + r, im = 3 * (int64_t)c[3 + a] + r;
            jmp[r] += w * (U[ip] - U[im]);
            if (lam) lj[r] += w * ((dir_u[ip] ? 0.0 : lam[ip]) - (dir_u[im] ? 0.0 : lam[im]));
        }
    }
    const double *nv = g + 1, *e1 = g + 4, *e2 = g + 7;
    const double dn = nv[0] * jmp[0] + nv[1] * jmp[1] + nv[2] * jmp[2];
    const double d1 = e1[0] * jmp[0] + e1[1] * jmp[1] + e1[2] * jmp[2];
    const double d2 = e2[0] * jmp[0] + e2[1] * jmp[1] + e2[2] * jmp[2];
    const double *tz = t0 + 3 * iq, *dio = die_old + 2 * iq, *an = a_new + 2 * iq;
    const double gap = dn - tz[0] / kn;
    const double tn = gap < 0.0 ? -kn * gap : 0.0;
    const double dtn = gap < 0.0 ? -kn : 0.0;
    const double tr1 = tz[1] + ks * (d1 - dio[0]), tr2 = tz[2] + ks * (d2 - dio[1]);
    const double trn = sqrt(tr1 * tr1 + tr2 * tr2);
    // stick defaults
    double Dn[2] = {0, 0};                      // ddie/dd_n
    double Ds[2][2] = {{0, 0}, {0, 0}};         // ddie/dd_s
    double Do[2][2] = {{1, 0}, {0, 1}};         // ddie/ddie_old
    double To[2][2] = {{-ks, 0}, {0, -ks}};     // dt_s/ddie_old
    if (trn - fr * tn > 0.0) {
        const double u[2] = {tr1 / trn, tr2 / trn};
        const double cc = fr * tn / trn;
        for (int i = 0; i < 2; ++i) {
            Dn[i] = -(fr / ks) * u[i] * dtn;
            for (int j = 0; j < 2; ++j) {
                const double Pij = (i == j ? 1.0 : 0.0) - u[i] * u[j];
                Ds[i][j] = (i == j ? 1.0 : 0.0) - cc * Pij;
                Do[i][j] = cc * Pij;
                To[i][j] = -ks * cc * Pij;
            }
        }
    }
    if (qpG) {
        // local (ddie/dd)^T a_new, then back to the global frame
        const double ln = Dn[0] * an[0] + Dn[1] * an[1];
        const double l1 = Ds[0][0] * an[0] + Ds[1][0] * an[1];
        const double l2 = Ds[0][1] * an[0] + Ds[1][1] * an[1];
        for (int r = 0; r < 3; ++r) qpG[3 * iq + r] = ln * nv[r] + l1 * e1[r] + l2 * e2[r];
    }
    if (a_old) {
        const double w = g[0] / 3.0;
        const double ls1 = e1[0] * lj[0] + e1[1] * lj[1] + e1[2] * lj[2];
        const double ls2 = e2[0] * lj[0] + e2[1] * lj[1] + e2[2] * lj[2];
        for (int j = 0; j < 2; ++j)
            a_old[2 * iq + j] = Do[0][j] * an[0] + Do[1][j] * an[1] - w * (To[0][j] * ls1 + To[1][j] * ls2);
    }
}

// gU per fault row: +-sum over incident elements and points of N_a(q) qpG_q (+ lip, - lip).
__global__ void k_slip_adj_rows(int64_t nfr, const int32_t *__restrict__ frows, const int32_t *__restrict__ fadj_ptr,
                                const int32_t *__restrict__ fadj, const double *__restrict__ qpG,
                                const uint8_t *__restrict__ dir_u, double *gU)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nfr) return;
    const int64_t row = frows[k];
    double acc[3] = {0, 0, 0};
    for (int m = fadj_ptr[k]; m < fadj_ptr[k + 1]; ++m) {
        const int64_t t = fadj[m] / 6;
        const int la = fadj[m] % 6, va = la % 3;
        const double sg = la < 3 ? 1.0 : -1.0;
        for (int q = 0; q < 3; ++q) {
            const double cq = sg * bary(q, va);
            for (int r = 0; r < 3; ++r) acc[r] += cq * qpG[3 * (3 * t + q) + r];
        }
    }
    for (int r = 0; r < 3; ++r) gU[3 * row + r] = dir_u[3 * row + r] ? 0.0 : acc[r];
}

}  // namespace

void slip_adjoint(fg_system *S, const double *U_int, const double *die_old, const double *t0, const double *a_new,
                  const double *lam_int, double *gU_int, double *a_old, hipStream_t st)
{
    if (gU_int) vfill(gU_int, 0.0, 3 * S->Npad, st);
    if (S->nq == 0) return;
    LAUNCH(k_slip_adj_qp, (S->nq + WG - 1) / WG, WG, st, S->nq, S->coh, S->tri_geo, U_int, die_old, t0, S->gprm,
           S->slice_group, a_new, lam_int, S->dir_u, gU_int ? S->qpT : nullptr, a_old);
    if (gU_int)
        LAUNCH(k_slip_adj_rows, (S->nfr + WG - 1) / WG, WG, st, S->nfr, S->frows, S->fadj_ptr, S->fadj, S->qpT,
               S->dir_u, gU_int);
}

}  // namespace fg
