// Launchers of the libfg device kernels (implemented in fg_kernels.hip).
#pragma once

#include "fg_internal.h"

namespace fg {

// caller order <-> internal order
void perm_in(const fg_system *S, int bs, const double *nat, double *in, hipStream_t st);
void perm_out(const fg_system *S, int bs, const double *in, double *nat, hipStream_t st);
void perm_in_u8(const fg_system *S, int bs, const uint8_t *nat, uint8_t *in, hipStream_t st);

// assembly: the per-tetrahedron slot table (once per mesh), then every assembly
fg_status tet_slots(fg_system *S, hipStream_t st);
void assemble_all(fg_system *S, const double *E, const double *logk, hipStream_t st);
void refresh_k32(fg_system *S, hipStream_t st);
void stick_tangent(fg_system *S, hipStream_t st);

// interface
void cohesive_qp(fg_system *S, const double *U_int, const double *die_n, const double *t0, double *trac,
                 double *die, uint8_t *flag, hipStream_t st);
void cohesive_rows(fg_system *S, double *fcoh_int, int write_tangent, hipStream_t st);

// adjoint: y = N^T x (slip part of the exact interface tangent, last interface update)
void apply_NT(fg_system *S, const double *x, double *y, hipStream_t st);
// dJ/dE and dJ/dln k per tetrahedron (caller order) from the state and the multipliers,
// written, or added to dE / dlogk with accumulate
void slip_adjoint(fg_system *S, const double *U_int, const double *die_old, const double *t0, const double *a_new,
                  const double *lam_int, double *gU_int, double *a_old, hipStream_t st);
void sensitivity(fg_system *S, const double *U, const double *P, const double *lu, const double *lp, double *dE,
                 double *dlogk, const double *logk, bool accumulate, hipStream_t st);

// coupling products, internal order, masked on both sides
void apply_Apu(fg_system *S, const double *p, double *out, hipStream_t st);
void apply_Aup(fg_system *S, const double *u, double *out, hipStream_t st);

// products: which in {FG_K, FG_A22, FG_KBULK, FG_C}
void spmv(fg_system *S, int which, const double *x, double *y, hipStream_t st);
void spmv_k32(fg_system *S, const float *x, float *y, hipStream_t st);

// vector helpers (internal order, n elements)
void vfill(double *y, double v, int64_t n, hipStream_t st);
// y = a*x + b*y
void vaxpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t st);
void vscale(int64_t n, double a, double *y, hipStream_t st);  // y = a y
// y[i] = mask[i] ? 0 : y[i]
void vmask(int64_t n, const uint8_t *mask, double *y, hipStream_t st);
// red[slot+k] = dot(a_k, b_k) for k < nd; synchronous result in host[0..nd)
void vdots(fg_system *S, int64_t n, int nd, const double *const *a, const double *const *b, double *host,
           hipStream_t st);

// CG on internal-order vectors.  bs = 3 (K) or 1 (A22).  The right-hand side
// must already be in S->wr (FP64) or S->fr (FP32); the solution is left in
// S->wx / S->fx.  Returns the final status and fills iters/relres.
// Mixed-precision K solve with reliable updates (FP32 CG, FP64 residual replacement).
fg_status cg_reliable(fg_system *S, const double *b, double *x, double tol, int64_t maxit, int check_every,
                      double delta, int64_t *iters, int64_t *updates, double *relres, hipStream_t st);
fg_status cg_run(fg_system *S, int which, int precision, double tol, int64_t maxit, int check_every,
                 int64_t *iters, double *relres, hipStream_t st);

// Block-Jacobi data of the current K (built on first use after K changed), and its
// FP32 copy for FP32 CG.
void bj_ready(fg_system *S, hipStream_t st);
void bj_ready32(fg_system *S, hipStream_t st);
// q = K p with the CG product kernel (reads the stop flag of S->sc; partials of
// p.q in row 0 of S->partials); returns the number of partials.
int64_t cg_spmv_k(fg_system *S, const double *p, double *q, hipStream_t st);

// Chebyshev-over-block-Jacobi PCG on K (fg_cheb.hip): b, x internal order.
fg_status cheb_cg(fg_system *S, const double *b, double *x, double tol, int64_t maxit, int check_every, int64_t *iters,
                  double *relres, hipStream_t st);
// Spectrum interval of the Chebyshev preconditioner for the current K (estimated if stale).
fg_status cheb_interval_ready(fg_system *S, hipStream_t st);
// Smallest and largest Ritz values of `steps` block-Jacobi CG steps on the probe vector.
fg_status lanczos_bounds(fg_system *S, int steps, double *lo, double *hi, hipStream_t st);
// Smoothed-aggregation AMG (fg_amg.hip): hierarchy for the current K (symbolic part
// once per mesh, numeric part when K changed), PCG with its V-cycle on internal
// vectors (f32: the cycle on FP32 copies of every level inside the FP64 CG), and
// release.
fg_status amg_ready(fg_system *S, hipStream_t st);
fg_status amg_pcg(fg_system *S, const double *b, double *x, double tol, int64_t maxit, bool f32, int64_t *iters,
                  double *relres, hipStream_t st);
void amg_apply(fg_system *S, const double *r, double *z, hipStream_t st);   // one FP64 V-cycle
fg_status amg_ready_f32(fg_system *S, hipStream_t st);                      // hierarchy and its FP32 copies
void amg_apply32(fg_system *S, const double *r, double *z, hipStream_t st); // one FP32 V-cycle
void amg_destroy(fg_system *S);
void amg_levels(const fg_system *S, int *nlev, int64_t *nodes);  // nodes[6]
fg_status amg_aggregates(const fg_system *S, int level, int32_t *out);  // host out, level's nodes
// out = M^-1 in with the block-Jacobi data (bj_ready first).
void bj_apply(fg_system *S, const double *in, double *out, hipStream_t st);
// One step of the AMG cycle's level-0 smoother (degree-2 Chebyshev over block Jacobi),
// FP64 or FP32 (the FP32 copy of the blocks: bj_ready32 first).  step 0:
// d = M^-1 b * inv_theta, x = d (acc: x += d); step 1, kd = K d:
// x += c2 M^-1 (b - kd) + c1 d.
void bj_smooth(fg_system *S, int step, int acc, double inv_theta, double c1, double c2, const double *b,
               const double *kd, double *d, double *x, hipStream_t st);
void bj_smooth(fg_system *S, int step, int acc, double inv_theta, double c1, double c2, const float *b,
               const float *kd, float *d, float *x, hipStream_t st);

// Length of S->bx: five BiCGStab work vectors and room for its device scalars.
constexpr int64_t BX_TAIL = 16;
inline int64_t bx_len(const fg_system *S) { return 15 * S->Npad + BX_TAIL; }

// Exact interface tangent (fg_exact.hip): y += N x or y += N^T x (slip part of the
// last interface update), y = (K_t + N) x or (K_t + N^T) x, and BiCGStab on
// either (internal order).
void apply_N_add(fg_system *S, const double *x, double *y, hipStream_t st);
void apply_NT_add(fg_system *S, const double *x, double *y, hipStream_t st);
void spmv_exact(fg_system *S, const double *x, double *y, bool transposed, hipStream_t st);
// f32 (with "k_precond" 3): the V-cycle preconditioner in FP32.
fg_status bicgstab_exact(fg_system *S, const double *b, double *x, double tol, int64_t maxit, bool transposed,
                         int64_t *iters, double *relres, hipStream_t st, bool f32 = false);

// float <-> double conversions with a scale: y = (T)(s * x)
void to_f32(int64_t n, double s, const double *x, float *y, hipStream_t st);
// y += s * (double)x
void add_f32(int64_t n, double s, const float *x, double *y, hipStream_t st);

fg_status check_hip(const char *where);

// Destroy the captured CG batches (after a change of launch parameters).
void drop_graphs(fg_system *S);

// Block solves of many right-hand sides on K (fg_block.hip).
fg_status block_solve(fg_system *S, int nrhs, const double *b, double *x, int precision, double tol, int64_t maxit,
                      int check_every, fg_pcg_info *info, hipStream_t st);
fg_status mr_reserve(fg_system *S, int nrhs);
void drop_mr_graphs(fg_system *S);

// Batched systems (fg_group.hip): per-group CG with the right-hand side in
// S->wr / S->fr and the solution left in S->wx / S->fx, as cg_run.
fg_status cg_run_grouped(fg_system *S, int which, int precision, double tol, int64_t maxit, int check_every,
                         int64_t *iters, double *relres, hipStream_t st);
fg_status cg_reliable_grouped(fg_system *S, const double *rhs, double *x, double tol, int64_t maxit, int check_every,
                              double delta, int64_t *iters, int64_t *updates, double *worst_rel, hipStream_t st);
void group_norms(fg_system *S, int bs, const double *a, double *host, hipStream_t st);
void group_to_f32(fg_system *S, const double *scale, const double *x, float *y, hipStream_t st);
void group_add_f32(fg_system *S, const double *scale, const float *x, double *y, hipStream_t st);
void drop_group_graphs(fg_system *S);

// Device address of the allocation-free solve's scratch on `device` (fg_noalloc.hip);
// called once per device by fg_ctx_create.
fg_status noalloc_init(int device);

}  // namespace fg
