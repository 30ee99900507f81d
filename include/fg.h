/*
 * fg.h -- C-ABI of libfg, an MI355X (gfx950) implementation of the hot path of
 * the fully implicit flow / geomechanics scheme of Gallyamov et al., "A
 * Parallelized 3D Geomechanical Solver for Fluid-induced Fault Slip in
 * Poroelastic Media" (arXiv 2410.17133): the assembled linear-tetrahedron
 * poroelastic stiffness with zero-thickness cohesive fault elements, the scalar
 * pressure system with double-node fracture flow, and the preconditioned CG
 * solves that the partitioned (Prevost) iteration runs in every Newton step.
 *
 * Conventions shared by every entry point
 *  - Ownership.  Pointers named *_h are host memory, all others are device
 *    memory on the context's GPU.  Every buffer is owned by the caller; libfg
 *    owns only the opaque fg_ctx / fg_system objects and their workspaces,
 *    freed by the matching *_destroy call.  No call hands out memory the
 *    caller must free.
 *  - Ordering.  Nodes are numbered by the caller; displacement vectors are
 *    node-major [u0x,u0y,u0z,u1x,...] (length 3N), pressure vectors have length
 *    N.  libfg permutes internally; inputs and outputs are always in the
 *    caller's order.  Interface quadrature points are numbered 3*t+q for
 *    cohesive element t and point q of the interior 3-point Gauss rule
 *    (barycentric (2/3,1/6,1/6) and its permutations, weights area/3).
 *  - Mesh.  tets[e*4..e*4+3] are the four vertices of a linear tetrahedron.
 *    coh[t*6..t*6+5] = [+a,+b,+c,-a,-b,-c] is a zero-thickness interface element
 *    (Sec. 3.1.1): the same triangle seen from the + lip and the - lip, with
 *    (x_b-x_a) x (x_c-x_a) pointing from the - lip to the + lip.  That cross
 *    product defines the element normal n; t1 is the unit projection of +z on
 *    the plane (of +x if the plane is horizontal) and t2 = n x t1.  Geometry is
 *    frozen at the reference configuration (small deformation).
 *  - Unknowns.  U and P are the displacement and pressure changes since t = 0
 *    (the initial state is in equilibrium, Sec. 2.1); held DOFs (dir_u, dir_p)
 *    stay zero and are eliminated symmetrically (zero row and column, unit
 *    diagonal).
 *  - Streams.  Every call is ordered on `stream` (a hipStream_t; 0 = the null
 *    stream).  Calls that report scalars (iterations, residuals) synchronise
 *    that stream before returning.
 *  - Errors.  Every call returns an fg_status; on error fg_last_error() returns
 *    a message for the calling thread.  No C++ exception crosses the ABI.
 *    Outputs are unspecified after an error other than FG_NOT_CONVERGED.
 */
#ifndef FG_H
#define FG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int fg_status;
#define FG_OK 0
#define FG_NOT_CONVERGED 1   /* result valid, tolerance not reached within max_iter */
#define FG_ERR_ARG (-1)      /* bad argument: null pointer, size mismatch, malformed mesh */
#define FG_ERR_OOM (-2)      /* device or host allocation failed */
#define FG_ERR_BREAKDOWN (-3) /* CG breakdown: p.Ap <= 0 (matrix not SPD), or a singular preconditioner */
#define FG_ERR_NAN (-4)      /* NaN or Inf met in a residual or a CG scalar */
#define FG_ERR_HIP (-5)      /* HIP runtime error (launch, copy) */
#define FG_ERR_STATE (-6)    /* call out of order (e.g. solve before fg_assemble) */

/* Which operator a solve or product uses. */
#define FG_K 0      /* tangent stiffness K = K_bulk + interface tangent (3 DOFs per node) */
#define FG_A22 1    /* pressure operator A22 = S + dt C (eq. prevost_system) */
#define FG_KBULK 2  /* bulk stiffness only (products and export, not solves) */
#define FG_C 3      /* conductivity C (products and export) */
#define FG_K_EXACT 4 /* exact tangent K_t + N: K plus the slip term the symmetric tangent omits
                 (fg_spmv and fg_exact_solve only) */

/* Arithmetic of a K solve. */
#define FG_F64 0    /* FP64 storage and arithmetic */
#define FG_F32 1    /* FP32 matrix and vectors throughout (no refinement) */
#define FG_MIXED 2  /* FP32 PCG with FP64 residual replacement: whenever the FP32 residual has dropped
                      tenfold, the FP32 solution is added to the FP64 one, b - K x is formed in FP64
                      and replaces the FP32 residual, and CG continues (reliable updates; per
                      column in the block solve, per group on batched systems).  With the AMG
                      preconditioner ("k_precond" 3, see fg_tune): FP64 CG (on the exact tangent:
                      FP64 BiCGStab) whose V-cycle runs in FP32 */
#define FG_MIXED_F32VAL 3  /* inner PCG on the FP32 matrix values with FP64 vectors and arithmetic,
                              FP64 residual and refinement (single right-hand side, unbatched) */

typedef struct fg_ctx fg_ctx;
typedef struct fg_system fg_system;

/* Material, fluid, fault and time-step scalars (SI units).  nu, alpha: Poisson
 * ratio and Biot coefficient (eq. stress); biot_M: Biot modulus (eq.
 * fluid_content); mu: viscosity (eq. darcy_matrix); k_par, k_perp: fault
 * permeabilities along and across the plane, w0: default hydraulic aperture,
 * M_F: fracture Biot modulus, S_F = 1/M_F (eq. flux_decompose_operators,
 * discrete_mass_fracture); k_n, k_s [Pa/m]: normal and shear penalties,
 * friction: Coulomb coefficient (eq. normal_traction, yield_function); dt:
 * backward-Euler step (eq. time_disc). */
typedef struct {
    double nu, alpha, biot_M, mu, k_par, k_perp, w0, M_F, k_n, k_s, friction, dt;
} fg_params;

/* Mesh and boundary masks, all host arrays, copied by fg_system_create. */
typedef struct {
    int64_t n_nodes, n_tets, n_coh;
    const double *xyz_h;     /* [n_nodes*3] coordinates */
    const int32_t *tets_h;   /* [n_tets*4] */
    const int32_t *coh_h;    /* [n_coh*6], may be NULL when n_coh == 0 */
    const uint8_t *dir_u_h;  /* [3*n_nodes], 1 = displacement DOF held at zero */
    const uint8_t *dir_p_h;  /* [n_nodes], 1 = pressure DOF held at zero */
    const int32_t *group_h;  /* [n_nodes] or NULL: instance of each node in a batch of independent
                                problems (0..63); no element may couple two groups */
} fg_mesh;

typedef struct {
    double tol;          /* stop when ||b - A x||_2 <= tol ||b||_2 (K solves: FP64 residual for FG_MIXED) */
    int64_t max_iter;    /* CG iterations (inner iterations in total for FG_MIXED) */
    int precision;       /* FG_F64 / FG_F32 / FG_MIXED / FG_MIXED_F32VAL (K only; A22 solves are FP64) */
    int check_every;     /* iterations between convergence polls by the host (0 = default 32) */
    double inner_tol;    /* FG_MIXED_F32VAL (restarted refinement): relative tolerance of each
                            inner solve (0 = default 1e-4) */
} fg_pcg_opts;

typedef struct {
    int64_t iters;       /* CG iterations performed (sum over refinement cycles) */
    int64_t cycles;      /* FG_MIXED: FP64 residual replacements (or refinement cycles), else 1 */
    double relres;       /* final ||b - A x|| / ||b|| as tracked by the solver */
    int status;          /* same value as returned */
} fg_pcg_info;

/* Statistics of a partitioned solve or a step. */
typedef struct {
    int64_t newton_iters, outer_iters, inner_k_iters, inner_a22_iters;  /* newton_iters: defect iterations for the adjoint */
    double outer_relres;  /* last Prevost ||r||/||r0|| */
    double res_m, res_f;  /* scaled Newton residual norms at exit (fg_step) */
    int status;
    int64_t step_cuts;    /* fg_step: halvings of the Newton step taken by the line search */
} fg_solve_info;

/* Thread-local message of the last failing call ("" if none). */
const char *fg_last_error(void);

/* Create / destroy a context bound to HIP device `device`. */
fg_status fg_ctx_create(fg_ctx **ctx, int device);
fg_status fg_ctx_destroy(fg_ctx *ctx);

/* Plan a mesh: builds the node graph of the tetrahedra and interface elements,
 * a locality-preserving row permutation, the sliced block-ELL storage of 3x3
 * blocks (K) and scalars (A22, C) on that graph, a colouring of the tetrahedra
 * (no two tetrahedra of a colour share a node) and the interface adjacency of
 * fault nodes; uploads everything to the device.  Host work, once per mesh.
 * Errors: FG_ERR_ARG for out-of-range node ids or degenerate interface
 * triangles, FG_ERR_OOM. */
fg_status fg_system_create(fg_ctx *ctx, const fg_mesh *mesh, fg_system **sys);
/* Frees the system's device memory; valid even after its context was destroyed. */
fg_status fg_system_destroy(fg_system *sys);

/* Assemble (Sec. 3.2): K_bulk = sum_e V B^T D(E_e, nu) B (eq. discrete_balance),
 * the storage S = (1/M) int N N plus fracture storage (w0/M_F) int <r><p>,
 * the conductivity C = (k_e/mu) int grad N . grad N plus fracture longitudinal
 * (w0 k_par/mu) int grad<r>.grad<p> and transverse (k_perp/(mu w0)) int [[r]][[p]]
 * (eq. discrete_mass, discrete_mass_fracture), A22 = S + dt C, Dirichlet
 * elimination, and the point-Jacobi diagonals.  K starts as K_bulk plus the
 * stick tangent of the interface.
 * E [n_tets] Young modulus per tetrahedron, log_k [n_tets] natural log of the
 * matrix permeability per tetrahedron (device, caller order).
 * Errors: FG_ERR_ARG (null pointers, non-positive volume). */
fg_status fg_assemble(fg_ctx *ctx, fg_system *sys, const fg_params *params, const double *E, const double *log_k,
                      void *stream);

/* fg_assemble for a batch system (fg_mesh.group_h set) whose instances carry
 * their own parameters: params[g] applies to every element of group g.  The
 * penalties of Sec. 2.2.1 scale with the element size, so instances of different
 * resolution need their own k_n and k_s.  n_params is 1 (all groups share
 * params[0], same as fg_assemble) or the number of groups.  params is host
 * memory, read before the call returns.
 * Errors: FG_ERR_ARG for another n_params or for groups with different dt (the
 * time step enters the host-side flow residual and is shared by the batch). */
fg_status fg_assemble_groups(fg_ctx *ctx, fg_system *sys, const fg_params *params, int n_params, const double *E,
                             const double *log_k, void *stream);

/* Interface update at every quadrature point (Sec. 2.2.1, eq. normal_traction to
 * eq. corrector): opening delta = sum_a N_a (U_a+ - U_a-) resolved on (n,t1,t2);
 * normal traction t'_n = k_n max(-(delta_n - t'_n0/k_n), 0); elastic trial
 * t_tr = k_s (t'_s0/k_s + delta_s - die_n); Coulomb yield F = |t_tr| - f t'_n;
 * if F > 0 a single-step projection with dlambda = F/k_s along t_tr.
 *   U      [3N]   displacement since t = 0
 *   die_n  [nq*2] inelastic slip at the start of the step (t1, t2 components)
 *   t0     [nq*3] initial effective traction (t'_n0, t'_s0 along t1, t2)
 * Out:
 *   trac   [nq*3] (t'_n, t_s1, t_s2);  die [nq*2];  flag [nq] 0 stick, 1 slip, 2 open
 *   f_coh  [3N]   interface force sum_q w_q N_a (T_q - T_0q) on + lips and its
 *                 negative on - lips, T = -t'_n n + t_s1 t1 + t_s2 t2; zero on held DOFs
 * write_tangent != 0 also rewrites the fault rows of K with K_bulk plus the
 * symmetric interface tangent: k_n n(x)n in contact, plus k_s (t1(x)t1 + t2(x)t2)
 * in stick or k_s (f t'_n/|t_tr|)(I_t - tau(x)tau) in slip; zero when open. */
fg_status fg_cohesive_update(fg_ctx *ctx, fg_system *sys, const double *U, const double *die_n, const double *t0,
                             double *trac, double *die, uint8_t *flag, double *f_coh, int write_tangent,
                             void *stream);

/* Point-Jacobi preconditioned CG (Hestenes-Stiefel, Sec. 3.3.2) on `which`
 * (FG_K or FG_A22) from x0 = 0.  b, x: nrhs column vectors, each of length 3N
 * (FG_K) or N (FG_A22), stored one after the other.  precision applies to FG_K.
 * With FG_K and nrhs > 1 (a power of two up to 64) the columns are solved
 * together: independent CG recurrences (own alpha, beta, stop test) advanced in
 * lockstep so that each iteration streams the matrix once per tile of columns
 * (block product); converged columns are masked out.  FG_MIXED replaces each
 * column's FP32 residual by its FP64 one whenever it has dropped by the
 * mixed_update factor (reliable updates, all columns at the same points).
 * Returns FG_OK, FG_NOT_CONVERGED (x holds the last iterate),
 * FG_ERR_BREAKDOWN, FG_ERR_NAN.  info (host) receives the worst column. */
fg_status fg_pcg_solve(fg_ctx *ctx, fg_system *sys, int which, int nrhs, const double *b, double *x,
                       const fg_pcg_opts *opts, fg_pcg_info *info_h, void *stream);

/* fg_pcg_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  One
 * right-hand side, FG_K or FG_A22, FP64, point Jacobi (the paper's; "k_precond"
 * and "exact_tangent" are ignored), kernels launched one by one.  The CG's work
 * memory (device scalars, reduction partials and the x, r, p, q vectors) comes
 * from one fixed 64 MiB array per GPU that the library holds until the process
 * ends; the call allocates nothing and must not be given a solve that needs more
 * (4 vectors of 3N (FG_K) or N (FG_A22) doubles plus the partials: about 2.09 M
 * unknowns), which returns FG_ERR_ARG.  Every call on one GPU shares that array:
 * calls that overlap on one GPU (other threads or streams) race and give wrong
 * results.  Results equal fg_pcg_solve's with the default preconditioner.
 * Arguments, returns and info as fg_pcg_solve (nrhs = 1); opts->precision must
 * be FG_F64 (opts may be NULL: tol 1e-10).  Synchronises the stream. */
fg_status fg_pcg_solve_noalloc(fg_ctx *ctx, fg_system *sys, int which, const double *b, double *x,
                               const fg_pcg_opts *opts, fg_pcg_info *info_h, void *stream);

/* One partitioned solve of the Newton system (eq. linear_system,
 * eq. prevost_system, eq. schur_system):
 *   [ K      -A_pu ] [du]   [b_u]
 *   [ A_up    A22  ] [dp] = [b_p]
 * by CG on the Schur complement A22 + A_up K^-1 A_pu preconditioned with
 * A22^-1, with matrix-free coupling products A_pu p and A_up u = A_pu^T u
 * (Appendix A, Appendix B) and inner Jacobi-PCG solves with K and A22.
 * b_u [3N], b_p [N] in; du [3N], dp [N] out. */
fg_status fg_flow_solve(fg_ctx *ctx, fg_system *sys, const double *b_u, const double *b_p, double *du, double *dp,
                        const fg_pcg_opts *inner_k, const fg_pcg_opts *inner_p, double outer_tol,
                        int64_t outer_max_iter, fg_solve_info *info_h, void *stream);

/* One implicit step (Sec. 3.3, eq. nonlinear_system): Newton on (U, P) from the
 * state at t_n, each iterate with an interface update from die_n and a
 * partitioned solve; residuals in total form
 *   R_m = K_bulk U + f_coh(U) - A_pu P - F_u
 *   R_f = A_up (U - U_n) + A22 (P - P_n) + dt (C P_n - f_p).
 * Stops when ||R_m|| <= tol s_m and ||R_f|| <= tol s_f, with
 * s_m = max(||R_m^0||, ||A_pu P||, ||F_u||) and s_f = max(||R_f^0||, dt ||f_p||).
 * Newton steps are globalised by backtracking (on by default, fg_tune
 * "line_search"): with s* = max(s_m, ||A_pu (P + dP)||) the merit
 * (||R_m||/s*)^2 + (||R_f||/s_f)^2 must drop; step lengths 1, 1/2, ... 1/64 are
 * tried in turn (1/64 is taken if none lowers it).  Full steps overshoot once
 * slip spreads, because the Newton tangent omits the non-symmetric slip term.
 * In/out: U [3N], P [N], die [nq*2] (start-of-step inelastic slip in, final out).
 * Out: trac [nq*3], flag [nq].  In: t0 [nq*3], F_u [3N] total external force
 * change at t_n+1, f_p [N] volumetric sources. */
fg_status fg_step(fg_ctx *ctx, fg_system *sys, double *U, double *P, double *die, double *trac, uint8_t *flag,
                  const double *t0, const double *F_u, const double *f_p, double newton_tol,
                  int64_t newton_max_iter, const fg_pcg_opts *inner_k, const fg_pcg_opts *inner_p,
                  double outer_tol, int64_t outer_max_iter, fg_solve_info *info_h, void *stream);

/* Adjoint of one converged implicit step and the gradient of an objective J(U, P)
 * with respect to the per-tetrahedron Young modulus and log-permeability.  The
 * step's residual R(U, P; E, ln k) = 0 (fg_step) gives dJ/dtheta = -lambda^T dR/dtheta
 * with the multipliers of the transposed Newton Jacobian (Sec. 3.3.1):
 *   [ K_exact^T   A_pu ] [lam_u]   [dJ/dU]
 *   [ -A_up       A22  ] [lam_p] = [dJ/dP]
 * solved as the forward partitioned CG (Sec. 3.3.2) on mu = -lam_u, with the slip
 * part of the exact interface tangent, N = sum w N_a N_b (-f k_n tau (x) n), lagged
 * (defect correction) in refinement form: each iteration computes the true residual
 * of the exact transposed system with the FP64 operators and solves only for the
 * correction with the symmetric tangent, to relative tolerance outer_tol with the
 * inner_k / inner_p solves.  Loose values (outer 0.05, inner 1e-3) make every
 * correction cheap; the accuracy of the result is set by defect_tol, the stop test
 * on the relative change of each multiplier block.  Then
 * dJ/dE_e = -lam_u^T (K_e/E_e) U_e and dJ/dln k_e = -dt lam_p^T C_e P_e.
 * info: newton_iters = defect iterations, outer/inner iterations summed over them,
 * outer_relres = last relative change.
 *   U, P       converged state of fg_step (changes since t = 0), caller order
 *   die_n, t0  the step's start-of-step inelastic slip and initial tractions
 *   log_k      [n_tets] the log-permeability given to fg_assemble
 *   dJdU, dJdP [3N], [N] objective gradient
 * Out: dJ_dE, dJ_dlogk [n_tets] (caller order); lam_u [3N], lam_p [N] (may be NULL).
 * Uses the operators of the last fg_assemble (it must be the step's assembly).
 * Returns FG_NOT_CONVERGED when max_defect_iters is reached. */
fg_status fg_adjoint_solve(fg_ctx *ctx, fg_system *sys, const double *U, const double *P, const double *die_n,
                           const double *t0, const double *log_k, const double *dJdU, const double *dJdP,
                           double *dJ_dE, double *dJ_dlogk, double *lam_u, double *lam_p,
                           const fg_pcg_opts *inner_k, const fg_pcg_opts *inner_p, double outer_tol,
                           double defect_tol, int64_t max_defect_iters, fg_solve_info *info_h, void *stream);

/* Adjoint through the inelastic slip a time loop carries from step to step.  A
 * step maps its start-of-step slip die_old to die_new = Phi(U, die_old) by the
 * return map of Sec. 2.2.1 (eq. plastic_slip_increment, eq. corrector) at every
 * interface point, and its interface force reads die_old through the trial
 * traction (see fg_cohesive_update).  For a reverse sweep over the steps:
 *   gU    = (dPhi/dU)^T a_new                       [3N], added to the step's dJ/dU
 *   a_old = (dPhi/ddie_old)^T a_new - (df_coh/ddie_old)^T lam_u    [nq*2]
 *   U        [3N]   the step's converged displacement (caller order)
 *   die_old  [nq*2] its start-of-step slip;  t0 [nq*3] initial tractions
 *   a_new    [nq*2] adjoint of the slip the step produced
 *   lam_u    [3N]   the step's displacement multipliers (fg_adjoint_solve), or NULL
 *                   (read as zero: a_old then omits the force term)
 * Either output may be NULL (not both).  gU is zero on held DOFs.  Derivatives
 * are taken branch by branch (stick, slip; open points follow the slip branch
 * with zero normal traction), like the step's own tangent.
 * Errors: FG_ERR_ARG, FG_ERR_STATE (before fg_assemble). */
fg_status fg_slip_adjoint(fg_ctx *ctx, fg_system *sys, const double *U, const double *die_old, const double *t0,
                          const double *a_new, const double *lam_u, double *gU, double *a_old, void *stream);

/* One step of the reverse sweep through a time loop of implicit steps (the adjoint
 * of Sec. 3.3.1 carried backwards over the backward-Euler steps of eq. time_disc),
 * for an objective J = sum_n j_n(U_n, P_n).  Going n = T..1, step n solves
 *   J_n^T lam_n = dj_n/dy_n - (dR_{n+1}/dy_n)^T lam_{n+1} + (dPhi_n/dU_n)^T a_n
 * where the next step's flow residual reads y_n = (U_n, P_n) through -A_up U_n and
 * -(A22 - dt C) P_n (fg_step's R_f), so its multipliers add A_pu lam_{n+1,p} to
 * the displacement block and (A22 - dt C) lam_{n+1,p} to the pressure block, and
 * Phi_n is the return map that carries the slip (fg_slip_adjoint).  The system is
 * solved as in fg_adjoint_solve (same options and stop test); then
 *   a_{n-1} = (dPhi_n/ddie_{n-1})^T a_n - (df_coh/ddie_{n-1})^T lam_{n,u}
 * and the step's share -lam_n^T dR_n/dtheta is ADDED to dJ_dE and dJ_dlogk.
 *   U, P, die_old  step n's converged state and its start-of-step slip
 *   t0, log_k      initial tractions and the log-permeability of the assembly
 *   dJdU, dJdP     [3N], [N] dj_n/dU_n, dj_n/dP_n
 *   lam_p_next     [N] lam_{n+1,p} (lam_p of the previous call), NULL for the last step
 *   a              [nq*2] in: a_n (zero for the last step), out: a_{n-1}
 *   dJ_dE, dJ_dlogk [n_tets] accumulated gradient (caller order)
 *   lam_u, lam_p   [3N], [N] out, this step's multipliers (each may be NULL)
 * All device pointers, caller order.  Returns as fg_adjoint_solve; outputs are
 * unspecified after an error. */
fg_status fg_adjoint_loop_step(fg_ctx *ctx, fg_system *sys, const double *U, const double *P, const double *die_old,
                               const double *t0, const double *log_k, const double *dJdU, const double *dJdP,
                               const double *lam_p_next, double *a, double *dJ_dE, double *dJ_dlogk, double *lam_u,
                               double *lam_p, const fg_pcg_opts *inner_k, const fg_pcg_opts *inner_p,
                               double outer_tol, double defect_tol, int64_t max_defect_iters, fg_solve_info *info,
                               void *stream);

/* (K_t + N) x = b: the exact interface tangent.  K_t is the current K (its
 * interface rows written by the last fg_cohesive_update with write_tangent); N is
 * the part of the exact slip tangent that K_t omits, from the point states of
 * the last fg_cohesive_update: at a slip point the return map of Sec. 2.2.1 makes
 * the shear traction's magnitude f t'_n follow the normal opening, d t_s /
 * d delta_n = -f k_n tau, so the force on the + / - lip of an interface element
 * gets +-sum_q (A/3) N_a(q) (-f k_n tau_q)(n . jump(x)(q)) (zero at stick and
 * open points; held DOFs are neither read nor written).  Solved by BiCGStab (van
 * der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992) from x0 = 0 with the K
 * preconditioner chosen by fg_tune "k_precond" (0 point Jacobi, 1 or 2 block
 * Jacobi) applied on the right, stopping on the recursive residual
 * ||r|| <= opts->tol ||b|| (default 1e-10) or after opts->max_iter iterations
 * (two products each).  b, x: [3N] device, caller order.  opts->precision must be
 * FG_F64; check_every and inner_tol are ignored; opts may be NULL.  The
 * iteration's scalars stay in device memory; the host polls every 16 iterations.  info (host, may be NULL): iters,
 * relres (recursive), status.  Returns FG_OK, FG_NOT_CONVERGED, or
 * FG_ERR_BREAKDOWN (rh.r, rh.v, t.t or omega vanished, or a singular block),
 * FG_ERR_NAN, FG_ERR_ARG (also for batched systems), FG_ERR_STATE. */
fg_status fg_exact_solve(fg_ctx *ctx, fg_system *sys, const double *b, double *x, const fg_pcg_opts *opts,
                         fg_pcg_info *info, void *stream);

/* Interval [lo, hi] (host outputs) of the Chebyshev preconditioner of K
 * ("k_precond" 2, see fg_tune) for the current K, estimated now if K changed
 * since the last estimate: hi = 1.1 x the largest Ritz value of the Lanczos
 * matrix that "cheb_lanczos" block-Jacobi CG steps on the probe vector give
 * (Saad, Sec. 6.7.3: T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_j,j+1 =
 * sqrt(beta_j)/alpha_j), lo = hi / "cheb_ratio".  The probe is, per caller-order
 * DOF i, SplitMix64 (Steele, Lea and Flood 2014) of counter i mapped to
 * [-1/2, 1/2) as (z >> 11) 2^-53 - 1/2, zero on held DOFs.  Synchronises the
 * stream.  Errors: FG_ERR_ARG, FG_ERR_STATE (before fg_assemble, or k_precond is
 * not 2), FG_ERR_BREAKDOWN (singular block, K not SPD, or the probe vanished). */
fg_status fg_cheb_interval(fg_ctx *ctx, fg_system *sys, double *lo, double *hi, void *stream);

/* Extreme eigenvalue estimates of the block-Jacobi preconditioned tangent M^-1 K
 * (M as "k_precond" 1): the smallest and largest Ritz values (host outputs) of the
 * Lanczos matrix of `steps` block-Jacobi CG steps on the SplitMix64 probe vector
 * of fg_cheb_interval (Saad, Sec. 6.7.3).  hi / lo estimates the condition
 * number that bounds the forward error of a K solve (the Ritz values lie inside
 * the spectrum, so the estimate is a lower bound).  steps in [2, 100000]; fewer
 * steps are taken if r.z vanishes first.  Synchronises the stream.
 * Errors: FG_ERR_ARG (also for batched systems), FG_ERR_STATE (before
 * fg_assemble), FG_ERR_BREAKDOWN (singular block or K not SPD), FG_ERR_OOM. */
fg_status fg_lanczos_bounds(fg_ctx *ctx, fg_system *sys, int steps, double *lo, double *hi, void *stream);

/* Sizes of the smoothed-aggregation hierarchy of "k_precond" 3 for the current K
 * (built now if needed): *nlev levels, nodes[l] (host, 6 entries) nodes of level
 * l (level 0: the mesh nodes, 3 DOFs each; below: aggregates, 6 DOFs each; unused
 * entries 0).  Synchronises the stream.  Errors: FG_ERR_ARG, FG_ERR_STATE (before
 * fg_assemble, or k_precond is not 3), FG_ERR_BREAKDOWN (singular block or
 * coarsest matrix not SPD), FG_ERR_OOM. */
fg_status fg_amg_levels(fg_ctx *ctx, fg_system *sys, int *nlev, int64_t *nodes, void *stream);

/* The aggregate of every node of level `level` (0 to nlev-2) of that hierarchy
 * (built now if needed): agg (host, int32, nodes[level] entries; level 0 in the
 * caller's node numbering) receives aggregate numbers 0 .. nodes[level+1]-1, the
 * integer output of the aggregation passes.  Synchronises the stream.  Errors:
 * FG_ERR_ARG (level out of range), FG_ERR_STATE (before fg_assemble, or
 * k_precond is not 3), and those of fg_amg_levels. */
fg_status fg_amg_aggregates(fg_ctx *ctx, fg_system *sys, int level, int32_t *agg, void *stream);

/* Products on the assembled system, caller order: y = A x for which in
 * {FG_K, FG_A22, FG_KBULK, FG_C, FG_K_EXACT} (FG_K_EXACT: see fg_exact_solve). */
fg_status fg_spmv(fg_ctx *ctx, fg_system *sys, int which, const double *x, double *y, void *stream);

/* Coupling products (Appendix A eq. Apdp / Adpd, Appendix B eq. afdpd and its
 * transpose): transpose == 0: y[3N] = A_pu x[N]; transpose != 0: y[N] = A_up x[3N],
 * masked on held DOFs on both sides. */
fg_status fg_coupling(fg_ctx *ctx, fg_system *sys, int transpose, const double *x, double *y, void *stream);

/* Residuals R_m [3N], R_f [N] of fg_step's definition at (U, P) given the state
 * at t_n (U_n, P_n), f_coh from fg_cohesive_update, F_u and f_p. */
fg_status fg_residual(fg_ctx *ctx, fg_system *sys, const double *U, const double *P, const double *U_n,
                      const double *P_n, const double *f_coh, const double *F_u, const double *f_p, double *R_m,
                      double *R_f, void *stream);

/* Sizes of the planned storage (host outputs, each may be NULL): stored node
 * pairs of the graph, blocks of the sliced storage including padding, slices
 * of 64 rows, and the total length of the per-slice halo lists (distinct
 * columns of each slice, staged in LDS by the products). */
fg_status fg_system_sizes(const fg_system *sys, int64_t *n_pairs_h, int64_t *n_padded_blocks_h,
                          int64_t *n_slices_h, int64_t *n_halo_h);

/* Export an assembled operator as node-pair blocks in caller order (host
 * arrays of n_pairs entries): rows_h, cols_h node ids; vals_h 9 (K, KBULK,
 * row-major 3x3) or 1 (A22, C) values per pair.  Synchronises the stream. */
fg_status fg_export(fg_ctx *ctx, fg_system *sys, int which, int32_t *rows_h, int32_t *cols_h, double *vals_h,
                    void *stream);

/* Per-group results of the last fg_pcg_solve on a batched system (fg_mesh.group_h):
 * each group is an independent problem with its own CG scalars and stop test.
 * Host arrays of n_groups entries (each may be NULL): CG iterations (summed over
 * refinement cycles), final relative residual, status. */
fg_status fg_group_stats(const fg_system *sys, int64_t *iters_h, double *relres_h, int *status_h, int *n_groups_h);

/* Tuning knobs of the products (the autotuner's search space).
 *   "halo_cap": largest per-slice halo whose x is staged in LDS; slices with a
 *               larger halo gather x from global memory (0 = never stage).
 *               Default: the largest halo, up to 384.  Clipped to what 64 KB
 *               of LDS per 4-wavefront workgroup holds.
 *   "graphs":   1 (default) replays each batch of CG iterations as a captured
 *               HIP graph, 0 launches the kernels one by one (same results).
 *   "line_search": 1 (default) backtracking on the Newton steps of fg_step,
 *               0 full steps.
 *   "k_precond": preconditioner of the single-right-hand-side K solves
 *               (fg_pcg_solve, and the K solves inside fg_flow_solve, fg_step and
 *               fg_adjoint_solve): 0 (default) point Jacobi; 1 block Jacobi, the
 *               inverse of every node's 3x3 diagonal block except that the two
 *               lips' nodes at one interface point share the inverse of their
 *               6x6 block (the penalty stiffness couples them), also in the FP32
 *               CG of FG_F32 and FG_MIXED (FP32 copy of the blocks); 2 as 1, and
 *               FP64 solves are preconditioned by the Chebyshev polynomial over
 *               block Jacobi: z = p(M^-1 K) M^-1 r with 1 - t p(t) the Chebyshev
 *               polynomial of degree "cheb_degree" scaled to the interval
 *               [hi/"cheb_ratio", hi] (Saad, Iterative Methods for Sparse Linear
 *               Systems, Sec. 12.3), hi = 1.1 x the largest Ritz value of
 *               "cheb_lanczos" block-Jacobi CG steps on a fixed SplitMix64 probe
 *               vector (fg_cheb_interval).  Each CG iteration then costs
 *               cheb_degree products with K and reduces twice.  Blocks and
 *               interval are rebuilt after every change of K; FG_ERR_BREAKDOWN if
 *               a block is singular.  Block solves (nrhs > 1) and
 *               batched systems apply the block-Jacobi stage (1 and 2 alike) to
 *               every column / group, in FP64 and in the FP32 CG of FG_F32 /
 *               FG_MIXED; FG_MIXED_F32VAL solves keep point Jacobi.
 *               3: the FP64 single-right-hand-side K solves use CG preconditioned
 *               by a smoothed-aggregation AMG V-cycle (Vanek, Mandel and Brezina,
 *               Computing 56, 1996): aggregates of the node graph (the two lips of
 *               a fault pair together), the six rigid-body modes as near-null
 *               space, prolongator (I - w D^-1 A) P_tent with w = 4/(3 rho), rho
 *               the Gershgorin bound of D^-1 A, Galerkin coarse operators down to
 *               "amg_coarse" nodes (at most 6 levels, the last inverted), and
 *               degree-2 Chebyshev smoothing over block Jacobi (level 0: the
 *               blocks of stage 1 on [hi/30, hi] with hi as for stage 2; below:
 *               6x6 blocks on [rho/30, rho]).  The patterns are built on the host
 *               once per mesh, the values on the GPU after every change of K;
 *               the BiCGStab of fg_exact_solve and of the exact-tangent solves
 *               (see "exact_tangent") is preconditioned by one V-cycle of the
 *               same hierarchy (built on the symmetric tangent K_t; FP32 under
 *               FG_MIXED, its input scaled on the device by a power of two); other
 *               solves behave as with 1.  FG_MIXED single-right-hand-side
 *               K solves run the same FP64 CG with the V-cycle in FP32: every
 *               level's values rounded once per change of K (level 0: K's FP32
 *               copy and the FP32 blocks of stage 1), the cycle's input scaled
 *               to unit norm by the last residual norm and its output scaled
 *               back, and beta = r_{k+1}.(z_{k+1} - z_k) / r_k.z_k, the
 *               flexible form that tolerates the rounding's asymmetry (Golub
 *               and Ye, SIAM J. Sci. Comput. 21, 1999); info.cycles is 1.
 *   "exact_tangent": 1 makes the FP64 K solves inside fg_flow_solve and fg_step
 *               solve the exact tangent K_t + N by BiCGStab (as fg_exact_solve),
 *               so that Newton uses the exact Jacobian of the interface force;
 *               the outer partitioned CG then runs on a Schur complement that
 *               is not exactly symmetric.  0 (default): the symmetric tangent.
 *               fg_adjoint_solve then solves its FP64 corrections with K_t + N^T
 *               (BiCGStab, the transposed exact tangent) instead of the
 *               symmetric tangent: the same multipliers (the refinement runs on
 *               the true residual of the exact transposed system either way) in
 *               fewer corrections.  If a correction breaks down (the Schur
 *               complement of K_t + N^T need not be positive definite at slip
 *               points), it and the later ones use the symmetric tangent.  fg_pcg_solve always uses the symmetric
 *               tangent; mixed-precision K solves stay symmetric, except with
 *               "k_precond" 3, where FG_MIXED solves the exact tangent by FP64
 *               BiCGStab with the V-cycle in FP32.
 *   "cheb_degree": degree of the Chebyshev polynomial, 1 to 16 (default 4;
 *               1 is block Jacobi scaled by 1/theta: same iterates).
 *   "cheb_ratio": hi / lo of the interval, 2 to 1000000 (default 300).
 *   "cheb_lanczos": CG steps of the spectrum estimate, 5 to 500 (default 40).
 *   "amg_coarse": "k_precond" 3 coarsens down to at most this many nodes, 1 to
 *               1000 (default 64).
 *   "spmv_unroll": slots per unrolled step of the CG product: 1, 2 (default),
 *               3, 4 or 6.
 *   "mixed_update": FG_MIXED: factor by which the FP32 residual (of the
 *               solve, a column or a group) must drop before the FP64
 *               residual replaces it: 2 to 100 (default 10).  Longer FP32
 *               phases drift: larger factors multiplied the FP32 iterations
 *               and, at 1000, let an FP32 recurrence diverge.
 *   "vec_grid": workgroups of the CG vector kernels: 512 (default), 1024 or
 *               2048 (each adds the previous kernel's partial sums itself).
 *   "spmv_wpb": slices (one wavefront each) per workgroup of the CG
 *               product: 1, 2 or 4 (default); the slices of a workgroup
 *               share its LDS and its staging barrier.
 *   "spmv_nt":  access mask of the CG product: nontemporal loads of matrix
 *               values (1), column indices (2), halo lists (4), nontemporal
 *               product stores (8), and (16) the next slots' loads issued
 *               before the current ones are used; 0, 1, 3, 7, 15 or 23
 *               (default).  Results are identical for every value.
 *   "rhs_tile": product of the block (many right-hand sides) solve.  0
 *               (default): with 8 or more columns, the columns of a row are
 *               spread over the lanes and the matrix is streamed once per
 *               product (fewer columns: tiles of 8).  1, 2, 4, 8 or 16: one
 *               lane per row with that many columns per pass, the matrix
 *               streamed once per tile.  Results agree to rounding.
 *   "mr_form":  slot loop of the rhs_tile 0 product.  0: one column-index
 *               load per slot.  Otherwise the columns of NR/2 slots are
 *               loaded at once and shared by lane shuffles, and U =
 *               mr_form & 7 (1, 2 or 4) slots' gathers are issued before any
 *               is used (default 2); +8: nontemporal matrix value and column loads;
 *               +16 (U 1 or 2): every lane loads a slot's nine values itself
 *               instead of receiving them by shuffles.  Valid values: 0, 1, 2,
 *               4, 9, 10, 12, 17, 18, 25, 26.  Results are identical for
 *               every value.
 * Returns FG_ERR_ARG for an unknown key or a negative value. */
fg_status fg_tune(fg_system *sys, const char *key, int64_t value);

/* Live timing of the CG product kernel (the hot loop's dominant kernel).
 * enable != 0: CG iterations launch kernel by kernel (no graph replay) and
 * record a timing-only HIP event (no system-scope fence) on the solve's stream
 * before and after each SpMV launch; durations are summed per operator slot:
 * 0 = K in FP64, 1 = K in FP32, 2 = A22, 3 = K with FP32 values and FP64 vectors.
 * fg_profile_read returns the number of
 * timed launches and their total milliseconds for `slot`, and clears the slot
 * when reset != 0. */
fg_status fg_profile(fg_system *sys, int enable);
fg_status fg_profile_read(fg_system *sys, int slot, int64_t *launches_h, double *milliseconds_h, int reset);

#ifdef __cplusplus
}
#endif
#endif /* FG_H */
