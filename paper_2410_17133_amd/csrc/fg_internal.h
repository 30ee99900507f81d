// Internal declarations shared by the libfg sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fg.h"

namespace fg {

// Rows per slice of the sliced block-ELL storage: one wavefront, one row per lane.
constexpr int SLICE = 64;
constexpr int WG = 256;  // threads per workgroup in most kernels
constexpr int MAX_GROUPS = 64;  // independent instances of one batched system

// Result of planning a mesh on the host (see fg_system_create).
struct Plan {
    int64_t N = 0, Npad = 0, nslices = 0, nblk_pad = 0, npairs = 0;
    int64_t ne = 0, nf = 0;
    std::vector<int32_t> perm;       // [Npad] internal row -> caller node, -1 for padding rows
    std::vector<int32_t> iperm;      // caller node -> internal row
    std::vector<int64_t> slice_ptr;  // [nslices+1] first block of each slice
    std::vector<int32_t> col;        // [nblk_pad] internal column node, padding = own row
    std::vector<uint8_t> rowlen;     // [Npad]
    std::vector<int32_t> diag_slot;  // [Npad] slot of the diagonal block, -1 for padding rows
    std::vector<int64_t> halo_ptr;   // [nslices+1] first halo entry of each slice
    std::vector<int32_t> halo;       // sorted distinct columns of each slice
    std::vector<uint16_t> lcol;      // [nblk_pad] column as an index into the slice's halo
    int64_t halo_max = 0;
    int ngroups = 1;
    std::vector<int64_t> group_slice_ptr;  // [ngroups+1] slice range of each group
    std::vector<int32_t> slice_group;      // [nslices]
    std::vector<int32_t> tets;       // [ne*4] internal node ids, grouped by colour
    std::vector<int32_t> tet_orig;   // [ne] caller index of each grouped tetrahedron
    std::vector<int64_t> colour_ptr; // [ncolours+1]
    std::vector<int32_t> coh;        // [nf*6] internal node ids, caller order
    std::vector<int32_t> frows;      // internal rows of interface nodes, ascending
    std::vector<int32_t> fadj_ptr;   // [nfr+1]
    std::vector<int32_t> fadj;       // 6*t + local vertex (0..5) of each incident interface element
    std::vector<int32_t> fslot;      // [Npad] index into frows, -1 for rows off the interface
    std::vector<int32_t> fpart;      // [nfr] internal row of the other lip's node at the same point, -1 if none
    std::vector<uint8_t> dir_u;      // [3*Npad] internal order, padding rows 0
    std::vector<double> xyz;         // [3*Npad] coordinates, internal order (host copy; AMG set-up)
    std::vector<uint8_t> dir_p;      // [Npad]
};

// Builds the plan; returns FG_OK or an error with a message in `err`.
fg_status build_plan(const fg_mesh &m, Plan &P, std::string &err);

// Per-solve scalars of a CG iteration, kept in device memory so that the
// iteration never returns to the host.
// Scalars of one device-resident CG.  rho and the iteration count are kept per
// iteration parity: the kernel that produces the next value reads the current
// slot and writes the other, so no block reads a slot another block of the
// same kernel writes.
struct CgScalars {
    double rho[2];    // r.z of the current iterate, by parity
    double pq;        // p.Ap
    double rr;        // r.r
    double bb;        // b.b
    double alpha, beta;
    double tol2;      // tol^2 * b.b
    int64_t iter[2];  // iterations done, by parity
    int64_t iters;    // iterations done (for the host)
    double rho_cur;   // rho of the iterate at which the stop test ended the iteration
    int64_t maxit;
    int32_t done, status;
};

void set_error(const std::string &msg);

struct AmgData;  // smoothed-aggregation hierarchy (fg_amg.hip)

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    int iters = 0, nrhs = 0, tile = 0;
};

// Per-column scalars of the block (many right-hand sides) CG.
constexpr int MR_MAX = 64;
struct MrScalars {
    double rho[MR_MAX], pq[MR_MAX], rr[MR_MAX], bb[MR_MAX], alpha[MR_MAX], beta[MR_MAX], tol2[MR_MAX];
    int64_t iter[MR_MAX];
    int32_t done[MR_MAX], status[MR_MAX];
    int32_t upd[MR_MAX];  // column advanced by this iteration's alpha (x += alpha p is still due)
    // Block CG with residual replacement: a column is ready for the next replacement
    // once r.r <= tol2 and keeps iterating (instead of idling while the block
    // product still costs the same) until r.r <= soft2 = overrun2 tol2.
    // overrun2 = 1 (plain block CG): ready and done coincide.
    double soft2[MR_MAX];
    int32_t ready[MR_MAX];
    double overrun2;
    int64_t maxit;
    int32_t nrhs, pad;
};

}  // namespace fg

// Opaque objects of the C-ABI.
struct fg_ctx {
    int device = 0;
    int n_cu = 0;
};

struct fg_system {
    fg_ctx *ctx = nullptr;
    int device = 0;  // own copy: the system may outlive its context object
    fg::Plan plan;  // host copy (sizes, colours, permutation)
    int64_t N = 0, Npad = 0, nslices = 0, nblk = 0, ne = 0, nf = 0, nq = 0, nfr = 0;
    int ncolours = 0;
    bool assembled = false;
    fg_params prm{};                   // group 0's parameters (the time step is shared by all groups)
    fg_params *gprm = nullptr;         // [ngroups] per-group parameters on the device
    // device graph
    int64_t *slice_ptr = nullptr;
    int32_t *col = nullptr;
    uint8_t *rowlen = nullptr;
    int max_rowlen = 0;         // longest row (stored blocks)
    int32_t *diag_slot = nullptr;
    int32_t *perm = nullptr;  // [Npad] internal -> caller, -1 for padding rows
    int ngroups = 1;
    int32_t *slice_group = nullptr;  // [nslices]
    int64_t *group_slice_ptr = nullptr;
    fg::MrScalars *gsc = nullptr, *gsc_host = nullptr;  // per-group CG scalars
    double *gpart = nullptr;                             // per-slice partials [2][nslices]
    double *gred = nullptr, *gred_host = nullptr;        // [MAX_GROUPS]
    fg::GraphCache g_graph[3];
    std::vector<int64_t> grp_iters;   // per-group results of the last solve (fg_group_stats)
    std::vector<double> grp_relres;
    std::vector<int> grp_status;
    int64_t *halo_ptr = nullptr;
    int32_t *halo = nullptr;
    uint16_t *lcol = nullptr;
    int halo_cap = 0;         // largest halo staged in LDS; larger slices gather from global memory
    // device mesh (internal numbering)
    double *xyz = nullptr;
    int32_t *tets = nullptr, *tet_orig = nullptr;
    uint8_t *tslot = nullptr;   // [ne*16] slot of block (a, b) of each grouped tetrahedron in row a
    int64_t *rinc_ptr = nullptr; // [Npad+1] per row, its range of rinc
    uint32_t *rinc = nullptr;   // [6 * 4ne] per row, in increasing element order: the element's 4 nodes, its caller index, the 4 slots of the row
    int32_t *coh = nullptr;
    int32_t *frows = nullptr, *fadj_ptr = nullptr, *fadj = nullptr;
    int32_t *fslot = nullptr, *fpart = nullptr;  // fault-pair map (block-Jacobi preconditioner of K)
    double *bjA = nullptr;      // [Npad*6] symmetric 3x3 inverse blocks, xx yy zz yz xz xy
    double *bjB = nullptr;      // [nfr*9] pair coupling blocks of the inverse, row-major
    double *wz = nullptr;       // [3*Npad] z = M^-1 r of the block-preconditioned CG
    float *bjA32 = nullptr, *bjB32 = nullptr, *wz32 = nullptr;  // FP32 copies (FP32 CG of the mixed mode)
    bool bj32_valid = false;
    bool bj_valid = false;      // bjA/bjB built from the current K
    bool bj_singular = false;   // the last build met a singular block
    int k_precond = 0;          // fg_tune "k_precond": 0 point Jacobi, 1 nodal + fault-pair block Jacobi,
                                // 2 Chebyshev polynomial over block Jacobi (FP64 single-system K solves)
    int64_t bj_epoch = 0;       // builds of bjA/bjB so far
    double *chd = nullptr, *chs = nullptr, *chq = nullptr;  // [3*Npad] Chebyshev d, s and K d
    int cheb_degree = 4;        // fg_tune "cheb_degree": degree of the Chebyshev polynomial
    int cheb_ratio = 300;       // fg_tune "cheb_ratio": lower end of the interval = upper end / ratio
    int cheb_lanczos = 40;      // fg_tune "cheb_lanczos": CG steps of the spectrum estimate
    double cheb_lo = 0, cheb_hi = 0;  // interval of the last estimate
    int64_t cheb_epoch = -1;    // bj_epoch of the last estimate
    int exact_tangent = 0;      // fg_tune "exact_tangent": FP64 K solves of the forward path on K_t + N
    fg::AmgData *amg = nullptr; // "k_precond" 3: the smoothed-aggregation hierarchy (symbolic part once per mesh)
    int64_t amg_coarse = 64;    // fg_tune "amg_coarse": coarsening stops at this many nodes
    double *bx = nullptr;       // [5*3*Npad] BiCGStab work vectors (rh, ph, s, sh, t)
    uint8_t *dir_u = nullptr, *dir_p = nullptr;
    double *tri_geo = nullptr;  // [nf*10]: area, n[3], t1[3], t2[3]
    // operators
    double *K = nullptr;        // [nblk*9] tangent stiffness, sliced block-ELL
    float *K32 = nullptr;       // [nblk*9] FP32 copy (mixed precision)
    double *Kfb = nullptr;      // [nfr*maxw*9] bulk blocks of interface rows
    int fault_w = 0;            // slots saved per interface row
    double *A22 = nullptr;      // [nblk]
    double *Cm = nullptr;       // [nblk] conductivity
    double *dinvK = nullptr;    // [3*Npad]
    float *dinvK32 = nullptr;   // [3*Npad]
    double *dinvA = nullptr;    // [Npad]
    bool k32_valid = false;
    // interface quadrature-point scratch
    double *qpD = nullptr;      // [nq*6] symmetric global tangent
    double *qpT = nullptr;      // [nq*3] T - T0
    double *qpNs = nullptr;     // [nq*3] -f k_n tau at slip points, else 0 (adjoint)
    double *qpS = nullptr;      // [nq] scratch of the N^T product
    double *adj_trac = nullptr, *adj_die = nullptr;  // [nq*3], [nq*2] scratch of the adjoint's interface update
    uint8_t *adj_flag = nullptr;                      // [nq]
    // solver workspaces (internal order)
    double *wx = nullptr, *wr = nullptr, *wp = nullptr, *wq = nullptr;  // [3*Npad]
    float *fx = nullptr, *fr = nullptr, *fp = nullptr, *fq = nullptr;   // [3*Npad]
    double *v1 = nullptr, *v2 = nullptr, *v3 = nullptr, *v4 = nullptr;  // [3*Npad] scratch
    double *pv1 = nullptr, *pv2 = nullptr;                              // [3*Npad] scratch
    double *ui = nullptr, *ui0 = nullptr, *fi = nullptr, *rm = nullptr, *du = nullptr, *fc = nullptr;  // [3*Npad]
    double *s1 = nullptr, *s2 = nullptr, *s3 = nullptr, *s4 = nullptr, *s5 = nullptr, *s6 = nullptr;  // [Npad]
    double *s7 = nullptr, *s8 = nullptr, *pi = nullptr, *pi0 = nullptr, *qi = nullptr, *rf = nullptr, *dpv = nullptr;
    double *die0 = nullptr;      // [nq*2] start-of-step inelastic slip
    double *partials = nullptr;  // reduction partials
    int64_t npartials = 0;
    fg::CgScalars *sc = nullptr;      // device scalars
    fg::CgScalars *sc_host = nullptr; // pinned host mirror
    double *red = nullptr;            // device reduction results [8]
    double *red_host = nullptr;       // pinned [8]
    uint32_t *red_counter = nullptr;
    // captured CG batches per operator slot: K FP64, K FP32, A22
    bool use_graphs = true;
    bool line_search = true;  // fg_tune "line_search": backtracking on the Newton steps of fg_step
    hipStream_t cap_stream = nullptr;
    fg::GraphCache cg_graph[4];  // K FP64, K FP32, A22, K with FP32 values and FP64 vectors
    // block solves (many right-hand sides), column-interleaved workspaces
    int mr_cap = 0;   // columns allocated
    int spmv_unroll = 2;  // fg_tune "spmv_unroll": slots per unrolled step of the CG product (2, 3, 4, 6)
    int mixed_update = 10;  // fg_tune "mixed_update": FP32 residual reduction between FP64 replacements
    int vec_grid = 512;   // fg_tune "vec_grid": workgroups of the CG vector kernels (512, 1024, 2048)
    int spmv_wpb = 4;     // fg_tune "spmv_wpb": slices (wavefronts) per workgroup of the CG product (1, 2, 4)
    int spmv_nt = 23;     // fg_tune "spmv_nt": access mask of the CG product (nontemporal values 1, indices 2,
                          // halo lists 4, product stores 8; 16 software-pipelined staged rows)
    int mr_tile = 0;  // fg_tune "rhs_tile": 0 = row-group product, else columns per column-tile pass
    int mr_form = 2;  // fg_tune "mr_form": slot-loop form of the row-group product
    double *mx = nullptr, *mr = nullptr, *mp = nullptr, *mq = nullptr, *mb = nullptr, *mx64 = nullptr, *mr64 = nullptr;
    float *mfx = nullptr, *mfr = nullptr, *mfp = nullptr, *mfq = nullptr;
    double *mz = nullptr;  // block-Jacobi z of the block solve (FP64 CG)
    float *mfz = nullptr;  // and of its FP32 CG
    fg::MrScalars *msc = nullptr, *msc_host = nullptr;
    double *mpart = nullptr;
    int64_t mpart_stride = 0;
    double *mred = nullptr, *mred_host = nullptr;
    fg::GraphCache mr_graph[2];  // FP64, FP32
    // live kernel timing (fg_profile)
    bool prof = false;
    std::vector<hipEvent_t> prof_ev[4];  // per operator slot: pairs (start, stop), one per launch of a batch
    int prof_pending = 0;
    int prof_slot = 0;
    int64_t prof_count[4] = {0, 0, 0, 0};
    double prof_ms[4] = {0, 0, 0, 0};
};
