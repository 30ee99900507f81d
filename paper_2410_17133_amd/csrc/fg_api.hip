// C-ABI of libfg: object lifetime, drivers of the partitioned solve and of the
// Newton step.  The drivers run on the host and keep every vector on the
// device; only scalars (dot products, CG status) come back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "fg_kernels.h"

namespace fg {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

}  // namespace fg

using namespace fg;

namespace {

// Every entry point first discards a HIP error left pending by other code on
// this thread (torch, the caller), so that check_hip reports only libfg's own
// failures, then makes the context's device current.
struct Guard {
    explicit Guard(int dev)
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) fprintf(stderr, "libfg: discarding a HIP error raised before this call: %s\n", hipGetErrorString(e));
        hipSetDevice(dev);
    }
};

template <class T>
fg_status dalloc(T **p, int64_t n)
{
    *p = nullptr;
    if (n <= 0) n = 1;
    if (hipMalloc((void **)p, sizeof(T) * (size_t)n) != hipSuccess) {
        hipGetLastError();
        set_error("device allocation of " + std::to_string(sizeof(T) * (size_t)n) + " bytes failed");
        return FG_ERR_OOM;
    }
    return FG_OK;
}

template <class T>
fg_status upload(T **p, const std::vector<T> &v)
{
    fg_status e = dalloc(p, (int64_t)v.size());
    if (e) return e;
    if (!v.empty() && hipMemcpy(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("host to device copy failed");
        return FG_ERR_HIP;
    }
    return FG_OK;
}

void dfree(void *p)
{
    if (p) hipFree(p);
}

#define TRY(x)                       \
    do {                             \
        fg_status _e = (x);          \
        if (_e < 0) return _e;       \
    } while (0)

hipStream_t S_(void *s) { return (hipStream_t)s; }

double vnorm(fg_system *S, int64_t n, const double *a, hipStream_t st)
{
    const double *A[1] = {a};
    double r;
    vdots(S, n, 1, A, A, &r, st);
    return std::sqrt(r);
}

double vdot1(fg_system *S, int64_t n, const double *a, const double *b, hipStream_t st)
{
    const double *A[1] = {a}, *B[1] = {b};
    double r;
    vdots(S, n, 1, A, B, &r, st);
    return r;
}

fg_pcg_opts defaults(const fg_pcg_opts *o, double tol)
{
    fg_pcg_opts d{};
    d.tol = tol;
    d.max_iter = 1000000;
    d.precision = FG_F64;
    d.check_every = 32;
    d.inner_tol = 0;
    if (o) {
        d = *o;
        if (d.check_every <= 0) d.check_every = 32;
        if (d.max_iter <= 0) d.max_iter = 1000000;
    }
    // inner solves of the refinement stop at 1e-4: each cycle gains about what the
    // FP32 matrix values allow, with FP32 or FP64 vectors alike
    if (d.inner_tol <= 0) d.inner_tol = 1e-4;
    return d;
}

// Holds the K solves on the symmetric tangent for its lifetime (restores fg_tune
// "exact_tangent" on every return path).
struct SymmetricSolves {
    fg_system *S;
    int saved;
    explicit SymmetricSolves(fg_system *s) : S(s), saved(s->exact_tangent) { S->exact_tangent = 0; }
    ~SymmetricSolves() { S->exact_tangent = saved; }
};

// The adjoint's K solves for its lifetime: K_t + N^T (exact_tangent 2, BiCGStab)
// when fg_tune "exact_tangent" is on, else the symmetric tangent.
struct AdjointSolves {
    fg_system *S;
    int saved;
    explicit AdjointSolves(fg_system *s) : S(s), saved(s->exact_tangent) { S->exact_tangent = saved ? 2 : 0; }
    ~AdjointSolves() { S->exact_tangent = saved; }
};

// K solve on internal vectors: rhs (3 Npad) -> out (3 Npad).
fg_status k_solve(fg_system *S, const double *rhs, double *out, const fg_pcg_opts &o, fg_pcg_info *info, hipStream_t st)
{
    const int64_t n = 3 * S->Npad;
    if (S->k_precond == 3 && !S->exact_tangent && S->ngroups == 1 &&
        (o.precision == FG_F64 || o.precision == FG_MIXED)) {
        // AMG-PCG in FP64; FG_MIXED runs its V-cycle in FP32
        int64_t it = 0;
        double rr = 0;
        fg_status s = amg_pcg(S, rhs, out, o.tol, o.max_iter, o.precision == FG_MIXED, &it, &rr, st);
        if (info) {
            info->iters = it;
            info->cycles = 1;
            info->relres = rr;
            info->status = s;
        }
        return s;
    }
    if (S->k_precond == 3 && S->exact_tangent && S->ngroups == 1 && o.precision == FG_MIXED) {
        // the exact tangent by FP64 BiCGStab with the V-cycle in FP32
        int64_t it = 0;
        double rr = 0;
        fg_status s = bicgstab_exact(S, rhs, out, o.tol, o.max_iter, S->exact_tangent == 2, &it, &rr, st, true);
        if (info) {
            info->iters = it;
            info->cycles = 1;
            info->relres = rr;
            info->status = s;
        }
        return s;
    }
    if (o.precision == FG_F64 || o.precision == FG_F32) {
        int64_t it = 0;
        double rr = 0;
        fg_status s;
        if (o.precision == FG_F64 && S->exact_tangent && S->ngroups == 1) {
            s = bicgstab_exact(S, rhs, out, o.tol, o.max_iter, S->exact_tangent == 2, &it, &rr, st);
        } else if (o.precision == FG_F64 && S->k_precond == 2 && S->ngroups == 1) {
            s = cheb_cg(S, rhs, out, o.tol, o.max_iter, o.check_every, &it, &rr, st);
        } else if (o.precision == FG_F64) {
            hipMemcpyAsync(S->wr, rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st);
            s = cg_run(S, FG_K, FG_F64, o.tol, o.max_iter, o.check_every, &it, &rr, st);
            hipMemcpyAsync(out, S->wx, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        } else {
            to_f32(n, 1.0, rhs, S->fr, st);
            s = cg_run(S, FG_K, FG_F32, o.tol, o.max_iter, o.check_every, &it, &rr, st);
            vfill(out, 0.0, n, st);
            add_f32(n, 1.0, S->fx, out, st);
        }
        if (info) {
            info->iters = it;
            info->cycles = 1;
            info->relres = rr;
            info->status = s;
        }
        return s;
    }
    // FG_MIXED_F32VAL: inner CG on the correction equation with the FP32 matrix and
    // FP64 vectors, FP64 true residual and accumulation (iterative refinement with
    // restarts).
    if (!S->k32_valid) refresh_k32(S, st);
    if (S->ngroups > 1) {
        // every group by reliable updates of its own (FG_MIXED_F32VAL is rejected for groups)
        int64_t it = 0, up = 0;
        double rel = 0;
        fg_status s = cg_reliable_grouped(S, rhs, out, o.tol, o.max_iter, o.check_every, 1.0 / S->mixed_update, &it,
                                          &up, &rel, st);
        if (info) {
            info->iters = it;
            info->cycles = up;
            info->relres = rel;
            info->status = s;
        }
        return s;
    }
    if (o.precision == FG_MIXED) {
        // FP32 CG with reliable updates: the FP64 residual replaces the FP32 one each
        // time the latter has dropped tenfold, and the search direction carries over
        int64_t it = 0, up = 0;
        double rel = 0;
        fg_status s = cg_reliable(S, rhs, S->v3, o.tol, o.max_iter, o.check_every, 1.0 / S->mixed_update, &it, &up,
                                  &rel, st);
        hipMemcpyAsync(out, S->v3, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        if (info) {
            info->iters = it;
            info->cycles = up;
            info->relres = rel;
            info->status = s;
        }
        return s;
    }
    double *x = S->v3, *r = S->v4;
    const double bn = vnorm(S, n, rhs, st);
    vfill(x, 0.0, n, st);
    hipMemcpyAsync(r, rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    int64_t total = 0, cycles = 0;
    double rel = bn > 0 ? 1.0 : 0.0;
    fg_status s = FG_OK;
    while (bn > 0) {
        const double rn = vnorm(S, n, r, st);
        rel = rn / bn;
        if (!std::isfinite(rel)) {
            s = FG_ERR_NAN;
            set_error("fg_pcg_solve: NaN in the mixed-precision residual");
            break;
        }
        if (rel <= o.tol) {
            s = FG_OK;
            break;
        }
        if (total >= o.max_iter || cycles >= 200) {
            s = FG_NOT_CONVERGED;
            break;
        }
        const bool f32vec = o.precision == FG_MIXED;
        if (f32vec) {
            to_f32(n, 1.0 / rn, r, S->fr, st);
        } else {
            hipMemcpyAsync(S->wr, r, n * sizeof(double), hipMemcpyDeviceToDevice, st);
            vscale(n, 1.0 / rn, S->wr, st);
        }
        int64_t it = 0;
        double rr = 0;
        fg_status si = cg_run(S, FG_K, f32vec ? FG_F32 : FG_MIXED_F32VAL, std::max(o.inner_tol, o.tol * bn / rn),
                              o.max_iter - total, o.check_every, &it, &rr, st);
        total += it;
        cycles++;
        if (si < 0) {
            s = si;
            break;
        }
        if (f32vec)
            add_f32(n, rn, S->fx, x, st);
        else
            vaxpby(n, rn, S->wx, 1.0, x, st);
        spmv(S, FG_K, x, S->wq, st);
        hipMemcpyAsync(r, rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        vaxpby(n, -1.0, S->wq, 1.0, r, st);
    }
    hipMemcpyAsync(out, x, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (info) {
        info->iters = total;
        info->cycles = cycles;
        info->relres = rel;
        info->status = s;
    }
    return s;
}

fg_status a_solve(fg_system *S, const double *rhs, double *out, const fg_pcg_opts &o, int64_t *iters, hipStream_t st)
{
    const int64_t n = S->Npad;
    hipMemcpyAsync(S->wr, rhs, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    int64_t it = 0;
    double rr = 0;
    fg_status s = cg_run(S, FG_A22, FG_F64, o.tol, o.max_iter, o.check_every, &it, &rr, st);
    hipMemcpyAsync(out, S->wx, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (iters) *iters += it;
    return s;
}

// Partitioned CG (Sec. 3.3.2) on internal vectors.  b1, x1: 3 Npad; b2, x2: Npad.
fg_status prevost(fg_system *S, const double *b1, const double *b2, double *x1, double *x2, const fg_pcg_opts &ok,
                  const fg_pcg_opts &op, double tol, int64_t maxit, fg_solve_info *info, hipStream_t st)
{
    const int64_t n1 = 3 * S->Npad, n2 = S->Npad;
    double *y = S->v1, *w = S->v2, *t1 = S->pv1;
    double *r = S->s1, *z = S->s2, *zn = S->s3, *d = S->s4, *Sd = S->s5, *t2 = S->s6;
    fg_pcg_info ki{};
    fg_status s = k_solve(S, b1, y, ok, &ki, st);  // y0 = K^-1 b1
    info->inner_k_iters += ki.iters;
    if (s < 0) return s;
    apply_Aup(S, y, t2, st);
    hipMemcpyAsync(r, b2, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
    vaxpby(n2, -1.0, t2, 1.0, r, st);
    vfill(x2, 0.0, n2, st);
    const double r0 = vnorm(S, n2, r, st);
    double rel = 0;
    fg_status st_out = FG_OK;
    if (r0 > 0) {
        s = a_solve(S, r, z, op, &info->inner_a22_iters, st);
        if (s < 0) return s;
        hipMemcpyAsync(d, z, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
        double rz = vdot1(S, n2, r, z, st);
        int64_t outer = 0;
        for (;;) {
            apply_Apu(S, d, t1, st);
            s = k_solve(S, t1, w, ok, &ki, st);  // w = K^-1 A_pu d
            info->inner_k_iters += ki.iters;
            if (s < 0) return s;
            apply_Aup(S, w, t2, st);
            spmv(S, FG_A22, d, Sd, st);
            vaxpby(n2, 1.0, t2, 1.0, Sd, st);
            const double dSd = vdot1(S, n2, d, Sd, st);
            if (!std::isfinite(dSd)) {
                set_error("fg_flow_solve: NaN in the Schur-complement product");
                return FG_ERR_NAN;
            }
            if (!(dSd > 0)) {
                set_error("fg_flow_solve: Schur complement not positive (d.S d <= 0)");
                return FG_ERR_BREAKDOWN;
            }
            const double al = rz / dSd;
            vaxpby(n2, al, d, 1.0, x2, st);
            vaxpby(n2, -al, Sd, 1.0, r, st);
            vaxpby(n1, al, w, 1.0, y, st);
            outer++;
            rel = vnorm(S, n2, r, st) / r0;
            if (rel <= tol) break;
            if (outer >= maxit) {
                st_out = FG_NOT_CONVERGED;
                break;
            }
            s = a_solve(S, r, zn, op, &info->inner_a22_iters, st);
            if (s < 0) return s;
            const double *A[2] = {r, r}, *B[2] = {zn, z};
            double dd[2];
            vdots(S, n2, 2, A, B, dd, st);
            const double be = (dd[0] - dd[1]) / rz;  // flexible (Polak-Ribiere) beta
            vaxpby(n2, 1.0, zn, be, d, st);
            hipMemcpyAsync(z, zn, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
            rz = dd[0];
        }
        info->outer_iters += outer;
    }
    info->outer_relres = rel;
    hipMemcpyAsync(x1, y, n1 * sizeof(double), hipMemcpyDeviceToDevice, st);
    return st_out;
}

// Residuals of the Newton system (internal order).
void residual_int(fg_system *S, const double *U, const double *P, const double *Un, const double *Pn,
                  const double *fcoh, const double *Fu, const double *fp, double *Rm, double *Rf, hipStream_t st)
{
    const int64_t n1 = 3 * S->Npad, n2 = S->Npad;
    double *t1 = S->pv1, *du = S->pv2, *t2 = S->s7, *dp = S->s8;
    spmv(S, FG_KBULK, U, Rm, st);
    apply_Apu(S, P, t1, st);
    vaxpby(n1, 1.0, fcoh, 1.0, Rm, st);
    vaxpby(n1, -1.0, t1, 1.0, Rm, st);
    vaxpby(n1, -1.0, Fu, 1.0, Rm, st);
    vmask(n1, S->dir_u, Rm, st);
    hipMemcpyAsync(du, U, n1 * sizeof(double), hipMemcpyDeviceToDevice, st);
    vaxpby(n1, -1.0, Un, 1.0, du, st);
    hipMemcpyAsync(dp, P, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
    vaxpby(n2, -1.0, Pn, 1.0, dp, st);
    apply_Aup(S, du, Rf, st);
    spmv(S, FG_A22, dp, t2, st);
    vaxpby(n2, 1.0, t2, 1.0, Rf, st);
    spmv(S, FG_C, Pn, t2, st);
    vaxpby(n2, S->prm.dt, t2, 1.0, Rf, st);
    vaxpby(n2, -S->prm.dt, fp, 1.0, Rf, st);
    vmask(n2, S->dir_p, Rf, st);
}

bool ready(fg_system *S)
{
    if (!S || !S->assembled) {
        set_error("call fg_assemble first");
        return false;
    }
    return true;
}

}  // namespace

extern "C" {

const char *fg_last_error(void) { return fg::g_err.c_str(); }

fg_status fg_ctx_create(fg_ctx **ctx, int device)
{
    if (!ctx) {
        set_error("fg_ctx_create: null output");
        return FG_ERR_ARG;
    }
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        hipGetLastError();
        set_error("fg_ctx_create: no such HIP device");
        return FG_ERR_ARG;
    }
    Guard g(device);
    fg_status e = noalloc_init(device);
    if (e) return e;
    fg_ctx *c = new fg_ctx;
    c->device = device;
    hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device);
    *ctx = c;
    return FG_OK;
}

fg_status fg_ctx_destroy(fg_ctx *ctx)
{
    delete ctx;
    return FG_OK;
}

fg_status fg_system_destroy(fg_system *S)
{
    if (!S) return FG_OK;
    Guard g(S->device);
    hipDeviceSynchronize();
    void *ptrs[] = {S->gprm, S->slice_group, S->group_slice_ptr, S->gsc, S->gpart, S->gred, S->halo_ptr, S->halo, S->lcol, S->slice_ptr, S->col, S->rowlen, S->diag_slot, S->perm, S->xyz, S->tets, S->tet_orig, S->tslot, S->rinc_ptr, S->rinc, S->coh,
                    S->frows, S->fadj_ptr, S->fadj, S->dir_u, S->dir_p, S->tri_geo, S->K, S->K32, S->Kfb, S->A22,
                    S->Cm, S->dinvK, S->dinvK32, S->dinvA, S->qpD, S->qpT, S->qpNs, S->qpS, S->adj_trac, S->adj_die, S->adj_flag, S->wx, S->wr, S->wp, S->wq, S->fx,
                    S->fr, S->fp, S->fq, S->v1, S->v2, S->v3, S->v4, S->pv1, S->pv2, S->ui, S->ui0, S->fi, S->rm,
                    S->du, S->fc, S->s1, S->s2, S->s3, S->s4, S->s5, S->s6, S->s7, S->s8, S->pi, S->pi0, S->qi,
                    S->rf, S->dpv, S->die0, S->partials, S->sc, S->red, S->red_counter, S->fslot, S->fpart,
                    S->bjA, S->bjB, S->wz, S->bjA32, S->bjB32, S->wz32, S->chd, S->chs, S->chq, S->bx};
    for (void *p : ptrs) dfree(p);
    drop_graphs(S);
    drop_mr_graphs(S);
    drop_group_graphs(S);
    amg_destroy(S);
    void *mr_ptrs[] = {S->mx, S->mr, S->mp, S->mq, S->mb, S->mx64, S->mr64, S->mz, S->mfx, S->mfr, S->mfp, S->mfq,
                       S->mfz, S->msc, S->mpart, S->mred};
    for (void *p : mr_ptrs) dfree(p);
    if (S->msc_host) hipHostFree(S->msc_host);
    if (S->gsc_host) hipHostFree(S->gsc_host);
    if (S->gred_host) hipHostFree(S->gred_host);
    if (S->mred_host) hipHostFree(S->mred_host);
    if (S->cap_stream) hipStreamDestroy(S->cap_stream);
    for (auto &pool : S->prof_ev)
        for (hipEvent_t ev : pool) hipEventDestroy(ev);
    if (S->sc_host) hipHostFree(S->sc_host);
    if (S->red_host) hipHostFree(S->red_host);
    delete S;
    return FG_OK;
}

fg_status fg_system_create(fg_ctx *ctx, const fg_mesh *mesh, fg_system **out)
{
    if (!ctx || !mesh || !out) {
        set_error("fg_system_create: null argument");
        return FG_ERR_ARG;
    }
    Guard g(ctx->device);
    fg_system *S = new fg_system;
    S->ctx = ctx;
    S->device = ctx->device;
    std::string err;
    fg_status e = build_plan(*mesh, S->plan, err);
    if (e) {
        set_error(err);
        delete S;
        return e;
    }
    const Plan &P = S->plan;
    S->N = P.N;
    S->Npad = P.Npad;
    S->nslices = P.nslices;
    S->nblk = P.nblk_pad;
    S->ne = P.ne;
    S->nf = P.nf;
    S->nq = 3 * P.nf;
    S->nfr = (int64_t)P.frows.size();
    S->ncolours = (int)P.colour_ptr.size() - 1;
    int fw = 0;
    for (int32_t r : P.frows) fw = std::max(fw, (int)P.rowlen[r]);
    S->fault_w = fw;
    const int64_t n1 = 3 * S->Npad, n2 = S->Npad;
#define CK(x)                       \
    do {                            \
        fg_status _e = (x);         \
        if (_e) {                   \
            fg_system_destroy(S);   \
            return _e;              \
        }                           \
    } while (0)
    CK(upload(&S->slice_ptr, P.slice_ptr));
    CK(upload(&S->col, P.col));
    CK(upload(&S->rowlen, P.rowlen));
    CK(upload(&S->diag_slot, P.diag_slot));
    CK(upload(&S->perm, P.perm));
    CK(upload(&S->halo_ptr, P.halo_ptr));
    CK(upload(&S->halo, P.halo));
    CK(upload(&S->lcol, P.lcol));
    // LDS window per wavefront: the largest halo up to 384 nodes (37 KB per 4-wave workgroup of FP64
    // 3-vectors, so that four workgroups share a CU); slices with larger halos gather from memory
    S->halo_cap = (int)std::min<int64_t>(P.halo_max, 384);
    std::vector<double> xyz(3 * S->Npad, 0.0);
    for (int64_t r = 0; r < S->Npad; ++r)
        if (P.perm[r] >= 0)
            for (int c = 0; c < 3; ++c) xyz[3 * r + c] = mesh->xyz_h[3 * (int64_t)P.perm[r] + c];
    S->ngroups = P.ngroups;
    CK(upload(&S->slice_group, P.slice_group));
    CK(upload(&S->group_slice_ptr, P.group_slice_ptr));
    CK(upload(&S->xyz, xyz));
    S->plan.xyz = xyz;
    CK(upload(&S->tets, P.tets));
    CK(upload(&S->tet_orig, P.tet_orig));
    CK(upload(&S->coh, P.coh));
    CK(upload(&S->frows, P.frows));
    CK(upload(&S->fadj_ptr, P.fadj_ptr));
    CK(upload(&S->fadj, P.fadj));
    if (!P.fslot.empty()) CK(upload(&S->fslot, P.fslot));
    if (!P.fpart.empty()) CK(upload(&S->fpart, P.fpart));
    CK(upload(&S->dir_u, P.dir_u));
    CK(upload(&S->dir_p, P.dir_p));
    CK(dalloc(&S->gprm, S->ngroups));
    CK(dalloc(&S->tri_geo, 10 * S->nf));
    CK(dalloc(&S->K, 9 * S->nblk));
    CK(dalloc(&S->K32, 9 * S->nblk));
    CK(dalloc(&S->Kfb, 9 * S->nfr * std::max(fw, 1)));
    CK(dalloc(&S->A22, S->nblk));
    CK(dalloc(&S->Cm, S->nblk));
    CK(dalloc(&S->dinvK, n1));
    CK(dalloc(&S->dinvK32, n1));
    CK(dalloc(&S->dinvA, n2));
    CK(dalloc(&S->qpD, 6 * S->nq));
    CK(dalloc(&S->qpT, 3 * S->nq));
    CK(dalloc(&S->qpNs, 3 * S->nq));
    CK(dalloc(&S->qpS, S->nq));
    CK(dalloc(&S->adj_trac, 3 * S->nq));
    CK(dalloc(&S->adj_die, 2 * S->nq));
    CK(dalloc(&S->adj_flag, S->nq));
    double **d3[] = {&S->wx, &S->wr, &S->wp, &S->wq, &S->v1, &S->v2, &S->v3, &S->v4, &S->pv1, &S->pv2,
                     &S->ui, &S->ui0, &S->fi, &S->rm, &S->du, &S->fc};
    for (double **p : d3) CK(dalloc(p, n1));
    float **f3[] = {&S->fx, &S->fr, &S->fp, &S->fq};
    for (float **p : f3) CK(dalloc(p, n1));
    double **d1[] = {&S->s1, &S->s2, &S->s3, &S->s4, &S->s5, &S->s6, &S->s7, &S->s8,
                     &S->pi, &S->pi0, &S->qi, &S->rf, &S->dpv};
    for (double **p : d1) CK(dalloc(p, n2));
    CK(dalloc(&S->die0, 2 * S->nq));
    S->npartials = 1 << 17;
    CK(dalloc(&S->partials, 4 * S->npartials));
    CK(dalloc(&S->sc, 1));
    CK(dalloc(&S->red, 8));
    CK(dalloc(&S->red_counter, 4));
    hipMemset(S->red_counter, 0, 4 * sizeof(uint32_t));
    hipMemset(S->sc, 0, sizeof(CgScalars));
    S->grp_iters.assign(S->ngroups, 0);
    S->grp_relres.assign(S->ngroups, 0.0);
    S->grp_status.assign(S->ngroups, 0);
    if (dalloc(&S->gsc, 1) || dalloc(&S->gpart, 2 * S->nslices) || dalloc(&S->gred, 2 * MAX_GROUPS) ||
        hipHostMalloc((void **)&S->gsc_host, sizeof(MrScalars)) != hipSuccess ||
        hipHostMalloc((void **)&S->gred_host, MAX_GROUPS * sizeof(double)) != hipSuccess) {
        set_error("allocation of the batched-solve scalars failed");
        fg_system_destroy(S);
        return FG_ERR_OOM;
    }
    S->mpart_stride = std::max<int64_t>((S->nslices + 7) / 8 * 8, 2048) + 8;  // one partial per slice at most
    if (dalloc(&S->mpart, 2 * (int64_t)MR_MAX * S->mpart_stride) || dalloc(&S->msc, 1) || dalloc(&S->mred, 2 * MR_MAX) ||
        hipHostMalloc((void **)&S->msc_host, sizeof(MrScalars)) != hipSuccess ||
        hipHostMalloc((void **)&S->mred_host, MR_MAX * sizeof(double)) != hipSuccess) {
        set_error("allocation of the block-solve scalars failed");
        fg_system_destroy(S);
        return FG_ERR_OOM;
    }
    if (hipStreamCreateWithFlags(&S->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        set_error("stream creation failed");
        fg_system_destroy(S);
        return FG_ERR_HIP;
    }
    if (hipHostMalloc((void **)&S->sc_host, sizeof(CgScalars)) != hipSuccess ||
        hipHostMalloc((void **)&S->red_host, 8 * sizeof(double)) != hipSuccess) {
        set_error("pinned host allocation failed");
        fg_system_destroy(S);
        return FG_ERR_OOM;
    }
#undef CK
    if ((S->nslices + 3) / 4 + 8 > S->npartials) {
        set_error("fg_system_create: mesh too large for the reduction workspace");
        fg_system_destroy(S);
        return FG_ERR_ARG;
    }
    if (dalloc(&S->tslot, 16 * std::max<int64_t>(S->ne, 1))) {
        set_error("fg_system_create: allocation of the tetrahedron slot table failed");
        fg_system_destroy(S);
        return FG_ERR_OOM;
    }
    {
        // row incidence list of the assembly: per internal row, an entry for every
        // element t whose local node a is the row's node, in increasing t; the host
        // leaves 4 t + a in each entry, tet_slots fills in the rest on the device
        if (4 * S->ne >= (int64_t(1) << 32)) {
            set_error("fg_system_create: more than 2^30 tetrahedra");
            fg_system_destroy(S);
            return FG_ERR_ARG;
        }
        const std::vector<int32_t> &T = S->plan.tets;
        for (uint8_t w : S->plan.rowlen) S->max_rowlen = std::max(S->max_rowlen, (int)w);
        std::vector<int64_t> rp(S->Npad + 1, 0);
        for (int64_t k = 0; k < 4 * S->ne; ++k) rp[T[k] + 1]++;
        for (int64_t r = 0; r < S->Npad; ++r) rp[r + 1] += rp[r];
        std::vector<uint32_t> ri(6 * std::max<int64_t>(4 * S->ne, 1), 0);
        std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
        for (int64_t k = 0; k < 4 * S->ne; ++k) ri[6 * fill[T[k]]++] = (uint32_t)k;  // k = 4 t + a
        if (upload(&S->rinc_ptr, rp) || upload(&S->rinc, ri)) {
            set_error("fg_system_create: allocation of the assembly incidence list failed");
            fg_system_destroy(S);
            return FG_ERR_OOM;
        }
    }
    {
        fg_status e = tet_slots(S, nullptr);
        if (e) {
            fg_system_destroy(S);
            return e;
        }
    }
    *out = S;
    return check_hip("fg_system_create");
}

fg_status fg_system_sizes(const fg_system *S, int64_t *n_pairs, int64_t *n_blk, int64_t *n_slices, int64_t *n_halo)
{
    if (!S) return FG_ERR_ARG;
    if (n_halo) *n_halo = S->plan.halo_ptr.empty() ? 0 : S->plan.halo_ptr.back();
    if (n_pairs) *n_pairs = S->plan.npairs;
    if (n_blk) *n_blk = S->nblk;
    if (n_slices) *n_slices = S->nslices;
    return FG_OK;
}

fg_status fg_assemble(fg_ctx *ctx, fg_system *S, const fg_params *prm, const double *E, const double *log_k, void *stream)
{
    return fg_assemble_groups(ctx, S, prm, 1, E, log_k, stream);
}

fg_status fg_assemble_groups(fg_ctx *ctx, fg_system *S, const fg_params *prm, int n_params, const double *E,
                             const double *log_k, void *stream)
{
    if (!ctx || !S || !prm || !E || !log_k) {
        set_error("fg_assemble: null argument");
        return FG_ERR_ARG;
    }
    if (n_params != 1 && n_params != S->ngroups) {
        set_error("fg_assemble_groups: n_params must be 1 or the number of groups");
        return FG_ERR_ARG;
    }
    for (int g = 1; g < n_params; ++g)
        if (prm[g].dt != prm[0].dt) {
            set_error("fg_assemble_groups: every group must use the same time step dt");
            return FG_ERR_ARG;
        }
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    std::vector<fg_params> gp(S->ngroups);
    for (int i = 0; i < S->ngroups; ++i) gp[i] = prm[n_params == 1 ? 0 : i];
    // synchronous upload: the parameters are host data owned by the caller
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(S->gprm, gp.data(), gp.size() * sizeof(fg_params), hipMemcpyHostToDevice) != hipSuccess)
        return check_hip("fg_assemble parameters");
    S->prm = prm[0];
    S->k32_valid = false;
    S->bj_valid = S->bj32_valid = false;
    assemble_all(S, E, log_k, st);
    TRY(check_hip("fg_assemble"));
    int bad = 0;
    hipMemcpyAsync(&bad, (int *)S->red_counter + 1, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    if (bad) {
        set_error(bad == 1 ? "fg_assemble: tetrahedron with non-positive volume" : "fg_assemble: graph slot missing");
        return FG_ERR_ARG;
    }
    S->assembled = true;
    stick_tangent(S, st);  // K = K_bulk + stick-and-contact interface tangent
    return check_hip("fg_assemble");
}

fg_status fg_cohesive_update(fg_ctx *ctx, fg_system *S, const double *U, const double *die_n, const double *t0,
                             double *trac, double *die, uint8_t *flag, double *f_coh, int write_tangent, void *stream)
{
    if (!ctx || !S || !U || (S->nq && (!die_n || !t0 || !trac || !die || !flag)) || !f_coh) {
        set_error("fg_cohesive_update: null argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    perm_in(S, 3, U, S->ui, st);
    cohesive_qp(S, S->ui, die_n, t0, trac, die, flag, st);
    cohesive_rows(S, S->fc, write_tangent, st);
    perm_out(S, 3, S->fc, f_coh, st);
    return check_hip("fg_cohesive_update");
}

fg_status fg_pcg_solve(fg_ctx *ctx, fg_system *S, int which, int nrhs, const double *b, double *x,
                       const fg_pcg_opts *opts, fg_pcg_info *info, void *stream)
{
    if (!ctx || !S || !b || !x || nrhs < 1 || (which != FG_K && which != FG_A22)) {
        set_error("fg_pcg_solve: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    SymmetricSolves sym(S);  // CG: always the symmetric tangent
    hipStream_t st = S_(stream);
    fg_pcg_opts o = defaults(opts, 1e-10);
    if (opts && !(opts->tol > 0)) {
        set_error("fg_pcg_solve: tol must be positive");
        return FG_ERR_ARG;
    }
    if (o.precision < FG_F64 || o.precision > FG_MIXED_F32VAL ||
        (o.precision == FG_MIXED_F32VAL && (nrhs > 1 || S->ngroups > 1))) {
        set_error("fg_pcg_solve: bad precision (FG_MIXED_F32VAL takes one right-hand side on an unbatched system)");
        return FG_ERR_ARG;
    }
    const int bs = which == FG_K ? 3 : 1;
    const int64_t nn = bs * S->N;
    std::fill(S->grp_iters.begin(), S->grp_iters.end(), 0);
    if (which == FG_K && nrhs > 1) {
        fg_pcg_info bi{};
        fg_status s = block_solve(S, nrhs, b, x, o.precision, o.tol, o.max_iter, o.check_every, &bi, st);
        if (info) *info = bi;
        return s;
    }
    fg_status worst = FG_OK;
    fg_pcg_info wi{};
    for (int c = 0; c < nrhs; ++c) {
        fg_pcg_info ci{};
        fg_status s;
        if (which == FG_K) {
            perm_in(S, 3, b + c * nn, S->pv1, st);
            s = k_solve(S, S->pv1, S->pv2, o, &ci, st);
            perm_out(S, 3, S->pv2, x + c * nn, st);
        } else {
            perm_in(S, 1, b + c * nn, S->s7, st);
            int64_t it = 0;
            hipMemcpyAsync(S->wr, S->s7, S->Npad * sizeof(double), hipMemcpyDeviceToDevice, st);
            double rr = 0;
            s = cg_run(S, FG_A22, FG_F64, o.tol, o.max_iter, o.check_every, &it, &rr, st);
            perm_out(S, 1, S->wx, x + c * nn, st);
            ci.iters = it;
            ci.cycles = 1;
            ci.relres = rr;
            ci.status = s;
        }
        if (s < 0) {
            if (info) *info = ci;
            return s;
        }
        if (s > worst || ci.relres > wi.relres || c == 0) wi = ci;
        if (s > worst) worst = s;
    }
    hipStreamSynchronize(st);
    if (info) {
        *info = wi;
        info->status = worst;
    }
    fg_status e = check_hip("fg_pcg_solve");
    return e ? e : worst;
}

fg_status fg_flow_solve(fg_ctx *ctx, fg_system *S, const double *b_u, const double *b_p, double *du, double *dp,
                        const fg_pcg_opts *inner_k, const fg_pcg_opts *inner_p, double outer_tol,
                        int64_t outer_max_iter, fg_solve_info *info, void *stream)
{
    if (!ctx || !S || !b_u || !b_p || !du || !dp || !(outer_tol > 0)) {
        set_error("fg_flow_solve: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    fg_pcg_opts ok = defaults(inner_k, 1e-12), op = defaults(inner_p, 1e-12);
    fg_solve_info si{};
    perm_in(S, 3, b_u, S->rm, st);
    perm_in(S, 1, b_p, S->rf, st);
    fg_status s = prevost(S, S->rm, S->rf, S->du, S->dpv, ok, op, outer_tol, outer_max_iter > 0 ? outer_max_iter : 1000,
                          &si, st);
    perm_out(S, 3, S->du, du, st);
    perm_out(S, 1, S->dpv, dp, st);
    hipStreamSynchronize(st);
    si.status = s;
    if (info) *info = si;
    fg_status e = check_hip("fg_flow_solve");
    return e ? e : s;
}

fg_status fg_residual(fg_ctx *ctx, fg_system *S, const double *U, const double *P, const double *U_n,
                      const double *P_n, const double *f_coh, const double *F_u, const double *f_p, double *R_m,
                      double *R_f, void *stream)
{
    if (!ctx || !S || !U || !P || !U_n || !P_n || !f_coh || !F_u || !f_p || !R_m || !R_f) {
        set_error("fg_residual: null argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    perm_in(S, 3, U, S->ui, st);
    perm_in(S, 3, U_n, S->ui0, st);
    perm_in(S, 1, P, S->pi, st);
    perm_in(S, 1, P_n, S->pi0, st);
    perm_in(S, 3, f_coh, S->fc, st);
    perm_in(S, 3, F_u, S->fi, st);
    perm_in(S, 1, f_p, S->qi, st);
    residual_int(S, S->ui, S->pi, S->ui0, S->pi0, S->fc, S->fi, S->qi, S->rm, S->rf, st);
    perm_out(S, 3, S->rm, R_m, st);
    perm_out(S, 1, S->rf, R_f, st);
    return check_hip("fg_residual");
}

// Newton globalisation of fg_step: merit phi = (||R_m|| / s*)^2 + (||R_f|| / s_f)^2
// with s* = max(s_m, ||A_pu (P + dP)||) fixed for the iteration (1 if zero) and
// s_f the flow scale (1 if zero); step lengths 1, 1/2, ..., 1/64 are tried and the
// first that lowers phi is taken (1/64 if none does).  Trial states use the
// interface forces only (no tangent); they leave S->ui, S->pi, du, dpv intact.
static double newton_step_length(fg_system *S, double rm, double rf, double sm, double sf, const double *t0,
                                 int64_t *cuts, hipStream_t st)
{
    const int64_t n1 = 3 * S->Npad, n2 = S->Npad;
    double *ut = S->v1, *rmt = S->v2, *ap = S->pv2, *pt = S->s1, *rft = S->s2;
    hipMemcpyAsync(pt, S->pi, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
    vaxpby(n2, 1.0, S->dpv, 1.0, pt, st);
    apply_Apu(S, pt, ap, st);
    double s_star = std::max(sm, vnorm(S, n1, ap, st));
    if (!(s_star > 0)) s_star = 1.0;
    const double sfn = sf > 0 ? sf : 1.0;
    auto phi = [&](double a, double b) { return (a / s_star) * (a / s_star) + (b / sfn) * (b / sfn); };
    const double m0 = phi(rm, rf);
    double step = 1.0;
    for (;;) {
        hipMemcpyAsync(ut, S->ui, n1 * sizeof(double), hipMemcpyDeviceToDevice, st);
        vaxpby(n1, step, S->du, 1.0, ut, st);
        hipMemcpyAsync(pt, S->pi, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
        vaxpby(n2, step, S->dpv, 1.0, pt, st);
        cohesive_qp(S, ut, S->die0, t0, S->adj_trac, S->adj_die, S->adj_flag, st);
        cohesive_rows(S, S->fc, 0, st);
        residual_int(S, ut, pt, S->ui0, S->pi0, S->fc, S->fi, S->qi, rmt, rft, st);
        if (phi(vnorm(S, n1, rmt, st), vnorm(S, n2, rft, st)) < m0 || step <= 1.0 / 64) break;
        step *= 0.5;
        ++*cuts;
    }
    return step;
}

fg_status fg_step(fg_ctx *ctx, fg_system *S, double *U, double *P, double *die, double *trac, uint8_t *flag,
                  const double *t0, const double *F_u, const double *f_p, double newton_tol, int64_t newton_max_iter,
                  const fg_pcg_opts *inner_k, const fg_pcg_opts *inner_p, double outer_tol, int64_t outer_max_iter,
                  fg_solve_info *info, void *stream)
{
    if (!ctx || !S || !U || !P || !F_u || !f_p || (S->nq && (!die || !trac || !flag || !t0))) {
        set_error("fg_step: null argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    const int64_t n1 = 3 * S->Npad, n2 = S->Npad;
    fg_pcg_opts ok = defaults(inner_k, 1e-12), op = defaults(inner_p, 1e-12);
    fg_solve_info si{};
    perm_in(S, 3, U, S->ui, st);
    perm_in(S, 1, P, S->pi, st);
    hipMemcpyAsync(S->ui0, S->ui, n1 * sizeof(double), hipMemcpyDeviceToDevice, st);
    hipMemcpyAsync(S->pi0, S->pi, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
    perm_in(S, 3, F_u, S->fi, st);
    perm_in(S, 1, f_p, S->qi, st);
    if (S->nq) hipMemcpyAsync(S->die0, die, 2 * S->nq * sizeof(double), hipMemcpyDeviceToDevice, st);
    double sm = 0, sf = 0, em = 0, ef = 0;
    int64_t it = 0, cuts = 0;
    fg_status status = FG_NOT_CONVERGED;
    for (;;) {
        cohesive_qp(S, S->ui, S->die0, t0, trac, die, flag, st);
        cohesive_rows(S, S->fc, 1, st);
        residual_int(S, S->ui, S->pi, S->ui0, S->pi0, S->fc, S->fi, S->qi, S->rm, S->rf, st);
        const double rm = vnorm(S, n1, S->rm, st), rf = vnorm(S, n2, S->rf, st);
        apply_Apu(S, S->pi, S->pv1, st);
        const double ap = vnorm(S, n1, S->pv1, st);
        if (it == 0) {
            sm = std::max(rm, std::max(ap, vnorm(S, n1, S->fi, st)));
            sf = std::max(rf, S->prm.dt * vnorm(S, n2, S->qi, st));
        } else {
            sm = std::max(sm, ap);
        }
        em = sm > 0 ? rm / sm : rm;
        ef = sf > 0 ? rf / sf : rf;
        if (!std::isfinite(em) || !std::isfinite(ef)) {
            set_error("fg_step: NaN in the Newton residual");
            status = FG_ERR_NAN;
            break;
        }
        if (em <= newton_tol && ef <= newton_tol) {
            status = FG_OK;
            break;
        }
        if (it >= newton_max_iter) {
            status = FG_NOT_CONVERGED;
            break;
        }
        vscale(n1, -1.0, S->rm, st);
        vscale(n2, -1.0, S->rf, st);
        fg_status s = prevost(S, S->rm, S->rf, S->du, S->dpv, ok, op, outer_tol,
                              outer_max_iter > 0 ? outer_max_iter : 1000, &si, st);
        if (s < 0) {
            status = s;
            break;
        }
        const double step = S->line_search ? newton_step_length(S, rm, rf, sm, sf, t0, &cuts, st) : 1.0;
        vaxpby(n1, step, S->du, 1.0, S->ui, st);
        vaxpby(n2, step, S->dpv, 1.0, S->pi, st);
        it++;
    }
    perm_out(S, 3, S->ui, U, st);
    perm_out(S, 1, S->pi, P, st);
    hipStreamSynchronize(st);
    si.newton_iters = it;
    si.res_m = em;
    si.res_f = ef;
    si.status = status;
    si.step_cuts = cuts;
    if (info) *info = si;
    fg_status e = check_hip("fg_step");
    return e ? e : status;
}

// The transposed Newton system of one converged step and its gradient (the body of
// fg_adjoint_solve).  On entry S->ui, S->pi hold the state and S->fi, S->qi the
// objective gradient (internal order, zero on held DOFs).  On success the
// multipliers are left in S->ui0 (lam_u) and S->pi0 (lam_p), and the gradient is
// written to (or, with accumulate, added to) dJ_dE, dJ_dlogk.
static fg_status adjoint_core(fg_system *S, const double *die_n, const double *t0, const double *log_k,
                              double *dJ_dE, double *dJ_dlogk, bool accumulate, double *lam_u, double *lam_p,
                              const fg_pcg_opts *inner_k, const fg_pcg_opts *inner_p, double outer_tol,
                              double defect_tol, int64_t max_defect_iters, fg_solve_info *info, hipStream_t st)
{
    // the corrections solve with the symmetric tangent, or with K_t + N^T when the
    // exact tangent is on; either way the true residual below carries N^T
    AdjointSolves adj(S);
    const int64_t n1 = 3 * S->Npad, n2 = S->Npad;
    fg_pcg_opts ok = defaults(inner_k, 1e-12), op = defaults(inner_p, 1e-12);
    fg_solve_info si{};
    // interface state and symmetric tangent at the converged state
    cohesive_qp(S, S->ui, die_n, t0, S->adj_trac, S->adj_die, S->adj_flag, st);
    cohesive_rows(S, S->fc, 1, st);
    // right-hand sides: b1 = -dJ/dU - N^T mu, b2 = dJ/dP
    // Defect correction in refinement form: the true residual of the exact transposed
    // system, r = f - [(K + N^T) mu - A_pu lp ; A_up mu + A22 lp], is computed with the
    // FP64 operators and only the correction is solved, with the symmetric tangent,
    // to the caller's (possibly loose) tolerances.  The fixed point is that of the
    // plain iteration K mu_k+1 - A_pu lp = -dJ/dU - N^T mu_k.
    double *mu = S->ui0, *lp = S->pi0, *r1 = S->rm, *r2 = S->rf, *dmu = S->du, *dlp = S->dpv;
    vfill(mu, 0.0, n1, st);
    vfill(lp, 0.0, n2, st);
    hipMemcpyAsync(r1, S->fi, n1 * sizeof(double), hipMemcpyDeviceToDevice, st);
    vscale(n1, -1.0, r1, st);  // r1 = -dJ/dU
    hipMemcpyAsync(r2, S->qi, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
    fg_status status = FG_NOT_CONVERGED;
    double change = 0;
    int64_t k = 0, outer = 0, kit = 0, ait = 0;
    while (k < max_defect_iters) {
        fg_solve_info sk{};
        fg_status s = prevost(S, r1, r2, dmu, dlp, ok, op, outer_tol, 1000, &sk, st);
        if (s == FG_ERR_BREAKDOWN && S->exact_tangent == 2) {
            // with K_t + N^T the Schur complement's symmetric part can be indefinite at
            // slip points (d.S d <= 0): redo this correction, and the later ones, with the
            // symmetric tangent; the true residual above still carries N^T, so the fixed
            // point is the same
            S->exact_tangent = 0;
            outer += sk.outer_iters;
            kit += sk.inner_k_iters;
            ait += sk.inner_a22_iters;
            sk = fg_solve_info{};
            s = prevost(S, r1, r2, dmu, dlp, ok, op, outer_tol, 1000, &sk, st);
        }
        outer += sk.outer_iters;
        kit += sk.inner_k_iters;
        ait += sk.inner_a22_iters;
        if (s < 0) {
            status = s;
            break;
        }
        ++k;
        vaxpby(n1, 1.0, dmu, 1.0, mu, st);
        vaxpby(n2, 1.0, dlp, 1.0, lp, st);
        // relative change of each block (a block that is zero does not count)
        const double *A1[2] = {dmu, mu}, *A2[2] = {dlp, lp};
        double d1[2], d2[2];
        vdots(S, n1, 2, A1, A1, d1, st);
        vdots(S, n2, 2, A2, A2, d2, st);
        change = std::max(d1[1] > 0 ? std::sqrt(d1[0] / d1[1]) : 0.0, d2[1] > 0 ? std::sqrt(d2[0] / d2[1]) : 0.0);
        if (!std::isfinite(change)) {
            set_error("fg_adjoint_solve: NaN in the defect correction");
            status = FG_ERR_NAN;
            break;
        }
        if (change <= defect_tol) {
            status = FG_OK;
            break;
        }
        // r1 = -dJ/dU - K mu - N^T mu + A_pu lp;  r2 = dJ/dP - A_up mu - A22 lp
        spmv(S, FG_K, mu, S->v1, st);
        apply_NT(S, mu, S->v2, st);
        apply_Apu(S, lp, S->pv1, st);
        hipMemcpyAsync(r1, S->fi, n1 * sizeof(double), hipMemcpyDeviceToDevice, st);
        vscale(n1, -1.0, r1, st);
        vaxpby(n1, -1.0, S->v1, 1.0, r1, st);
        vaxpby(n1, -1.0, S->v2, 1.0, r1, st);
        vaxpby(n1, 1.0, S->pv1, 1.0, r1, st);
        apply_Aup(S, mu, S->s7, st);
        spmv(S, FG_A22, lp, S->s8, st);
        hipMemcpyAsync(r2, S->qi, n2 * sizeof(double), hipMemcpyDeviceToDevice, st);
        vaxpby(n2, -1.0, S->s7, 1.0, r2, st);
        vaxpby(n2, -1.0, S->s8, 1.0, r2, st);
    }
    si.outer_iters = outer;
    si.inner_k_iters = kit;
    si.inner_a22_iters = ait;
    if (status >= 0) {
        vscale(n1, -1.0, mu, st);  // lam_u = -mu
        sensitivity(S, S->ui, S->pi, mu, lp, dJ_dE, dJ_dlogk, log_k, accumulate, st);
        if (lam_u) perm_out(S, 3, mu, lam_u, st);
        if (lam_p) perm_out(S, 1, lp, lam_p, st);
    }
    hipStreamSynchronize(st);
    si.newton_iters = k;
    si.outer_relres = change;
    si.status = status;
    if (info) *info = si;
    return status;
}

fg_status fg_adjoint_solve(fg_ctx *ctx, fg_system *S, const double *U, const double *P, const double *die_n,
                           const double *t0, const double *log_k, const double *dJdU, const double *dJdP,
                           double *dJ_dE, double *dJ_dlogk, double *lam_u, double *lam_p,
                           const fg_pcg_opts *inner_k, const fg_pcg_opts *inner_p, double outer_tol,
                           double defect_tol, int64_t max_defect_iters, fg_solve_info *info, void *stream)
{
    if (!ctx || !S || !U || !P || !log_k || !dJdU || !dJdP || !dJ_dE || !dJ_dlogk ||
        (S->nq && (!die_n || !t0)) || !(outer_tol > 0) || !(defect_tol > 0)) {
        set_error("fg_adjoint_solve: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    perm_in(S, 3, U, S->ui, st);
    perm_in(S, 1, P, S->pi, st);
    perm_in(S, 3, dJdU, S->fi, st);
    vmask(3 * S->Npad, S->dir_u, S->fi, st);
    perm_in(S, 1, dJdP, S->qi, st);
    vmask(S->Npad, S->dir_p, S->qi, st);
    fg_status status = adjoint_core(S, die_n, t0, log_k, dJ_dE, dJ_dlogk, false, lam_u, lam_p, inner_k, inner_p,
                                    outer_tol, defect_tol, max_defect_iters, info, st);
    fg_status e = check_hip("fg_adjoint_solve");
    return e ? e : status;
}

fg_status fg_adjoint_loop_step(fg_ctx *ctx, fg_system *S, const double *U, const double *P, const double *die_old,
                               const double *t0, const double *log_k, const double *dJdU, const double *dJdP,
                               const double *lam_p_next, double *a, double *dJ_dE, double *dJ_dlogk, double *lam_u,
                               double *lam_p, const fg_pcg_opts *inner_k, const fg_pcg_opts *inner_p,
                               double outer_tol, double defect_tol, int64_t max_defect_iters, fg_solve_info *info,
                               void *stream)
{
    if (!ctx || !S || !U || !P || !log_k || !dJdU || !dJdP || !dJ_dE || !dJ_dlogk ||
        (S->nq && (!die_old || !t0 || !a)) || !(outer_tol > 0) || !(defect_tol > 0)) {
        set_error("fg_adjoint_loop_step: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    const int64_t n1 = 3 * S->Npad, n2 = S->Npad;
    perm_in(S, 3, U, S->ui, st);
    perm_in(S, 1, P, S->pi, st);
    perm_in(S, 3, dJdU, S->fi, st);
    vmask(n1, S->dir_u, S->fi, st);
    perm_in(S, 1, dJdP, S->qi, st);
    vmask(n2, S->dir_p, S->qi, st);
    if (lam_p_next) {
        // the next step's flow residual reads this state through -A_up U_n and
        // -(A22 - dt C) P_n: its multipliers add A_pu lam and (A22 - dt C) lam
        double *lam = S->s7, *a22 = S->s8, *cl = S->s6;
        perm_in(S, 1, lam_p_next, lam, st);
        apply_Apu(S, lam, S->pv1, st);
        vaxpby(n1, 1.0, S->pv1, 1.0, S->fi, st);
        spmv(S, FG_A22, lam, a22, st);
        spmv(S, FG_C, lam, cl, st);
        vaxpby(n2, -S->prm.dt, cl, 1.0, a22, st);
        vmask(n2, S->dir_p, a22, st);
        vaxpby(n2, 1.0, a22, 1.0, S->qi, st);
    }
    if (S->nq) {
        // the slip this step produced, through the return map: (dPhi/dU)^T a
        slip_adjoint(S, S->ui, die_old, t0, a, nullptr, S->v2, nullptr, st);
        vaxpby(n1, 1.0, S->v2, 1.0, S->fi, st);
    }
    fg_status status = adjoint_core(S, die_old, t0, log_k, dJ_dE, dJ_dlogk, true, lam_u, lam_p, inner_k, inner_p,
                                    outer_tol, defect_tol, max_defect_iters, info, st);
    if (status >= 0 && S->nq) {
        // the adjoint of the slip the step started from (lam_u is in S->ui0)
        slip_adjoint(S, S->ui, die_old, t0, a, S->ui0, nullptr, S->adj_die, st);
        hipMemcpyAsync(a, S->adj_die, 2 * S->nq * sizeof(double), hipMemcpyDeviceToDevice, st);
    }
    fg_status e = check_hip("fg_adjoint_loop_step");
    return e ? e : status;
}

fg_status fg_slip_adjoint(fg_ctx *ctx, fg_system *S, const double *U, const double *die_old, const double *t0,
                          const double *a_new, const double *lam_u, double *gU, double *a_old, void *stream)
{
    if (!ctx || !S || !U || (S->nq && (!die_old || !t0 || !a_new)) || (!gU && !a_old)) {
        set_error("fg_slip_adjoint: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    perm_in(S, 3, U, S->ui, st);
    if (lam_u) perm_in(S, 3, lam_u, S->v1, st);
    slip_adjoint(S, S->ui, die_old, t0, a_new, lam_u ? S->v1 : nullptr, gU ? S->v2 : nullptr, S->nq ? a_old : nullptr,
                 st);
    if (gU) perm_out(S, 3, S->v2, gU, st);
    return check_hip("fg_slip_adjoint");
}

fg_status fg_exact_solve(fg_ctx *ctx, fg_system *S, const double *b, double *x, const fg_pcg_opts *opts,
                         fg_pcg_info *info, void *stream)
{
    if (!ctx || !S || !b || !x) {
        set_error("fg_exact_solve: bad argument");
        return FG_ERR_ARG;
    }
    const fg_pcg_opts o = defaults(opts, 1e-10);
    if (o.precision != FG_F64) {
        set_error("fg_exact_solve: only FG_F64 is supported");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    if (S->ngroups > 1) {
        set_error("fg_exact_solve: batched systems are not supported");
        return FG_ERR_ARG;
    }
    if (!S->bx && dalloc(&S->bx, bx_len(S))) {
        set_error("fg_exact_solve: device allocation of the BiCGStab work vectors failed");
        return FG_ERR_OOM;
    }
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    perm_in(S, 3, b, S->pv2, st);
    int64_t it = 0;
    double rel = 0;
    fg_status s = bicgstab_exact(S, S->pv2, S->wx, o.tol, o.max_iter, false, &it, &rel, st);
    perm_out(S, 3, S->wx, x, st);
    if (info) {
        info->iters = it;
        info->cycles = 1;
        info->relres = rel;
        info->status = s;
    }
    fg_status e = check_hip("fg_exact_solve");
    return e ? e : s;
}

// The block-Jacobi data and the Chebyshev work vectors (allocated on first use).
static fg_status precond_buffers(fg_system *S, bool cheb)
{
    if (cheb && !S->chd) {
        if (dalloc(&S->chd, 3 * S->Npad) || dalloc(&S->chs, 3 * S->Npad) || dalloc(&S->chq, 3 * S->Npad)) {
            set_error("device allocation for the Chebyshev preconditioner failed");
            return FG_ERR_OOM;
        }
    }
    if (!S->bjA) {
        if (dalloc(&S->bjA, 6 * S->Npad) || dalloc(&S->bjB, 9 * std::max<int64_t>(S->nfr, 1)) ||
            dalloc(&S->wz, 3 * S->Npad) || dalloc(&S->bjA32, 6 * S->Npad) ||
            dalloc(&S->bjB32, 9 * std::max<int64_t>(S->nfr, 1)) || dalloc(&S->wz32, 3 * S->Npad)) {
            set_error("device allocation for the block-Jacobi preconditioner failed");
            return FG_ERR_OOM;
        }
        S->bj_valid = false;
    }
    return FG_OK;
}

fg_status fg_lanczos_bounds(fg_ctx *ctx, fg_system *S, int steps, double *lo, double *hi, void *stream)
{
    if (!ctx || !S || !lo || !hi || steps < 2 || steps > 100000) {
        set_error("fg_lanczos_bounds: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    if (S->ngroups > 1) {
        set_error("fg_lanczos_bounds: batched systems are not supported");
        return FG_ERR_ARG;
    }
    Guard g(ctx->device);
    fg_status e = precond_buffers(S, true);
    if (e) return e;
    e = lanczos_bounds(S, steps, lo, hi, S_(stream));
    if (e) return e;
    return check_hip("fg_lanczos_bounds");
}

fg_status fg_amg_levels(fg_ctx *ctx, fg_system *S, int *nlev, int64_t *nodes, void *stream)
{
    if (!ctx || !S || !nlev || !nodes) {
        set_error("fg_amg_levels: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    if (S->k_precond != 3) {
        set_error("fg_amg_levels: the AMG preconditioner is not selected (fg_tune k_precond 3)");
        return FG_ERR_STATE;
    }
    Guard g(ctx->device);
    fg_status e = amg_ready(S, S_(stream));
    if (e) return e;
    amg_levels(S, nlev, nodes);
    return check_hip("fg_amg_levels");
}

fg_status fg_amg_aggregates(fg_ctx *ctx, fg_system *S, int level, int32_t *agg, void *stream)
{
    if (!ctx || !S || !agg) {
        set_error("fg_amg_aggregates: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    if (S->k_precond != 3) {
        set_error("fg_amg_aggregates: the AMG preconditioner is not selected (fg_tune k_precond 3)");
        return FG_ERR_STATE;
    }
    Guard g(ctx->device);
    fg_status e = amg_ready(S, S_(stream));
    if (e) return e;
    hipStreamSynchronize(S_(stream));
    return amg_aggregates(S, level, agg);
}

fg_status fg_cheb_interval(fg_ctx *ctx, fg_system *S, double *lo, double *hi, void *stream)
{
    if (!ctx || !S || !lo || !hi) {
        set_error("fg_cheb_interval: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    if (S->k_precond != 2) {
        set_error("fg_cheb_interval: the Chebyshev preconditioner is not selected (fg_tune k_precond 2)");
        return FG_ERR_STATE;
    }
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    fg_status e = cheb_interval_ready(S, st);
    if (e) return e;
    *lo = S->cheb_lo;
    *hi = S->cheb_hi;
    return check_hip("fg_cheb_interval");
}

fg_status fg_spmv(fg_ctx *ctx, fg_system *S, int which, const double *x, double *y, void *stream)
{
    if (!ctx || !S || !x || !y || which < 0 || which > FG_K_EXACT) {
        set_error("fg_spmv: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    const int bs = (which == FG_K || which == FG_KBULK || which == FG_K_EXACT) ? 3 : 1;
    double *xi = bs == 3 ? S->pv1 : S->s7, *yi = bs == 3 ? S->pv2 : S->s8;
    perm_in(S, bs, x, xi, st);
    if (which == FG_K_EXACT)
        spmv_exact(S, xi, yi, false, st);
    else
        spmv(S, which, xi, yi, st);
    perm_out(S, bs, yi, y, st);
    return check_hip("fg_spmv");
}

fg_status fg_coupling(fg_ctx *ctx, fg_system *S, int transpose, const double *x, double *y, void *stream)
{
    if (!ctx || !S || !x || !y) {
        set_error("fg_coupling: null argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    if (!transpose) {
        perm_in(S, 1, x, S->s7, st);
        apply_Apu(S, S->s7, S->pv1, st);
        perm_out(S, 3, S->pv1, y, st);
    } else {
        perm_in(S, 3, x, S->pv1, st);
        apply_Aup(S, S->pv1, S->s7, st);
        perm_out(S, 1, S->s7, y, st);
    }
    return check_hip("fg_coupling");
}

fg_status fg_export(fg_ctx *ctx, fg_system *S, int which, int32_t *rows, int32_t *cols, double *vals, void *stream)
{
    if (!ctx || !S || !rows || !cols || !vals || which < 0 || which > 3) {
        set_error("fg_export: bad argument");
        return FG_ERR_ARG;
    }
    if (!ready(S)) return FG_ERR_STATE;
    Guard g(ctx->device);
    hipStream_t st = S_(stream);
    const Plan &P = S->plan;
    const int bs = (which == FG_K || which == FG_KBULK) ? 9 : 1;
    std::vector<double> v((size_t)S->nblk * bs);
    const double *src = which == FG_K || which == FG_KBULK ? S->K : (which == FG_A22 ? S->A22 : S->Cm);
    hipMemcpyAsync(v.data(), src, v.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    std::vector<double> kfb;
    if (which == FG_KBULK && S->nfr) {
        kfb.resize((size_t)S->nfr * S->fault_w * 9);
        hipMemcpyAsync(kfb.data(), S->Kfb, kfb.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    }
    hipStreamSynchronize(st);
    TRY(check_hip("fg_export"));
    std::vector<int32_t> fidx(S->Npad, -1);
    for (size_t k = 0; k < P.frows.size(); ++k) fidx[P.frows[k]] = (int32_t)k;
    int64_t m = 0;
    for (int64_t r = 0; r < S->Npad; ++r) {
        if (P.perm[r] < 0) continue;
        const int64_t s = r / SLICE, l = r % SLICE, base = P.slice_ptr[s];
        for (int j = 0; j < P.rowlen[r]; ++j) {
            const int64_t c = P.col[base + (int64_t)j * SLICE + l];
            rows[m] = P.perm[r];
            cols[m] = P.perm[c];
            if (bs == 1) {
                vals[m] = v[base + (int64_t)j * SLICE + l];
            } else if (which == FG_KBULK && fidx[r] >= 0) {
                for (int e = 0; e < 9; ++e) vals[9 * m + e] = kfb[((size_t)fidx[r] * S->fault_w + j) * 9 + e];
            } else {
                for (int e = 0; e < 9; ++e) vals[9 * m + e] = v[9 * base + (int64_t)(9 * j + e) * SLICE + l];
            }
            ++m;
        }
    }
    return FG_OK;
}

fg_status fg_group_stats(const fg_system *S, int64_t *iters, double *relres, int *status, int *n_groups)
{
    if (!S) {
        set_error("fg_group_stats: null system");
        return FG_ERR_ARG;
    }
    for (int g = 0; g < S->ngroups; ++g) {
        if (iters) iters[g] = S->grp_iters[g];
        if (relres) relres[g] = S->grp_relres[g];
        if (status) status[g] = S->grp_status[g];
    }
    if (n_groups) *n_groups = S->ngroups;
    return FG_OK;
}

fg_status fg_tune(fg_system *S, const char *key, int64_t value)
{
    if (!S || !key || value < 0) {
        set_error("fg_tune: bad argument");
        return FG_ERR_ARG;
    }
    Guard g(S->device);
    if (std::strcmp(key, "halo_cap") == 0) {
        S->halo_cap = (int)std::min<int64_t>(value, 65536 / (4 * 3 * (int64_t)sizeof(double)));
        drop_graphs(S);
        drop_group_graphs(S);
        return FG_OK;
    }
    if (std::strcmp(key, "graphs") == 0) {
        S->use_graphs = value != 0;
        drop_graphs(S);
        drop_mr_graphs(S);
        drop_group_graphs(S);
        return FG_OK;
    }
    if (std::strcmp(key, "k_precond") == 0) {
        if (value > 3) {
            set_error("fg_tune: k_precond must be 0 (point Jacobi), 1 (nodal and fault-pair block Jacobi), 2 "
                      "(Chebyshev polynomial over block Jacobi) or 3 (smoothed-aggregation AMG)");
            return FG_ERR_ARG;
        }
        if (value >= 1) {
            fg_status e = precond_buffers(S, value >= 2);
            if (e) return e;
        }
        S->k_precond = (int)value;
        drop_graphs(S);
        return FG_OK;
    }
    if (std::strcmp(key, "amg_coarse") == 0) {
        if (value < 1 || value > 1000) {
            set_error("fg_tune: amg_coarse must be 1 to 1000 nodes");
            return FG_ERR_ARG;
        }
        if (value != S->amg_coarse) amg_destroy(S);
        S->amg_coarse = value;
        return FG_OK;
    }
    if (std::strcmp(key, "line_search") == 0) {
        S->line_search = value != 0;
        return FG_OK;
    }
    if (std::strcmp(key, "spmv_unroll") == 0) {
        if (value != 1 && value != 2 && value != 3 && value != 4 && value != 6) {
            set_error("fg_tune: spmv_unroll must be 1, 2, 3, 4 or 6");
            return FG_ERR_ARG;
        }
        S->spmv_unroll = (int)value;
        drop_graphs(S);
        return FG_OK;
    }
    if (std::strcmp(key, "exact_tangent") == 0) {
        if (value > 1) {
            set_error("fg_tune: exact_tangent must be 0 or 1");
            return FG_ERR_ARG;
        }
        if (value == 1 && !S->bx && dalloc(&S->bx, bx_len(S))) {
            set_error("fg_tune: device allocation of the BiCGStab work vectors failed");
            return FG_ERR_OOM;
        }
        S->exact_tangent = (int)value;
        return FG_OK;
    }
    if (std::strcmp(key, "cheb_degree") == 0) {
        if (value < 1 || value > 16) {
            set_error("fg_tune: cheb_degree must be in [1, 16]");
            return FG_ERR_ARG;
        }
        S->cheb_degree = (int)value;
        return FG_OK;
    }
    if (std::strcmp(key, "cheb_ratio") == 0) {
        if (value < 2 || value > 1000000) {
            set_error("fg_tune: cheb_ratio must be in [2, 1000000]");
            return FG_ERR_ARG;
        }
        S->cheb_ratio = (int)value;
        S->cheb_epoch = -1;
        return FG_OK;
    }
    if (std::strcmp(key, "cheb_lanczos") == 0) {
        if (value < 5 || value > 500) {
            set_error("fg_tune: cheb_lanczos must be in [5, 500]");
            return FG_ERR_ARG;
        }
        S->cheb_lanczos = (int)value;
        S->cheb_epoch = -1;
        return FG_OK;
    }
    if (std::strcmp(key, "mixed_update") == 0) {
        // longer FP32 phases lose the recurrence: on the 64^3 fault problem a factor
        // of 300 tripled the FP32 iterations and 1000 let a column diverge
        if (value < 2 || value > 100) {
            set_error("fg_tune: mixed_update must be in [2, 100]");
            return FG_ERR_ARG;
        }
        S->mixed_update = (int)value;
        return FG_OK;
    }
    if (std::strcmp(key, "vec_grid") == 0) {
        if (value != 512 && value != 1024 && value != 2048) {
            set_error("fg_tune: vec_grid must be 512, 1024 or 2048");
            return FG_ERR_ARG;
        }
        S->vec_grid = (int)value;
        drop_graphs(S);
        return FG_OK;
    }
    if (std::strcmp(key, "spmv_wpb") == 0) {
        if (value != 1 && value != 2 && value != 4) {
            set_error("fg_tune: spmv_wpb must be 1, 2 or 4");
            return FG_ERR_ARG;
        }
        if ((S->nslices + value - 1) / value + 8 > S->npartials) {
            set_error("fg_tune: spmv_wpb too small for the partial-sum buffer of this system");
            return FG_ERR_ARG;
        }
        S->spmv_wpb = (int)value;
        drop_graphs(S);
        return FG_OK;
    }
    if (std::strcmp(key, "spmv_nt") == 0) {
        if (value != 0 && value != 1 && value != 3 && value != 7 && value != 15 && value != 23) {
            set_error("fg_tune: spmv_nt must be 0, 1, 3, 7, 15 or 23");
            return FG_ERR_ARG;
        }
        S->spmv_nt = (int)value;
        drop_graphs(S);
        return FG_OK;
    }
    if (std::strcmp(key, "rhs_tile") == 0) {
        if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8 && value != 16) {
            set_error("fg_tune: rhs_tile must be 0, 1, 2, 4, 8 or 16");
            return FG_ERR_ARG;
        }
        S->mr_tile = (int)value;
        drop_mr_graphs(S);
        return FG_OK;
    }
    if (std::strcmp(key, "mr_form") == 0) {
        const int ok[] = {0, 1, 2, 4, 9, 10, 12, 17, 18, 25, 26};
        if (std::find(std::begin(ok), std::end(ok), (int)value) == std::end(ok) || value != (int)value) {
            set_error("fg_tune: mr_form must be 0, 1, 2, 4, 9, 10, 12, 17, 18, 25 or 26");
            return FG_ERR_ARG;
        }
        S->mr_form = (int)value;
        drop_mr_graphs(S);
        return FG_OK;
    }
    set_error(std::string("fg_tune: unknown key ") + key);
    return FG_ERR_ARG;
}

fg_status fg_profile(fg_system *S, int enable)
{
    if (!S) {
        set_error("fg_profile: null system");
        return FG_ERR_ARG;
    }
    S->prof = enable != 0;
    return FG_OK;
}

fg_status fg_profile_read(fg_system *S, int slot, int64_t *launches, double *ms, int reset)
{
    if (!S || slot < 0 || slot > 3) {
        set_error("fg_profile_read: bad argument");
        return FG_ERR_ARG;
    }
    if (launches) *launches = S->prof_count[slot];
    if (ms) *ms = S->prof_ms[slot];
    if (reset) {
        S->prof_count[slot] = 0;
        S->prof_ms[slot] = 0;
    }
    return FG_OK;
}

}  // extern "C"
