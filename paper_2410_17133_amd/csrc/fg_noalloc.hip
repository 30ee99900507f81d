// Point-Jacobi CG for callers that cannot allocate device memory.
//
// fg_pcg_solve keeps its CG vectors, reduction partials and device scalars in
// workspaces the library allocates; fg_pcg_solve_noalloc runs the same kernels
// with all of that work memory taken from `scratch`, one fixed array per GPU
// that lives as long as the process, and launches them one by one (no graph
// capture or instantiation).  It calls no allocating routine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "fg_internal.h"
#include "fg_kernels.h"

// CG work memory of the allocation-free solve: device scalars, reduction
// partials and the four CG vectors.  64 MiB hold the FP64 K solve of a mesh of
// up to about 690,000 nodes (2.09 M unknowns), e.g. the 64^3 cube.
constexpr size_t FG_NOALLOC_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[FG_NOALLOC_BYTES];

namespace fg {

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char *g_scratch[MAX_DEVICES] = {};  // device address of `scratch` on each device

inline size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of scratch a solve with `which` on S needs.
size_t need_bytes(const fg_system *S, int which)
{
    const size_t n = (size_t)(which == FG_K ? 3 : 1) * (size_t)S->Npad;
    return round256(sizeof(CgScalars)) + round256(4 * (size_t)S->npartials * sizeof(double)) +
           4 * round256(n * sizeof(double));
}

}  // namespace

// Device address of `scratch` on `device`, taken once per device with that device
// current (the host-side name of a __device__ array is not a device address).
fg_status noalloc_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("fg_ctx_create: device index beyond the allocation-free solve's table");
        return FG_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return FG_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        hipGetLastError();
        set_error(std::string("fg_ctx_create: hipGetSymbolAddress of the solve scratch failed: ") +
                  hipGetErrorString(e));
        return FG_ERR_HIP;
    }
    g_scratch[device] = (unsigned char *)p;
    return FG_OK;
}

}  // namespace fg

using namespace fg;

extern "C" fg_status fg_pcg_solve_noalloc(fg_ctx *ctx, fg_system *S, int which, const double *b, double *x,
                                          const fg_pcg_opts *opts, fg_pcg_info *info, void *stream)
{
    if (!ctx || !S || !b || !x || (which != FG_K && which != FG_A22)) {
        set_error("fg_pcg_solve_noalloc: bad argument");
        return FG_ERR_ARG;
    }
    if (opts && (!(opts->tol > 0) || opts->precision != FG_F64)) {
        set_error("fg_pcg_solve_noalloc: tol must be positive and precision FG_F64");
        return FG_ERR_ARG;
    }
    if (!S->assembled) {
        set_error("fg_pcg_solve_noalloc: call fg_assemble first");
        return FG_ERR_STATE;
    }
    if (S->ngroups > 1) {
        set_error("fg_pcg_solve_noalloc: batched systems are not supported");
        return FG_ERR_ARG;
    }
    const size_t need = need_bytes(S, which);
    if (need > FG_NOALLOC_BYTES) {
        set_error("fg_pcg_solve_noalloc: the solve needs " + std::to_string(need) + " bytes of scratch, more than the " +
                  std::to_string(FG_NOALLOC_BYTES) + " bytes the library holds per GPU (use fg_pcg_solve)");
        return FG_ERR_ARG;
    }
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (ctx->device >= 0 && ctx->device < MAX_DEVICES) base = g_scratch[ctx->device];
    }
    if (!base) {
        set_error("fg_pcg_solve_noalloc: the context's device has no solve scratch (fg_ctx_create failed?)");
        return FG_ERR_STATE;
    }
    int prev_dev = 0;
    hipGetDevice(&prev_dev);
    if (hipSetDevice(ctx->device) != hipSuccess) return check_hip("fg_pcg_solve_noalloc set device");
    const fg_pcg_opts o = opts ? *opts : fg_pcg_opts{1e-10, 1000000, FG_F64, 32, 0.0};
    const int64_t max_iter = o.max_iter > 0 ? o.max_iter : 1000000;
    const int check_every = o.check_every > 0 ? o.check_every : 32;
    hipStream_t st = (hipStream_t)stream;
    const int bs = which == FG_K ? 3 : 1;
    const size_t nb = round256((size_t)bs * S->Npad * sizeof(double));

    // carve the scratch: scalars | partials | x r p q
    unsigned char *q = base;
    CgScalars *sc = (CgScalars *)q;
    q += round256(sizeof(CgScalars));
    double *part = (double *)q;
    q += round256(4 * (size_t)S->npartials * sizeof(double));
    double *wx = (double *)q, *wr = (double *)(q + nb), *wp = (double *)(q + 2 * nb), *wq = (double *)(q + 3 * nb);

    // run the library's CG kernels on the scratch buffers: the system's workspace
    // pointers, launch mode and preconditioner are swapped for the call and restored
    double *s_wx = S->wx, *s_wr = S->wr, *s_wp = S->wp, *s_wq = S->wq, *s_part = S->partials;
    CgScalars *s_sc = S->sc;
    const bool s_graphs = S->use_graphs, s_prof = S->prof;
    const int s_prec = S->k_precond, s_exact = S->exact_tangent;
    S->wx = wx;
    S->wr = wr;
    S->wp = wp;
    S->wq = wq;
    S->partials = part;
    S->sc = sc;
    S->use_graphs = false;
    S->prof = false;
    S->k_precond = 0;
    S->exact_tangent = 0;
    perm_in(S, bs, b, wr, st);
    int64_t it = 0;
    double rr = 0;
    fg_status s = cg_run(S, which, FG_F64, o.tol, max_iter, check_every, &it, &rr, st);
    perm_out(S, bs, wx, x, st);
    hipStreamSynchronize(st);
    S->wx = s_wx;
    S->wr = s_wr;
    S->wp = s_wp;
    S->wq = s_wq;
    S->partials = s_part;
    S->sc = s_sc;
    S->use_graphs = s_graphs;
    S->prof = s_prof;
    S->k_precond = s_prec;
    S->exact_tangent = s_exact;
    if (info) {
        info->iters = it;
        info->cycles = 1;
        info->relres = rr;
        info->status = s;
    }
    fg_status e = check_hip("fg_pcg_solve_noalloc");
    hipSetDevice(prev_dev);
    return e ? e : s;
}
