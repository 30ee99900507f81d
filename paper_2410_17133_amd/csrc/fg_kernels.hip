// Device kernels of libfg (gfx950).
//
// Storage: the stiffness K is a sliced block-ELL matrix of 3x3 blocks.  Rows
// (nodes, in the planner's internal order) come in slices of 64, one per
// wavefront, one row per lane.  For slice s with width w (blocks per row) the
// column of slot j of lane l is col[slice_ptr[s] + 64 j + l] and entry (r,c)
// of that block is val[9 slice_ptr[s] + 64 (9 j + 3 r + c) + l]: every load
// of a wavefront reads 64 consecutive values.  Scalar operators (A22, C) use
// the same slots with one value each.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "fg_device.h"
#include "fg_kernels.h"

namespace fg {

namespace {

constexpr int STICK = 0, SLIP = 1, OPEN = 2;

// ----------------------------------------------------------------- permutation
__global__ void k_perm_in(int64_t N, int64_t Npad, int bs, const int32_t *__restrict__ perm,
                          const double *__restrict__ nat, double *__restrict__ in)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Npad * bs; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i / bs;
        int c = (int)(i - r * bs);
        const int32_t o = perm[r];
        in[i] = o >= 0 ? nat[(int64_t)o * bs + c] : 0.0;
    }
}

__global__ void k_perm_out(int64_t Npad, int bs, const int32_t *__restrict__ perm, const double *__restrict__ in,
                           double *__restrict__ nat)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Npad * bs; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i / bs;
        int c = (int)(i - r * bs);
        const int32_t o = perm[r];
        if (o >= 0) nat[(int64_t)o * bs + c] = in[i];
    }
}

__global__ void k_perm_in_u8(int64_t N, int64_t Npad, int bs, const int32_t *__restrict__ perm,
                             const uint8_t *__restrict__ nat, uint8_t *__restrict__ in)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Npad * bs; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = i / bs;
        int c = (int)(i - r * bs);
        const int32_t o = perm[r];
        in[i] = o >= 0 ? nat[(int64_t)o * bs + c] : 0;
    }
}

// ----------------------------------------------------------------- geometry
struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 crs(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ __forceinline__ double dt3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 scl(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ V3 ld3(const double *p) { return {p[0], p[1], p[2]}; }
__device__ __forceinline__ double cmp(V3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// Linear tetrahedron: gradients of the barycentric shape functions from the
// face normals, grad N_1 = (e2 x e3)/det etc., grad N_0 = -sum, V = |det|/6.
__device__ __forceinline__ double tet_grads(const double *xyz, const int32_t *nd, V3 g[4])
{
    V3 x0 = ld3(xyz + 3 * (int64_t)nd[0]);
    V3 e1 = sub(ld3(xyz + 3 * (int64_t)nd[1]), x0);
    V3 e2 = sub(ld3(xyz + 3 * (int64_t)nd[2]), x0);
    V3 e3 = sub(ld3(xyz + 3 * (int64_t)nd[3]), x0);
    V3 c23 = crs(e2, e3), c31 = crs(e3, e1), c12 = crs(e1, e2);
    double det = dt3(e1, c23);
    double inv = 1.0 / det;
    g[1] = scl(c23, inv);
    g[2] = scl(c31, inv);
    g[3] = scl(c12, inv);
    g[0] = {-(g[1].x + g[2].x + g[3].x), -(g[1].y + g[2].y + g[3].y), -(g[1].z + g[2].z + g[3].z)};
    return fabs(det) / 6.0;
}

__device__ __forceinline__ int find_slot(const int32_t *colrow, int len, int32_t c)
{
    for (int j = 0; j < len; ++j)
        if (colrow[(int64_t)j * SLICE] == c) return j;
    return -1;
}

// Shape function a of the interface triangle at quadrature point q.
__device__ __forceinline__ double qpN(int q, int a) { return q == a ? 2.0 / 3.0 : 1.0 / 6.0; }

// Parameters of the instance that owns internal row r (slices never mix instances).
__device__ __forceinline__ const fg_params &group_params(const fg_params *gprm, const int32_t *sgrp, int64_t r)
{
    return gprm[sgrp[r / SLICE]];
}

// ----------------------------------------------------------------- assembly
// Slot of block (a, b) of every tetrahedron in row a: tslot[16 t + 4 a + b] = j with
// col[slice_ptr[s] + 64 j + l] = node b (row a = 64 s + l).  Once per mesh, so that
// every assembly scatters without searching the rows.
__global__ void k_tet_slots(int64_t ne, const int32_t *__restrict__ tets, const int64_t *__restrict__ slice_ptr,
                            const int32_t *__restrict__ col, const uint8_t *__restrict__ rowlen, uint8_t *tslot,
                            int *bad)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ne) return;
    const int32_t *nd = tets + 4 * t;
    for (int a = 0; a < 4; ++a) {
        const int64_t row = nd[a];
        const int64_t base = slice_ptr[row / SLICE] + row % SLICE;
        const int len = rowlen[row];
        for (int b = 0; b < 4; ++b) {
            const int j = find_slot(col + base, len, nd[b]);
            if (j < 0) *bad = 1;
            tslot[16 * t + 4 * a + b] = (uint8_t)(j < 0 ? 0 : j);
        }
    }
}

// Entries of the row incidence list: the host leaves 4 t + a in word 0 of each
// 6-word entry; this writes the element's 4 nodes starting with the row's own node
// (a, then the other three in order), its caller index, and the slots of those four
// blocks of row a in the same order, so the assembly reads one contiguous run per
// row and the row's node is always local node 0.
__global__ void k_rinc_fill(int64_t nent, const int32_t *__restrict__ tets, const int32_t *__restrict__ orig,
                            const uint8_t *__restrict__ tslot, uint32_t *rinc)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nent) return;
    uint32_t *en = rinc + 6 * k;
    const uint32_t ta = en[0];
    const int64_t t = ta >> 2;
    const int a = (int)(ta & 3u);
    uint32_t sl = 0;
    for (int v = 0; v < 4; ++v) {
        const int src = v == 0 ? a : (v - 1) + (v - 1 >= a ? 1 : 0);
        en[v] = (uint32_t)tets[4 * t + src];
        sl |= (uint32_t)tslot[16 * t + 4 * a + src] << (8 * v);
    }
    en[4] = (uint32_t)orig[t];
    en[5] = sl;
}

// Element terms gathered per row: element stiffness V [lam g_a g_b^T + G (g_b g_a^T + (g_a.g_b) I)],
// storage (V/(20 M))(1 + delta_ab) and conductivity (k/mu) V g_a.g_b.  One thread per
// internal row and group of four consecutive slots (blockIdx.y): it sums, over the
// elements containing the row's node in increasing element order (the node first in
// each entry), the element's blocks of that row that fall in its slots, in registers,
// and writes each of its entries once.  Lanes are consecutive rows of a slice, so the stores are coalesced.
__global__ __launch_bounds__(WG) void k_assemble_rows(int64_t Npad, const int64_t *__restrict__ rinc_ptr, const uint32_t *__restrict__ rinc,
                                const uint8_t *__restrict__ rowlen, const double *__restrict__ xyz,
                                const double *__restrict__ E, const double *__restrict__ logk,
                                const fg_params *__restrict__ gprm, const int32_t *__restrict__ sgrp,
                                const int64_t *__restrict__ slice_ptr, double *__restrict__ K,
                                double *__restrict__ A22, double *__restrict__ Cm, int *bad)
{
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= Npad) return;
    const int j0 = 4 * (int)blockIdx.y, len = rowlen[row];
    if (j0 >= len) return;
    double acc[4][11];
    for (int q = 0; q < 4; ++q)
        for (int m = 0; m < 11; ++m) acc[q][m] = 0.0;
    const int64_t k1 = rinc_ptr[row + 1];
    for (int64_t k = rinc_ptr[row]; k < k1; ++k) {
        const uint32_t *en = rinc + 6 * k;
        const uint32_t sl = en[5];
        bool hit = false;
#pragma unroll
        for (int b = 0; b < 4; ++b) hit |= (unsigned)((int)((sl >> (8 * b)) & 0xffu) - j0) < 4u;
        if (!hit) continue;
        const int32_t nd[4] = {(int32_t)en[0], (int32_t)en[1], (int32_t)en[2], (int32_t)en[3]};
        const int64_t e = en[4];
        V3 g[4];
        const double V = tet_grads(xyz, nd, g);
        if (!(V > 0)) {
            *bad = 1;
            continue;
        }
        const fg_params &prm = group_params(gprm, sgrp, nd[0]);
        const double Ee = E[e], nu = prm.nu;
        const double lam = Ee * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        const double G = Ee / (2.0 * (1.0 + nu));
        const double kmu = exp(logk[e]) / prm.mu;
        const double sm = V / (20.0 * prm.biot_M);
        const V3 ga = g[0];   // the row's node
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int jq = (int)((sl >> (8 * b)) & 0xffu) - j0;
            if ((unsigned)jq >= 4u) continue;
            const double gg = dt3(ga, g[b]);
            double t[11];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    t[3 * r + c] = V * (lam * cmp(ga, r) * cmp(g[b], c) + G * (cmp(ga, c) * cmp(g[b], r) + (r == c ? gg : 0.0)));
            const double cab = kmu * V * gg;
            t[9] = sm * (b == 0 ? 2.0 : 1.0) + prm.dt * cab;
            t[10] = cab;
            for (int q = 0; q < 4; ++q)     // constant register indices: acc stays in registers
                if (jq == q)
                    for (int m = 0; m < 11; ++m) acc[q][m] += t[m];
        }
    }
    const int64_t l = row % SLICE, base = slice_ptr[row / SLICE];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (j0 + q >= len) break;
        const int64_t js = (int64_t)(j0 + q) * SLICE;
        double *kb = K + 9 * (base + js) + l;
        for (int m = 0; m < 9; ++m) kb[(int64_t)m * SLICE] = acc[q][m];
        A22[base + js + l] = acc[q][9];
        Cm[base + js + l] = acc[q][10];
    }
}

// Reference geometry of each interface element: area, normal, t1, t2.
__global__ void k_tri_geo(int64_t nf, const int32_t *__restrict__ coh, const double *__restrict__ xyz, double *geo)
{
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nf) return;
    const int32_t *c = coh + 6 * t;
    V3 x0 = ld3(xyz + 3 * (int64_t)c[3]);
    V3 cr = crs(sub(ld3(xyz + 3 * (int64_t)c[4]), x0), sub(ld3(xyz + 3 * (int64_t)c[5]), x0));
    double twoA = sqrt(dt3(cr, cr));
    V3 n = scl(cr, 1.0 / twoA);
    V3 v = {-n.z * n.x, -n.z * n.y, 1.0 - n.z * n.z};  // e_z minus its normal part
    double vn = sqrt(dt3(v, v));
    if (vn < 1e-8) {
        v = {1.0 - n.x * n.x, -n.x * n.y, -n.x * n.z};
        vn = sqrt(dt3(v, v));
    }
    V3 t1 = scl(v, 1.0 / vn);
    V3 t2 = crs(n, t1);
    double *o = geo + 10 * t;
    o[0] = 0.5 * twoA;
    o[1] = n.x, o[2] = n.y, o[3] = n.z;
    o[4] = t1.x, o[5] = t1.y, o[6] = t1.z;
    o[7] = t2.x, o[8] = t2.y, o[9] = t2.z;
}

// Fracture flow (double-node operators) gathered per interface row and slot:
// storage (w0/M_F) int <r><p>, longitudinal (w0 k_par/mu) int grad<r>.grad<p>
// and transverse (k_perp/(mu w0)) int [[r]][[p]] with int N_a N_b = A(1+d_ab)/12.
__global__ void k_fault_flow(int64_t nfr, int fw, const int32_t *__restrict__ frows, const int32_t *__restrict__ fadj_ptr,
                             const int32_t *__restrict__ fadj, const int32_t *__restrict__ coh,
                             const double *__restrict__ geo, const double *__restrict__ xyz,
                             const fg_params *__restrict__ gprm, const int32_t *__restrict__ sgrp,
                             const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ col,
                             const uint8_t *__restrict__ rowlen, double *A22, double *Cm)
{
    int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nfr * fw) return;
    const int64_t k = id / fw;
    const int j = (int)(id - k * fw);
    const int64_t row = frows[k];
    const int64_t s = row / SLICE, l = row % SLICE, base = slice_ptr[s];
    if (j >= rowlen[row]) return;
    const int32_t cj = col[base + (int64_t)j * SLICE + l];
    const fg_params &prm = group_params(gprm, sgrp, row);
    const double cs = prm.w0 / prm.M_F, cl = prm.w0 * prm.k_par / prm.mu, ct = prm.k_perp / (prm.mu * prm.w0);
    double sacc = 0, cacc = 0;
    for (int m = fadj_ptr[k]; m < fadj_ptr[k + 1]; ++m) {
        const int64_t t = fadj[m] / 6;
        const int la = fadj[m] % 6, sa = la / 3, va = la % 3;
        const int32_t *c = coh + 6 * t;
        for (int lb = 0; lb < 6; ++lb) {
            if (c[lb] != cj) continue;
            const int sb = lb / 3, vb = lb % 3;
            const double A = geo[10 * t];
            const V3 n = ld3(geo + 10 * t + 1);
            // in-plane gradients from the - lip vertices: grad N_a = n x (x_c - x_b) / (2A)
            V3 X[3] = {ld3(xyz + 3 * (int64_t)c[3]), ld3(xyz + 3 * (int64_t)c[4]), ld3(xyz + 3 * (int64_t)c[5])};
            V3 ga = scl(crs(n, sub(X[(va + 2) % 3], X[(va + 1) % 3])), 0.5 / A);
            V3 gb = scl(crs(n, sub(X[(vb + 2) % 3], X[(vb + 1) % 3])), 0.5 / A);
            const double m3 = A * (va == vb ? 2.0 : 1.0) / 12.0;
            const double cg = A * dt3(ga, gb);
            sacc += 0.25 * cs * m3;
            cacc += 0.25 * cl * cg + (sa == sb ? 1.0 : -1.0) * ct * m3;
        }
    }
    const int64_t kk = base + (int64_t)j * SLICE + l;
    A22[kk] += sacc + prm.dt * cacc;
    Cm[kk] += cacc;
}

// Symmetric elimination of held DOFs (zero row and column, unit diagonal),
// then point-Jacobi inverse diagonals.
__global__ void k_dirichlet(int64_t Npad, const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ col,
                            const uint8_t *__restrict__ rowlen, const uint8_t *__restrict__ dir_u,
                            const uint8_t *__restrict__ dir_p, double *K, double *A22, double *dinvK, double *dinvA)
{
    int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= Npad) return;
    const int64_t s = row / SLICE, l = row % SLICE, base = slice_ptr[s];
    const int len = rowlen[row];
    double dK[3] = {0, 0, 0}, dA = 0;
    for (int j = 0; j < len; ++j) {
        const int64_t c = col[base + (int64_t)j * SLICE + l];
        double *kb = K + 9 * base + (int64_t)9 * j * SLICE + l;
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) {
                const bool hr = dir_u[3 * row + r], hc = dir_u[3 * c + cc];
                if (hr || hc) kb[(int64_t)(3 * r + cc) * SLICE] = (c == row && r == cc) ? 1.0 : 0.0;
            }
        double *ab = A22 + base + (int64_t)j * SLICE + l;
        if (dir_p[row] || dir_p[c]) *ab = (c == row) ? 1.0 : 0.0;
        if (c == row) {
            for (int r = 0; r < 3; ++r) dK[r] = kb[(int64_t)(4 * r) * SLICE];
            dA = *ab;
        }
    }
    for (int r = 0; r < 3; ++r) dinvK[3 * row + r] = len ? 1.0 / dK[r] : 0.0;
    dinvA[row] = len ? 1.0 / dA : 0.0;
}

__global__ void k_save_fault_bulk(int64_t nfr, int fw, const int32_t *__restrict__ frows,
                                  const int64_t *__restrict__ slice_ptr, const uint8_t *__restrict__ rowlen,
                                  const double *__restrict__ K, double *Kfb)
{
    int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nfr * fw) return;
    const int64_t k = id / fw;
    const int j = (int)(id - k * fw);
    const int64_t row = frows[k];
    const int64_t s = row / SLICE, l = row % SLICE, base = slice_ptr[s];
    for (int e = 0; e < 9; ++e)
        Kfb[id * 9 + e] = j < rowlen[row] ? K[9 * base + (int64_t)(9 * j + e) * SLICE + l] : 0.0;
}

__global__ void k_to_f32(int64_t n, double s, const double *__restrict__ x, float *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)(s * x[i]);
}

__global__ void k_add_f32(int64_t n, double s, const float *__restrict__ x, double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += s * (double)x[i];
}

// ----------------------------------------------------------------- interface
// Elastic predictor / plastic corrector (Sec. 2.2.1) at one quadrature point.
// Inputs: opening (dn, ds1, ds2) of the displacement since t = 0, inelastic slip
// die at the start of the step, initial tractions (tn0, ts01, ts02).  Outputs
// the tractions, new inelastic slip, state and the local symmetric tangent
// (Dn on n(x)n, S on the tangent plane).
struct QpOut {
    double tn, ts1, ts2, die1, die2, Dn, S11, S12, S22;
    int flag;
};

__device__ QpOut return_map(double dn, double ds1, double ds2, double die1, double die2, double tn0, double ts01,
                            double ts02, double kn, double ks, double f)
{
    QpOut o;
    const double gap = dn - tn0 / kn;  // normal opening including the initial penetration
    o.tn = gap < 0.0 ? -kn * gap : 0.0;
    const double tr1 = ts01 + ks * (ds1 - die1);
    const double tr2 = ts02 + ks * (ds2 - die2);
    const double trn = sqrt(tr1 * tr1 + tr2 * tr2);
    const double F = trn - f * o.tn;
    o.Dn = gap <= 0.0 ? kn : 0.0;
    if (F <= 0.0) {
        o.ts1 = tr1, o.ts2 = tr2;
        o.die1 = die1, o.die2 = die2;
        o.flag = gap > 0.0 ? OPEN : STICK;
        const double k = o.flag == STICK ? ks : 0.0;
        o.S11 = k, o.S12 = 0.0, o.S22 = k;
    } else {
        const double u1 = tr1 / trn, u2 = tr2 / trn;
        const double dl = F / ks;
        o.die1 = die1 + dl * u1, o.die2 = die2 + dl * u2;
        o.ts1 = f * o.tn * u1, o.ts2 = f * o.tn * u2;
        o.flag = gap > 0.0 ? OPEN : SLIP;
        const double k = o.flag == SLIP ? ks * f * o.tn / trn : 0.0;
        o.S11 = k * (1.0 - u1 * u1), o.S12 = -k * u1 * u2, o.S22 = k * (1.0 - u2 * u2);
    }
    return o;
}

__global__ void k_cohesive_qp(int64_t nq, const int32_t *__restrict__ coh, const double *__restrict__ geo,
                              const double *__restrict__ U, const double *__restrict__ die_n,
                              const double *__restrict__ t0, const fg_params *__restrict__ gprm,
                              const int32_t *__restrict__ sgrp, double *trac,
                              double *die, uint8_t *flag, double *qpT, double *qpD, double *qpNs)
{
    int64_t iq = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (iq >= nq) return;
    const int64_t t = iq / 3;
    const int q = (int)(iq - 3 * t);
    const int32_t *c = coh + 6 * t;
    const double *gp = geo + 10 * t;
    const fg_params &prm = group_params(gprm, sgrp, c[0]);
    const double kn = prm.k_n, ks = prm.k_s, f = prm.friction;
    const V3 n = ld3(gp + 1), e1 = ld3(gp + 4), e2 = ld3(gp + 7);
    V3 jmp = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        const double Na = qpN(q, a);
        V3 d = sub(ld3(U + 3 * (int64_t)c[a]), ld3(U + 3 * (int64_t)c[3 + a]));
        jmp = {jmp.x + Na * d.x, jmp.y + Na * d.y, jmp.z + Na * d.z};
    }
    const double *tz = t0 + 3 * iq;
    QpOut o = return_map(dt3(n, jmp), dt3(e1, jmp), dt3(e2, jmp), die_n[2 * iq], die_n[2 * iq + 1], tz[0], tz[1],
                         tz[2], kn, ks, f);
    trac[3 * iq] = o.tn, trac[3 * iq + 1] = o.ts1, trac[3 * iq + 2] = o.ts2;
    die[2 * iq] = o.die1, die[2 * iq + 1] = o.die2;
    flag[iq] = (uint8_t)o.flag;
    // force conjugate to the opening, relative to the initial state
    const double fn = -(o.tn - tz[0]), f1 = o.ts1 - tz[1], f2 = o.ts2 - tz[2];
    qpT[3 * iq] = fn * n.x + f1 * e1.x + f2 * e2.x;
    qpT[3 * iq + 1] = fn * n.y + f1 * e1.y + f2 * e2.y;
    qpT[3 * iq + 2] = fn * n.z + f1 * e1.z + f2 * e2.z;
    // the part of the exact tangent the symmetric one omits: at slip points
    // d t_s / d delta_n = -f k_n tau, stored as the vector -f k_n tau (global frame)
    {
        const double ttr1 = tz[1] + ks * (dt3(e1, jmp) - die_n[2 * iq]);
        const double ttr2 = tz[2] + ks * (dt3(e2, jmp) - die_n[2 * iq + 1]);
        const double tn_ = sqrt(ttr1 * ttr1 + ttr2 * ttr2);
        const double c = (o.flag == SLIP && tn_ > 0.0) ? -f * kn / tn_ : 0.0;
        qpNs[3 * iq] = c * (ttr1 * e1.x + ttr2 * e2.x);
        qpNs[3 * iq + 1] = c * (ttr1 * e1.y + ttr2 * e2.y);
        qpNs[3 * iq + 2] = c * (ttr1 * e1.z + ttr2 * e2.z);
    }
    // global tangent Dn n n^T + sum S_ab t_a t_b^T, stored xx yy zz yz xz xy
    const double nn[3] = {n.x, n.y, n.z}, a1[3] = {e1.x, e1.y, e1.z}, a2[3] = {e2.x, e2.y, e2.z};
    const int I[6] = {0, 1, 2, 1, 0, 0}, J[6] = {0, 1, 2, 2, 2, 1};
    for (int m = 0; m < 6; ++m) {
        const int i = I[m], jj = J[m];
        qpD[6 * iq + m] = o.Dn * nn[i] * nn[jj] + o.S11 * a1[i] * a1[jj] + o.S22 * a2[i] * a2[jj] +
                          o.S12 * (a1[i] * a2[jj] + a2[i] * a1[jj]);
    }
}

// Stick-and-contact tangent k_n n(x)n + k_s (t1(x)t1 + t2(x)t2) at every point.
__global__ void k_stick_tangent(int64_t nq, const int32_t *__restrict__ coh, const double *__restrict__ geo,
                                const fg_params *__restrict__ gprm, const int32_t *__restrict__ sgrp, double *qpD)
{
    int64_t iq = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (iq >= nq) return;
    const double *gp = geo + 10 * (iq / 3);
    const fg_params &prm = group_params(gprm, sgrp, coh[6 * (iq / 3)]);
    const double kn = prm.k_n, ks = prm.k_s;
    const int I[6] = {0, 1, 2, 1, 0, 0}, J[6] = {0, 1, 2, 2, 2, 1};
    for (int m = 0; m < 6; ++m)
        qpD[6 * iq + m] = kn * gp[1 + I[m]] * gp[1 + J[m]] +
                          ks * (gp[4 + I[m]] * gp[4 + J[m]] + gp[7 + I[m]] * gp[7 + J[m]]);
}

__device__ __forceinline__ double symD(const double *d, int r, int c)
{
    // xx yy zz yz xz xy
    if (r == c) return d[r];
    const int s = r + c;  // 1: xy, 2: xz, 3: yz
    return s == 3 ? d[3] : (s == 2 ? d[4] : d[5]);
}

// Interface force per fault row: sum over incident elements and quadrature
// points of +-w N_a (T - T0).
__global__ void k_cohesive_force(int64_t nfr, const int32_t *__restrict__ frows, const int32_t *__restrict__ fadj_ptr,
                                 const int32_t *__restrict__ fadj, const double *__restrict__ geo,
                                 const double *__restrict__ qpT, const uint8_t *__restrict__ dir_u, double *fcoh)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nfr) return;
    const int64_t row = frows[k];
    double acc[3] = {0, 0, 0};
    for (int m = fadj_ptr[k]; m < fadj_ptr[k + 1]; ++m) {
        const int64_t t = fadj[m] / 6;
        const int la = fadj[m] % 6, va = la % 3;
        const double sg = la < 3 ? 1.0 : -1.0;
        const double w = geo[10 * t] / 3.0;
        for (int q = 0; q < 3; ++q) {
            const double c = sg * w * qpN(q, va);
            for (int r = 0; r < 3; ++r) acc[r] += c * qpT[3 * (3 * t + q) + r];
        }
    }
    for (int r = 0; r < 3; ++r) fcoh[3 * row + r] = dir_u[3 * row + r] ? 0.0 : acc[r];
}

// Fault rows of K = saved bulk blocks + interface tangent, with the held DOFs
// eliminated again; one thread per (fault row, slot).
__global__ void k_cohesive_tangent(int64_t nfr, int fw, const int32_t *__restrict__ frows,
                                   const int32_t *__restrict__ fadj_ptr, const int32_t *__restrict__ fadj,
                                   const int32_t *__restrict__ coh, const double *__restrict__ geo,
                                   const double *__restrict__ qpD, const double *__restrict__ Kfb,
                                   const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ col,
                                   const uint8_t *__restrict__ rowlen, const uint8_t *__restrict__ dir_u, double *K,
                                   float *K32, double *dinvK, float *dinvK32)
{
    int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= nfr * fw) return;
    const int64_t k = id / fw;
    const int j = (int)(id - k * fw);
    const int64_t row = frows[k];
    const int64_t s = row / SLICE, l = row % SLICE, base = slice_ptr[s];
    if (j >= rowlen[row]) return;
    const int64_t cj = col[base + (int64_t)j * SLICE + l];
    double acc[9];
    for (int e = 0; e < 9; ++e) acc[e] = Kfb[id * 9 + e];
    for (int m = fadj_ptr[k]; m < fadj_ptr[k + 1]; ++m) {
        const int64_t t = fadj[m] / 6;
        const int la = fadj[m] % 6, va = la % 3;
        const int32_t *c = coh + 6 * t;
        const double w = geo[10 * t] / 3.0;
        for (int lb = 0; lb < 6; ++lb) {
            if (c[lb] != cj) continue;
            const int vb = lb % 3;
            const double sg = ((la < 3) == (lb < 3)) ? 1.0 : -1.0;
            for (int q = 0; q < 3; ++q) {
                const double cq = sg * w * qpN(q, va) * qpN(q, vb);
                const double *d = qpD + 6 * (3 * t + q);
                for (int r = 0; r < 3; ++r)
                    for (int cc = 0; cc < 3; ++cc) acc[3 * r + cc] += cq * symD(d, r, cc);
            }
        }
    }
    double *kb = K + 9 * base + (int64_t)9 * j * SLICE + l;
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) {
            double v = acc[3 * r + cc];
            if (dir_u[3 * row + r] || dir_u[3 * cj + cc]) v = (cj == row && r == cc) ? 1.0 : 0.0;
            kb[(int64_t)(3 * r + cc) * SLICE] = v;
            if (K32) K32[9 * base + (int64_t)(9 * j + 3 * r + cc) * SLICE + l] = (float)v;
            if (cj == row && r == cc) {
                dinvK[3 * row + r] = 1.0 / v;
                if (dinvK32) dinvK32[3 * row + r] = (float)(1.0 / v);
            }
        }
}

// ----------------------------------------------------------------- adjoint
// N^T x, step 1: per point s_q = (-f k_n tau) . [[x]](q) (zero away from slip points).
__global__ void k_nt_qp(int64_t nq, const int32_t *__restrict__ coh, const double *__restrict__ qpNs,
                        const double *__restrict__ x, const uint8_t *__restrict__ dir_u, double *qpS)
{
    int64_t iq = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (iq >= nq) return;
    const int64_t t = iq / 3;
    const int q = (int)(iq - 3 * t);
    const int32_t *c = coh + 6 * t;
    double s = 0;
    for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r) {
            const int64_t ip = 3 * (int64_t)c[a] + r, im = 3 * (int64_t)c[3 + a] + r;
            s += qpNs[3 * iq + r] * qpN(q, a) * ((dir_u[ip] ? 0.0 : x[ip]) - (dir_u[im] ? 0.0 : x[im]));
        }
    qpS[iq] = s;
}

// N^T x, step 2: per fault row, +-sum_q w N_a s_q n on the + / - lip.
__global__ void k_nt_rows(int64_t nfr, const int32_t *__restrict__ frows, const int32_t *__restrict__ fadj_ptr,
                          const int32_t *__restrict__ fadj, const double *__restrict__ geo,
                          const double *__restrict__ qpS, const uint8_t *__restrict__ dir_u, double *y)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nfr) return;
    const int64_t row = frows[k];
    double acc[3] = {0, 0, 0};
    for (int m = fadj_ptr[k]; m < fadj_ptr[k + 1]; ++m) {
        const int64_t t = fadj[m] / 6;
        const int la = fadj[m] % 6, va = la % 3;
        const double w = (la < 3 ? 1.0 : -1.0) * geo[10 * t] / 3.0;
        double s = 0;
        for (int q = 0; q < 3; ++q) s += w * qpN(q, va) * qpS[3 * t + q];
        for (int r = 0; r < 3; ++r) acc[r] += s * geo[10 * t + 1 + r];
    }
    for (int r = 0; r < 3; ++r) y[3 * row + r] = dir_u[3 * row + r] ? 0.0 : acc[r];
}

// Parameter sensitivities per tetrahedron: dJ/dE_e = -lam_u^T (K_e/E_e) U_e, written as
// -V [lam1 tr eps(U) tr eps(lam) + 2 G1 eps(U):eps(lam)] with the E = 1 Lame constants, and
// dJ/dln k_e = -dt lam_p^T C_e P_e = -dt (k_e/mu) V grad(lam_p) . grad(P).
__global__ void k_sensitivity(int64_t ne, const int32_t *__restrict__ tets, const int32_t *__restrict__ orig,
                              const double *__restrict__ xyz, const double *__restrict__ logk,
                              const fg_params *__restrict__ gprm, const int32_t *__restrict__ sgrp,
                              const double *__restrict__ U, const double *__restrict__ P,
                              const double *__restrict__ lu, const double *__restrict__ lp,
                              const uint8_t *__restrict__ dir_u, const uint8_t *__restrict__ dir_p, double *dE,
                              double *dlogk, int accumulate)
{
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ne) return;
    const int32_t *nd = tets + 4 * t;
    V3 g[4];
    const double V = tet_grads(xyz, nd, g);
    double eu[3][3] = {{0}}, el[3][3] = {{0}};
    V3 gp = {0, 0, 0}, gl = {0, 0, 0};
    for (int a = 0; a < 4; ++a) {
        const int64_t o = 3 * (int64_t)nd[a];
        double ua[3], la[3];
        for (int r = 0; r < 3; ++r) {
            ua[r] = dir_u[o + r] ? 0.0 : U[o + r];
            la[r] = dir_u[o + r] ? 0.0 : lu[o + r];
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                eu[i][j] += 0.5 * (ua[i] * cmp(g[a], j) + ua[j] * cmp(g[a], i));
                el[i][j] += 0.5 * (la[i] * cmp(g[a], j) + la[j] * cmp(g[a], i));
            }
        const double pa = dir_p[nd[a]] ? 0.0 : P[nd[a]];
        const double qa = dir_p[nd[a]] ? 0.0 : lp[nd[a]];
        gp = {gp.x + pa * g[a].x, gp.y + pa * g[a].y, gp.z + pa * g[a].z};
        gl = {gl.x + qa * g[a].x, gl.y + qa * g[a].y, gl.z + qa * g[a].z};
    }
    const fg_params &prm = group_params(gprm, sgrp, nd[0]);
    const double nu = prm.nu;
    const double lam1 = nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), G1 = 1.0 / (2.0 * (1.0 + nu));
    double tru = eu[0][0] + eu[1][1] + eu[2][2], trl = el[0][0] + el[1][1] + el[2][2], dd = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dd += eu[i][j] * el[i][j];
    const int64_t e = orig[t];
    const double ge = -V * (lam1 * tru * trl + 2.0 * G1 * dd);
    const double gk = -prm.dt * exp(logk[e]) / prm.mu * V * dt3(gl, gp);
    dE[e] = accumulate ? dE[e] + ge : ge;
    dlogk[e] = accumulate ? dlogk[e] + gk : gk;
}

// ----------------------------------------------------------------- coupling
// A^m_pu p: per tetrahedron alpha (V/4) grad N_a sum_b p_b (eq. Apdp), one colour.
__global__ void k_apu_tets(int64_t t0, int64_t t1, const int32_t *__restrict__ tets, const double *__restrict__ xyz,
                           const fg_params *__restrict__ gprm, const int32_t *__restrict__ sgrp,
                           const double *__restrict__ p, const uint8_t *__restrict__ dir_p, double *out)
{
    int64_t t = t0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= t1) return;
    const int32_t *nd = tets + 4 * t;
    V3 g[4];
    const double V = tet_grads(xyz, nd, g);
    double sp = 0;
    for (int b = 0; b < 4; ++b) sp += dir_p[nd[b]] ? 0.0 : p[nd[b]];
    const double c = group_params(gprm, sgrp, nd[0]).alpha * 0.25 * V * sp;
    for (int a = 0; a < 4; ++a) {
        double *o = out + 3 * (int64_t)nd[a];
        o[0] += c * g[a].x;
        o[1] += c * g[a].y;
        o[2] += c * g[a].z;
    }
}

// A^m_up u: per tetrahedron alpha (V/4) div u added to each vertex (eq. Adpd), one colour.
__global__ void k_aup_tets(int64_t t0, int64_t t1, const int32_t *__restrict__ tets, const double *__restrict__ xyz,
                           const fg_params *__restrict__ gprm, const int32_t *__restrict__ sgrp,
                           const double *__restrict__ u, const uint8_t *__restrict__ dir_u, double *out)
{
    int64_t t = t0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= t1) return;
    const int32_t *nd = tets + 4 * t;
    V3 g[4];
    const double V = tet_grads(xyz, nd, g);
    double dv = 0;
    for (int a = 0; a < 4; ++a) {
        const int64_t o = 3 * (int64_t)nd[a];
        dv += (dir_u[o] ? 0.0 : u[o]) * g[a].x + (dir_u[o + 1] ? 0.0 : u[o + 1]) * g[a].y +
              (dir_u[o + 2] ? 0.0 : u[o + 2]) * g[a].z;
    }
    const double c = group_params(gprm, sgrp, nd[0]).alpha * 0.25 * V * dv;
    for (int b = 0; b < 4; ++b) out[nd[b]] += c;
}

// A^f_pu p per fault row: +-(1/2) int N_a N_b (p_b+ + p_b-) n (transpose of eq. afdpd).
__global__ void k_apu_fault(int64_t nfr, const int32_t *__restrict__ frows, const int32_t *__restrict__ fadj_ptr,
                            const int32_t *__restrict__ fadj, const int32_t *__restrict__ coh,
                            const double *__restrict__ geo, const double *__restrict__ p,
                            const uint8_t *__restrict__ dir_p, double *out)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nfr) return;
    const int64_t row = frows[k];
    double acc[3] = {0, 0, 0};
    for (int m = fadj_ptr[k]; m < fadj_ptr[k + 1]; ++m) {
        const int64_t t = fadj[m] / 6;
        const int la = fadj[m] % 6, va = la % 3;
        const int32_t *c = coh + 6 * t;
        const double A = geo[10 * t];
        double sp = 0;
        for (int b = 0; b < 3; ++b) {
            const double pb = (dir_p[c[b]] ? 0.0 : p[c[b]]) + (dir_p[c[3 + b]] ? 0.0 : p[c[3 + b]]);
            sp += 0.5 * A * (va == b ? 2.0 : 1.0) / 12.0 * pb;
        }
        const double sg = la < 3 ? sp : -sp;
        for (int r = 0; r < 3; ++r) acc[r] += sg * geo[10 * t + 1 + r];
    }
    for (int r = 0; r < 3; ++r) out[3 * row + r] += acc[r];
}

// A^f_up u per fault row (eq. afdpd): (1/2) int N_b n.(u+ - u-) on both lips.
__global__ void k_aup_fault(int64_t nfr, const int32_t *__restrict__ frows, const int32_t *__restrict__ fadj_ptr,
                            const int32_t *__restrict__ fadj, const int32_t *__restrict__ coh,
                            const double *__restrict__ geo, const double *__restrict__ u,
                            const uint8_t *__restrict__ dir_u, double *out)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nfr) return;
    const int64_t row = frows[k];
    double acc = 0;
    for (int m = fadj_ptr[k]; m < fadj_ptr[k + 1]; ++m) {
        const int64_t t = fadj[m] / 6;
        const int vb = (fadj[m] % 6) % 3;
        const int32_t *c = coh + 6 * t;
        const double A = geo[10 * t];
        for (int a = 0; a < 3; ++a) {
            double jn = 0;
            for (int r = 0; r < 3; ++r) {
                const int64_t ip = 3 * (int64_t)c[a] + r, im = 3 * (int64_t)c[3 + a] + r;
                jn += geo[10 * t + 1 + r] * ((dir_u[ip] ? 0.0 : u[ip]) - (dir_u[im] ? 0.0 : u[im]));
            }
            acc += 0.5 * A * (vb == a ? 2.0 : 1.0) / 12.0 * jn;
        }
    }
    out[row] += acc;
}

// ----------------------------------------------------------------- vectors
__global__ void k_fill(double *y, double v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = v;
}

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i] + b * y[i];
}

__global__ void k_scale(int64_t n, double a, double *y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] *= a;
}

__global__ void k_mask(int64_t n, const uint8_t *__restrict__ m, double *y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (m[i]) y[i] = 0.0;
}

struct DotArgs {
    const double *a[4];
    const double *b[4];
};

template <int ND>
__global__ void k_dots(int64_t n, DotArgs args, double *partials, int64_t stride)
{
    double v[ND];
    for (int k = 0; k < ND; ++k) v[k] = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int k = 0; k < ND; ++k) v[k] += args.a[k][i] * args.b[k][i];
    block_partials<ND>(v, partials, stride);
}

template <int ND>
__global__ __launch_bounds__(FIN) void k_dots_fin(const double *partials, int64_t stride, int64_t nparts, double *res)
{
    double tot[ND];
    finalize_sum<ND>(partials, stride, nparts, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < ND; ++k) res[k] = tot[k];
}

// ----------------------------------------------------------------- SpMV
template <int BS, typename T, typename TV>
__global__ __launch_bounds__(WG) void k_spmv(SpmvArgs a, const TV *__restrict__ val, const T *__restrict__ x,
                                             T *__restrict__ y)
{
    extern __shared__ unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T *xs = (T *)smem + (int64_t)wave * a.cap * BS;
    const int64_t s = xcd_block() * (WG / SLICE) + wave;
    bool staged = false;
    if (s < a.nslices) staged = stage_halo<BS, T>(s, lane, a.halo_ptr, a.halo, a.cap, x, xs);
    __syncthreads();
    if (s < a.nslices) slice_spmv<BS, T, TV>(s, lane, staged, a.slice_ptr, a.col, a.lcol, a.diag_slot, val, x, xs, y);
}

// Fault rows of K_bulk x from the saved bulk blocks (overwrites y on those rows).
__global__ void k_spmv_fault_bulk(int64_t nfr, int fw, const int32_t *__restrict__ frows,
                                  const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ col,
                                  const uint8_t *__restrict__ rowlen, const double *__restrict__ Kfb,
                                  const double *__restrict__ x, double *y)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nfr) return;
    const int64_t row = frows[k];
    const int64_t s = row / SLICE, l = row % SLICE, base = slice_ptr[s];
    double a[3] = {0, 0, 0};
    for (int j = 0; j < rowlen[row]; ++j) {
        const int64_t cj = col[base + (int64_t)j * SLICE + l];
        const double *b = Kfb + (k * fw + j) * 9;
        for (int r = 0; r < 3; ++r) a[r] += b[3 * r] * x[3 * cj] + b[3 * r + 1] * x[3 * cj + 1] + b[3 * r + 2] * x[3 * cj + 2];
    }
    for (int r = 0; r < 3; ++r) y[3 * row + r] = a[r];
}

// ----------------------------------------------------------------- CG
// The iteration lives on the device: alpha, beta, rho and the stop flag are in
// CgScalars; every kernel returns at once when the flag is set, so the host
// can launch iterations in batches and poll the flag between batches.
template <typename T>
__global__ __launch_bounds__(WG) void k_cg_init(int64_t n, const T *__restrict__ dinv, T *__restrict__ x,
                                                const T *__restrict__ r, T *__restrict__ p, double *partials,
                                                int64_t stride)
{
    double v[2] = {0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T ri = r[i], zi = dinv[i] * ri;
        x[i] = 0;
        p[i] = zi;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    block_partials<2>(v, partials, stride);
}

__global__ __launch_bounds__(FIN) void k_cg_init_fin(const double *partials, int64_t stride, int64_t nparts,
                                                    CgScalars *sc, double tol)
{
    double tot[2];
    finalize_sum<2>(partials, stride, nparts, tot);
    if (threadIdx.x != 0) return;
    sc->rho[0] = tot[0];
    sc->rr = tot[1];
    sc->bb = tot[1];
    sc->tol2 = tol * tol * tot[1];
    sc->iter[0] = 0;
    sc->iters = 0;
    sc->status = FG_OK;
    sc->done = 0;
    if (!isfinite(tot[1])) {
        sc->status = FG_ERR_NAN;
        sc->done = 1;
    } else if (!isfinite(tot[0])) {   // finite r, non-finite r.z: a zero diagonal entry
        sc->status = FG_ERR_BREAKDOWN;
        sc->done = 1;
    } else if (tot[1] == 0.0) {
        sc->done = 1;
    } else if (sc->maxit <= 0) {
        sc->status = FG_NOT_CONVERGED;
        sc->done = 1;
    }
}

// q = A p and the per-block partials of p.q.
template <int BS, typename T, typename TV, int UNR, int NT, int WPB>
__global__ __launch_bounds__(WG) void k_cg_spmv(SpmvArgs a, const TV *__restrict__ val, const T *__restrict__ p,
                                                T *__restrict__ q, double *partials, int64_t stride,
                                                const CgScalars *sc)
{
    if (sc->done) return;
    extern __shared__ unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T *xs = (T *)smem + (int64_t)wave * a.cap * BS;
    const int64_t s = xcd_block() * WPB + wave;
    bool staged = false;
    if (s < a.nslices) staged = stage_halo<BS, T, (NT & 4) != 0>(s, lane, a.halo_ptr, a.halo, a.cap, p, xs);
    __syncthreads();
    double v[1] = {0};
    if (s < a.nslices)
        v[0] = slice_spmv<BS, T, TV, UNR, NT & 27>(s, lane, staged, a.slice_ptr, a.col, a.lcol, a.diag_slot, val, p, xs, q);
    block_partials<1>(v, partials, stride);
}

// x += alpha p, r -= alpha q, z = D^-1 r and the per-block partials of r.z, r.r
// (written to rows 2 and 3 of the partials).  alpha = rho / (p.q) is formed by
// every block from the product's partials in the same fixed order, so all blocks
// hold the same value; block 0 records it and any breakdown.
template <typename T>
__global__ __launch_bounds__(WG) void k_cg_update(int64_t n, int par, const T *__restrict__ dinv, T *__restrict__ x,
                                                  T *__restrict__ r, const T *__restrict__ p,
                                                  const T *__restrict__ q, double *partials, int64_t stride,
                                                  int64_t nparts, CgScalars *sc)
{
    // block 0 may set the flag while this kernel runs: take it once per block
    if (__syncthreads_or(sc->done)) return;
    double tot[1];
    finalize_sum<1>(partials, stride, nparts, tot);
    const double pq = tot[0];
    const bool ok = isfinite(pq) && pq > 0.0;
    const double alpha = sc->rho[par] / pq;
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
    const T al = (T)alpha;
    double v[2] = {0, 0};
#pragma unroll 4
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += al * p[i];
        const T ri = r[i] - al * q[i];
        r[i] = ri;
        const T zi = dinv[i] * ri;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    block_partials<2>(v, partials + 2 * stride, stride);
}

// Stop test and p = z + beta p.  Every block forms r.z and r.r from the update's
// partials in the same fixed order and takes the same decision; block 0 records
// the iteration count, the new rho (slot par^1) and the status.
template <typename T>
__global__ __launch_bounds__(WG) void k_cg_pupdate(int64_t n, int par, const T *__restrict__ dinv,
                                                   const T *__restrict__ r, T *__restrict__ p,
                                                   const double *partials, int64_t stride, int64_t nparts,
                                                   CgScalars *sc)
{
    if (__syncthreads_or(sc->done)) return;
    double tot[2];
    finalize_sum<2>(partials + 2 * stride, stride, nparts, tot);
    const int64_t it = sc->iter[par] + 1;
    const bool finite = isfinite(tot[0]) && isfinite(tot[1]);
    const bool stop = !finite || tot[1] <= sc->tol2 || it >= sc->maxit;
    const double beta = tot[0] / sc->rho[par];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->iter[par ^ 1] = it;
        sc->iters = it;
        sc->rr = tot[1];
        sc->rho_cur = sc->rho[par];
        if (!finite) {
            // finite r with a non-finite r.z: the preconditioner is singular
            sc->status = isfinite(tot[1]) ? FG_ERR_BREAKDOWN : FG_ERR_NAN;
            sc->done = 1;
        } else if (tot[1] <= sc->tol2) {
            sc->status = FG_OK;
            sc->done = 1;
        } else if (it >= sc->maxit) {
            sc->status = FG_NOT_CONVERGED;
            sc->done = 1;
        } else {
            sc->beta = beta;
            sc->rho[par ^ 1] = tot[0];
        }
    }
    if (stop) return;
    const T be = (T)beta;
#pragma unroll 4
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = dinv[i] * r[i] + be * p[i];
}

// ----------------------------------------------------------------- block Jacobi
// Preconditioner of K built from its own blocks: the 3x3 diagonal block of every
// node, and for the two lips' nodes at the same interface point the 6x6 block of
// the pair (their diagonal blocks and the coupling the penalty stiffness puts
// between them), inverted.  Row u keeps the symmetric 3x3 part A_u of its inverse
// and, on the interface, the coupling part B_u (z_u = A_u r_u + B_u r_partner).
template <typename T>
struct BlockJacobi {
    const T *A;            // [Npad*6] xx yy zz yz xz xy
    const T *B;            // [nfr*9] row-major
    const int32_t *fslot;  // [Npad] index into the fault rows, -1 off the interface
    const int32_t *fpart;  // [nfr] partner row, -1 if none
    T *z;                  // [3*Npad]
};

// In-place inverse of an n x n matrix (row-major, n <= 6), Gauss-Jordan with
// partial pivoting; false if a pivot vanishes.
template <int NN>
__device__ bool small_inverse(double (&a)[NN * NN], double (&inv)[NN * NN])
{
    for (int i = 0; i < NN * NN; ++i) inv[i] = (i / NN == i % NN) ? 1.0 : 0.0;
    for (int c = 0; c < NN; ++c) {
        int pr = c;
        double pv = fabs(a[c * NN + c]);
        for (int r = c + 1; r < NN; ++r)
            if (fabs(a[r * NN + c]) > pv) pv = fabs(a[r * NN + c]), pr = r;
        if (!(pv > 0.0)) return false;
        if (pr != c)
            for (int k = 0; k < NN; ++k) {
                double t = a[c * NN + k];
                a[c * NN + k] = a[pr * NN + k], a[pr * NN + k] = t;
                t = inv[c * NN + k];
                inv[c * NN + k] = inv[pr * NN + k], inv[pr * NN + k] = t;
            }
        const double d = 1.0 / a[c * NN + c];
        for (int k = 0; k < NN; ++k) a[c * NN + k] *= d, inv[c * NN + k] *= d;
        for (int r = 0; r < NN; ++r) {
            if (r == c) continue;
            const double m = a[r * NN + c];
            if (m == 0.0) continue;
            for (int k = 0; k < NN; ++k) a[r * NN + k] -= m * a[c * NN + k], inv[r * NN + k] -= m * inv[c * NN + k];
        }
    }
    return true;
}

__device__ __forceinline__ void k_block(const double *K, const int64_t *slice_ptr, int64_t row, int slot, double (&b)[9])
{
    const int64_t s = row / SLICE, l = row % SLICE, base = slice_ptr[s];
    for (int e = 0; e < 9; ++e) b[e] = K[9 * base + (int64_t)(9 * slot + e) * SLICE + l];
}

__global__ void k_bj_build(int64_t Npad, const double *__restrict__ K, const int64_t *__restrict__ slice_ptr,
                           const int32_t *__restrict__ col, const uint8_t *__restrict__ rowlen,
                           const int32_t *__restrict__ diag_slot, const int32_t *__restrict__ fslot,
                           const int32_t *__restrict__ fpart, double *A, double *B, int *bad)
{
    const int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (u >= Npad) return;
    const int dj = diag_slot[u];
    if (dj < 0) {  // padding row: its residual is always zero
        for (int e = 0; e < 6; ++e) A[6 * u + e] = 0.0;
        return;
    }
    double D[9];
    k_block(K, slice_ptr, u, dj, D);
    const int k = fslot[u];
    const int64_t v = k >= 0 ? fpart[k] : -1;
    int cslot = -1;
    if (v >= 0) {
        const int64_t s = u / SLICE, l = u % SLICE, base = slice_ptr[s];
        for (int j = 0; j < rowlen[u]; ++j)
            if (col[base + (int64_t)j * SLICE + l] == v) cslot = j;
    }
    if (cslot < 0) {
        double a[9], inv[9];
        for (int e = 0; e < 9; ++e) a[e] = D[e];
        if (!small_inverse<3>(a, inv)) *bad = 1;
        const double sym[6] = {inv[0], inv[4], inv[8], 0.5 * (inv[5] + inv[7]), 0.5 * (inv[2] + inv[6]),
                               0.5 * (inv[1] + inv[3])};
        for (int e = 0; e < 6; ++e) A[6 * u + e] = sym[e];
        if (k >= 0)
            for (int e = 0; e < 9; ++e) B[9 * k + e] = 0.0;
        return;
    }
    double C[9], Dp[9];
    k_block(K, slice_ptr, u, cslot, C);
    k_block(K, slice_ptr, v, diag_slot[v], Dp);
    double a[36], inv[36];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            a[6 * r + c] = D[3 * r + c];
            a[6 * r + 3 + c] = C[3 * r + c];
            a[6 * (3 + r) + c] = C[3 * c + r];  // K is symmetric: the partner row's block is C^T
            a[6 * (3 + r) + 3 + c] = Dp[3 * r + c];
        }
    if (!small_inverse<6>(a, inv)) *bad = 1;
    const double sym[6] = {inv[0], inv[7], inv[14], 0.5 * (inv[8] + inv[13]), 0.5 * (inv[2] + inv[12]),
                           0.5 * (inv[1] + inv[6])};
    for (int e = 0; e < 6; ++e) A[6 * u + e] = sym[e];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) B[9 * k + 3 * r + c] = inv[6 * r + 3 + c];
}

// z of one unit (a node, or both nodes of a pair) from its residual values rr
// (rows u and v); writes z, returns r.z.
template <typename T>
__device__ __forceinline__ T symT(const T *d, int r, int c)
{
    // xx yy zz yz xz xy
    if (r == c) return d[r];
    const int s = r + c;  // 1: xy, 2: xz, 3: yz
    return s == 3 ? d[3] : (s == 2 ? d[4] : d[5]);
}

template <typename T>
__device__ __forceinline__ double bj_unit_z(const BlockJacobi<T> &bj, int64_t u, int64_t v, int ku, int kv,
                                            const T (&rr)[6], int nr)
{
    double rz = 0;
    for (int m = 0; m < nr; ++m) {
        const int64_t row = m == 0 ? u : v;
        const int kk = m == 0 ? ku : kv;
        const T *a = bj.A + 6 * row;
        const T *ro = rr + 3 * m, *rp = rr + 3 * (1 - m);
        for (int c = 0; c < 3; ++c) {
            T z = symT(a, c, 0) * ro[0] + symT(a, c, 1) * ro[1] + symT(a, c, 2) * ro[2];
            if (nr == 2) {
                const T *b = bj.B + 9 * kk + 3 * c;
                z += b[0] * rp[0] + b[1] * rp[1] + b[2] * rp[2];
            }
            bj.z[3 * row + c] = z;
            rz += (double)ro[c] * (double)z;
        }
    }
    return rz;
}

// Start of the block-preconditioned CG: z = M^-1 r, p = z, x = 0; partials of r.z, r.r.
// One thread per unit: a node off the interface pairs, or a pair (taken by its lower row).
// With x == nullptr (a resumption after a residual replacement) only z and the
// partials are formed.
template <typename T>
__global__ __launch_bounds__(WG) void k_cg_init_bj(int64_t Npad, BlockJacobi<T> bj, T *__restrict__ x,
                                                   const T *__restrict__ r, T *__restrict__ p, double *partials,
                                                   int64_t stride)
{
    double v[2] = {0, 0};
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < Npad; u += (int64_t)gridDim.x * blockDim.x) {
        const int ku = bj.fslot[u];
        const int64_t w = ku >= 0 ? bj.fpart[ku] : -1;
        if (w >= 0 && w < u) continue;
        const int nr = w >= 0 ? 2 : 1;
        const int kw = w >= 0 ? bj.fslot[w] : -1;
        T rr[6] = {0, 0, 0, 0, 0, 0};
        for (int m = 0; m < nr; ++m)
            for (int c = 0; c < 3; ++c) {
                const int64_t i = 3 * (m == 0 ? u : w) + c;
                rr[3 * m + c] = r[i];
                if (x) x[i] = 0;
            }
        v[0] += bj_unit_z(bj, u, w, ku, kw, rr, nr);
        for (int m = 0; m < nr; ++m)
            for (int c = 0; c < 3; ++c) {
                const int64_t i = 3 * (m == 0 ? u : w) + c;
                if (x) p[i] = bj.z[i];
                v[1] += (double)rr[3 * m + c] * (double)rr[3 * m + c];
            }
    }
    block_partials<2>(v, partials, stride);
}

// k_cg_update with the block preconditioner: x, r of a unit updated by the thread
// that owns it, then z = M^-1 r of the unit from those values (no other thread
// writes them), stored for k_cg_pupdate_bj.
template <typename T>
__global__ __launch_bounds__(WG) void k_cg_update_bj(int64_t Npad, int par, BlockJacobi<T> bj, T *__restrict__ x,
                                                     T *__restrict__ r, const T *__restrict__ p,
                                                     const T *__restrict__ q, double *partials, int64_t stride,
                                                     int64_t nparts, CgScalars *sc)
{
    if (__syncthreads_or(sc->done)) return;
    double tot[1];
    finalize_sum<1>(partials, stride, nparts, tot);
    const double pq = tot[0];
    const bool ok = isfinite(pq) && pq > 0.0;
    const double alpha = sc->rho[par] / pq;
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
    const T al = (T)alpha;
    double v[2] = {0, 0};
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < Npad; u += (int64_t)gridDim.x * blockDim.x) {
        const int ku = bj.fslot[u];
        const int64_t w = ku >= 0 ? bj.fpart[ku] : -1;
        if (w >= 0 && w < u) continue;
        const int nr = w >= 0 ? 2 : 1;
        const int kw = w >= 0 ? bj.fslot[w] : -1;
        T rr[6] = {0, 0, 0, 0, 0, 0};
        for (int m = 0; m < nr; ++m)
            for (int c = 0; c < 3; ++c) {
                const int64_t i = 3 * (m == 0 ? u : w) + c;
                x[i] += al * p[i];
                const T ri = r[i] - al * q[i];
                r[i] = ri;
                rr[3 * m + c] = ri;
                v[1] += (double)ri * (double)ri;
            }
        v[0] += bj_unit_z(bj, u, w, ku, kw, rr, nr);
    }
    block_partials<2>(v, partials + 2 * stride, stride);
}

// k_cg_pupdate with the stored z.
template <typename T>
__global__ __launch_bounds__(WG) void k_cg_pupdate_bj(int64_t n, int par, const T *__restrict__ z,
                                                      T *__restrict__ p, const double *partials, int64_t stride,
                                                      int64_t nparts, CgScalars *sc)
{
    if (__syncthreads_or(sc->done)) return;
    double tot[2];
    finalize_sum<2>(partials + 2 * stride, stride, nparts, tot);
    const int64_t it = sc->iter[par] + 1;
    const bool finite = isfinite(tot[0]) && isfinite(tot[1]);
    const bool stop = !finite || tot[1] <= sc->tol2 || it >= sc->maxit;
    const double beta = tot[0] / sc->rho[par];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->iter[par ^ 1] = it;
        sc->iters = it;
        sc->rr = tot[1];
        sc->rho_cur = sc->rho[par];
        if (!finite) {
            // finite r with a non-finite r.z: the preconditioner is singular
            sc->status = isfinite(tot[1]) ? FG_ERR_BREAKDOWN : FG_ERR_NAN;
            sc->done = 1;
        } else if (tot[1] <= sc->tol2) {
            sc->status = FG_OK;
            sc->done = 1;
        } else if (it >= sc->maxit) {
            sc->status = FG_NOT_CONVERGED;
            sc->done = 1;
        } else {
            sc->beta = beta;
            sc->rho[par ^ 1] = tot[0];
        }
    }
    if (stop) return;
    const T be = (T)beta;
#pragma unroll 4
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + be * p[i];
}

// p = z + beta p after a residual replacement (k_cg_resume_p with the stored z).
template <typename T>
__global__ __launch_bounds__(WG) void k_cg_resume_p_bj(int64_t n, const T *__restrict__ z, T *__restrict__ p,
                                                       const CgScalars *sc)
{
    if (sc->done) return;
    const T be = (T)sc->beta;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z[i] + be * p[i];
}

// Resumption of a stopped CG after its residual was replaced (reliable update):
// partials of r.z and r.r of the new residual, then the scalars (beta against the
// rho at which the iteration stopped, the next stop threshold, parity slot 0),
// then p = z + beta p, so the search direction carries over.
template <typename T>
__global__ __launch_bounds__(WG) void k_cg_resume(int64_t n, const T *__restrict__ dinv, const T *__restrict__ r,
                                                  double *partials, int64_t stride)
{
    double v[2] = {0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T ri = r[i], zi = dinv[i] * ri;
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    block_partials<2>(v, partials, stride);
}

__global__ __launch_bounds__(FIN) void k_cg_resume_fin(const double *partials, int64_t stride, int64_t nparts,
                                                      CgScalars *sc, double tol2)
{
    double tot[2];
    finalize_sum<2>(partials, stride, nparts, tot);
    if (threadIdx.x != 0) return;
    sc->beta = tot[0] / sc->rho_cur;
    sc->rho[0] = tot[0];
    sc->rr = tot[1];
    sc->tol2 = tol2;
    sc->iter[0] = sc->iters;
    sc->status = FG_OK;
    sc->done = 0;
    if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(sc->beta)) {
        sc->status = FG_ERR_NAN;
        sc->done = 1;
    } else if (sc->iters >= sc->maxit) {
        sc->status = FG_NOT_CONVERGED;
        sc->done = 1;
    }
}

template <typename T>
__global__ __launch_bounds__(WG) void k_cg_resume_p(int64_t n, const T *__restrict__ dinv, const T *__restrict__ r,
                                                    T *__restrict__ p, const CgScalars *sc)
{
    if (sc->done) return;
    const T be = (T)sc->beta;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = dinv[i] * r[i] + be * p[i];
}

}  // namespace

// =================================================================== launchers
fg_status check_hip(const char *where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string(where) + ": " + hipGetErrorString(e));
        return FG_ERR_HIP;
    }
    return FG_OK;
}

void perm_in(const fg_system *S, int bs, const double *nat, double *in, hipStream_t st)
{
    LAUNCH(k_perm_in, grid_elems(S->Npad * bs), WG, st, S->N, S->Npad, bs, S->perm, nat, in);
}

void perm_out(const fg_system *S, int bs, const double *in, double *nat, hipStream_t st)
{
    LAUNCH(k_perm_out, grid_elems(S->Npad * bs), WG, st, S->Npad, bs, S->perm, in, nat);
}

void perm_in_u8(const fg_system *S, int bs, const uint8_t *nat, uint8_t *in, hipStream_t st)
{
    LAUNCH(k_perm_in_u8, grid_elems(S->Npad * bs), WG, st, S->N, S->Npad, bs, S->perm, nat, in);
}

void vfill(double *y, double v, int64_t n, hipStream_t st) { LAUNCH(k_fill, grid_elems(n), WG, st, y, v, n); }

void vaxpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t st)
{
    LAUNCH(k_axpby, grid_elems(n), WG, st, n, a, x, b, y);
}

void vscale(int64_t n, double a, double *y, hipStream_t st) { LAUNCH(k_scale, grid_elems(n), WG, st, n, a, y); }

void vmask(int64_t n, const uint8_t *mask, double *y, hipStream_t st) { LAUNCH(k_mask, grid_elems(n), WG, st, n, mask, y); }

void to_f32(int64_t n, double s, const double *x, float *y, hipStream_t st)
{
    LAUNCH(k_to_f32, grid_elems(n), WG, st, n, s, x, y);
}

void add_f32(int64_t n, double s, const float *x, double *y, hipStream_t st)
{
    LAUNCH(k_add_f32, grid_elems(n), WG, st, n, s, x, y);
}

void vdots(fg_system *S, int64_t n, int nd, const double *const *a, const double *const *b, double *host, hipStream_t st)
{
    DotArgs args{};
    for (int k = 0; k < nd; ++k) {
        args.a[k] = a[k];
        args.b[k] = b[k];
    }
    const int64_t g = grid_elems(n);
    switch (nd) {
    case 1:
        LAUNCH(k_dots<1>, g, WG, st, n, args, S->partials, S->npartials);
        LAUNCH(k_dots_fin<1>, 1, FIN, st, S->partials, S->npartials, g, S->red);
        break;
    case 2:
        LAUNCH(k_dots<2>, g, WG, st, n, args, S->partials, S->npartials);
        LAUNCH(k_dots_fin<2>, 1, FIN, st, S->partials, S->npartials, g, S->red);
        break;
    case 3:
        LAUNCH(k_dots<3>, g, WG, st, n, args, S->partials, S->npartials);
        LAUNCH(k_dots_fin<3>, 1, FIN, st, S->partials, S->npartials, g, S->red);
        break;
    default:
        LAUNCH(k_dots<4>, g, WG, st, n, args, S->partials, S->npartials);
        LAUNCH(k_dots_fin<4>, 1, FIN, st, S->partials, S->npartials, g, S->red);
        break;
    }
    hipMemcpyAsync(S->red_host, S->red, nd * sizeof(double), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    for (int k = 0; k < nd; ++k) host[k] = S->red_host[k];
}

void assemble_all(fg_system *S, const double *E, const double *logk, hipStream_t st)
{
    hipMemsetAsync(S->K, 0, S->nblk * 9 * sizeof(double), st);
    hipMemsetAsync(S->A22, 0, S->nblk * sizeof(double), st);
    hipMemsetAsync(S->Cm, 0, S->nblk * sizeof(double), st);
    int *bad = (int *)S->red_counter + 1;
    hipMemsetAsync(bad, 0, sizeof(int), st);
    if (S->ne > 0)
        LAUNCH(k_assemble_rows, dim3((unsigned)((S->Npad + WG - 1) / WG), (unsigned)((S->max_rowlen + 3) / 4)), WG, st,
               S->Npad, S->rinc_ptr, S->rinc, S->rowlen, S->xyz, E, logk, S->gprm, S->slice_group, S->slice_ptr, S->K,
               S->A22, S->Cm, bad);
    if (S->nf > 0) {
        LAUNCH(k_tri_geo, (S->nf + WG - 1) / WG, WG, st, S->nf, S->coh, S->xyz, S->tri_geo);
        LAUNCH(k_fault_flow, (S->nfr * S->fault_w + WG - 1) / WG, WG, st, S->nfr, S->fault_w, S->frows, S->fadj_ptr,
               S->fadj, S->coh, S->tri_geo, S->xyz, S->gprm, S->slice_group, S->slice_ptr, S->col, S->rowlen, S->A22, S->Cm);
    }
    LAUNCH(k_dirichlet, (S->Npad + WG - 1) / WG, WG, st, S->Npad, S->slice_ptr, S->col, S->rowlen, S->dir_u, S->dir_p,
           S->K, S->A22, S->dinvK, S->dinvA);
    if (S->nf > 0)
        LAUNCH(k_save_fault_bulk, (S->nfr * S->fault_w + WG - 1) / WG, WG, st, S->nfr, S->fault_w, S->frows,
               S->slice_ptr, S->rowlen, S->K, S->Kfb);
}

fg_status tet_slots(fg_system *S, hipStream_t st)
{
    int *bad = (int *)S->red_counter + 1;
    hipMemsetAsync(bad, 0, sizeof(int), st);
    if (S->ne > 0) {
        LAUNCH(k_tet_slots, (S->ne + WG - 1) / WG, WG, st, S->ne, S->tets, S->slice_ptr, S->col, S->rowlen, S->tslot,
               bad);
        LAUNCH(k_rinc_fill, (4 * S->ne + WG - 1) / WG, WG, st, 4 * S->ne, S->tets, S->tet_orig, S->tslot, S->rinc);
    }
    int h = 0;
    hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    fg_status e = check_hip("tetrahedron slot table");
    if (e) return e;
    if (h) {
        set_error("fg_system_create: a tetrahedron's node pair is missing from the planned graph");
        return FG_ERR_ARG;
    }
    return FG_OK;
}

void stick_tangent(fg_system *S, hipStream_t st)
{
    S->bj_valid = S->bj32_valid = false;
    if (S->nq == 0) return;
    LAUNCH(k_stick_tangent, (S->nq + WG - 1) / WG, WG, st, S->nq, S->coh, S->tri_geo, S->gprm, S->slice_group,
           S->qpD);
    cohesive_rows(S, S->fc, 1, st);
}

void refresh_k32(fg_system *S, hipStream_t st)
{
    to_f32(S->nblk * 9, 1.0, S->K, S->K32, st);
    to_f32(3 * S->Npad, 1.0, S->dinvK, S->dinvK32, st);
    S->k32_valid = true;
}

void cohesive_qp(fg_system *S, const double *U_int, const double *die_n, const double *t0, double *trac, double *die,
                 uint8_t *flag, hipStream_t st)
{
    if (S->nq == 0) return;
    LAUNCH(k_cohesive_qp, (S->nq + WG - 1) / WG, WG, st, S->nq, S->coh, S->tri_geo, U_int, die_n, t0, S->gprm,
           S->slice_group, trac, die, flag, S->qpT, S->qpD, S->qpNs);
}

void cohesive_rows(fg_system *S, double *fcoh_int, int write_tangent, hipStream_t st)
{
    if (write_tangent) S->bj_valid = S->bj32_valid = false;
    vfill(fcoh_int, 0.0, 3 * S->Npad, st);
    if (S->nq == 0) return;
    LAUNCH(k_cohesive_force, (S->nfr + WG - 1) / WG, WG, st, S->nfr, S->frows, S->fadj_ptr, S->fadj, S->tri_geo,
           S->qpT, S->dir_u, fcoh_int);
    if (write_tangent)
        LAUNCH(k_cohesive_tangent, (S->nfr * S->fault_w + WG - 1) / WG, WG, st, S->nfr, S->fault_w, S->frows,
               S->fadj_ptr, S->fadj, S->coh, S->tri_geo, S->qpD, S->Kfb, S->slice_ptr, S->col, S->rowlen, S->dir_u,
               S->K, S->k32_valid ? S->K32 : nullptr, S->dinvK, S->k32_valid ? S->dinvK32 : nullptr);
}

void apply_NT(fg_system *S, const double *x, double *y, hipStream_t st)
{
    vfill(y, 0.0, 3 * S->Npad, st);
    if (S->nq == 0) return;
    LAUNCH(k_nt_qp, (S->nq + WG - 1) / WG, WG, st, S->nq, S->coh, S->qpNs, x, S->dir_u, S->qpS);
    LAUNCH(k_nt_rows, (S->nfr + WG - 1) / WG, WG, st, S->nfr, S->frows, S->fadj_ptr, S->fadj, S->tri_geo, S->qpS,
           S->dir_u, y);
}

void sensitivity(fg_system *S, const double *U, const double *P, const double *lu, const double *lp, double *dE,
                 double *dlogk, const double *logk, bool accumulate, hipStream_t st)
{
    LAUNCH(k_sensitivity, (S->ne + WG - 1) / WG, WG, st, S->ne, S->tets, S->tet_orig, S->xyz, logk, S->gprm, S->slice_group, U, P, lu,
           lp, S->dir_u, S->dir_p, dE, dlogk, accumulate ? 1 : 0);
}

void apply_Apu(fg_system *S, const double *p, double *out, hipStream_t st)
{
    const Plan &P = S->plan;
    vfill(out, 0.0, 3 * S->Npad, st);
    for (size_t c = 0; c + 1 < P.colour_ptr.size(); ++c) {
        const int64_t a = P.colour_ptr[c], b = P.colour_ptr[c + 1];
        if (b > a) LAUNCH(k_apu_tets, (b - a + WG - 1) / WG, WG, st, a, b, S->tets, S->xyz, S->gprm, S->slice_group, p,
                          S->dir_p, out);
    }
    if (S->nf > 0)
        LAUNCH(k_apu_fault, (S->nfr + WG - 1) / WG, WG, st, S->nfr, S->frows, S->fadj_ptr, S->fadj, S->coh, S->tri_geo,
               p, S->dir_p, out);
    vmask(3 * S->Npad, S->dir_u, out, st);
}

void apply_Aup(fg_system *S, const double *u, double *out, hipStream_t st)
{
    const Plan &P = S->plan;
    vfill(out, 0.0, S->Npad, st);
    for (size_t c = 0; c + 1 < P.colour_ptr.size(); ++c) {
        const int64_t a = P.colour_ptr[c], b = P.colour_ptr[c + 1];
        if (b > a) LAUNCH(k_aup_tets, (b - a + WG - 1) / WG, WG, st, a, b, S->tets, S->xyz, S->gprm, S->slice_group, u,
                          S->dir_u, out);
    }
    if (S->nf > 0)
        LAUNCH(k_aup_fault, (S->nfr + WG - 1) / WG, WG, st, S->nfr, S->frows, S->fadj_ptr, S->fadj, S->coh, S->tri_geo,
               u, S->dir_u, out);
    vmask(S->Npad, S->dir_p, out, st);
}

void spmv(fg_system *S, int which, const double *x, double *y, hipStream_t st)
{
    const int64_t g = grid_xcd((S->nslices + 3) / 4);
    const SpmvArgs a = spmv_args(S);
    if (which == FG_K || which == FG_KBULK) {
        LAUNCH_SH((k_spmv<3, double, double>), g, WG, (spmv_lds<3, double>(S)), st, a, S->K, x, y);
        if (which == FG_KBULK && S->nf > 0)
            LAUNCH(k_spmv_fault_bulk, (S->nfr + WG - 1) / WG, WG, st, S->nfr, S->fault_w, S->frows, S->slice_ptr,
                   S->col, S->rowlen, S->Kfb, x, y);
    } else {
        const double *v = which == FG_A22 ? S->A22 : S->Cm;
        LAUNCH_SH((k_spmv<1, double, double>), g, WG, (spmv_lds<1, double>(S)), st, a, v, x, y);
    }
}

void spmv_k32(fg_system *S, const float *x, float *y, hipStream_t st)
{
    const int64_t g = grid_xcd((S->nslices + 3) / 4);
    LAUNCH_SH((k_spmv<3, float, float>), g, WG, (spmv_lds<3, float>(S)), st, spmv_args(S), S->K32, x, y);
}

// Sum the durations of the timed launches of the last batch (stream already
// synchronised); only the first `worked` launches ran a real iteration, the
// rest returned at once because the solve had stopped.
static void prof_collect(fg_system *S, int64_t worked)
{
    const int n = (int)std::min<int64_t>(S->prof_pending, std::max<int64_t>(worked, 0));
    const std::vector<hipEvent_t> &ev = S->prof_ev[S->prof_slot];
    for (int i = 0; i < n; ++i) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) {
            S->prof_ms[S->prof_slot] += ms;
            S->prof_count[S->prof_slot] += 1;
        } else {
            hipGetLastError();  // an untimed launch is not an error of the solve
        }
    }
    S->prof_pending = 0;
}

// The CG product with the tuned slot unroll depth, access hints and waves per workgroup.
template <int BS, typename T, typename TV>
static void cg_spmv_launch(fg_system *S, int64_t gs, const TV *val, const T *p, T *q, hipStream_t st)
{
    const size_t lds = (size_t)S->spmv_wpb * S->halo_cap * BS * sizeof(T);
    const SpmvArgs a = spmv_args(S);
#define FG_CG_SPMV_W(U, N, W)                                                                               \
    LAUNCH_SH((k_cg_spmv<BS, T, TV, U, N, W>), gs, 64 * W, lds, st, a, val, p, q, S->partials, S->npartials, \
              S->sc)
#define FG_CG_SPMV(U, N)                  \
    switch (S->spmv_wpb) {                \
    case 1: FG_CG_SPMV_W(U, N, 1); break; \
    case 2: FG_CG_SPMV_W(U, N, 2); break; \
    default: FG_CG_SPMV_W(U, N, 4); break; \
    }
#define FG_CG_SPMV_NT(U)                   \
    switch (S->spmv_nt) {                  \
    case 0: FG_CG_SPMV(U, 0); break;       \
    case 1: FG_CG_SPMV(U, 1); break;       \
    case 3: FG_CG_SPMV(U, 3); break;       \
    case 7: FG_CG_SPMV(U, 7); break;       \
    case 15: FG_CG_SPMV(U, 15); break;     \
    default: FG_CG_SPMV(U, 23); break;     \
    }
    switch (S->spmv_unroll) {
    case 1: FG_CG_SPMV_NT(1); break;
    case 2: FG_CG_SPMV_NT(2); break;
    case 4: FG_CG_SPMV_NT(4); break;
    case 6: FG_CG_SPMV_NT(6); break;
    default: FG_CG_SPMV_NT(3); break;
    }
#undef FG_CG_SPMV_NT
#undef FG_CG_SPMV
#undef FG_CG_SPMV_W
}

// q = K p with the CG product kernel and launch parameters (stops with the solve's
// flag in S->sc); the per-block partials of p.q go to row 0 of S->partials.
// Returns the number of blocks (partials).
int64_t cg_spmv_k(fg_system *S, const double *p, double *q, hipStream_t st)
{
    const int64_t gs = grid_xcd((S->nslices + S->spmv_wpb - 1) / S->spmv_wpb);
    cg_spmv_launch<3, double, double>(S, gs, S->K, p, q, st);
    return gs;
}

template <typename T>
static BlockJacobi<T> bj_args(fg_system *S);
template <>
BlockJacobi<double> bj_args<double>(fg_system *S)
{
    return BlockJacobi<double>{S->bjA, S->bjB, S->fslot, S->fpart, S->wz};
}
template <>
BlockJacobi<float> bj_args<float>(fg_system *S)
{
    return BlockJacobi<float>{S->bjA32, S->bjB32, S->fslot, S->fpart, S->wz32};
}

template <int BS, typename T, typename TV>
static void cg_launch_batch(fg_system *S, const TV *val, const T *dinv, T *x, T *r, T *p, T *q, int iters, int slot,
                            bool prof, hipStream_t st)
{
    const std::vector<hipEvent_t> &ev = S->prof_ev[slot];
    const int64_t n = BS * S->Npad;
    const int64_t gs = grid_xcd((S->nslices + S->spmv_wpb - 1) / S->spmv_wpb);
    const int64_t ge = std::min<int64_t>(grid_vec(n) * S->vec_grid / 512, std::max<int64_t>((n + WG - 1) / WG, 1));
    for (int it = 0; it < iters; ++it) {
        const int par = it & 1;  // batches have an even length and start at parity 0
        if (prof) hipEventRecord(ev[2 * it], st);
        cg_spmv_launch<BS, T, TV>(S, gs, val, p, q, st);
        if (prof) hipEventRecord(ev[2 * it + 1], st);
        if constexpr (BS == 3 && std::is_same<T, TV>::value) {
            if (S->k_precond) {
                const BlockJacobi<T> bj = bj_args<T>(S);
                LAUNCH((k_cg_update_bj<T>), ge, WG, st, S->Npad, par, bj, x, r, p, q, S->partials, S->npartials, gs,
                       S->sc);
                LAUNCH((k_cg_pupdate_bj<T>), ge, WG, st, n, par, bj.z, p, S->partials, S->npartials, ge, S->sc);
                continue;
            }
        }
        LAUNCH((k_cg_update<T>), ge, WG, st, n, par, dinv, x, r, p, q, S->partials, S->npartials, gs, S->sc);
        LAUNCH((k_cg_pupdate<T>), ge, WG, st, n, par, dinv, r, p, S->partials, S->npartials, ge, S->sc);
    }
}

// One batch of CG iterations.  With graphs enabled the batch is captured once
// per (operator slot, batch length) on the system's capture stream and
// replayed on `st`: every kernel argument is a fixed workspace pointer of the
// system, so the graph stays valid until fg_tune changes a launch parameter or
// the system is destroyed.  Timed batches (fg_profile) launch kernel by kernel
// with fence-free events on `st` around each SpMV: event records captured into
// a graph are not ordered against the kernels between them.
template <int BS, typename T, typename TV>
static fg_status cg_batch(fg_system *S, const TV *val, const T *dinv, T *x, T *r, T *p, T *q, int iters, int slot,
                          hipStream_t st)
{
    if (S->prof) {
        std::vector<hipEvent_t> &ev = S->prof_ev[slot];
        while ((int)ev.size() < 2 * iters) {
            hipEvent_t e;
            hipEventCreateWithFlags(&e, hipEventDisableSystemFence);  // no cache write-back around the kernel
            ev.push_back(e);
        }
        S->prof_slot = slot;
        S->prof_pending = iters;
        cg_launch_batch<BS, T, TV>(S, val, dinv, x, r, p, q, iters, slot, true, st);
        return check_hip("cg batch");
    }
    if (!S->use_graphs) {
        cg_launch_batch<BS, T, TV>(S, val, dinv, x, r, p, q, iters, slot, false, st);
        return check_hip("cg batch");
    }
    GraphCache &g = S->cg_graph[slot];
    if (!g.exec || g.iters != iters) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(S->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return check_hip("cg graph capture");
        cg_launch_batch<BS, T, TV>(S, val, dinv, x, r, p, q, iters, slot, false, S->cap_stream);
        if (hipStreamEndCapture(S->cap_stream, &graph) != hipSuccess) return check_hip("cg graph capture end");
        hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g.exec = nullptr;
            return check_hip("cg graph instantiate");
        }
        g.iters = iters;
    }
    hipGraphLaunch(g.exec, st);
    return check_hip("cg graph launch");
}

void drop_graphs(fg_system *S)
{
    for (GraphCache &g : S->cg_graph) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.iters = 0;
    }
}

// Block-Jacobi data of the current K, built on first use after K changed.
void bj_ready(fg_system *S, hipStream_t st)
{
    if (S->bj_valid) return;
    int *bad = (int *)S->red_counter + 2;
    hipMemsetAsync(bad, 0, sizeof(int), st);
    LAUNCH(k_bj_build, (S->Npad + WG - 1) / WG, WG, st, S->Npad, S->K, S->slice_ptr, S->col, S->rowlen, S->diag_slot,
           S->fslot, S->fpart, S->bjA, S->bjB, bad);
    int h = 0;
    hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    S->bj_singular = h != 0;
    S->bj_valid = true;
    ++S->bj_epoch;
    S->bj32_valid = false;
}

// FP32 copy of the block-Jacobi data (FP32 CG of the mixed-precision solve).
void bj_ready32(fg_system *S, hipStream_t st)
{
    bj_ready(S, st);
    if (S->bj32_valid) return;
    to_f32(6 * S->Npad, 1.0, S->bjA, S->bjA32, st);
    if (S->nfr > 0) to_f32(9 * S->nfr, 1.0, S->bjB, S->bjB32, st);
    S->bj32_valid = true;
}

// Batches of CG iterations on the state the init (or a resume) left, polled every
// check_every iterations until the device-side stop flag is set.
static fg_status cg_loop(fg_system *S, int which, int precision, int check_every, hipStream_t st)
{
    const bool f32 = (which == FG_K && precision == FG_F32);
    const bool f32val = (which == FG_K && precision == FG_MIXED_F32VAL);
    // even batches keep the scalars' parity at 0 between polls
    const int batch = check_every > 0 ? (check_every + 1) / 2 * 2 : 32;
    int64_t iter0 = -1;
    S->prof_pending = 0;
    fg_status e;
    for (;;) {
        hipMemcpyAsync(S->sc_host, S->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, st);
        hipStreamSynchronize(st);
        e = check_hip("cg poll");
        if (e) return e;
        if (S->prof_pending && iter0 >= 0) prof_collect(S, S->sc_host->iters - iter0);
        if (S->sc_host->done) break;
        iter0 = S->sc_host->iters;
        if (f32)
            e = cg_batch<3, float, float>(S, S->K32, S->dinvK32, S->fx, S->fr, S->fp, S->fq, batch, 1, st);
        else if (f32val)
            e = cg_batch<3, double, float>(S, S->K32, S->dinvK, S->wx, S->wr, S->wp, S->wq, batch, 3, st);
        else if (which == FG_K)
            e = cg_batch<3, double, double>(S, S->K, S->dinvK, S->wx, S->wr, S->wp, S->wq, batch, 0, st);
        else
            e = cg_batch<1, double, double>(S, S->A22, S->dinvA, S->wx, S->wr, S->wp, S->wq, batch, 2, st);
        if (e) return e;
    }
    const CgScalars &h = *S->sc_host;
    if (h.status == FG_ERR_BREAKDOWN)
        set_error("fg_pcg_solve: CG breakdown (p.Ap <= 0, or a zero diagonal entry under point Jacobi): operator not SPD");
    if (h.status == FG_ERR_NAN) set_error("fg_pcg_solve: NaN or Inf in the CG iteration");
    return h.status;
}

static void cg_init(fg_system *S, int which, int precision, double tol, int64_t maxit, hipStream_t st)
{
    const int bs = which == FG_K ? 3 : 1;
    const int64_t n = bs * S->Npad;
    CgScalars init{};
    init.maxit = maxit;
    hipMemcpyAsync(S->sc, &init, sizeof init, hipMemcpyHostToDevice, st);
    const bool f32 = (which == FG_K && precision == FG_F32);
    const bool f32val = (which == FG_K && precision == FG_MIXED_F32VAL);
    if (f32 || f32val)
        if (!S->k32_valid) refresh_k32(S, st);
    if (f32 && S->k_precond) {
        bj_ready32(S, st);
        LAUNCH((k_cg_init_bj<float>), grid_elems(n), WG, st, S->Npad, bj_args<float>(S), S->fx, S->fr, S->fp,
               S->partials, S->npartials);
    } else if (f32) {
        LAUNCH((k_cg_init<float>), grid_elems(n), WG, st, n, S->dinvK32, S->fx, S->fr, S->fp, S->partials, S->npartials);
    } else if (which == FG_K && !f32val && S->k_precond) {
        bj_ready(S, st);
        LAUNCH((k_cg_init_bj<double>), grid_elems(n), WG, st, S->Npad, bj_args<double>(S), S->wx, S->wr, S->wp,
               S->partials, S->npartials);
    } else if (which == FG_K) {
        LAUNCH((k_cg_init<double>), grid_elems(n), WG, st, n, S->dinvK, S->wx, S->wr, S->wp, S->partials, S->npartials);
    } else {
        LAUNCH((k_cg_init<double>), grid_elems(n), WG, st, n, S->dinvA, S->wx, S->wr, S->wp, S->partials, S->npartials);
    }
    LAUNCH(k_cg_init_fin, 1, FIN, st, S->partials, S->npartials, grid_elems(n), S->sc, tol);
}

fg_status cg_run(fg_system *S, int which, int precision, double tol, int64_t maxit, int check_every, int64_t *iters,
                 double *relres, hipStream_t st)
{
    if (S->ngroups > 1) return cg_run_grouped(S, which, precision, tol, maxit, check_every, iters, relres, st);
    cg_init(S, which, precision, tol, maxit, st);
    fg_status e = check_hip("cg init");
    if (e) return e;
    if (which == FG_K && (precision == FG_F64 || precision == FG_F32) && S->k_precond && S->bj_singular) {
        set_error("fg_pcg_solve: a diagonal or fault-pair block of K is singular (block Jacobi)");
        return FG_ERR_BREAKDOWN;
    }
    e = cg_loop(S, which, precision, check_every, st);
    const CgScalars &h = *S->sc_host;
    *iters = h.iters;
    *relres = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    return e;
}

// Mixed-precision K solve with reliable updates: FP32 CG (matrix, vectors and
// arithmetic) on the residual equation scaled by 1/||b||; whenever its recursive
// residual has dropped by `delta` since the last update, the FP32 solution is
// added to the FP64 one, the true residual b - K x is formed with the FP64
// operator and replaces the FP32 residual, and CG continues with its search
// direction (no restart).  Stops on the FP64 true residual.
static double norm2(fg_system *S, int64_t n, const double *a, hipStream_t st)
{
    const double *A[1] = {a};
    double r = 0;
    vdots(S, n, 1, A, A, &r, st);
    return std::sqrt(r);
}

fg_status cg_reliable(fg_system *S, const double *b, double *x, double tol, int64_t maxit, int check_every,
                      double delta, int64_t *iters, int64_t *updates, double *relres, hipStream_t st)
{
    const int64_t n = 3 * S->Npad;
    double *r = S->v4;
    *iters = 0;
    *updates = 0;
    vfill(x, 0.0, n, st);
    const double bn = norm2(S, n, b, st);
    *relres = bn > 0 ? 1.0 : 0.0;
    if (!(bn > 0)) return std::isfinite(bn) ? FG_OK : FG_ERR_NAN;
    if (!S->k32_valid) refresh_k32(S, st);
    to_f32(n, 1.0 / bn, b, S->fr, st);
    cg_init(S, FG_K, FG_F32, delta, maxit, st);
    fg_status e = check_hip("mixed cg init");
    if (e) return e;
    for (;;) {
        fg_status s = cg_loop(S, FG_K, FG_F32, check_every, st);
        if (s < 0) return s;
        *iters = S->sc_host->iters;
        // fold the FP32 correction into x and replace the residual by the FP64 one
        add_f32(n, bn, S->fx, x, st);
        hipMemsetAsync(S->fx, 0, n * sizeof(float), st);
        spmv(S, FG_K, x, S->wq, st);
        hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, st);
        vaxpby(n, -1.0, S->wq, 1.0, r, st);
        ++*updates;
        const double rel = norm2(S, n, r, st) / bn;
        *relres = rel;
        if (!std::isfinite(rel)) {
            set_error("fg_pcg_solve: NaN in the mixed-precision residual");
            return FG_ERR_NAN;
        }
        if (rel <= tol) return FG_OK;
        if (s == FG_NOT_CONVERGED || *iters >= maxit) return FG_NOT_CONVERGED;
        to_f32(n, 1.0 / bn, r, S->fr, st);
        const double next = std::max(delta * rel, 0.5 * tol);
        if (S->k_precond) {
            const BlockJacobi<float> bj = bj_args<float>(S);
            LAUNCH((k_cg_init_bj<float>), grid_elems(n), WG, st, S->Npad, bj, (float *)nullptr, S->fr, (float *)nullptr,
                   S->partials, S->npartials);
            LAUNCH(k_cg_resume_fin, 1, FIN, st, S->partials, S->npartials, grid_elems(n), S->sc, next * next);
            LAUNCH((k_cg_resume_p_bj<float>), grid_elems(n), WG, st, n, bj.z, S->fp, S->sc);
        } else {
            LAUNCH((k_cg_resume<float>), grid_elems(n), WG, st, n, S->dinvK32, S->fr, S->partials, S->npartials);
            LAUNCH(k_cg_resume_fin, 1, FIN, st, S->partials, S->npartials, grid_elems(n), S->sc, next * next);
            LAUNCH((k_cg_resume_p<float>), grid_elems(n), WG, st, n, S->dinvK32, S->fr, S->fp, S->sc);
        }
        e = check_hip("mixed cg resume");
        if (e) return e;
    }
}

}  // namespace fg
