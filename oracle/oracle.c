/*
 * CPU ORACLE (test infrastructure, not product code).
 *
 * A plain, slow, FP64 reference of the solver's hot path: element matrices of
 * linear tetrahedra and zero-thickness interface triangles, scalar-CSR
 * assembly, the Coulomb return map, matrix-free coupling products, point-Jacobi
 * CG, the partitioned (Prevost) CG on the pressure Schur complement and the
 * Newton loop of one implicit step.  It shares no code with the HIP library.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.
 *
 * Paper: Gallyamov et al., "A Parallelized 3D Geomechanical Solver for
 * Fluid-induced Fault Slip in Poroelastic Media" (arXiv 2410.17133).
 * Each routine names the section / equation it follows.
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *  - element matrices are the 3D analogues of the 2D operators of Appendix A
 *    (Voigt order xx,yy,zz,yz,xz,xy with engineering shear strains);
 *  - storage mass is consistent, fracture storage uses S_F = 1/M_F;
 *  - fracture normals, areas and tangents are frozen at the reference geometry;
 *  - 3-point interior Gauss rule on interface triangles;
 *  - the Newton tangent keeps only the symmetric part of the slip tangent;
 *  - the fracture coupling A^f_pu is the transpose of A^f_up (eq. afdpd), i.e.
 *    a factor 1/2 on the mean pressure acting on each lip;
 *  - Dirichlet DOFs are eliminated symmetrically (row and column zero, unit
 *    diagonal) and the coupling operators are masked on both sides.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double nu, alpha, biot_M, mu, k_par, k_perp, w0, M_F, k_n, k_s, friction, dt;
} or_params;

typedef struct {
    int64_t n, nnz;
    int64_t *rowptr;
    int32_t *col;
    double *val;
} or_csr;

typedef struct {
    int64_t N, ne, nf;
    double *xyz;
    int32_t *tets, *coh;
    double *E, *logk;
    uint8_t *dir_u, *dir_p;
    or_params p;
    or_csr Kb, Kt, A22, C;
    /* reference interface geometry per triangle */
    double *tri_A, *tri_n, *tri_t1, *tri_t2;
    /* last interface update's qp states (for the adjoint's non-symmetric correction) */
    double *qp_trac, *qp_ttr, *qp_tau;
    uint8_t *qp_flag;
} or_problem;

enum { OR_STICK = 0, OR_SLIP = 1, OR_OPEN = 2 };

/* ------------------------------------------------------------------ */
/* small dense helpers                                                 */
/* ------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Linear tetrahedron: volume and gradients of the four shape functions.
 * With J = [x1-x0, x2-x0, x3-x0] (edge vectors as columns), x = x0 + J xi, the
 * gradient of N_{c+1} = xi_c is row c of J^{-1} and grad N_0 = -sum (Sec. 3.1,
 * first-order elements; Appendix A gives the 2D B_p). */
void or_tet_grad(const double *X /*[4][3]*/, double *V, double *g /*[4][3]*/)
{
    double J[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J[r][c] = X[3 * (c + 1) + r] - X[r];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    *V = fabs(det) / 6.0;
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) g[3 * (c + 1) + r] = inv[c][r];
    for (int r = 0; r < 3; ++r) g[r] = -(g[3 + r] + g[6 + r] + g[9 + r]);
}

/* Bulk stiffness K_e = V B^T D B (eq. discrete_balance, first term; Appendix A
 * B_u in 3D).  Ke is 12x12 row-major, DOF order (node a, component i) -> 3a+i. */
void or_tet_stiffness(const double *X, double E, double nu, double *Ke)
{
    double V, g[12];
    or_tet_grad(X, &V, g);
    double B[6][12];
    memset(B, 0, sizeof B);
    for (int a = 0; a < 4; ++a) {
        const double *ga = g + 3 * a;
        B[0][3 * a + 0] = ga[0];
        B[1][3 * a + 1] = ga[1];
        B[2][3 * a + 2] = ga[2];
        B[3][3 * a + 1] = ga[2]; /* gamma_yz */
        B[3][3 * a + 2] = ga[1];
        B[4][3 * a + 0] = ga[2]; /* gamma_xz */
        B[4][3 * a + 2] = ga[0];
        B[5][3 * a + 0] = ga[1]; /* gamma_xy */
        B[5][3 * a + 1] = ga[0];
    }
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double G = E / (2.0 * (1.0 + nu));
    double D[6][6];
    memset(D, 0, sizeof D);
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) D[i][j] = lam;
        D[i][i] = lam + 2.0 * G;
        D[3 + i][3 + i] = G;
    }
    double DB[6][12];
    for (int i = 0; i < 6; ++i)
        for (int c = 0; c < 12; ++c) {
            double s = 0;
            for (int k = 0; k < 6; ++k) s += D[i][k] * B[k][c];
            DB[i][c] = s;
        }
    for (int r = 0; r < 12; ++r)
        for (int c = 0; c < 12; ++c) {
            double s = 0;
            for (int k = 0; k < 6; ++k) s += B[k][r] * DB[k][c];
            Ke[12 * r + c] = V * s;
        }
}

/* Matrix coupling block A^m_pu,e (eq. Apdp): alpha * int B_u^T m N_p with one
 * integration point; int N_b = V/4 for a linear tetrahedron.  Ae is 12x4. */
void or_tet_coupling(const double *X, double alpha, double *Ae)
{
    double V, g[12];
    or_tet_grad(X, &V, g);
    for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 4; ++b) Ae[4 * (3 * a + i) + b] = alpha * 0.25 * V * g[3 * a + i];
}

/* Matrix flow blocks (eq. discrete_mass): storage S_e = (1/M) int N_a N_b
 * (consistent mass, V(1+delta_ab)/20) and conductivity C_e = (k/mu) V grad N_a . grad N_b. */
void or_tet_flow(const double *X, double perm_over_mu, double inv_M, double *Se, double *Ce)
{
    double V, g[12];
    or_tet_grad(X, &V, g);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            Se[4 * a + b] = inv_M * V * (a == b ? 2.0 : 1.0) / 20.0;
            Ce[4 * a + b] = perm_over_mu * V * dot3(g + 3 * a, g + 3 * b);
        }
}

/* Interface triangle geometry in the reference configuration (Sec. 3.1.1):
 * area, unit normal n (from the - lip to the + lip, given the vertex order),
 * in-plane tangent t1 (projection of +z, else of +x) and t2 = n x t1, and the
 * in-plane gradients of the three linear shape functions. */
void or_tri_geom(const double *X /*[3][3]*/, double *A, double *n, double *t1, double *t2, double *gG /*[3][3]*/)
{
    double e1[3], e2[3], c[3];
    for (int r = 0; r < 3; ++r) {
        e1[r] = X[3 + r] - X[r];
        e2[r] = X[6 + r] - X[r];
    }
    cross3(e1, e2, c);
    double cn = sqrt(dot3(c, c));
    *A = 0.5 * cn;
    for (int r = 0; r < 3; ++r) n[r] = c[r] / cn;
    double ez[3] = {0, 0, 1}, ex[3] = {1, 0, 0};
    double v[3];
    double s = dot3(ez, n);
    for (int r = 0; r < 3; ++r) v[r] = ez[r] - s * n[r];
    double vn = sqrt(dot3(v, v));
    if (vn < 1e-8) {
        s = dot3(ex, n);
        for (int r = 0; r < 3; ++r) v[r] = ex[r] - s * n[r];
        vn = sqrt(dot3(v, v));
    }
    for (int r = 0; r < 3; ++r) t1[r] = v[r] / vn;
    cross3(n, t1, t2);
    /* grad N_a = n x (x_c - x_b) / (2A) for (a,b,c) cyclic */
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, cc = (a + 2) % 3;
        double d[3];
        for (int r = 0; r < 3; ++r) d[r] = X[3 * cc + r] - X[3 * b + r];
        cross3(n, d, gG + 3 * a);
        for (int r = 0; r < 3; ++r) gG[3 * a + r] /= (2.0 * *A);
    }
}

/* Fracture flow on one interface element (eq. discrete_mass_fracture with the
 * double-node operators of eq. operators).  6x6 blocks in the order
 * [+a,+b,+c,-a,-b,-c]:  storage w0 S_F int <r><p>;  longitudinal
 * (w0 k_par/mu) int grad<r>.grad<p>;  transverse (k_perp/(mu w0)) int [[r]][[p]]. */
void or_tri_flow(const double *X, const or_params *p, double *Sf, double *Cf)
{
    double A, n[3], t1[3], t2[3], gG[9];
    or_tri_geom(X, &A, n, t1, t2, gG);
    double M3[3][3], CG[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            M3[a][b] = A * (a == b ? 2.0 : 1.0) / 12.0;
            CG[a][b] = A * dot3(gG + 3 * a, gG + 3 * b);
        }
    double cs = p->w0 / p->M_F, cl = p->w0 * p->k_par / p->mu, ct = p->k_perp / (p->mu * p->w0);
    for (int sa = 0; sa < 2; ++sa)
        for (int sb = 0; sb < 2; ++sb) {
            double jump = (sa == sb) ? 1.0 : -1.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    int r = 3 * sa + a, c = 3 * sb + b;
                    Sf[6 * r + c] = cs * 0.25 * M3[a][b];
                    Cf[6 * r + c] = cl * 0.25 * CG[a][b] + ct * jump * M3[a][b];
                }
        }
}

/* Elastic predictor / plastic corrector at one interface quadrature point
 * (Sec. 2.2.1: eq. normal_traction, yield_function, slip_split,
 * plastic_slip_increment, kuhn-tucker, corrector).
 *   d[3]    opening (n, t1, t2 components) of the displacement since t = 0
 *   die_n   inelastic slip at the start of the step
 *   t0[3]   initial effective traction (t'_n0, t'_s0 along t1, t2)
 * Out: trac = (t'_n, t_s1, t_s2), die, flag, and the local 3x3 symmetric
 * tangent Dl (frame n,t1,t2).  Returns the trial-traction norm. */
double or_return_map(const double *d, const double *die_n, const double *t0, double kn, double ks, double f,
                     double *trac, double *die, uint8_t *flag, double *Dl)
{
    double dn0 = -t0[0] / kn;
    double ds0[2] = {t0[1] / ks, t0[2] / ks};
    double dnt = dn0 + d[0];
    double tn = dnt < 0 ? -kn * dnt : 0.0;
    double ttr[2] = {ks * (ds0[0] + d[1] - die_n[0]), ks * (ds0[1] + d[2] - die_n[1])};
    double nt = sqrt(ttr[0] * ttr[0] + ttr[1] * ttr[1]);
    double F = nt - f * tn;
    memset(Dl, 0, 9 * sizeof(double));
    if (F <= 0.0) {
        trac[1] = ttr[0];
        trac[2] = ttr[1];
        die[0] = die_n[0];
        die[1] = die_n[1];
        *flag = dnt > 0 ? OR_OPEN : OR_STICK;
        if (*flag == OR_STICK) {
            Dl[4] = ks;
            Dl[8] = ks;
        }
    } else {
        double tau[2] = {1.0, 0.0};
        if (nt > 0) {
            tau[0] = ttr[0] / nt;
            tau[1] = ttr[1] / nt;
        }
        double dl = F / ks;
        die[0] = die_n[0] + dl * tau[0];
        die[1] = die_n[1] + dl * tau[1];
        trac[1] = f * tn * tau[0];
        trac[2] = f * tn * tau[1];
        *flag = dnt > 0 ? OR_OPEN : OR_SLIP;
        if (*flag == OR_SLIP) {
            double c = ks * f * tn / nt;
            Dl[4] = c * (1.0 - tau[0] * tau[0]);
            Dl[5] = c * (-tau[0] * tau[1]);
            Dl[7] = c * (-tau[1] * tau[0]);
            Dl[8] = c * (1.0 - tau[1] * tau[1]);
        }
    }
    trac[0] = tn;
    if (dnt <= 0) Dl[0] = kn;
    return nt;
}

/* ------------------------------------------------------------------ */
/* CSR                                                                 */
/* ------------------------------------------------------------------ */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int64_t csr_find(const or_csr *A, int64_t row, int32_t col)
{
    int64_t lo = A->rowptr[row], hi = A->rowptr[row + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int32_t c = A->col[mid];
        if (c == col) return mid;
        if (c < col) lo = mid + 1;
        else hi = mid - 1;
    }
    abort(); /* entry outside the element graph: a bug in the caller */
}

static void csr_free(or_csr *A)
{
    free(A->rowptr);
    free(A->col);
    free(A->val);
    memset(A, 0, sizeof *A);
}

/* Node graph: nodes coupled through a tetrahedron or an interface element. */
static void node_graph(const or_problem *P, int64_t **rp_out, int32_t **adj_out)
{
    int64_t N = P->N;
    int64_t *cnt = calloc(N + 1, sizeof(int64_t));
    for (int64_t e = 0; e < P->ne; ++e)
        for (int a = 0; a < 4; ++a) cnt[P->tets[4 * e + a] + 1] += 4;
    for (int64_t t = 0; t < P->nf; ++t)
        for (int a = 0; a < 6; ++a) cnt[P->coh[6 * t + a] + 1] += 6;
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    int32_t *lst = malloc(cnt[N] * sizeof(int32_t));
    int64_t *pos = malloc(N * sizeof(int64_t));
    memcpy(pos, cnt, N * sizeof(int64_t));
    for (int64_t e = 0; e < P->ne; ++e)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) lst[pos[P->tets[4 * e + a]]++] = P->tets[4 * e + b];
    for (int64_t t = 0; t < P->nf; ++t)
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) lst[pos[P->coh[6 * t + a]]++] = P->coh[6 * t + b];
    int64_t *rp = calloc(N + 1, sizeof(int64_t));
    for (int64_t i = 0; i < N; ++i) {
        int32_t *row = lst + cnt[i];
        int64_t len = cnt[i + 1] - cnt[i];
        qsort(row, len, sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t k = 0; k < len; ++k)
            if (u == 0 || row[k] != row[u - 1]) row[u++] = row[k];
        rp[i + 1] = u;
    }
    for (int64_t i = 0; i < N; ++i) rp[i + 1] += rp[i];
    int32_t *adj = malloc(rp[N] * sizeof(int32_t));
    for (int64_t i = 0; i < N; ++i) {
        int64_t len = rp[i + 1] - rp[i];
        memcpy(adj + rp[i], lst + cnt[i], len * sizeof(int32_t));
    }
    free(lst);
    free(pos);
    free(cnt);
    *rp_out = rp;
    *adj_out = adj;
}

/* Expand the node graph to a scalar CSR with `d` DOFs per node. */
static void csr_from_graph(or_csr *A, int64_t N, const int64_t *rp, const int32_t *adj, int d)
{
    A->n = N * d;
    A->nnz = rp[N] * d * d;
    A->rowptr = malloc((A->n + 1) * sizeof(int64_t));
    A->col = malloc(A->nnz * sizeof(int32_t));
    A->val = calloc(A->nnz, sizeof(double));
    A->rowptr[0] = 0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t len = rp[i + 1] - rp[i];
        for (int c = 0; c < d; ++c) {
            int64_t r = i * d + c, base = rp[i] * d * d + c * len * d;
            A->rowptr[r + 1] = base + len * d;
            for (int64_t k = 0; k < len; ++k)
                for (int cc = 0; cc < d; ++cc) A->col[base + k * d + cc] = adj[rp[i] + k] * d + cc;
        }
    }
}

static void csr_copy_values(or_csr *dst, const or_csr *src)
{
    if (!dst->rowptr) {
        dst->n = src->n;
        dst->nnz = src->nnz;
        dst->rowptr = malloc((src->n + 1) * sizeof(int64_t));
        dst->col = malloc(src->nnz * sizeof(int32_t));
        dst->val = malloc(src->nnz * sizeof(double));
        memcpy(dst->rowptr, src->rowptr, (src->n + 1) * sizeof(int64_t));
        memcpy(dst->col, src->col, src->nnz * sizeof(int32_t));
    }
    memcpy(dst->val, src->val, src->nnz * sizeof(double));
}

/* Symmetric elimination of masked DOFs: zero row and column, unit diagonal. */
static void csr_eliminate(or_csr *A, const uint8_t *mask)
{
    for (int64_t r = 0; r < A->n; ++r)
        for (int64_t k = A->rowptr[r]; k < A->rowptr[r + 1]; ++k) {
            int32_t c = A->col[k];
            if (mask[r] || mask[c]) A->val[k] = (r == c && mask[r]) ? 1.0 : 0.0;
        }
}

/* Loops shorter than this run on one thread: on the small test meshes the
 * threads' start and barrier cost more than the loop itself.  Only the grouping
 * of the partial sums of dot products depends on it. */
#define OR_PAR_MIN 4096

void or_csr_spmv(const or_csr *A, const double *x, double *y)
{
#pragma omp parallel for schedule(static) if (A->n > OR_PAR_MIN)
    for (int64_t r = 0; r < A->n; ++r) {
        double s = 0;
        for (int64_t k = A->rowptr[r]; k < A->rowptr[r + 1]; ++k) s += A->val[k] * x[A->col[k]];
        y[r] = s;
    }
}

static double vdot(int64_t n, const double *a, const double *b)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static) if (n > OR_PAR_MIN)
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------ */
/* problem set-up and assembly                                         */
/* ------------------------------------------------------------------ */
static void tet_coords(const or_problem *P, int64_t e, double *X)
{
    for (int a = 0; a < 4; ++a)
        for (int r = 0; r < 3; ++r) X[3 * a + r] = P->xyz[3 * (int64_t)P->tets[4 * e + a] + r];
}

static void tri_coords(const or_problem *P, int64_t t, double *X)
{
    /* reference geometry: the - lip (lips coincide at t = 0) */
    for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r) X[3 * a + r] = P->xyz[3 * (int64_t)P->coh[6 * t + 3 + a] + r];
}

/* Assemble K_bulk (Sec. 3.2.1), S and C (Sec. 3.2.2-3.2.3) and A22 = S + dt C
 * (eq. prevost_system), with Dirichlet elimination. */
or_problem *or_create(int64_t N, int64_t ne, int64_t nf, const double *xyz, const int32_t *tets,
                      const int32_t *coh, const double *E, const double *logk, const uint8_t *dir_u,
                      const uint8_t *dir_p, const double *params)
{
    or_problem *P = calloc(1, sizeof *P);
    P->N = N;
    P->ne = ne;
    P->nf = nf;
    P->xyz = malloc(N * 3 * sizeof(double));
    memcpy(P->xyz, xyz, N * 3 * sizeof(double));
    P->tets = malloc(ne * 4 * sizeof(int32_t));
    memcpy(P->tets, tets, ne * 4 * sizeof(int32_t));
    P->coh = malloc((nf ? nf : 1) * 6 * sizeof(int32_t));
    if (nf) memcpy(P->coh, coh, nf * 6 * sizeof(int32_t));
    P->E = malloc(ne * sizeof(double));
    memcpy(P->E, E, ne * sizeof(double));
    P->logk = malloc(ne * sizeof(double));
    memcpy(P->logk, logk, ne * sizeof(double));
    P->dir_u = malloc(3 * N);
    memcpy(P->dir_u, dir_u, 3 * N);
    P->dir_p = malloc(N);
    memcpy(P->dir_p, dir_p, N);
    memcpy(&P->p, params, sizeof(or_params));

    int64_t *rp;
    int32_t *adj;
    node_graph(P, &rp, &adj);
    csr_from_graph(&P->Kb, N, rp, adj, 3);
    csr_from_graph(&P->A22, N, rp, adj, 1);
    csr_from_graph(&P->C, N, rp, adj, 1);
    free(rp);
    free(adj);

    double *S = calloc(P->A22.nnz, sizeof(double));
    for (int64_t e = 0; e < ne; ++e) {
        double X[12], Ke[144], Se[16], Ce[16];
        tet_coords(P, e, X);
        or_tet_stiffness(X, P->E[e], P->p.nu, Ke);
        or_tet_flow(X, exp(P->logk[e]) / P->p.mu, 1.0 / P->p.biot_M, Se, Ce);
        const int32_t *nd = P->tets + 4 * e;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        P->Kb.val[csr_find(&P->Kb, 3 * (int64_t)nd[a] + i, 3 * nd[b] + j)] += Ke[12 * (3 * a + i) + 3 * b + j];
                int64_t k = csr_find(&P->A22, nd[a], nd[b]);
                S[k] += Se[4 * a + b];
                P->C.val[k] += Ce[4 * a + b];
            }
    }
    P->tri_A = malloc((nf ? nf : 1) * sizeof(double));
    P->tri_n = malloc((nf ? nf : 1) * 3 * sizeof(double));
    P->tri_t1 = malloc((nf ? nf : 1) * 3 * sizeof(double));
    P->tri_t2 = malloc((nf ? nf : 1) * 3 * sizeof(double));
    for (int64_t t = 0; t < nf; ++t) {
        double X[9], Sf[36], Cf[36], gG[9];
        tri_coords(P, t, X);
        or_tri_geom(X, P->tri_A + t, P->tri_n + 3 * t, P->tri_t1 + 3 * t, P->tri_t2 + 3 * t, gG);
        or_tri_flow(X, &P->p, Sf, Cf);
        const int32_t *nd = P->coh + 6 * t;
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) {
                int64_t k = csr_find(&P->A22, nd[a], nd[b]);
                S[k] += Sf[6 * a + b];
                P->C.val[k] += Cf[6 * a + b];
            }
    }
    for (int64_t k = 0; k < P->A22.nnz; ++k) P->A22.val[k] = S[k] + P->p.dt * P->C.val[k];
    free(S);
    csr_eliminate(&P->Kb, P->dir_u);
    csr_eliminate(&P->A22, P->dir_p);
    /* C enters only through the residual; rows of held pressures are dropped there */
    csr_copy_values(&P->Kt, &P->Kb);
    int64_t nq = 3 * (nf ? nf : 1);
    P->qp_trac = calloc(nq * 3, sizeof(double));
    P->qp_ttr = calloc(nq, sizeof(double));
    P->qp_tau = calloc(nq * 3, sizeof(double));
    P->qp_flag = calloc(nq, 1);
    return P;
}

void or_free(or_problem *P)
{
    if (!P) return;
    csr_free(&P->Kb);
    csr_free(&P->Kt);
    csr_free(&P->A22);
    csr_free(&P->C);
    free(P->xyz);
    free(P->tets);
    free(P->coh);
    free(P->E);
    free(P->logk);
    free(P->dir_u);
    free(P->dir_p);
    free(P->tri_A);
    free(P->tri_n);
    free(P->tri_t1);
    free(P->tri_t2);
    free(P->qp_trac);
    free(P->qp_ttr);
    free(P->qp_tau);
    free(P->qp_flag);
    free(P);
}

/* which: 0 = K_bulk, 1 = K tangent, 2 = A22, 3 = C */
static or_csr *pick(or_problem *P, int which)
{
    switch (which) {
    case 0: return &P->Kb;
    case 1: return &P->Kt;
    case 2: return &P->A22;
    default: return &P->C;
    }
}

int64_t or_nnz(or_problem *P, int which) { return pick(P, which)->nnz; }

void or_get_csr(or_problem *P, int which, int64_t *rowptr, int32_t *col, double *val)
{
    or_csr *A = pick(P, which);
    memcpy(rowptr, A->rowptr, (A->n + 1) * sizeof(int64_t));
    memcpy(col, A->col, A->nnz * sizeof(int32_t));
    memcpy(val, A->val, A->nnz * sizeof(double));
}

void or_spmv(or_problem *P, int which, const double *x, double *y) { or_csr_spmv(pick(P, which), x, y); }

/* Quadrature on the interface triangle: interior 3-point Gauss rule, weights A/3. */
static const double QP_N[3][3] = {{2.0 / 3, 1.0 / 6, 1.0 / 6}, {1.0 / 6, 2.0 / 3, 1.0 / 6}, {1.0 / 6, 1.0 / 6, 2.0 / 3}};

/* Interface update (Sec. 2.2.1 and eq. discrete_balance_full, fracture term):
 * opening at every quadrature point from the displacement U since t = 0,
 * return map from the start-of-step inelastic slip, the cohesive force
 * sum_q w N_a (T_q - T_0q) (+ lip) / its negative (- lip), where
 * T = -t'_n n + t_s1 t1 + t_s2 t2, and the symmetric tangent added to K_bulk. */
void or_cohesive(or_problem *P, const double *U, const double *die_n, const double *t0, double *trac, double *die,
                 uint8_t *flag, double *fcoh)
{
    int64_t N = P->N;
    memset(fcoh, 0, 3 * N * sizeof(double));
    csr_copy_values(&P->Kt, &P->Kb);
    const double kn = P->p.k_n, ks = P->p.k_s, f = P->p.friction;
    for (int64_t t = 0; t < P->nf; ++t) {
        const int32_t *nd = P->coh + 6 * t;
        const double *n = P->tri_n + 3 * t, *t1 = P->tri_t1 + 3 * t, *t2 = P->tri_t2 + 3 * t;
        double w = P->tri_A[t] / 3.0;
        double Kc[18][18];
        memset(Kc, 0, sizeof Kc);
        for (int q = 0; q < 3; ++q) {
            int64_t iq = 3 * t + q;
            double jump[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a)
                for (int r = 0; r < 3; ++r)
                    jump[r] += QP_N[q][a] * (U[3 * (int64_t)nd[a] + r] - U[3 * (int64_t)nd[3 + a] + r]);
            double d[3] = {dot3(n, jump), dot3(t1, jump), dot3(t2, jump)};
            double Dl[9];
            double nt = or_return_map(d, die_n + 2 * iq, t0 + 3 * iq, kn, ks, f, trac + 3 * iq, die + 2 * iq, flag + iq, Dl);
            P->qp_ttr[iq] = nt;
            P->qp_flag[iq] = flag[iq];
            {
                /* slip direction in global coordinates (from the trial traction) */
                double a = 1.0, b = 0.0;
                if (nt > 0) {
                    double tt1 = ks * (t0[3 * iq + 1] / ks + d[1] - die_n[2 * iq]);
                    double tt2 = ks * (t0[3 * iq + 2] / ks + d[2] - die_n[2 * iq + 1]);
                    a = tt1 / nt;
                    b = tt2 / nt;
                }
                for (int r = 0; r < 3; ++r) P->qp_tau[3 * iq + r] = a * t1[r] + b * t2[r];
            }
            memcpy(P->qp_trac + 3 * iq, trac + 3 * iq, 3 * sizeof(double));
            const double *tr = trac + 3 * iq, *tz = t0 + 3 * iq;
            double T[3];
            for (int r = 0; r < 3; ++r)
                T[r] = -(tr[0] - tz[0]) * n[r] + (tr[1] - tz[1]) * t1[r] + (tr[2] - tz[2]) * t2[r];
            /* global tangent D = R Dl R^T with R = [n t1 t2] */
            const double *R[3] = {n, t1, t2};
            double Dg[3][3];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double s = 0;
                    for (int k = 0; k < 3; ++k)
                        for (int l = 0; l < 3; ++l) s += R[k][r] * Dl[3 * k + l] * R[l][c];
                    Dg[r][c] = s;
                }
            for (int a = 0; a < 3; ++a) {
                double wa = w * QP_N[q][a];
                for (int r = 0; r < 3; ++r) {
                    fcoh[3 * (int64_t)nd[a] + r] += wa * T[r];
                    fcoh[3 * (int64_t)nd[3 + a] + r] -= wa * T[r];
                }
                for (int b = 0; b < 3; ++b) {
                    double wab = wa * QP_N[q][b];
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < 3; ++c) {
                            double v = wab * Dg[r][c];
                            Kc[3 * a + r][3 * b + c] += v;
                            Kc[3 * a + r][9 + 3 * b + c] -= v;
                            Kc[9 + 3 * a + r][3 * b + c] -= v;
                            Kc[9 + 3 * a + r][9 + 3 * b + c] += v;
                        }
                }
            }
        }
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b)
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        int64_t row = 3 * (int64_t)nd[a] + r, col = 3 * (int64_t)nd[b] + c;
                        if (P->dir_u[row] || P->dir_u[col]) continue;
                        P->Kt.val[csr_find(&P->Kt, row, (int32_t)col)] += Kc[3 * a + r][3 * b + c];
                    }
    }
    for (int64_t i = 0; i < 3 * N; ++i)
        if (P->dir_u[i]) fcoh[i] = 0;
}

/* A_pu p = (A^m_pu + A^f_pu) p, masked on held displacement rows and held
 * pressure columns (eq. Apdp and eq. afpdp read as the transpose of eq. afdpd). */
void or_apply_Apu(or_problem *P, const double *p_in, double *out)
{
    int64_t N = P->N;
    double *p = malloc(N * sizeof(double));
    for (int64_t i = 0; i < N; ++i) p[i] = P->dir_p[i] ? 0.0 : p_in[i];
    memset(out, 0, 3 * N * sizeof(double));
    for (int64_t e = 0; e < P->ne; ++e) {
        double X[12], Ae[48];
        tet_coords(P, e, X);
        or_tet_coupling(X, P->p.alpha, Ae);
        const int32_t *nd = P->tets + 4 * e;
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i) {
                double s = 0;
                for (int b = 0; b < 4; ++b) s += Ae[4 * (3 * a + i) + b] * p[nd[b]];
                out[3 * (int64_t)nd[a] + i] += s;
            }
    }
    for (int64_t t = 0; t < P->nf; ++t) {
        const int32_t *nd = P->coh + 6 * t;
        const double *n = P->tri_n + 3 * t;
        double A = P->tri_A[t];
        for (int a = 0; a < 3; ++a) {
            double s = 0;
            for (int b = 0; b < 3; ++b) s += 0.5 * A * (a == b ? 2.0 : 1.0) / 12.0 * (p[nd[b]] + p[nd[3 + b]]);
            for (int r = 0; r < 3; ++r) {
                out[3 * (int64_t)nd[a] + r] += s * n[r];
                out[3 * (int64_t)nd[3 + a] + r] -= s * n[r];
            }
        }
    }
    for (int64_t i = 0; i < 3 * N; ++i)
        if (P->dir_u[i]) out[i] = 0;
    free(p);
}

/* A_up u = (A^m_up + A^f_up) u (eq. Adpd and eq. afdpd), the exact transpose of or_apply_Apu. */
void or_apply_Aup(or_problem *P, const double *u_in, double *out)
{
    int64_t N = P->N;
    double *u = malloc(3 * N * sizeof(double));
    for (int64_t i = 0; i < 3 * N; ++i) u[i] = P->dir_u[i] ? 0.0 : u_in[i];
    memset(out, 0, N * sizeof(double));
    for (int64_t e = 0; e < P->ne; ++e) {
        double X[12], Ae[48];
        tet_coords(P, e, X);
        or_tet_coupling(X, P->p.alpha, Ae);
        const int32_t *nd = P->tets + 4 * e;
        for (int b = 0; b < 4; ++b) {
            double s = 0;
            for (int a = 0; a < 4; ++a)
                for (int i = 0; i < 3; ++i) s += Ae[4 * (3 * a + i) + b] * u[3 * (int64_t)nd[a] + i];
            out[nd[b]] += s;
        }
    }
    for (int64_t t = 0; t < P->nf; ++t) {
        const int32_t *nd = P->coh + 6 * t;
        const double *n = P->tri_n + 3 * t;
        double A = P->tri_A[t];
        for (int b = 0; b < 3; ++b) {
            double s = 0;
            for (int a = 0; a < 3; ++a) {
                double dn = 0;
                for (int r = 0; r < 3; ++r) dn += n[r] * (u[3 * (int64_t)nd[a] + r] - u[3 * (int64_t)nd[3 + a] + r]);
                s += 0.5 * A * (a == b ? 2.0 : 1.0) / 12.0 * dn;
            }
            out[nd[b]] += s;
            out[nd[3 + b]] += s;
        }
    }
    for (int64_t i = 0; i < N; ++i)
        if (P->dir_p[i]) out[i] = 0;
    free(u);
}

/* ------------------------------------------------------------------ */
/* solvers                                                             */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t iters;
    double relres;
    int status; /* 0 converged, 1 not converged, -3 breakdown */
} or_cg_info;

/* Point-Jacobi preconditioned CG (Hestenes-Stiefel, cited in Sec. 3.3.2),
 * x0 = 0, stop on the unpreconditioned ||r||/||b||. */
static or_cg_info pcg(const or_csr *A, const double *b, double *x, double tol, int64_t maxit)
{
    int64_t n = A->n;
    or_cg_info info = {0, 0.0, 0};
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double)), *dinv = malloc(n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        double d = 0;
        for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            if (A->col[k] == i) d = A->val[k];
        dinv[i] = 1.0 / d;
        x[i] = 0;
        r[i] = b[i];
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    double bn = sqrt(vdot(n, b, b));
    if (bn == 0.0) goto done;
    double rho = vdot(n, r, z);
    for (;;) {
        double rn = sqrt(vdot(n, r, r));
        info.relres = rn / bn;
        if (info.relres <= tol) break;
        if (info.iters >= maxit) {
            info.status = 1;
            break;
        }
        or_csr_spmv(A, p, q);
        double pq = vdot(n, p, q);
        if (!(pq > 0.0)) {
            info.status = -3;
            break;
        }
        double al = rho / pq;
#pragma omp parallel for schedule(static) if (n > OR_PAR_MIN)
        for (int64_t i = 0; i < n; ++i) {
            x[i] += al * p[i];
            r[i] -= al * q[i];
            z[i] = dinv[i] * r[i];
        }
        double rho2 = vdot(n, r, z);
        double be = rho2 / rho;
        rho = rho2;
#pragma omp parallel for schedule(static) if (n > OR_PAR_MIN)
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + be * p[i];
        info.iters++;
    }
done:
    free(r);
    free(z);
    free(p);
    free(q);
    free(dinv);
    return info;
}

int or_pcg(or_problem *P, int which, const double *b, double *x, double tol, int64_t maxit, int64_t *iters, double *relres)
{
    or_cg_info in = pcg(pick(P, which), b, x, tol, maxit);
    *iters = in.iters;
    *relres = in.relres;
    return in.status;
}

/* Partitioned CG of Prevost (Sec. 3.3.2, eq. prevost_system and schur_system):
 * solve [[K, -A],[A^T, A22]] [x1; x2] = [b1; b2] through CG on the Schur
 * complement A22 + A^T K^{-1} A preconditioned by A22^{-1}, never forming it;
 * K^{-1} and A22^{-1} are inner Jacobi-PCG solves.  The Polak-Ribiere form of
 * beta keeps the outer iteration stable under inexact inner solves.
 * stats: [outer iters, inner K iters, inner A22 iters, outer relres, status] */
int or_prevost(or_problem *P, const double *b1, const double *b2, double *x1, double *x2, double tol_outer,
               double tol_inner, int64_t maxit_outer, int64_t maxit_inner, double *stats)
{
    int64_t n1 = 3 * P->N, n2 = P->N;
    or_csr *K = &P->Kt, *A22 = &P->A22;
    double *y = calloc(n1, sizeof(double)), *w = calloc(n1, sizeof(double)), *t1 = calloc(n1, sizeof(double));
    double *r = calloc(n2, sizeof(double)), *z = calloc(n2, sizeof(double)), *zn = calloc(n2, sizeof(double));
    double *d = calloc(n2, sizeof(double)), *Sd = calloc(n2, sizeof(double)), *t2 = calloc(n2, sizeof(double));
    int64_t itK = 0, itA = 0, outer = 0;
    int status = 0;
    or_cg_info ci;

    ci = pcg(K, b1, y, tol_inner, maxit_inner); /* y0 = K^-1 b1 */
    itK += ci.iters;
    if (ci.status < 0) status = ci.status;
    or_apply_Aup(P, y, t2);
    for (int64_t i = 0; i < n2; ++i) {
        r[i] = b2[i] - t2[i];
        x2[i] = 0;
    }
    double r0 = sqrt(vdot(n2, r, r));
    double relres = 0;
    if (r0 > 0 && status == 0) {
        ci = pcg(A22, r, z, tol_inner, maxit_inner);
        itA += ci.iters;
        memcpy(d, z, n2 * sizeof(double));
        double rz = vdot(n2, r, z);
        for (;;) {
            or_apply_Apu(P, d, t1);
            ci = pcg(K, t1, w, tol_inner, maxit_inner); /* w = K^-1 A d */
            itK += ci.iters;
            if (ci.status < 0) {
                status = ci.status;
                break;
            }
            or_apply_Aup(P, w, t2);
            or_csr_spmv(A22, d, Sd);
            for (int64_t i = 0; i < n2; ++i) Sd[i] += t2[i];
            double dSd = vdot(n2, d, Sd);
            if (!(dSd > 0)) {
                status = -3;
                break;
            }
            double al = rz / dSd;
            for (int64_t i = 0; i < n2; ++i) {
                x2[i] += al * d[i];
                r[i] -= al * Sd[i];
            }
            for (int64_t i = 0; i < n1; ++i) y[i] += al * w[i];
            outer++;
            relres = sqrt(vdot(n2, r, r)) / r0;
            if (relres <= tol_outer) break;
            if (outer >= maxit_outer) {
                status = 1;
                break;
            }
            ci = pcg(A22, r, zn, tol_inner, maxit_inner);
            itA += ci.iters;
            double rzn = vdot(n2, r, zn);
            double rzo = 0;
            for (int64_t i = 0; i < n2; ++i) rzo += r[i] * z[i];
            double be = (rzn - rzo) / rz;
            for (int64_t i = 0; i < n2; ++i) d[i] = zn[i] + be * d[i];
            memcpy(z, zn, n2 * sizeof(double));
            rz = rzn;
        }
    }
    memcpy(x1, y, n1 * sizeof(double));
    stats[0] = (double)outer;
    stats[1] = (double)itK;
    stats[2] = (double)itA;
    stats[3] = relres;
    stats[4] = (double)status;
    free(y);
    free(w);
    free(t1);
    free(r);
    free(z);
    free(zn);
    free(d);
    free(Sd);
    free(t2);
    return status;
}

static double vnorm(int64_t n, const double *a) { return sqrt(vdot(n, a, a)); }

/* Residuals of eq. nonlinear_system in total form with respect to t = 0:
 *   R_m = K_bulk U + f_coh(U) - A_pu P - F_u
 *   R_f = A_up (U - U_n) + A22 (P - P_n) + dt (C P_n - f_p)
 * rows of held DOFs are zero. */
void or_residual(or_problem *P, const double *U, const double *P_, const double *Un, const double *Pn,
                 const double *fcoh, const double *Fu, const double *fp, double *Rm, double *Rf)
{
    int64_t N = P->N;
    double *t1 = malloc(3 * N * sizeof(double)), *du = malloc(3 * N * sizeof(double));
    double *t2 = malloc(N * sizeof(double)), *dp = malloc(N * sizeof(double));
    or_csr_spmv(&P->Kb, U, Rm);
    or_apply_Apu(P, P_, t1);
    for (int64_t i = 0; i < 3 * N; ++i) Rm[i] = P->dir_u[i] ? 0.0 : Rm[i] + fcoh[i] - t1[i] - Fu[i];
    for (int64_t i = 0; i < 3 * N; ++i) du[i] = U[i] - Un[i];
    for (int64_t i = 0; i < N; ++i) dp[i] = P_[i] - Pn[i];
    or_apply_Aup(P, du, Rf);
    or_csr_spmv(&P->A22, dp, t2);
    for (int64_t i = 0; i < N; ++i) Rf[i] += t2[i];
    or_csr_spmv(&P->C, Pn, t2);
    for (int64_t i = 0; i < N; ++i) Rf[i] = P->dir_p[i] ? 0.0 : Rf[i] + P->p.dt * (t2[i] - fp[i]);
    free(t1);
    free(t2);
    free(du);
    free(dp);
}

/* One implicit step (Sec. 3.3, eq. nonlinear_system and linear_system):
 * Newton on (U, P) from the state at t_n with an elastic-predictor /
 * plastic-corrector interface update at every iterate and a Prevost solve of
 * each Jacobian system.  Convergence: ||R_m|| <= tol s_m and ||R_f|| <= tol s_f
 * with s_m = max(||R_m^0||, ||A_pu P||, ||F_u||), s_f = max(||R_f^0||, dt ||f_p||).
 * In/out: U, P (totals since t = 0), die (inelastic slip per qp).
 * Out: trac, flag per qp.
 * info: [newton its, outer its, inner K its, inner A22 its, ||Rm||/s_m, ||Rf||/s_f, status] */
/* Newton globalisation (not in the paper; the symmetric slip tangent makes full
 * steps overshoot when slip spreads): the merit of an iterate is
 *   phi = (||R_m|| / s*)^2 + (||R_f|| / s_f)^2,
 * s* = max(s_m, ||A_pu (P + dP)||) fixed for the iteration (1 if zero), s_f the
 * flow scale (1 if zero).  Step lengths 1, 1/2, ..., 1/64 are tried in turn and
 * the first that lowers phi is taken; if none does, 1/64 is taken. */
static double merit(double rm, double rf, double s_star, double sf)
{
    const double a = rm / (s_star > 0 ? s_star : 1.0), b = rf / (sf > 0 ? sf : 1.0);
    return a * a + b * b;
}

int or_step(or_problem *P, double *U, double *Pp, double *die, double *trac, uint8_t *flag, const double *t0,
            const double *Fu, const double *fp, double tol_newton, int64_t max_newton, double tol_outer,
            double tol_inner, int64_t maxit_outer, int64_t maxit_inner, int line_search, double *info)
{
    int64_t N = P->N, nq = 3 * P->nf;
    double *Un = malloc(3 * N * sizeof(double)), *Pn = malloc(N * sizeof(double));
    memcpy(Un, U, 3 * N * sizeof(double));
    memcpy(Pn, Pp, N * sizeof(double));
    double *die_n = malloc((nq ? nq : 1) * 2 * sizeof(double));
    memcpy(die_n, die, nq * 2 * sizeof(double));
    double *fcoh = malloc(3 * N * sizeof(double)), *Rm = malloc(3 * N * sizeof(double)), *Rf = malloc(N * sizeof(double));
    double *du = malloc(3 * N * sizeof(double)), *dp = malloc(N * sizeof(double));
    double *t1 = malloc(3 * N * sizeof(double));
    double *Ut = malloc(3 * N * sizeof(double)), *Pt = malloc(N * sizeof(double));
    double *Rmt = malloc(3 * N * sizeof(double)), *Rft = malloc(N * sizeof(double));
    double *tract = malloc((nq ? nq : 1) * 3 * sizeof(double)), *diet = malloc((nq ? nq : 1) * 2 * sizeof(double));
    uint8_t *flagt = malloc(nq ? nq : 1);
    int64_t cuts = 0;
    double sm = 0, sf = 0;
    int64_t it = 0;
    int status = 1;
    double st[5], tot_outer = 0, tot_K = 0, tot_A = 0, em = 0, ef = 0;
    for (;;) {
        or_cohesive(P, U, die_n, t0, trac, die, flag, fcoh);
        or_residual(P, U, Pp, Un, Pn, fcoh, Fu, fp, Rm, Rf);
        double rm = vnorm(3 * N, Rm), rf = vnorm(N, Rf);
        if (it == 0) {
            or_apply_Apu(P, Pp, t1);
            sm = fmax(rm, fmax(vnorm(3 * N, t1), vnorm(3 * N, Fu)));
            sf = fmax(rf, P->p.dt * vnorm(N, fp));
        } else {
            or_apply_Apu(P, Pp, t1);
            sm = fmax(sm, vnorm(3 * N, t1));
        }
        em = sm > 0 ? rm / sm : rm;
        ef = sf > 0 ? rf / sf : rf;
        if (em <= tol_newton && ef <= tol_newton) {
            status = 0;
            break;
        }
        if (it >= max_newton) {
            status = 1;
            break;
        }
        for (int64_t i = 0; i < 3 * N; ++i) Rm[i] = -Rm[i];
        for (int64_t i = 0; i < N; ++i) Rf[i] = -Rf[i];
        int s = or_prevost(P, Rm, Rf, du, dp, tol_outer, tol_inner, maxit_outer, maxit_inner, st);
        tot_outer += st[0];
        tot_K += st[1];
        tot_A += st[2];
        if (s < 0) {
            status = s;
            break;
        }
        double step = 1.0;
        if (line_search) {
            for (int64_t i = 0; i < N; ++i) Pt[i] = Pp[i] + dp[i];
            or_apply_Apu(P, Pt, t1);
            const double s_star = fmax(sm, vnorm(3 * N, t1));
            const double m0 = merit(rm, rf, s_star, sf);
            for (;;) {
                for (int64_t i = 0; i < 3 * N; ++i) Ut[i] = U[i] + step * du[i];
                for (int64_t i = 0; i < N; ++i) Pt[i] = Pp[i] + step * dp[i];
                or_cohesive(P, Ut, die_n, t0, tract, diet, flagt, fcoh);
                or_residual(P, Ut, Pt, Un, Pn, fcoh, Fu, fp, Rmt, Rft);
                if (merit(vnorm(3 * N, Rmt), vnorm(N, Rft), s_star, sf) < m0 || step <= 1.0 / 64) break;
                step *= 0.5;
                cuts++;
            }
        }
        for (int64_t i = 0; i < 3 * N; ++i) U[i] += step * du[i];
        for (int64_t i = 0; i < N; ++i) Pp[i] += step * dp[i];
        it++;
    }
    info[0] = (double)it;
    info[1] = tot_outer;
    info[2] = tot_K;
    info[3] = tot_A;
    info[4] = em;
    info[5] = ef;
    info[6] = (double)status;
    info[7] = (double)cuts;
    free(Ut);
    free(Pt);
    free(Rmt);
    free(Rft);
    free(tract);
    free(diet);
    free(flagt);
    free(Un);
    free(Pn);
    free(die_n);
    free(fcoh);
    free(Rm);
    free(Rf);
    free(du);
    free(dp);
    free(t1);
    return status;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* adjoint                                                             */
/* ------------------------------------------------------------------ */
/* y = N^T x, N the part of the exact interface tangent that the symmetric
 * Newton tangent omits: at slip points in contact the shear traction
 * f t'_n tau changes with the normal opening, d t_s / d delta_n = -f k_n tau,
 * i.e. D_exact = D_sym + (-f k_n) tau (x) n.  Uses the points' states of the
 * last or_cohesive call.  Held displacement DOFs are masked on both sides. */
void or_apply_NT(or_problem *P, const double *x_in, double *y)
{
    int64_t N = P->N;
    memset(y, 0, 3 * N * sizeof(double));
    const double kn = P->p.k_n, f = P->p.friction;
    for (int64_t t = 0; t < P->nf; ++t) {
        const int32_t *nd = P->coh + 6 * t;
        const double *n = P->tri_n + 3 * t;
        double w = P->tri_A[t] / 3.0;
        for (int q = 0; q < 3; ++q) {
            int64_t iq = 3 * t + q;
            if (P->qp_flag[iq] != OR_SLIP) continue;
            const double *tau = P->qp_tau + 3 * iq;
            /* opening of x at the point, then D_ns^T jump = (-f k_n) n (tau . jump) */
            double jump[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a)
                for (int r = 0; r < 3; ++r) {
                    int64_t ip = 3 * (int64_t)nd[a] + r, im = 3 * (int64_t)nd[3 + a] + r;
                    double xp = P->dir_u[ip] ? 0.0 : x_in[ip], xm = P->dir_u[im] ? 0.0 : x_in[im];
                    jump[r] += QP_N[q][a] * (xp - xm);
                }
            double s = -f * kn * dot3(tau, jump);
            for (int a = 0; a < 3; ++a)
                for (int r = 0; r < 3; ++r) {
                    y[3 * (int64_t)nd[a] + r] += w * QP_N[q][a] * s * n[r];
                    y[3 * (int64_t)nd[3 + a] + r] -= w * QP_N[q][a] * s * n[r];
                }
        }
    }
    for (int64_t i = 0; i < 3 * N; ++i)
        if (P->dir_u[i]) y[i] = 0;
}

/* N x: the slip part of the exact interface tangent that the symmetric Newton
 * tangent omits (last or_cohesive call).  At a slip point the shear traction's
 * magnitude f t'_n follows the normal opening, d t_s / d delta_n = -f k_n tau, so
 * the force on the lips is +-w N_a tau (-f k_n)(n . jump(x)) (Sec. 2.2.1, return
 * map; the transpose of or_apply_NT). */
void or_apply_N(or_problem *P, const double *x_in, double *y)
{
    int64_t N = P->N;
    memset(y, 0, 3 * N * sizeof(double));
    const double kn = P->p.k_n, f = P->p.friction;
    for (int64_t t = 0; t < P->nf; ++t) {
        const int32_t *nd = P->coh + 6 * t;
        const double *n = P->tri_n + 3 * t;
        double w = P->tri_A[t] / 3.0;
        for (int q = 0; q < 3; ++q) {
            int64_t iq = 3 * t + q;
            if (P->qp_flag[iq] != OR_SLIP) continue;
            const double *tau = P->qp_tau + 3 * iq;
            double jump[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a)
                for (int r = 0; r < 3; ++r) {
                    int64_t ip = 3 * (int64_t)nd[a] + r, im = 3 * (int64_t)nd[3 + a] + r;
                    double xp = P->dir_u[ip] ? 0.0 : x_in[ip], xm = P->dir_u[im] ? 0.0 : x_in[im];
                    jump[r] += QP_N[q][a] * (xp - xm);
                }
            double s = -f * kn * dot3(n, jump);
            for (int a = 0; a < 3; ++a)
                for (int r = 0; r < 3; ++r) {
                    y[3 * (int64_t)nd[a] + r] += w * QP_N[q][a] * s * tau[r];
                    y[3 * (int64_t)nd[3 + a] + r] -= w * QP_N[q][a] * s * tau[r];
                }
        }
    }
    for (int64_t i = 0; i < 3 * N; ++i)
        if (P->dir_u[i]) y[i] = 0;
}

/* Adjoint of one converged step (the transposed Newton system, Sec. 3.3.1):
 *   [K_exact^T  A_pu ] [lam_u]   [g_u]
 *   [-A_up      A22  ] [lam_p] = [g_p]
 * With mu = -lam_u this is [[K_exact^T, -A_pu],[A_up, A22]] [mu; lam_p] = [-g_u; g_p],
 * the forward block structure; K_exact^T = K_sym + N^T is handled by defect
 * correction around the partitioned CG: solve with K_sym and the right-hand side
 * -g_u - N^T mu^k until mu stops changing.  Requires or_cohesive at the converged
 * state (tangent and point states).  stats: [defect its, outer its, K its, A22 its,
 * last relative change of mu, status]. */
int or_adjoint(or_problem *P, const double *g_u, const double *g_p, double *lam_u, double *lam_p, double tol_defect,
               int64_t max_defect, double tol_outer, double tol_inner, int64_t maxit_outer, int64_t maxit_inner,
               double *stats)
{
    int64_t n1 = 3 * P->N, n2 = P->N;
    double *mu = calloc(n1, sizeof(double)), *mu_new = calloc(n1, sizeof(double)), *b1 = calloc(n1, sizeof(double));
    double *b2 = calloc(n2, sizeof(double)), *ntm = calloc(n1, sizeof(double));
    for (int64_t i = 0; i < n2; ++i) b2[i] = P->dir_p[i] ? 0.0 : g_p[i];
    int status = 1;
    double change = 0, st[5], tot[3] = {0, 0, 0};
    int64_t k = 0;
    for (; k < max_defect; ++k) {
        or_apply_NT(P, mu, ntm);
        for (int64_t i = 0; i < n1; ++i) b1[i] = P->dir_u[i] ? 0.0 : -g_u[i] - ntm[i];
        int s = or_prevost(P, b1, b2, mu_new, lam_p, tol_outer, tol_inner, maxit_outer, maxit_inner, st);
        tot[0] += st[0];
        tot[1] += st[1];
        tot[2] += st[2];
        if (s < 0) {
            status = s;
            break;
        }
        double dn = 0, mn = 0;
        for (int64_t i = 0; i < n1; ++i) {
            dn += (mu_new[i] - mu[i]) * (mu_new[i] - mu[i]);
            mn += mu_new[i] * mu_new[i];
        }
        change = mn > 0 ? sqrt(dn / mn) : sqrt(dn);
        memcpy(mu, mu_new, n1 * sizeof(double));
        if (change <= tol_defect) {
            status = 0;
            k++;
            break;
        }
    }
    for (int64_t i = 0; i < n1; ++i) lam_u[i] = -mu[i];
    stats[0] = (double)k;
    stats[1] = tot[0];
    stats[2] = tot[1];
    stats[3] = tot[2];
    stats[4] = change;
    stats[5] = (double)status;
    free(mu);
    free(mu_new);
    free(b1);
    free(b2);
    free(ntm);
    return status;
}

/* Parameter sensitivities dJ/dtheta = -lam^T dR/dtheta at the converged state:
 *   dR_m/dE_e   = (K_e / E_e) U_e              (bulk stiffness is linear in E)
 *   dR_f/dlnk_e = dt C_e P_e                   (conductivity is linear in k = e^{ln k})
 * with held DOFs of lam, U and P taken as zero. */
void or_sensitivity(or_problem *P, const double *U, const double *Pp, const double *lam_u, const double *lam_p,
                    double *dJ_dE, double *dJ_dlogk)
{
#pragma omp parallel for schedule(static) if (P->ne > OR_PAR_MIN)
    for (int64_t e = 0; e < P->ne; ++e) {
        double X[12], Ke[144], Se[16], Ce[16], ue[12], le[12], pe[4], qe[4];
        tet_coords(P, e, X);
        or_tet_stiffness(X, 1.0, P->p.nu, Ke);
        or_tet_flow(X, exp(P->logk[e]) / P->p.mu, 1.0 / P->p.biot_M, Se, Ce);
        const int32_t *nd = P->tets + 4 * e;
        for (int a = 0; a < 4; ++a) {
            for (int r = 0; r < 3; ++r) {
                int64_t i = 3 * (int64_t)nd[a] + r;
                ue[3 * a + r] = P->dir_u[i] ? 0.0 : U[i];
                le[3 * a + r] = P->dir_u[i] ? 0.0 : lam_u[i];
            }
            pe[a] = P->dir_p[nd[a]] ? 0.0 : Pp[nd[a]];
            qe[a] = P->dir_p[nd[a]] ? 0.0 : lam_p[nd[a]];
        }
        double sE = 0, sk = 0;
        for (int r = 0; r < 12; ++r)
            for (int c = 0; c < 12; ++c) sE += le[r] * Ke[12 * r + c] * ue[c];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) sk += qe[a] * Ce[4 * a + b] * pe[b];
        dJ_dE[e] = -sE;
        dJ_dlogk[e] = -P->p.dt * sk;
    }
}

/* ------------------------------------------------------------------ */
/* adjoint through the inelastic slip state (time loop)                */
/* ------------------------------------------------------------------ */
/* The inelastic slip carried from step to step, die_new = Phi(U, die_old), is the
 * return map of Sec. 2.2.1 (eq. plastic_slip_increment, eq. corrector) applied at
 * every interface point, and the interface force of the step reads die_old through
 * the trial traction.  For a time loop of steps the adjoint needs, per point:
 *   gU    = (d Phi / d U)^T a_new                        (added to the step's dJ/dU)
 *   a_old = (d Phi / d die_old)^T a_new - (d f_coh / d die_old)^T lam_u
 * where a_new [nq*2] is the adjoint of the slip the step produced and lam_u [3N]
 * the step's displacement multipliers.  With the local opening d = (d_n, d_s) in
 * the frame (n, t1, t2), trial traction t_tr = k_s (d_s0 + d_s - die_old),
 * t'_n = k_n max(-(d_n0 + d_n), 0), Pi = I - tau tau^T:
 *   stick:  die = die_old;                 t_s = t_tr
 *   slip:   die = die_old + (|t_tr| - f t'_n)/k_s tau;  t_s = f t'_n tau
 * differentiated branch by branch (open points follow the slip branch with
 * t'_n = 0).  gU (or a_old) may be NULL; lam_u NULL reads as zero.  Held
 * displacement DOFs are zero in gU. */
void or_slip_adjoint(or_problem *P, const double *U, const double *die_old, const double *t0, const double *a_new,
                     const double *lam_u, double *gU, double *a_old)
{
    int64_t N = P->N;
    if (gU) memset(gU, 0, 3 * N * sizeof(double));
    const double kn = P->p.k_n, ks = P->p.k_s, f = P->p.friction;
    for (int64_t t = 0; t < P->nf; ++t) {
        const int32_t *nd = P->coh + 6 * t;
        const double *n = P->tri_n + 3 * t, *t1 = P->tri_t1 + 3 * t, *t2 = P->tri_t2 + 3 * t;
        const double *R[3] = {n, t1, t2};
        double w = P->tri_A[t] / 3.0;
        for (int q = 0; q < 3; ++q) {
            int64_t iq = 3 * t + q;
            double jump[3] = {0, 0, 0}, lj[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a)
                for (int r = 0; r < 3; ++r) {
                    int64_t ip = 3 * (int64_t)nd[a] + r, im = 3 * (int64_t)nd[3 + a] + r;
                    jump[r] += QP_N[q][a] * (U[ip] - U[im]);
                    if (lam_u) lj[r] += QP_N[q][a] * ((P->dir_u[ip] ? 0.0 : lam_u[ip]) - (P->dir_u[im] ? 0.0 : lam_u[im]));
                }
            double d[3] = {dot3(n, jump), dot3(t1, jump), dot3(t2, jump)};
            const double *dio = die_old + 2 * iq, *tz = t0 + 3 * iq;
            double dnt = -tz[0] / kn + d[0];
            double tn = dnt < 0 ? -kn * dnt : 0.0;
            double dtn = dnt < 0 ? -kn : 0.0; /* d t'_n / d d_n */
            double ttr[2] = {ks * (tz[1] / ks + d[1] - dio[0]), ks * (tz[2] / ks + d[2] - dio[1])};
            double nt = sqrt(ttr[0] * ttr[0] + ttr[1] * ttr[1]);
            /* D_d [2][3]: d die / d (d_n, d_s1, d_s2); D_o [2][2]: d die / d die_old;
             * T_o [2][2]: d t_s / d die_old */
            double D_d[2][3] = {{0, 0, 0}, {0, 0, 0}}, D_o[2][2] = {{1, 0}, {0, 1}}, T_o[2][2] = {{-ks, 0}, {0, -ks}};
            if (nt - f * tn > 0.0) {
                double tau[2] = {ttr[0] / nt, ttr[1] / nt};
                double Pi[2][2] = {{1 - tau[0] * tau[0], -tau[0] * tau[1]}, {-tau[1] * tau[0], 1 - tau[1] * tau[1]}};
                double c = f * tn / nt;
                for (int i = 0; i < 2; ++i) {
                    D_d[i][0] = -(f / ks) * tau[i] * dtn;
                    for (int j = 0; j < 2; ++j) {
                        D_d[i][1 + j] = (i == j ? 1.0 : 0.0) - c * Pi[i][j];
                        D_o[i][j] = c * Pi[i][j];
                        T_o[i][j] = -ks * c * Pi[i][j];
                    }
                }
            }
            const double *an = a_new + 2 * iq;
            if (gU) {
                /* (d die/d U)^T a: local (D_d^T a), rotated to global, spread with +-N_a */
                double loc[3];
                for (int k = 0; k < 3; ++k) loc[k] = D_d[0][k] * an[0] + D_d[1][k] * an[1];
                double g[3];
                for (int r = 0; r < 3; ++r) g[r] = R[0][r] * loc[0] + R[1][r] * loc[1] + R[2][r] * loc[2];
                for (int a = 0; a < 3; ++a)
                    for (int r = 0; r < 3; ++r) {
                        gU[3 * (int64_t)nd[a] + r] += QP_N[q][a] * g[r];
                        gU[3 * (int64_t)nd[3 + a] + r] -= QP_N[q][a] * g[r];
                    }
            }
            if (a_old) {
                /* f_coh on the lips is +- w N_a [t1 t2] t_s: its transpose applied to lam_u */
                double ls[2] = {dot3(t1, lj), dot3(t2, lj)};
                for (int j = 0; j < 2; ++j)
                    a_old[2 * iq + j] = D_o[0][j] * an[0] + D_o[1][j] * an[1] - w * (T_o[0][j] * ls[0] + T_o[1][j] * ls[1]);
            }
        }
    }
    if (gU)
        for (int64_t i = 0; i < 3 * N; ++i)
            if (P->dir_u[i]) gU[i] = 0;
}

/* ------------------------------------------------------------------ */
/* block-Jacobi preconditioned CG on K                                 */
/* ------------------------------------------------------------------ */
/* Inverse of an n x n matrix by Gauss-Jordan elimination with partial pivoting
 * (row-major, a destroyed).  Returns 0 if a pivot vanishes. */
static int gj_inverse(int n, double *a, double *inv)
{
    for (int i = 0; i < n * n; ++i) inv[i] = (i / n == i % n) ? 1.0 : 0.0;
    for (int c = 0; c < n; ++c) {
        int pr = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * n + c]) > fabs(a[pr * n + c])) pr = r;
        if (a[pr * n + c] == 0.0) return 0;
        for (int k = 0; k < n; ++k) {
            double t = a[c * n + k];
            a[c * n + k] = a[pr * n + k];
            a[pr * n + k] = t;
            t = inv[c * n + k];
            inv[c * n + k] = inv[pr * n + k];
            inv[pr * n + k] = t;
        }
        double d = a[c * n + c];
        for (int k = 0; k < n; ++k) {
            a[c * n + k] /= d;
            inv[c * n + k] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double m = a[r * n + c];
            for (int k = 0; k < n; ++k) {
                a[r * n + k] -= m * a[c * n + k];
                inv[r * n + k] -= m * inv[c * n + k];
            }
        }
    }
    return 1;
}

void or_gj_inverse(int n, double *a, double *inv, int *ok) { *ok = gj_inverse(n, a, inv); }

static double csr_at(const or_csr *A, int64_t row, int64_t col)
{
    for (int64_t k = A->rowptr[row]; k < A->rowptr[row + 1]; ++k)
        if (A->col[k] == col) return A->val[k];
    return 0.0;
}

/* Block-Jacobi preconditioner of K_t: the inverse of the 3x3 diagonal block of
 * every node, except that the two lips' nodes at the same interface point (+a, -a
 * of an interface element) share the inverse of their 6x6 block.  Per node: own
 * part Ai (3x3) and partner part Bi (3x3) of the rows of M^-1; partner[u] = -1
 * off the interface pairs.  Returns 1 if a block is singular. */
typedef struct {
    int64_t N;
    int32_t *partner;
    double *Ai, *Bi;
} or_bj;

static int bj_setup(const or_problem *P, or_bj *M)
{
    const or_csr *A = &P->Kt;
    int64_t N = P->N;
    int32_t *partner = malloc(N * sizeof(int32_t));
    for (int64_t i = 0; i < N; ++i) partner[i] = -1;
    for (int64_t t = 0; t < P->nf; ++t)
        for (int a = 0; a < 3; ++a) {
            int32_t u = P->coh[6 * t + a], v = P->coh[6 * t + 3 + a];
            partner[u] = (partner[u] == -1 || partner[u] == v) ? v : -2;
            partner[v] = (partner[v] == -1 || partner[v] == u) ? u : -2;
        }
    for (int64_t i = 0; i < N; ++i)
        if (partner[i] == -2 || partner[i] == i) partner[i] = -1;
    double *Ai = calloc(9 * N, sizeof(double)), *Bi = calloc(9 * N, sizeof(double));
    int singular = 0;
    for (int64_t u = 0; u < N; ++u) {
        int64_t v = partner[u];
        if (v >= 0 && partner[v] != u) v = -1;
        if (v < 0) {
            double m[9], inv[9];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) m[3 * r + c] = csr_at(A, 3 * u + r, 3 * u + c);
            if (!gj_inverse(3, m, inv)) singular = 1;
            memcpy(Ai + 9 * u, inv, sizeof inv);
        } else {
            double m[36], inv[36];
            int64_t nd[2] = {u, v};
            for (int bi = 0; bi < 2; ++bi)
                for (int bj = 0; bj < 2; ++bj)
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < 3; ++c)
                            m[6 * (3 * bi + r) + 3 * bj + c] = csr_at(A, 3 * nd[bi] + r, 3 * nd[bj] + c);
            if (!gj_inverse(6, m, inv)) singular = 1;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    Ai[9 * u + 3 * r + c] = inv[6 * r + c];
                    Bi[9 * u + 3 * r + c] = inv[6 * r + 3 + c];
                }
        }
        partner[u] = (int32_t)v;
    }
    M->N = N;
    M->partner = partner;
    M->Ai = Ai;
    M->Bi = Bi;
    return singular;
}

static void bj_free(or_bj *M)
{
    free(M->partner);
    free(M->Ai);
    free(M->Bi);
}

/* z = M^-1 r */
static void bj_apply(const or_bj *M, const double *r, double *z)
{
    for (int64_t u = 0; u < M->N; ++u)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += M->Ai[9 * u + 3 * c + k] * r[3 * u + k];
            if (M->partner[u] >= 0)
                for (int k = 0; k < 3; ++k) s += M->Bi[9 * u + 3 * c + k] * r[3 * M->partner[u] + k];
            z[3 * u + c] = s;
        }
}

/* PCG on K_t with a preconditioner z = prec(r).  Same recurrence and stop test as
 * or_pcg.  Returns 0, 1 (not converged) or -3 (p.Ap <= 0). */
typedef void (*or_prec_fn)(const or_problem *P, const or_bj *M, const void *ctx, const double *r, double *z);

static int pcg_prec(const or_problem *P, const or_bj *M, or_prec_fn prec, const void *ctx, const double *b,
                    double *x, double tol, int64_t maxit, int64_t *iters, double *relres)
{
    const or_csr *A = &P->Kt;
    int64_t n = 3 * P->N;
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
    int status = 0;
    int64_t it = 0;
    double rel = 0;
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 0;
        r[i] = b[i];
    }
    prec(P, M, ctx, r, z);
    memcpy(p, z, n * sizeof(double));
    double bn = sqrt(vdot(n, b, b));
    if (bn == 0.0) goto done;
    double rho = vdot(n, r, z);
    for (;;) {
        rel = sqrt(vdot(n, r, r)) / bn;
        if (rel <= tol) break;
        if (it >= maxit) {
            status = 1;
            break;
        }
        or_csr_spmv(A, p, q);
        double pq = vdot(n, p, q);
        if (!(pq > 0.0)) {
            status = -3;
            break;
        }
        double al = rho / pq;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += al * p[i];
            r[i] -= al * q[i];
        }
        prec(P, M, ctx, r, z);
        double rho2 = vdot(n, r, z);
        double be = rho2 / rho;
        rho = rho2;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + be * p[i];
        ++it;
    }
done:
    *iters = it;
    *relres = rel;
    free(r);
    free(z);
    free(p);
    free(q);
    return status;
}

static void prec_bj(const or_problem *P, const or_bj *M, const void *ctx, const double *r, double *z)
{
    (void)P;
    (void)ctx;
    bj_apply(M, r, z);
}

/* PCG on the current tangent K_t with the block-Jacobi preconditioner. */
int or_pcg_block(or_problem *P, const double *b, double *x, double tol, int64_t maxit, int64_t *iters, double *relres)
{
    or_bj M;
    int singular = bj_setup(P, &M);
    int status;
    if (singular) {
        memset(x, 0, 3 * P->N * sizeof(double));
        *iters = 0;
        *relres = 0;
        status = -3;
    } else {
        status = pcg_prec(P, &M, prec_bj, NULL, b, x, tol, maxit, iters, relres);
    }
    bj_free(&M);
    return status;
}

/* Chebyshev polynomial preconditioner over block Jacobi (Saad, Iterative Methods
 * for Sparse Linear Systems, Sec. 12.3, Chebyshev acceleration): z = p(M^-1 K)
 * M^-1 r is `degree` steps of the Chebyshev iteration for K z = r from z = 0 on
 * the interval [lo, hi] of the spectrum of M^-1 K, so that the residual
 * polynomial 1 - t p(t) is T_m((hi + lo - 2t)/(hi - lo)) / T_m((hi + lo)/(hi - lo)).
 * With theta = (hi + lo)/2, delta = (hi - lo)/2, sigma = theta/delta:
 *   d = M^-1 r / theta, z = d, s = r, rho = 1/sigma;
 *   repeat degree-1 times: s -= K d, rho' = 1/(2 sigma - rho),
 *                          d = rho' rho d + (2 rho'/delta) M^-1 s, z += d, rho = rho'. */
typedef struct {
    int degree;
    double lo, hi;
} or_cheb;

static void cheb_apply(const or_problem *P, const or_bj *M, const or_cheb *C, const double *r, double *z)
{
    int64_t n = 3 * P->N;
    double *d = malloc(n * sizeof(double)), *s = malloc(n * sizeof(double));
    double *w = malloc(n * sizeof(double)), *kd = malloc(n * sizeof(double));
    double theta = 0.5 * (C->hi + C->lo), delta = 0.5 * (C->hi - C->lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    bj_apply(M, r, d);
    for (int64_t i = 0; i < n; ++i) {
        d[i] /= theta;
        z[i] = d[i];
        s[i] = r[i];
    }
    for (int k = 1; k < C->degree; ++k) {
        or_csr_spmv(&P->Kt, d, kd);
        for (int64_t i = 0; i < n; ++i) s[i] -= kd[i];
        double rho1 = 1.0 / (2.0 * sigma - rho);
        bj_apply(M, s, w);
        for (int64_t i = 0; i < n; ++i) {
            d[i] = rho1 * rho * d[i] + (2.0 * rho1 / delta) * w[i];
            z[i] += d[i];
        }
        rho = rho1;
    }
    free(d);
    free(s);
    free(w);
    free(kd);
}

static void prec_cheb(const or_problem *P, const or_bj *M, const void *ctx, const double *r, double *z)
{
    cheb_apply(P, M, (const or_cheb *)ctx, r, z);
}

/* z = p(M^-1 K) M^-1 r for the current K_t (as above); returns -3 if a block is singular. */
int or_cheb_apply(or_problem *P, const double *r, double *z, int degree, double lo, double hi)
{
    or_bj M;
    int singular = bj_setup(P, &M);
    or_cheb C = {degree, lo, hi};
    if (!singular) cheb_apply(P, &M, &C, r, z);
    bj_free(&M);
    return singular ? -3 : 0;
}

/* PCG on K_t with the Chebyshev polynomial preconditioner of the given degree and interval. */
int or_pcg_cheb(or_problem *P, const double *b, double *x, double tol, int64_t maxit, int degree, double lo,
                double hi, int64_t *iters, double *relres)
{
    or_bj M;
    int singular = bj_setup(P, &M);
    or_cheb C = {degree, lo, hi};
    int status;
    if (singular) {
        memset(x, 0, 3 * P->N * sizeof(double));
        *iters = 0;
        *relres = 0;
        status = -3;
    } else {
        status = pcg_prec(P, &M, prec_cheb, &C, b, x, tol, maxit, iters, relres);
    }
    bj_free(&M);
    return status;
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) of counter i, as a double in
 * [-1/2, 1/2): the probe vector of the spectrum estimate, by caller-order DOF. */
static double splitmix_unit(uint64_t i)
{
    uint64_t z = (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

void or_probe_vector(or_problem *P, double *v)
{
    for (int64_t i = 0; i < 3 * P->N; ++i) v[i] = P->dir_u[i] ? 0.0 : splitmix_unit((uint64_t)i);
}

/* Lanczos coefficients of M^-1 K (block Jacobi) from `steps` PCG iterations on the
 * probe vector (Saad, Sec. 6.7.3: the CG coefficients alpha_j, beta_j give the
 * tridiagonal Lanczos matrix).  Returns the number of iterations taken (fewer if
 * the residual vanishes), or -3 on a singular block or p.Ap <= 0. */
int or_bj_lanczos(or_problem *P, int steps, double *alpha, double *beta)
{
    or_bj M;
    int64_t n = 3 * P->N;
    if (bj_setup(P, &M)) {
        bj_free(&M);
        return -3;
    }
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
    or_probe_vector(P, r);
    bj_apply(&M, r, z);
    memcpy(p, z, n * sizeof(double));
    double rho = vdot(n, r, z);
    int j = 0;
    for (; j < steps && rho > 0.0; ++j) {
        or_csr_spmv(&P->Kt, p, q);
        double pq = vdot(n, p, q);
        if (!(pq > 0.0)) {
            j = -3;
            break;
        }
        double al = rho / pq;
        for (int64_t i = 0; i < n; ++i) r[i] -= al * q[i];
        bj_apply(&M, r, z);
        double rho2 = vdot(n, r, z);
        alpha[j] = al;
        beta[j] = rho2 / rho;
        rho = rho2;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta[j] * p[i];
    }
    free(r);
    free(z);
    free(p);
    free(q);
    bj_free(&M);
    return j;
}

/* (K_t + N) x = b, the exact interface tangent of the last or_cohesive call, by
 * BiCGStab (van der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992) with the block-
 * Jacobi preconditioner M of K_t applied on the right (x = M^-1 y):
 *   r = b, rh = r, rho = alpha = omega = 1, v = p = 0;
 *   repeat: rho' = rh.r, beta = (rho'/rho)(alpha/omega), p = r + beta (p - omega v),
 *           ph = M^-1 p, v = A ph, alpha = rho'/(rh.v), s = r - alpha v,
 *           sh = M^-1 s, t = A sh, omega = (t.s)/(t.t),
 *           x += alpha ph + omega sh, r = s - omega t
 * until ||r|| <= tol ||b|| (r is the recursive residual).  Returns 0, 1 (not
 * converged) or -3 (a breakdown: rho', rh.v, t.t or omega zero, or a singular block). */
int or_bicgstab_exact(or_problem *P, const double *b, double *x, double tol, int64_t maxit, int64_t *iters,
                      double *relres)
{
    int64_t n = 3 * P->N;
    or_bj M;
    int status = 0;
    int64_t it = 0;
    double rel = 0;
    memset(x, 0, n * sizeof(double));
    if (bj_setup(P, &M)) {
        bj_free(&M);
        *iters = 0;
        *relres = 0;
        return -3;
    }
    double *r = malloc(n * sizeof(double)), *rh = malloc(n * sizeof(double)), *p = calloc(n, sizeof(double));
    double *v = calloc(n, sizeof(double)), *ph = malloc(n * sizeof(double)), *sv = malloc(n * sizeof(double));
    double *sh = malloc(n * sizeof(double)), *t = malloc(n * sizeof(double)), *w = malloc(n * sizeof(double));
    memcpy(r, b, n * sizeof(double));
    memcpy(rh, b, n * sizeof(double));
    double bn = sqrt(vdot(n, b, b)), rho = 1, alpha = 1, omega = 1;
    if (bn == 0.0) goto done;
    for (;;) {
        rel = sqrt(vdot(n, r, r)) / bn;
        if (rel <= tol) break;
        if (it >= maxit) {
            status = 1;
            break;
        }
        double rho1 = vdot(n, rh, r);
        if (rho1 == 0.0 || omega == 0.0) {
            status = -3;
            break;
        }
        double beta = (rho1 / rho) * (alpha / omega);
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        bj_apply(&M, p, ph);
        or_csr_spmv(&P->Kt, ph, v);
        or_apply_N(P, ph, w);
        for (int64_t i = 0; i < n; ++i) v[i] += w[i];
        double rv = vdot(n, rh, v);
        if (rv == 0.0) {
            status = -3;
            break;
        }
        alpha = rho1 / rv;
        for (int64_t i = 0; i < n; ++i) sv[i] = r[i] - alpha * v[i];
        bj_apply(&M, sv, sh);
        or_csr_spmv(&P->Kt, sh, t);
        or_apply_N(P, sh, w);
        for (int64_t i = 0; i < n; ++i) t[i] += w[i];
        double tt = vdot(n, t, t);
        if (tt == 0.0) {
            status = -3;
            break;
        }
        omega = vdot(n, t, sv) / tt;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * ph[i] + omega * sh[i];
            r[i] = sv[i] - omega * t[i];
        }
        rho = rho1;
        ++it;
    }
done:
    *iters = it;
    *relres = rel;
    free(r);
    free(rh);
    free(p);
    free(v);
    free(ph);
    free(sv);
    free(sh);
    free(t);
    free(w);
    bj_free(&M);
    return status;
}

/* ------------------------------------------------------------------ */
/* smoothed-aggregation AMG preconditioner of K_t                      */
/* ------------------------------------------------------------------ */
/* Smoothed aggregation (Vanek, Mandel and Brezina, Computing 56, 1996) with the
 * six rigid-body modes as near-null space, used as a preconditioner of the K_t
 * solves (the stronger preconditioner after block Jacobi and Chebyshev):
 *  - aggregates: three passes over the node graph of the level's matrix in
 *    increasing node order (the two lips of a fault pair count as one node):
 *    (1) a node whose neighbours are all free starts an aggregate with them;
 *    (2) a free node joins the aggregate of its lowest-numbered neighbour
 *    aggregated in pass 1; (3) a node still free starts an aggregate with its
 *    free neighbours;
 *  - tentative prolongator: per aggregate the near-null-space rows of its nodes
 *    (level 0: translations and rotations about the aggregate centroid, zero on
 *    held DOFs; below: the R factor of the aggregate's node), orthonormalised by
 *    modified Gram-Schmidt (a column that vanishes is dropped: zero column, zero
 *    R row); Q gives the prolongator's rows, R the coarse near-null space;
 *  - prolongator smoothing P = (I - w D^-1 A) Ptent, D the block diagonal,
 *    w = 4 / (3 rho), rho the Gershgorin bound max_r sum_c |(D^-1 A)_rc|;
 *  - Galerkin coarse operator A_c = P^T A P; a coarse DOF with an empty row gets a
 *    unit diagonal; coarsening stops at <= amg_coarse nodes or 6 levels, and the
 *    coarsest level is solved by a dense Cholesky factor;
 *  - V-cycle with pre- and post-smoothing by the degree-2 Chebyshev polynomial
 *    over block Jacobi (level 0: the nodal / fault-pair blocks of or_pcg_block on
 *    [hi0/30, hi0]; below: the 6x6 diagonal blocks on [rho/30, rho]), symmetric, so
 *    that CG can use it. */
#define OR_AMG_MAXLEV 6

typedef struct {
    int bs;             /* DOFs per node */
    int64_t nn, nc;     /* nodes of this level, aggregates (nodes of the next) */
    or_csr A;           /* this level's matrix (level 0: a copy of K_t) */
    or_csr P, R;        /* prolongator (bs nn x 6 nc) and its transpose */
    int32_t *agg;       /* node -> aggregate */
    double *Dinv;       /* [nn bs bs] inverse diagonal blocks */
    double rho;         /* Gershgorin bound of D^-1 A */
} or_amg_level;

typedef struct {
    int nlev;
    or_amg_level L[OR_AMG_MAXLEV];
    or_bj bj0;
    double hi0;
    double *chol;       /* dense Cholesky factor (row-major lower) of the coarsest matrix */
    int64_t nco;
} or_amg;

static void csr_alloc(or_csr *A, int64_t n, int64_t nnz)
{
    A->n = n;
    A->nnz = nnz;
    A->rowptr = calloc(n + 1, sizeof(int64_t));
    A->col = malloc((nnz ? nnz : 1) * sizeof(int32_t));
    A->val = malloc((nnz ? nnz : 1) * sizeof(double));
}

/* C = A B for scalar CSR (A: n x m, B: m x k) with a dense accumulator per row;
 * entries whose column is touched are kept even if they sum to zero. */
static void csr_matmul(const or_csr *A, const or_csr *B, int64_t k, or_csr *Cout)
{
    double *acc = calloc(k, sizeof(double));
    int32_t *mark = malloc(k * sizeof(int32_t)), *touched = malloc(k * sizeof(int32_t));
    for (int64_t j = 0; j < k; ++j) mark[j] = -1;
    int64_t cap = A->n * 8 + 16, nnz = 0;
    int32_t *col = malloc(cap * sizeof(int32_t));
    double *val = malloc(cap * sizeof(double));
    int64_t *rp = calloc(A->n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < A->n; ++i) {
        int nt = 0;
        for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
            const int32_t m = A->col[p];
            const double a = A->val[p];
            for (int64_t q = B->rowptr[m]; q < B->rowptr[m + 1]; ++q) {
                const int32_t c = B->col[q];
                if (mark[c] != (int32_t)i) {
                    mark[c] = (int32_t)i;
                    acc[c] = 0;
                    touched[nt++] = c;
                }
                acc[c] += a * B->val[q];
            }
        }
        qsort(touched, nt, sizeof(int32_t), cmp_i32);
        if (nnz + nt > cap) {
            while (nnz + nt > cap) cap *= 2;
            col = realloc(col, cap * sizeof(int32_t));
            val = realloc(val, cap * sizeof(double));
        }
        for (int t = 0; t < nt; ++t) {
            col[nnz] = touched[t];
            val[nnz] = acc[touched[t]];
            ++nnz;
        }
        rp[i + 1] = nnz;
    }
    Cout->n = A->n;
    Cout->nnz = nnz;
    Cout->rowptr = rp;
    Cout->col = col;
    Cout->val = val;
    free(acc);
    free(mark);
    free(touched);
}

static void csr_transpose(const or_csr *A, int64_t ncols, or_csr *T)
{
    csr_alloc(T, ncols, A->nnz);
    for (int64_t p = 0; p < A->nnz; ++p) T->rowptr[A->col[p] + 1]++;
    for (int64_t j = 0; j < ncols; ++j) T->rowptr[j + 1] += T->rowptr[j];
    int64_t *pos = malloc((ncols + 1) * sizeof(int64_t));
    memcpy(pos, T->rowptr, (ncols + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < A->n; ++i)
        for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
            const int64_t q = pos[A->col[p]]++;
            T->col[q] = (int32_t)i;
            T->val[q] = A->val[p];
        }
    free(pos);
}

/* Node graph of a level's matrix (bs DOFs per node): sorted neighbour lists
 * without the node itself. */
static void amg_node_graph(const or_csr *A, int bs, int64_t nn, int64_t **rp_out, int32_t **adj_out)
{
    int64_t *rp = calloc(nn + 1, sizeof(int64_t));
    int64_t cap = nn * 8 + 16, m = 0;
    int32_t *adj = malloc(cap * sizeof(int32_t));
    int32_t *mark = malloc(nn * sizeof(int32_t));
    for (int64_t i = 0; i < nn; ++i) mark[i] = -1;
    for (int64_t i = 0; i < nn; ++i) {
        int64_t start = m;
        for (int r = 0; r < bs; ++r)
            for (int64_t p = A->rowptr[bs * i + r]; p < A->rowptr[bs * i + r + 1]; ++p) {
                const int32_t j = A->col[p] / bs;
                if (j == i || mark[j] == (int32_t)i) continue;
                mark[j] = (int32_t)i;
                if (m == cap) {
                    cap *= 2;
                    adj = realloc(adj, cap * sizeof(int32_t));
                }
                adj[m++] = j;
            }
        qsort(adj + start, m - start, sizeof(int32_t), cmp_i32);
        rp[i + 1] = m;
    }
    free(mark);
    *rp_out = rp;
    *adj_out = adj;
}

/* The three aggregation passes; twin[i] is the other lip of a fault pair (or -1),
 * at level 0 only.  Returns the number of aggregates. */
static int64_t amg_aggregate(int64_t nn, const int64_t *rp, const int32_t *adj, const int32_t *twin, int32_t *agg)
{
    for (int64_t i = 0; i < nn; ++i) agg[i] = -1;
    /* members of the unit led by node i: i and its twin */
#define UNIT_MEMBERS(i, mem, nm)                                \
    int32_t mem[2] = {(int32_t)(i), -1};                        \
    int nm = 1;                                                 \
    if (twin && twin[i] >= 0) mem[nm++] = twin[i];
    int64_t na = 0;
    /* pass 1 */
    for (int64_t i = 0; i < nn; ++i) {
        if (twin && twin[i] >= 0 && twin[i] < i) continue;   /* the pair is led by its lower node */
        if (agg[i] >= 0) continue;
        UNIT_MEMBERS(i, mem, nm)
        int free_all = 1;
        for (int u = 0; u < nm && free_all; ++u)
            for (int64_t p = rp[mem[u]]; p < rp[mem[u] + 1]; ++p)
                if (agg[adj[p]] >= 0) {
                    free_all = 0;
                    break;
                }
        if (!free_all) continue;
        for (int u = 0; u < nm; ++u) {
            agg[mem[u]] = (int32_t)na;
            for (int64_t p = rp[mem[u]]; p < rp[mem[u] + 1]; ++p) {
                const int32_t j = adj[p];
                agg[j] = (int32_t)na;
                if (twin && twin[j] >= 0) agg[twin[j]] = (int32_t)na;
            }
        }
        ++na;
    }
    /* pass 2: join the lowest-numbered neighbour's pass-1 aggregate */
    int32_t *agg1 = malloc((nn ? nn : 1) * sizeof(int32_t));
    memcpy(agg1, agg, nn * sizeof(int32_t));
    for (int64_t i = 0; i < nn; ++i) {
        if (twin && twin[i] >= 0 && twin[i] < i) continue;
        if (agg[i] >= 0) continue;
        UNIT_MEMBERS(i, mem, nm)
        int32_t best = -1, bestj = INT32_MAX;
        for (int u = 0; u < nm; ++u)
            for (int64_t p = rp[mem[u]]; p < rp[mem[u] + 1]; ++p)
                if (agg1[adj[p]] >= 0 && adj[p] < bestj) {
                    bestj = adj[p];
                    best = agg1[adj[p]];
                }
        if (best >= 0)
            for (int u = 0; u < nm; ++u) agg[mem[u]] = best;
    }
    free(agg1);
    /* pass 3 */
    for (int64_t i = 0; i < nn; ++i) {
        if (twin && twin[i] >= 0 && twin[i] < i) continue;
        if (agg[i] >= 0) continue;
        UNIT_MEMBERS(i, mem, nm)
        for (int u = 0; u < nm; ++u) {
            agg[mem[u]] = (int32_t)na;
            for (int64_t p = rp[mem[u]]; p < rp[mem[u] + 1]; ++p) {
                const int32_t j = adj[p];
                if (agg[j] < 0) {
                    agg[j] = (int32_t)na;
                    if (twin && twin[j] >= 0) agg[twin[j]] = (int32_t)na;
                }
            }
        }
        ++na;
    }
#undef UNIT_MEMBERS
    return na;
}

/* Tentative prolongator of one level: B [bs nn x 6] near-null space rows; returns
 * Ptent (bs nn x 6 na, 6 columns per aggregate) and Bc [6 na x 6]. */
static void amg_tentative(int bs, int64_t nn, int64_t na, const int32_t *agg, const double *B, or_csr *Pt, double *Bc)
{
    int64_t *cnt = calloc(na + 1, sizeof(int64_t));
    for (int64_t i = 0; i < nn; ++i) cnt[agg[i] + 1]++;
    for (int64_t a = 0; a < na; ++a) cnt[a + 1] += cnt[a];
    int32_t *members = malloc((nn ? nn : 1) * sizeof(int32_t));
    int64_t *pos = malloc((na + 1) * sizeof(int64_t));
    memcpy(pos, cnt, (na + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < nn; ++i) members[pos[agg[i]]++] = (int32_t)i;   /* ascending within each aggregate */
    free(pos);
    double *Q = calloc(bs * nn * 6, sizeof(double));   /* row (bs i + r), col k */
    memset(Bc, 0, 6 * na * 6 * sizeof(double));
    for (int64_t a = 0; a < na; ++a) {
        const int64_t m0 = cnt[a], m1 = cnt[a + 1];
        const int64_t rows = (m1 - m0) * bs;
        double *M = malloc(rows * 6 * sizeof(double));
        for (int64_t t = m0; t < m1; ++t)
            for (int r = 0; r < bs; ++r)
                for (int k = 0; k < 6; ++k) M[((t - m0) * bs + r) * 6 + k] = B[((int64_t)members[t] * bs + r) * 6 + k];
        double Rm[36] = {0};
        for (int k = 0; k < 6; ++k) {
            double n0 = 0;
            for (int64_t q = 0; q < rows; ++q) n0 += M[q * 6 + k] * M[q * 6 + k];
            n0 = sqrt(n0);
            for (int j = 0; j < k; ++j) {
                double d = 0;
                for (int64_t q = 0; q < rows; ++q) d += M[q * 6 + j] * M[q * 6 + k];
                Rm[6 * j + k] = d;
                for (int64_t q = 0; q < rows; ++q) M[q * 6 + k] -= d * M[q * 6 + j];
            }
            double nk = 0;
            for (int64_t q = 0; q < rows; ++q) nk += M[q * 6 + k] * M[q * 6 + k];
            nk = sqrt(nk);
            if (!(nk > 1e-10 * n0) || nk == 0.0) {
                for (int64_t q = 0; q < rows; ++q) M[q * 6 + k] = 0;
                for (int j = 0; j < k; ++j) Rm[6 * j + k] = 0;   /* a dropped column: zero R row and column */
                Rm[6 * k + k] = 0;
            } else {
                for (int64_t q = 0; q < rows; ++q) M[q * 6 + k] /= nk;
                Rm[6 * k + k] = nk;
            }
        }
        for (int64_t t = m0; t < m1; ++t)
            for (int r = 0; r < bs; ++r)
                for (int k = 0; k < 6; ++k) Q[((int64_t)members[t] * bs + r) * 6 + k] = M[((t - m0) * bs + r) * 6 + k];
        for (int r = 0; r < 6; ++r)
            for (int k = 0; k < 6; ++k) Bc[(a * 6 + r) * 6 + k] = Rm[6 * r + k];
        free(M);
    }
    csr_alloc(Pt, bs * nn, bs * nn * 6);
    for (int64_t i = 0; i < nn; ++i)
        for (int r = 0; r < bs; ++r) {
            const int64_t row = bs * i + r;
            Pt->rowptr[row + 1] = Pt->rowptr[row] + 6;
            for (int k = 0; k < 6; ++k) {
                Pt->col[row * 6 + k] = (int32_t)(6 * agg[i] + k);
                Pt->val[row * 6 + k] = Q[row * 6 + k];
            }
        }
    free(Q);
    free(cnt);
    free(members);
}

/* Inverse diagonal blocks of a level and the Gershgorin bound of D^-1 A. */
static int amg_diag(const or_csr *A, int bs, int64_t nn, double *Dinv, double *rho_out)
{
    int singular = 0;
    double rho = 0;
    for (int64_t i = 0; i < nn; ++i) {
        double m[36], inv[36];
        for (int r = 0; r < bs; ++r)
            for (int c = 0; c < bs; ++c) m[bs * r + c] = csr_at(A, bs * i + r, bs * i + c);
        if (!gj_inverse(bs, m, inv)) singular = 1;
        memcpy(Dinv + (int64_t)bs * bs * i, inv, bs * bs * sizeof(double));
        for (int r = 0; r < bs; ++r) {
            double s = 0;
            /* row r of D_i^-1 [A rows of node i]: entries per column */
            int64_t p[6], e[6];
            for (int k = 0; k < bs; ++k) {
                p[k] = A->rowptr[bs * i + k];
                e[k] = A->rowptr[bs * i + k + 1];
            }
            /* rows of one node share a column pattern in these matrices; walk them together */
            for (int64_t q = 0; q < e[0] - p[0]; ++q) {
                double v = 0;
                for (int k = 0; k < bs; ++k) v += inv[bs * r + k] * A->val[p[k] + q];
                s += fabs(v);
            }
            rho = fmax(rho, s);
        }
    }
    *rho_out = rho;
    return singular;
}

static void amg_free(or_amg *G)
{
    for (int l = 0; l < G->nlev; ++l) {
        or_amg_level *L = &G->L[l];
        csr_free(&L->A);
        if (L->P.rowptr) csr_free(&L->P);
        if (L->R.rowptr) csr_free(&L->R);
        free(L->agg);
        free(L->Dinv);
    }
    bj_free(&G->bj0);
    free(G->chol);
    memset(G, 0, sizeof *G);
}

/* D^-1 (block diagonal) applied to the rows of a matrix with the level's block
 * pattern: Y = D^-1 X for X with node-aligned rows sharing a pattern. */
static void amg_dinv_rows(const double *Dinv, int bs, int64_t nn, or_csr *X)
{
    double *tmp = malloc(bs * sizeof(double));
    for (int64_t i = 0; i < nn; ++i) {
        const int64_t len = X->rowptr[bs * i + 1] - X->rowptr[bs * i];
        for (int64_t q = 0; q < len; ++q) {
            for (int r = 0; r < bs; ++r) {
                double s = 0;
                for (int k = 0; k < bs; ++k) s += Dinv[(int64_t)bs * bs * i + bs * r + k] * X->val[X->rowptr[bs * i + k] + q];
                tmp[r] = s;
            }
            for (int r = 0; r < bs; ++r) X->val[X->rowptr[bs * i + r] + q] = tmp[r];
        }
    }
    free(tmp);
}

/* Build the hierarchy for the current K_t.  hi0: upper end of the level-0 smoother
 * interval.  Returns 0, or -3 if a block of a smoother is singular. */
static int amg_setup(const or_problem *P, or_amg *G, double hi0, int64_t coarse_nodes)
{
    memset(G, 0, sizeof *G);
    G->hi0 = hi0;
    if (bj_setup(P, &G->bj0)) return -3;
    int64_t N = P->N;
    /* the fault pairs (the twin of each lip) */
    int32_t *twin = malloc(N * sizeof(int32_t));
    for (int64_t i = 0; i < N; ++i) twin[i] = G->bj0.partner[i];
    /* level-0 near-null space: translations and rotations, later taken about centroids */
    double *B = calloc(3 * N * 6, sizeof(double));
    int bs = 3;
    int64_t nn = N;
    or_csr A;
    csr_alloc(&A, 3 * N, P->Kt.nnz);
    memcpy(A.rowptr, P->Kt.rowptr, (3 * N + 1) * sizeof(int64_t));
    memcpy(A.col, P->Kt.col, P->Kt.nnz * sizeof(int32_t));
    memcpy(A.val, P->Kt.val, P->Kt.nnz * sizeof(double));
    int status = 0;
    for (int l = 0; l < OR_AMG_MAXLEV; ++l) {
        or_amg_level *L = &G->L[l];
        L->bs = bs;
        L->nn = nn;
        L->A = A;
        L->Dinv = malloc((int64_t)bs * bs * nn * sizeof(double));
        if (amg_diag(&A, bs, nn, L->Dinv, &L->rho)) status = -3;
        G->nlev = l + 1;
        if (nn <= coarse_nodes || l == OR_AMG_MAXLEV - 1) break;
        int64_t *rp;
        int32_t *adj;
        amg_node_graph(&A, bs, nn, &rp, &adj);
        L->agg = malloc(nn * sizeof(int32_t));
        const int64_t na = amg_aggregate(nn, rp, adj, l == 0 ? twin : NULL, L->agg);
        free(rp);
        free(adj);
        L->nc = na;
        if (l == 0) {
            /* rigid-body modes about each aggregate's centroid; zero on held DOFs */
            double *cen = calloc(3 * na, sizeof(double));
            int64_t *cnt = calloc(na, sizeof(int64_t));
            for (int64_t i = 0; i < N; ++i) {
                for (int c = 0; c < 3; ++c) cen[3 * L->agg[i] + c] += P->xyz[3 * i + c];
                cnt[L->agg[i]]++;
            }
            for (int64_t a = 0; a < na; ++a)
                for (int c = 0; c < 3; ++c) cen[3 * a + c] /= (double)cnt[a];
            for (int64_t i = 0; i < N; ++i) {
                const double *c0 = cen + 3 * L->agg[i];
                const double dx = P->xyz[3 * i] - c0[0], dy = P->xyz[3 * i + 1] - c0[1], dz = P->xyz[3 * i + 2] - c0[2];
                const double rows[3][6] = {{1, 0, 0, 0, dz, -dy}, {0, 1, 0, -dz, 0, dx}, {0, 0, 1, dy, -dx, 0}};
                for (int r = 0; r < 3; ++r)
                    for (int k = 0; k < 6; ++k) B[(3 * i + r) * 6 + k] = P->dir_u[3 * i + r] ? 0.0 : rows[r][k];
            }
            free(cen);
            free(cnt);
        }
        double *Bc = malloc(6 * na * 6 * sizeof(double));
        or_csr Pt, AP;
        amg_tentative(bs, nn, na, L->agg, B, &Pt, Bc);
        /* P = Pt - w D^-1 A Pt */
        csr_matmul(&A, &Pt, 6 * na, &AP);
        amg_dinv_rows(L->Dinv, bs, nn, &AP);
        const double w = 4.0 / (3.0 * L->rho);
        /* AP's pattern contains Pt's (every node neighbours itself) */
        for (int64_t row = 0; row < AP.n; ++row) {
            for (int64_t q = AP.rowptr[row]; q < AP.rowptr[row + 1]; ++q) AP.val[q] *= -w;
            for (int64_t q = Pt.rowptr[row]; q < Pt.rowptr[row + 1]; ++q) {
                int64_t lo = AP.rowptr[row], hi = AP.rowptr[row + 1] - 1;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) / 2;
                    if (AP.col[mid] < Pt.col[q]) lo = mid + 1;
                    else hi = mid;
                }
                AP.val[lo] += Pt.val[q];
            }
        }
        csr_free(&Pt);
        L->P = AP;
        csr_transpose(&L->P, 6 * na, &L->R);
        /* A_c = R (A P) */
        or_csr W, Ac;
        csr_matmul(&A, &L->P, 6 * na, &W);
        csr_matmul(&L->R, &W, 6 * na, &Ac);
        csr_free(&W);
        /* a coarse DOF whose prolongator column vanished keeps an empty row: unit diagonal */
        for (int64_t row = 0; row < Ac.n; ++row) {
            double s = 0;
            int64_t d = -1;
            for (int64_t q = Ac.rowptr[row]; q < Ac.rowptr[row + 1]; ++q) {
                s += fabs(Ac.val[q]);
                if (Ac.col[q] == row) d = q;
            }
            if (s == 0.0 && d >= 0) Ac.val[d] = 1.0;
        }
        free(B);
        B = Bc;
        A = Ac;
        bs = 6;
        nn = na;
    }
    free(B);
    free(twin);
    /* dense Cholesky of the coarsest matrix */
    or_amg_level *C = &G->L[G->nlev - 1];
    const int64_t n = (int64_t)C->bs * C->nn;
    G->nco = n;
    G->chol = calloc(n * n, sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t q = C->A.rowptr[i]; q < C->A.rowptr[i + 1]; ++q) G->chol[i * n + C->A.col[q]] = C->A.val[q];
    for (int64_t j = 0; j < n; ++j) {
        double d = G->chol[j * n + j];
        for (int64_t k = 0; k < j; ++k) d -= G->chol[j * n + k] * G->chol[j * n + k];
        if (!(d > 0)) {
            status = -3;
            d = 1.0;
        }
        d = sqrt(d);
        G->chol[j * n + j] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = G->chol[i * n + j];
            for (int64_t k = 0; k < j; ++k) s -= G->chol[i * n + k] * G->chol[j * n + k];
            G->chol[i * n + j] = s / d;
        }
        for (int64_t i = 0; i < j; ++i) G->chol[i * n + j] = 0;
    }
    return status;
}

/* x = p(M^-1 A) M^-1 b, the degree-2 Chebyshev polynomial on [hi/30, hi] (Saad,
 * Sec. 12.3; the recurrence of cheb_apply) with M the level's block Jacobi. */
static void amg_smooth(const or_amg *G, int l, const double *b, double *x)
{
    const or_amg_level *L = &G->L[l];
    const int64_t n = (int64_t)L->bs * L->nn;
    const double hi = l == 0 ? G->hi0 : L->rho, lo = hi / 30.0;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double *d = malloc(n * sizeof(double)), *s = malloc(n * sizeof(double)), *w = malloc(n * sizeof(double));
    double *kd = malloc(n * sizeof(double));
    /* M^-1 v */
#define AMG_MINV(v, out)                                                                                  \
    if (l == 0)                                                                                           \
        bj_apply(&G->bj0, v, out);                                                                        \
    else                                                                                                  \
        for (int64_t i = 0; i < L->nn; ++i)                                                               \
            for (int r = 0; r < 6; ++r) {                                                                 \
                double t_ = 0;                                                                            \
                for (int k = 0; k < 6; ++k) t_ += L->Dinv[36 * i + 6 * r + k] * v[6 * i + k];             \
                out[6 * i + r] = t_;                                                                      \
            }
    AMG_MINV(b, d)
    for (int64_t i = 0; i < n; ++i) {
        d[i] /= theta;
        x[i] = d[i];
        s[i] = b[i];
    }
    const double rho0 = 1.0 / sigma;
    or_csr_spmv(&L->A, d, kd);
    for (int64_t i = 0; i < n; ++i) s[i] -= kd[i];
    const double rho1 = 1.0 / (2.0 * sigma - rho0);
    AMG_MINV(s, w)
    for (int64_t i = 0; i < n; ++i) {
        d[i] = rho1 * rho0 * d[i] + (2.0 * rho1 / delta) * w[i];
        x[i] += d[i];
    }
#undef AMG_MINV
    free(d);
    free(s);
    free(w);
    free(kd);
}

static void amg_vcycle(const or_amg *G, int l, const double *b, double *x)
{
    const or_amg_level *L = &G->L[l];
    const int64_t n = (int64_t)L->bs * L->nn;
    if (l == G->nlev - 1) {
        /* L L^T x = b */
        for (int64_t i = 0; i < n; ++i) {
            double s = b[i];
            for (int64_t k = 0; k < i; ++k) s -= G->chol[i * n + k] * x[k];
            x[i] = s / G->chol[i * n + i];
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int64_t k = i + 1; k < n; ++k) s -= G->chol[k * n + i] * x[k];
            x[i] = s / G->chol[i * n + i];
        }
        return;
    }
    const int64_t nc = 6 * L->nc;
    double *r = malloc(n * sizeof(double)), *t = malloc(n * sizeof(double));
    double *bc = malloc(nc * sizeof(double)), *xc = calloc(nc, sizeof(double));
    amg_smooth(G, l, b, x);                                       /* pre-smoothing from zero */
    or_csr_spmv(&L->A, x, t);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    or_csr_spmv(&L->R, r, bc);                                    /* restriction */
    amg_vcycle(G, l + 1, bc, xc);
    or_csr_spmv(&L->P, xc, t);                                    /* prolongation */
    for (int64_t i = 0; i < n; ++i) x[i] += t[i];
    or_csr_spmv(&L->A, x, t);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    amg_smooth(G, l, r, t);                                       /* post-smoothing */
    for (int64_t i = 0; i < n; ++i) x[i] += t[i];
    free(r);
    free(t);
    free(bc);
    free(xc);
}

static void prec_amg(const or_problem *P, const or_bj *M, const void *ctx, const double *r, double *z)
{
    (void)P;
    (void)M;
    amg_vcycle((const or_amg *)ctx, 0, r, z);
}

/* PCG on K_t with the smoothed-aggregation V-cycle (hierarchy built for the current
 * K_t; hi0 the level-0 smoother's interval end; coarsening down to coarse_nodes).
 * stats (may be NULL): [levels, nodes of level 0..5 (6 entries)].  Returns 0, 1,
 * or -3 (singular block, coarse matrix not SPD or p.Ap <= 0). */
int or_pcg_amg(or_problem *P, const double *b, double *x, double tol, int64_t maxit, double hi0, int64_t coarse_nodes,
               int64_t *iters, double *relres, double *stats)
{
    or_amg G;
    int status = amg_setup(P, &G, hi0, coarse_nodes);
    if (stats) {
        stats[0] = G.nlev;
        for (int l = 0; l < OR_AMG_MAXLEV; ++l) stats[1 + l] = l < G.nlev ? (double)G.L[l].nn : 0.0;
    }
    if (status == 0) {
        status = pcg_prec(P, &G.bj0, prec_amg, &G, b, x, tol, maxit, iters, relres);
    } else {
        memset(x, 0, 3 * P->N * sizeof(double));
        *iters = 0;
        *relres = 0;
    }
    amg_free(&G);
    return status;
}

/* z = V-cycle(r) for the current K_t (one application of the preconditioner). */
int or_amg_apply(or_problem *P, const double *r, double *z, double hi0, int64_t coarse_nodes)
{
    or_amg G;
    int status = amg_setup(P, &G, hi0, coarse_nodes);
    if (status == 0) amg_vcycle(&G, 0, r, z);
    amg_free(&G);
    return status;
}

/* Export of level l of the hierarchy: which 0 = A_l, 1 = P_l, 2 = the aggregate of
 * each node of level l (into col, as int32; val unused).  With rowptr == NULL only
 * the sizes are returned in dims = [rows, cols, nnz]. */
int or_amg_export(or_problem *P, double hi0, int64_t coarse_nodes, int level, int which, int64_t *dims,
                  int64_t *rowptr, int32_t *col, double *val)
{
    or_amg G;
    int status = amg_setup(P, &G, hi0, coarse_nodes);
    if (level >= G.nlev || (which != 0 && level >= G.nlev - 1)) {
        amg_free(&G);
        return -1;
    }
    const or_amg_level *L = &G.L[level];
    if (which == 2) {
        dims[0] = L->nn;
        dims[1] = L->nc;
        dims[2] = L->nn;
        if (col) memcpy(col, L->agg, L->nn * sizeof(int32_t));
    } else {
        const or_csr *M = which == 0 ? &L->A : &L->P;
        dims[0] = M->n;
        dims[1] = which == 0 ? M->n : 6 * L->nc;
        dims[2] = M->nnz;
        if (rowptr) {
            memcpy(rowptr, M->rowptr, (M->n + 1) * sizeof(int64_t));
            memcpy(col, M->col, M->nnz * sizeof(int32_t));
            memcpy(val, M->val, M->nnz * sizeof(double));
        }
    }
    amg_free(&G);
    return status;
}
