/*
 * ddm_oracle.c -- plain FP64 complex CPU oracle for the additive overlapping
 * domain decomposition method (DDM) of Leng & Ju, "An Additive Overlapping
 * Domain Decomposition Method for the Helmholtz Equation" (arXiv 1807.04180).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only tests/, the smoke check and the benchmark's CPU-baseline leg
 * do.  It shares no code, header or table with the HIP library.
 *
 * What it computes (all in double complex, no blocking, no fusion):
 *   - the truncated PML operator of Sec. 3.1 (eq. PMLweak0) discretised by the
 *     5-point (2D) / 7-point (3D) finite-difference scheme of Sec. 4, in the
 *     unscaled form  L u = sum_j (1/alpha_j) d_j((1/alpha_j) d_j u) + k^2 u,
 *     which is J^{-1} div(A grad u) + k^2 u of eq. (PML) with A, J as given
 *     there (alpha_j = 1 + i sigma_j);
 *   - a banded LU with partial pivoting (the plain definition of a direct
 *     solve) for the global truncated problem and for every subdomain problem;
 *   - Algorithm 3.1 (truncated additive overlapping DDM) step by step:
 *     step 1 solves with f restricted to the cores, later steps solve with the
 *     8 (2D) / 26 (3D) transferred sources Psi of Sec. 2.2, edge sources lagged
 *     one step and corner sources two (3D: face 1, edge 2, vertex 3, Remark
 *     3.1), then U_a accumulates the local solutions and the DDM iterate is
 *     sum_a beta_{0;a} U_a (eq. tsum);
 *   - the relative residual ||f - L u|| / ||f|| used as stopping test in
 *     Sec. 4.2 and flexible GMRES with K DDM steps as right preconditioner
 *     (Sec. 4.2.2), classical Gram-Schmidt applied twice.
 *
 * Discrete readings (the paper states them only in the continuum):
 *   - per axis the physical interval [0, M h] has unknowns g = -n_pml+1 ...
 *     M+n_pml-1 and homogeneous Dirichlet nodes at g = -n_pml, M+n_pml;
 *     sigma(x) = sigma0 (t / n_pml)^2 with t the distance (in cells) outside
 *     [0, M];
 *   - cores are half-open: core i covers [i C, (i+1) C - 1] (C = M / N), the
 *     first core also takes the low global PML, the last the high one;
 *   - on every interior side a subdomain is extended by n_ov overlap cells with
 *     sigma = 0 (the shifted profile, eq. PMLprofile) followed by n_pml PML
 *     cells with sigma0 ((m - n_ov)/n_pml)^2, Dirichlet at m = n_ov + n_pml;
 *   - cut-off: side factor b(m) = 1 for m <= 1, beta0((m-1)/(n_ov-1)) for
 *     1 < m < n_ov, 0 for m >= n_ov, m = node offset outward from the core;
 *     beta0(t) = 1 - (10 t^3 - 15 t^4 + 6 t^5) (monotone, C^2, Sec. 2.2);
 *   - chi_{b->a} keeps the nodes of a's box on a's side of every axis on which
 *     b and a differ (a's first core layer included).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Banded LU with partial pivoting (row interchanges), column-major band     */
/* storage: A(i,j) lives at ab[(kl + ku + i - j) + j * ldab],                */
/* ldab = 2 kl + ku + 1; the extra kl rows hold the fill from pivoting.      */
/* ------------------------------------------------------------------------ */
typedef struct {
    long n;
    long kl, ku, ldab;
    cplx *ab;
    long *ipiv;
} band_lu;

static cplx *bl_at(band_lu *b, long i, long j) {
    return &b->ab[(b->kl + b->ku + i - j) + j * b->ldab];
}

static int bl_alloc(band_lu *b, long n, long kl, long ku) {
    b->n = n; b->kl = kl; b->ku = ku; b->ldab = 2 * kl + ku + 1;
    b->ab = (cplx *)calloc((size_t)(b->ldab * n), sizeof(cplx));
    b->ipiv = (long *)calloc((size_t)n, sizeof(long));
    return (b->ab && b->ipiv) ? 0 : -1;
}

static void bl_free(band_lu *b) {
    free(b->ab); free(b->ipiv);
    b->ab = NULL; b->ipiv = NULL;
}

/* Gaussian elimination with partial pivoting on the band; returns 0 or
 * (1 + j) if the pivot of column j is exactly zero. */
static int bl_factor(band_lu *b) {
    long n = b->n, kl = b->kl, ku = b->ku;
    long ju = 0;
    for (long j = 0; j < n; ++j) {
        long km = kl < n - 1 - j ? kl : n - 1 - j;
        long jp = 0;
        double best = cabs(*bl_at(b, j, j));
        for (long i = 1; i <= km; ++i) {
            double v = cabs(*bl_at(b, j + i, j));
            if (v > best) { best = v; jp = i; }
        }
        b->ipiv[j] = j + jp;
        if (best == 0.0) return (int)(1 + j);
        long jlim = j + ku + jp;
        if (jlim > n - 1) jlim = n - 1;
        if (jlim > ju) ju = jlim;
        if (jp != 0) {
            for (long c = j; c <= ju; ++c) {
                cplx t = *bl_at(b, j, c);
                *bl_at(b, j, c) = *bl_at(b, j + jp, c);
                *bl_at(b, j + jp, c) = t;
            }
        }
        cplx piv = *bl_at(b, j, j);
        for (long i = 1; i <= km; ++i) *bl_at(b, j + i, j) /= piv;
        for (long c = j + 1; c <= ju; ++c) {
            cplx ujc = *bl_at(b, j, c);
            if (ujc == 0.0) continue;
            for (long i = 1; i <= km; ++i)
                *bl_at(b, j + i, c) -= *bl_at(b, j + i, j) * ujc;
        }
    }
    return 0;
}

/* Solve A x = rhs in place (one right-hand side). */
static void bl_solve(band_lu *b, cplx *x) {
    long n = b->n, kl = b->kl, kuu = b->kl + b->ku;
    for (long j = 0; j < n; ++j) {
        long p = b->ipiv[j];
        if (p != j) { cplx t = x[j]; x[j] = x[p]; x[p] = t; }
        long km = kl < n - 1 - j ? kl : n - 1 - j;
        cplx xj = x[j];
        if (xj != 0.0)
            for (long i = 1; i <= km; ++i) x[j + i] -= *bl_at(b, j + i, j) * xj;
    }
    for (long j = n - 1; j >= 0; --j) {
        x[j] /= *bl_at(b, j, j);
        cplx xj = x[j];
        long top = j - kuu < 0 ? 0 : j - kuu;
        if (xj != 0.0)
            for (long i = top; i < j; ++i) x[i] -= *bl_at(b, i, j) * xj;
    }
}

/* ------------------------------------------------------------------------ */
/* Problem geometry                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int dim;
    int M[3], N[3], C[3];
    int G[3];          /* global unknowns per axis (1 on an unused axis)  */
    int glo[3];        /* physical index of global array entry 0          */
    int n_pml, n_ov;
    double h, sigma0;
    double *k2;        /* k(x)^2 on the global unknown grid, [z][y][x]     */
    long nglob;
    int nsub;
    int (*clo)[3], (*chi)[3];  /* core box per subdomain (physical index) */
    int (*elo)[3], (*ehi)[3];  /* extended box E_a                        */
    int (*sid)[3];             /* subdomain multi-index                   */
    long *nloc, *off;          /* |E_a| and packed offsets                */
    long etot;
    band_lu *lu;               /* local factors (after or_factor)         */
    int factored;
} or_ctx;

static double sq(double v) { return v * v; }

/* sigma of the global truncated problem (Sec. 3.1), x in cells. */
static double sigma_global(const or_ctx *c, int ax, double x) {
    if (ax >= c->dim) return 0.0;
    double t = 0.0;
    if (x < 0.0) t = -x;
    if (x > c->M[ax]) t = x - c->M[ax];
    return c->sigma0 * sq(t / c->n_pml);
}

/* sigma of subdomain a's truncated problem: the shifted profile (eq.
 * PMLprofile) on interior sides, the global profile elsewhere. */
static double sigma_local(const or_ctx *c, int a, int ax, double x) {
    if (ax >= c->dim) return 0.0;
    int i = c->sid[a][ax];
    if (i > 0 && x < c->clo[a][ax]) {
        double m = c->clo[a][ax] - x;
        double t = m - c->n_ov; if (t < 0) t = 0;
        return c->sigma0 * sq(t / c->n_pml);
    }
    if (i < c->N[ax] - 1 && x > c->chi[a][ax]) {
        double m = x - c->chi[a][ax];
        double t = m - c->n_ov; if (t < 0) t = 0;
        return c->sigma0 * sq(t / c->n_pml);
    }
    return sigma_global(c, ax, x);
}

/* Cut-off beta0 of Sec. 2.2 (monotone, C^2, 1 for t <= 0, 0 for t >= 1). */
static double beta0(double t) {
    if (t <= 0.0) return 1.0;
    if (t >= 1.0) return 0.0;
    return 1.0 - (10.0 * t * t * t - 15.0 * t * t * t * t + 6.0 * t * t * t * t * t);
}

/* Side factor at node offset m outward from a core. */
static double side_factor(const or_ctx *c, int m) {
    if (m <= 1) return 1.0;
    if (m >= c->n_ov) return 0.0;
    return beta0((double)(m - 1) / (double)(c->n_ov - 1));
}

/* beta_{0;a} at physical node q (eq. tsum weights). */
static double beta_zero(const or_ctx *c, int a, const int *q) {
    double v = 1.0;
    for (int ax = 0; ax < c->dim; ++ax) {
        if (q[ax] > c->chi[a][ax]) v *= side_factor(c, q[ax] - c->chi[a][ax]);
        else if (q[ax] < c->clo[a][ax]) v *= side_factor(c, c->clo[a][ax] - q[ax]);
    }
    return v;
}

/* beta_{b->a}: product over the axes where b and a differ of b's side factor
 * facing a (the beta of the transfer operators Psi in Sec. 2.2). */
static double beta_transfer(const or_ctx *c, int b, int a, const int *q) {
    double v = 1.0;
    for (int ax = 0; ax < c->dim; ++ax) {
        int db = c->sid[b][ax], da = c->sid[a][ax];
        if (db < da) v *= side_factor(c, q[ax] - c->chi[b][ax]);
        else if (db > da) v *= side_factor(c, c->clo[b][ax] - q[ax]);
    }
    return v;
}

/* chi_{b->a}: a's side of every axis on which b and a differ. */
static int chi_transfer(const or_ctx *c, int b, int a, const int *p) {
    for (int ax = 0; ax < c->dim; ++ax) {
        int db = c->sid[b][ax], da = c->sid[a][ax];
        if (db < da && p[ax] < c->clo[a][ax]) return 0;
        if (db > da && p[ax] > c->chi[a][ax]) return 0;
    }
    return 1;
}

static int in_box(const int *lo, const int *hi, const int *p) {
    for (int ax = 0; ax < 3; ++ax)
        if (p[ax] < lo[ax] || p[ax] > hi[ax]) return 0;
    return 1;
}

static long box_index(const int *lo, const int *hi, const int *p) {
    long n0 = hi[0] - lo[0] + 1, n1 = hi[1] - lo[1] + 1;
    return (p[0] - lo[0]) + n0 * ((p[1] - lo[1]) + n1 * (long)(p[2] - lo[2]));
}

static long glob_index(const or_ctx *c, const int *p) {
    return (p[0] - c->glo[0]) + (long)c->G[0] * ((p[1] - c->glo[1]) + (long)c->G[1] * (p[2] - c->glo[2]));
}

static void glob_lohi(const or_ctx *c, int *lo, int *hi) {
    for (int ax = 0; ax < 3; ++ax) { lo[ax] = c->glo[ax]; hi[ax] = c->glo[ax] + c->G[ax] - 1; }
}

/* ------------------------------------------------------------------------ */
/* Operator apply on a box with a given sigma function                       */
/* ------------------------------------------------------------------------ */
typedef double (*sigma_fn)(const or_ctx *, int, int, double);

static double sigma_global_fn(const or_ctx *c, int a, int ax, double x) {
    (void)a; return sigma_global(c, ax, x);
}

/* out = L u on box [lo, hi] (u = 0 outside the box): for each axis
 * (1/alpha(x)) [ (u(x+1)-u(x))/alpha(x+1/2) - (u(x)-u(x-1))/alpha(x-1/2) ] / h^2
 * plus k^2(x) u(x). */
static void apply_box(const or_ctx *c, int a, sigma_fn sf, const int *lo, const int *hi,
                      const cplx *u, cplx *out) {
    long n[3];
    for (int ax = 0; ax < 3; ++ax) n[ax] = hi[ax] - lo[ax] + 1;
    double ih2 = 1.0 / (c->h * c->h);
    int p[3];
    for (p[2] = lo[2]; p[2] <= hi[2]; ++p[2])
    for (p[1] = lo[1]; p[1] <= hi[1]; ++p[1])
    for (p[0] = lo[0]; p[0] <= hi[0]; ++p[0]) {
        long ip = box_index(lo, hi, p);
        cplx up = u[ip];
        cplx val = c->k2[glob_index(c, p)] * up;
        for (int ax = 0; ax < c->dim; ++ax) {
            double x = p[ax];
            cplx a0 = 1.0 + I * sf(c, a, ax, x);
            cplx ap = 1.0 + I * sf(c, a, ax, x + 0.5);
            cplx am = 1.0 + I * sf(c, a, ax, x - 0.5);
            long stride = ax == 0 ? 1 : (ax == 1 ? n[0] : n[0] * n[1]);
            cplx uplus = p[ax] < hi[ax] ? u[ip + stride] : 0.0;
            cplx uminus = p[ax] > lo[ax] ? u[ip - stride] : 0.0;
            val += ((uplus - up) / ap - (up - uminus) / am) / a0 * ih2;
        }
        out[ip] = val;
    }
}

/* Assemble the band matrix of L on a box (x fastest ordering). */
static int assemble_band(const or_ctx *c, int a, sigma_fn sf, const int *lo, const int *hi, band_lu *b) {
    long n[3];
    for (int ax = 0; ax < 3; ++ax) n[ax] = hi[ax] - lo[ax] + 1;
    long ntot = n[0] * n[1] * n[2];
    long bw = c->dim == 2 ? n[0] : n[0] * n[1];
    if (c->dim == 2 && n[2] != 1) return -1;
    if (bl_alloc(b, ntot, bw, bw)) return -2;
    double ih2 = 1.0 / (c->h * c->h);
    int p[3];
    for (p[2] = lo[2]; p[2] <= hi[2]; ++p[2])
    for (p[1] = lo[1]; p[1] <= hi[1]; ++p[1])
    for (p[0] = lo[0]; p[0] <= hi[0]; ++p[0]) {
        long ip = box_index(lo, hi, p);
        cplx diag = c->k2[glob_index(c, p)];
        for (int ax = 0; ax < c->dim; ++ax) {
            double x = p[ax];
            cplx a0 = 1.0 + I * sf(c, a, ax, x);
            cplx ap = 1.0 + I * sf(c, a, ax, x + 0.5);
            cplx am = 1.0 + I * sf(c, a, ax, x - 0.5);
            cplx cp = ih2 / (a0 * ap), cm = ih2 / (a0 * am);
            long stride = ax == 0 ? 1 : (ax == 1 ? n[0] : n[0] * n[1]);
            diag -= cp + cm;
            if (p[ax] < hi[ax]) *bl_at(b, ip, ip + stride) = cp;
            if (p[ax] > lo[ax]) *bl_at(b, ip, ip - stride) = cm;
        }
        *bl_at(b, ip, ip) = diag;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */
void or_destroy(or_ctx *c);

or_ctx *or_create(int dim, const int *M, double h, int n_pml, double sigma0,
                  const int *N, int n_ov, const double *k2) {
    if (dim != 2 && dim != 3) return NULL;
    if (n_ov < 2 || n_pml < 2) return NULL;
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    c->dim = dim; c->h = h; c->n_pml = n_pml; c->sigma0 = sigma0; c->n_ov = n_ov;
    c->nsub = 1;
    for (int ax = 0; ax < 3; ++ax) {
        if (ax < dim) {
            if (M[ax] % N[ax] != 0) { free(c); return NULL; }
            c->M[ax] = M[ax]; c->N[ax] = N[ax]; c->C[ax] = M[ax] / N[ax];
            if (N[ax] > 1 && c->C[ax] < n_ov + 2) { free(c); return NULL; }
            c->G[ax] = M[ax] + 2 * n_pml - 1; c->glo[ax] = -n_pml + 1;
        } else {
            c->M[ax] = 0; c->N[ax] = 1; c->C[ax] = 1; c->G[ax] = 1; c->glo[ax] = 0;
        }
        c->nsub *= c->N[ax];
    }
    c->nglob = (long)c->G[0] * c->G[1] * c->G[2];
    c->k2 = (double *)malloc(sizeof(double) * c->nglob);
    memcpy(c->k2, k2, sizeof(double) * c->nglob);
    int ns = c->nsub;
    c->clo = calloc(ns, sizeof(*c->clo)); c->chi = calloc(ns, sizeof(*c->chi));
    c->elo = calloc(ns, sizeof(*c->elo)); c->ehi = calloc(ns, sizeof(*c->ehi));
    c->sid = calloc(ns, sizeof(*c->sid));
    c->nloc = calloc(ns, sizeof(long)); c->off = calloc(ns, sizeof(long));
    c->lu = calloc(ns, sizeof(band_lu));
    long off = 0;
    for (int a = 0; a < ns; ++a) {
        int idx[3] = { a % c->N[0], (a / c->N[0]) % c->N[1], a / (c->N[0] * c->N[1]) };
        long cnt = 1;
        for (int ax = 0; ax < 3; ++ax) {
            c->sid[a][ax] = idx[ax];
            if (ax >= dim) { c->clo[a][ax] = c->chi[a][ax] = c->elo[a][ax] = c->ehi[a][ax] = 0; continue; }
            int i = idx[ax], Cc = c->C[ax], Nn = c->N[ax];
            int ext = n_ov + n_pml - 1;
            c->clo[a][ax] = i == 0 ? -n_pml + 1 : i * Cc;
            c->chi[a][ax] = i == Nn - 1 ? c->M[ax] + n_pml - 1 : (i + 1) * Cc - 1;
            c->elo[a][ax] = i == 0 ? c->clo[a][ax] : c->clo[a][ax] - ext;
            c->ehi[a][ax] = i == Nn - 1 ? c->chi[a][ax] : c->chi[a][ax] + ext;
            cnt *= c->ehi[a][ax] - c->elo[a][ax] + 1;
        }
        c->nloc[a] = cnt; c->off[a] = off; off += cnt;
    }
    c->etot = off;
    return c;
}

void or_destroy(or_ctx *c) {
    if (!c) return;
    if (c->lu) for (int a = 0; a < c->nsub; ++a) bl_free(&c->lu[a]);
    free(c->lu); free(c->k2); free(c->clo); free(c->chi); free(c->elo); free(c->ehi);
    free(c->sid); free(c->nloc); free(c->off); free(c);
}

long or_nglob(const or_ctx *c) { return c->nglob; }
long or_etot(const or_ctx *c) { return c->etot; }
int or_nsub(const or_ctx *c) { return c->nsub; }

/* Boxes of subdomain a: out[0..2] core lo, [3..5] core hi, [6..8] ext lo,
 * [9..11] ext hi, [12] packed offset (as int, < 2^31 for test sizes). */
void or_subdomain_info(const or_ctx *c, int a, long *out) {
    for (int ax = 0; ax < 3; ++ax) {
        out[ax] = c->clo[a][ax]; out[3 + ax] = c->chi[a][ax];
        out[6 + ax] = c->elo[a][ax]; out[9 + ax] = c->ehi[a][ax];
    }
    out[12] = c->off[a]; out[13] = c->nloc[a];
}

/* out = L_h u on the global grid, nrhs vectors of length nglob each. */
void or_apply_global(const or_ctx *c, int nrhs, const cplx *u, cplx *out) {
    int lo[3], hi[3];
    glob_lohi(c, lo, hi);
    for (int r = 0; r < nrhs; ++r)
        apply_box(c, -1, sigma_global_fn, lo, hi, u + r * c->nglob, out + r * c->nglob);
}

/* out = L_a u on subdomain a's box, one vector. */
void or_apply_local(const or_ctx *c, int a, const cplx *u, cplx *out) {
    apply_box(c, a, sigma_local, c->elo[a], c->ehi[a], u, out);
}

/* Dense 1D coefficient dump used by tests: sigma at node and half nodes. */
/* PML strength for a target reflection R (the profile sigma~ of Sec. 2.1 is
 * left open by the paper; reading: a wave of wave number k_ref crossing the
 * layer of width delta twice is damped by R).  With sigma0 (t/delta)^2 the
 * attenuation exponent is 2 k_ref times the layer integral of sigma,
 * 2 k_ref sigma0 delta / 3. */
double or_sigma0_for_reflection(double R, double k_ref, double delta) {
    double layer_integral_per_sigma0 = delta / 3.0;
    return log(1.0 / R) / (2.0 * k_ref * layer_integral_per_sigma0);
}

double or_sigma_local(const or_ctx *c, int a, int ax, double x) { return sigma_local(c, a, ax, x); }
double or_sigma_global(const or_ctx *c, int ax, double x) { return sigma_global(c, ax, x); }
double or_beta0(double t) { return beta0(t); }

/* Global truncated PML problem solved by banded LU; returns 0 or LU status. */
int or_global_solve(const or_ctx *c, int nrhs, const cplx *f, cplx *u) {
    int lo[3], hi[3];
    glob_lohi(c, lo, hi);
    band_lu b;
    int st = assemble_band(c, -1, sigma_global_fn, lo, hi, &b);
    if (st) return -100 + st;
    st = bl_factor(&b);
    if (st == 0) {
        for (int r = 0; r < nrhs; ++r) {
            memcpy(u + r * c->nglob, f + r * c->nglob, sizeof(cplx) * c->nglob);
            bl_solve(&b, u + r * c->nglob);
        }
    }
    bl_free(&b);
    return st;
}

/* Factor every subdomain operator L_a (banded LU). */
int or_factor(or_ctx *c) {
    int status = 0;
    #pragma omp parallel for schedule(dynamic)
    for (int a = 0; a < c->nsub; ++a) {
        bl_free(&c->lu[a]);
        int st = assemble_band(c, a, sigma_local, c->elo[a], c->ehi[a], &c->lu[a]);
        if (st == 0) st = bl_factor(&c->lu[a]);
        if (st) {
            #pragma omp critical
            status = status ? status : (st > 0 ? 1 + a : st);
        }
    }
    c->factored = status == 0;
    return status;
}

/* Packed subdomain vectors: [rhs][a][local box index], length etot per rhs. */
/* uhat = L_a^{-1} g for every subdomain and right-hand side. */
int or_local_solve(const or_ctx *c, int nrhs, const cplx *g, cplx *uhat) {
    if (!c->factored) return -5;
    #pragma omp parallel for collapse(2) schedule(dynamic)
    for (int r = 0; r < nrhs; ++r)
        for (int a = 0; a < c->nsub; ++a) {
            cplx *x = uhat + (long)r * c->etot + c->off[a];
            memcpy(x, g + (long)r * c->etot + c->off[a], sizeof(cplx) * c->nloc[a]);
            bl_solve(&c->lu[a], x);
        }
    return 0;
}

/* g_a = f restricted to the core of a (the f_{i,j} of Sec. 2.2). */
void or_restrict_core(const or_ctx *c, int nrhs, const cplx *f, cplx *g) {
    for (int r = 0; r < nrhs; ++r)
        for (int a = 0; a < c->nsub; ++a) {
            cplx *ga = g + (long)r * c->etot + c->off[a];
            int p[3];
            for (p[2] = c->elo[a][2]; p[2] <= c->ehi[a][2]; ++p[2])
            for (p[1] = c->elo[a][1]; p[1] <= c->ehi[a][1]; ++p[1])
            for (p[0] = c->elo[a][0]; p[0] <= c->ehi[a][0]; ++p[0]) {
                long ip = box_index(c->elo[a], c->ehi[a], p);
                ga[ip] = in_box(c->clo[a], c->chi[a], p) ? f[(long)r * c->nglob + glob_index(c, p)] : 0.0;
            }
        }
}

/* Transferred sources for the next step:
 *   g_a = sum_{b neighbour of a} Psi_{b->a}(uhat_b^{lag(b,a)}),
 *   Psi_{b->a}(v)(p) = -(L_a (beta_{b->a} v))(p) for p in chi_{b->a}, else 0,
 * with lag = number of axes on which b and a differ.  lagged[k] points to the
 * packed local solutions k+1 steps back (NULL = zero).
 * form 1 takes the Phi form of the source instead (eq. Phi, the remark after
 * the horizontal transfer in Sec. 2.2): the terms of L_a(beta v) in which
 * the derivatives fall on beta, i.e. the product-rule remainder
 *   Phi(v; beta) = L_a(beta v) - beta L_a(v),
 * written here as exactly that difference of two operator applications
 * (v is zero outside b's box). */
void or_transfer_form(const or_ctx *c, int nrhs, const cplx *const *lagged, cplx *g, int form) {
    long nmax = 0;
    for (int a = 0; a < c->nsub; ++a) if (c->nloc[a] > nmax) nmax = c->nloc[a];
    memset(g, 0, sizeof(cplx) * c->etot * nrhs);
    #pragma omp parallel
    {
        cplx *w = (cplx *)malloc(sizeof(cplx) * nmax);
        cplx *lw = (cplx *)malloc(sizeof(cplx) * nmax);
        cplx *v = form ? (cplx *)malloc(sizeof(cplx) * nmax) : NULL;
        cplx *lv = form ? (cplx *)malloc(sizeof(cplx) * nmax) : NULL;
        double *bw = form ? (double *)malloc(sizeof(double) * nmax) : NULL;
        #pragma omp for collapse(2) schedule(dynamic)
        for (int r = 0; r < nrhs; ++r)
        for (int a = 0; a < c->nsub; ++a) {
            cplx *ga = g + (long)r * c->etot + c->off[a];
            for (int b = 0; b < c->nsub; ++b) {
                if (b == a) continue;
                int lag = 0, far = 0;
                for (int ax = 0; ax < 3; ++ax) {
                    int d = c->sid[b][ax] - c->sid[a][ax];
                    if (d != 0) ++lag;
                    if (d > 1 || d < -1) far = 1;
                }
                if (far) continue;
                const cplx *src = lagged[lag - 1];
                if (!src) continue;
                const cplx *ub = src + (long)r * c->etot + c->off[b];
                /* w = beta_{b->a} uhat_b on E_a (zero outside E_b) */
                int p[3];
                for (p[2] = c->elo[a][2]; p[2] <= c->ehi[a][2]; ++p[2])
                for (p[1] = c->elo[a][1]; p[1] <= c->ehi[a][1]; ++p[1])
                for (p[0] = c->elo[a][0]; p[0] <= c->ehi[a][0]; ++p[0]) {
                    long ip = box_index(c->elo[a], c->ehi[a], p);
                    int inb = in_box(c->elo[b], c->ehi[b], p);
                    cplx vb = inb ? ub[box_index(c->elo[b], c->ehi[b], p)] : 0.0;
                    double be = inb ? beta_transfer(c, b, a, p) : 0.0;
                    w[ip] = be * vb;
                    if (form) { v[ip] = vb; bw[ip] = be; }
                }
                apply_box(c, a, sigma_local, c->elo[a], c->ehi[a], w, lw);
                if (form) apply_box(c, a, sigma_local, c->elo[a], c->ehi[a], v, lv);
                for (p[2] = c->elo[a][2]; p[2] <= c->ehi[a][2]; ++p[2])
                for (p[1] = c->elo[a][1]; p[1] <= c->ehi[a][1]; ++p[1])
                for (p[0] = c->elo[a][0]; p[0] <= c->ehi[a][0]; ++p[0]) {
                    if (!chi_transfer(c, b, a, p)) continue;
                    long ip = box_index(c->elo[a], c->ehi[a], p);
                    ga[ip] -= form ? lw[ip] - bw[ip] * lv[ip] : lw[ip];
                }
            }
        }
        free(w); free(lw); free(v); free(lv); free(bw);
    }
}

void or_transfer(const or_ctx *c, int nrhs, const cplx *const *lagged, cplx *g) {
    or_transfer_form(c, nrhs, lagged, g, 0);
}

/* u = sum_a beta_{0;a} U_a on the global grid (eq. tsum). */
void or_assemble(const or_ctx *c, int nrhs, const cplx *U, cplx *u) {
    memset(u, 0, sizeof(cplx) * c->nglob * nrhs);
    for (int r = 0; r < nrhs; ++r)
        for (int a = 0; a < c->nsub; ++a) {
            const cplx *Ua = U + (long)r * c->etot + c->off[a];
            int p[3];
            for (p[2] = c->elo[a][2]; p[2] <= c->ehi[a][2]; ++p[2])
            for (p[1] = c->elo[a][1]; p[1] <= c->ehi[a][1]; ++p[1])
            for (p[0] = c->elo[a][0]; p[0] <= c->ehi[a][0]; ++p[0]) {
                double bz = beta_zero(c, a, p);
                if (bz == 0.0) continue;
                u[(long)r * c->nglob + glob_index(c, p)] += bz * Ua[box_index(c->elo[a], c->ehi[a], p)];
            }
        }
}

/* ||f - L_h u||_2 / ||f||_2 per right-hand side (the stopping test of Sec.
 * 4.2); ||f|| = 0 gives ||r||. */
void or_relres(const or_ctx *c, int nrhs, const cplx *f, const cplx *u, double *relres) {
    cplx *lu = (cplx *)malloc(sizeof(cplx) * c->nglob * nrhs);
    or_apply_global(c, nrhs, u, lu);
    for (int r = 0; r < nrhs; ++r) {
        double rn = 0.0, fn = 0.0;
        for (long i = 0; i < c->nglob; ++i) {
            cplx d = f[r * c->nglob + i] - lu[r * c->nglob + i];
            rn += creal(d) * creal(d) + cimag(d) * cimag(d);
            fn += creal(f[r * c->nglob + i]) * creal(f[r * c->nglob + i]) + cimag(f[r * c->nglob + i]) * cimag(f[r * c->nglob + i]);
        }
        relres[r] = fn > 0 ? sqrt(rn / fn) : sqrt(rn);
    }
    free(lu);
}

/* Algorithm 3.1 run for nsteps (continued past N1+N2(+N3) steps with the
 * same recursion when used as an iterative solver, Sec. 4.2.1).
 *   u_out:   global DDM iterate after the last step (nrhs x nglob);
 *   relres:  nsteps x nrhs relative residuals after each step (may be NULL);
 *   uhat_out: packed local solutions of the last step (may be NULL);
 *   U_out:   packed accumulated U_a (may be NULL);
 *   g_out:   packed sources of the last step (may be NULL). */
int or_ddm_run(or_ctx *c, int nrhs, const cplx *f, int nsteps, cplx *u_out, double *relres,
               cplx *uhat_out, cplx *U_out, cplx *g_out) {
    if (!c->factored) { int st = or_factor(c); if (st) return st; }
    long pk = c->etot * nrhs;
    cplx *ring[4];
    for (int k = 0; k < 4; ++k) ring[k] = (cplx *)calloc(pk, sizeof(cplx));
    cplx *g = (cplx *)calloc(pk, sizeof(cplx));
    cplx *U = (cplx *)calloc(pk, sizeof(cplx));
    /* ring[(s) % 4] holds uhat^s; uhat^t = 0 for t <= 0 */
    for (int s = 1; s <= nsteps; ++s) {
        if (s == 1) {
            or_restrict_core(c, nrhs, f, g);
        } else {
            const cplx *lagged[3];
            for (int k = 0; k < 3; ++k) lagged[k] = (s - 1 - k >= 1) ? ring[(s - 1 - k) % 4] : NULL;
            or_transfer(c, nrhs, lagged, g);
        }
        cplx *us = ring[s % 4];
        or_local_solve(c, nrhs, g, us);
        for (long i = 0; i < pk; ++i) U[i] += us[i];
        if (relres || s == nsteps) {
            or_assemble(c, nrhs, U, u_out);
            if (relres) or_relres(c, nrhs, f, u_out, relres + (long)(s - 1) * nrhs);
        }
    }
    if (nsteps <= 0) memset(u_out, 0, sizeof(cplx) * c->nglob * nrhs);
    if (uhat_out && nsteps >= 1) memcpy(uhat_out, ring[nsteps % 4], sizeof(cplx) * pk);
    if (U_out) memcpy(U_out, U, sizeof(cplx) * pk);
    if (g_out) memcpy(g_out, g, sizeof(cplx) * pk);
    for (int k = 0; k < 4; ++k) free(ring[k]);
    free(g); free(U);
    return 0;
}

/* The DDM with K steps as a preconditioner: M_K(v) = sum_a beta_{0;a} U_a
 * after K steps of Algorithm 3.1 with source v (Sec. 4.2.2). */
int or_ddm_precond(or_ctx *c, int nrhs, const cplx *v, int K, cplx *z) {
    return or_ddm_run(c, nrhs, v, K, z, NULL, NULL, NULL, NULL);
}

static double norm2(const cplx *x, long n) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
    return sqrt(s);
}

static cplx dotc(const cplx *x, const cplx *y, long n) { /* x^H y */
    cplx s = 0.0;
    for (long i = 0; i < n; ++i) s += conj(x[i]) * y[i];
    return s;
}

/* Flexible GMRES(restart), right preconditioned by M_K (K > 0) or by the
 * identity (K = 0), x0 = 0, classical Gram-Schmidt applied twice.  One
 * right-hand side.  Stops when the Arnoldi residual estimate reaches tol and
 * the true residual ||f - L_h x|| / ||f|| confirms it, or after maxiter
 * Arnoldi steps.  iters_out = Arnoldi steps, relres_out = true residual. */
int or_fgmres(or_ctx *c, const cplx *f, int K, int restart, double tol, int maxiter,
              cplx *x, int *iters_out, double *relres_out) {
    long n = c->nglob;
    int m = restart;
    cplx *V = (cplx *)calloc((size_t)(m + 1) * n, sizeof(cplx));
    cplx *Z = (cplx *)calloc((size_t)m * n, sizeof(cplx));
    cplx *w = (cplx *)calloc(n, sizeof(cplx));
    cplx *H = (cplx *)calloc((size_t)(m + 1) * m, sizeof(cplx));  /* H[i*m + j] */
    cplx *cs = (cplx *)calloc(m, sizeof(cplx)), *sn = (cplx *)calloc(m, sizeof(cplx));
    cplx *gv = (cplx *)calloc(m + 1, sizeof(cplx)), *y = (cplx *)calloc(m, sizeof(cplx));
    double fn = norm2(f, n);
    int iters = 0;
    double rel = 1.0;
    memset(x, 0, sizeof(cplx) * n);
    if (fn == 0.0) { rel = 0.0; goto done; }
    while (iters < maxiter) {
        /* r = f - A x */
        or_apply_global(c, 1, x, w);
        for (long i = 0; i < n; ++i) V[i] = f[i] - w[i];
        double beta = norm2(V, n);
        rel = beta / fn;
        if (rel <= tol) break;
        for (long i = 0; i < n; ++i) V[i] /= beta;
        memset(gv, 0, sizeof(cplx) * (m + 1));
        gv[0] = beta;
        int j;
        for (j = 0; j < m && iters < maxiter; ++j) {
            cplx *vj = V + (long)j * n, *zj = Z + (long)j * n;
            if (K > 0) or_ddm_precond(c, 1, vj, K, zj);
            else memcpy(zj, vj, sizeof(cplx) * n);
            or_apply_global(c, 1, zj, w);
            for (int pass = 0; pass < 2; ++pass) {
                cplx hcol[m + 1];
                for (int i = 0; i <= j; ++i) hcol[i] = dotc(V + (long)i * n, w, n);
                for (int i = 0; i <= j; ++i) {
                    const cplx *vi = V + (long)i * n;
                    for (long q = 0; q < n; ++q) w[q] -= hcol[i] * vi[q];
                    H[i * m + j] = (pass == 0 ? 0.0 : H[i * m + j]) + hcol[i];
                }
            }
            double hn = norm2(w, n);
            H[(j + 1) * m + j] = hn;
            if (hn > 0) for (long q = 0; q < n; ++q) V[(long)(j + 1) * n + q] = w[q] / hn;
            /* apply previous rotations, then make a new one */
            for (int i = 0; i < j; ++i) {
                cplx a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = conj(cs[i]) * a + conj(sn[i]) * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            cplx a = H[j * m + j], b = H[(j + 1) * m + j];
            double r = sqrt(creal(a) * creal(a) + cimag(a) * cimag(a) + creal(b) * creal(b) + cimag(b) * cimag(b));
            if (r == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = a / r; sn[j] = b / r; }
            H[j * m + j] = r;
            H[(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = conj(cs[j]) * gv[j];
            ++iters;
            if (cabs(gv[j + 1]) / fn <= tol || hn == 0.0) { ++j; break; }
        }
        /* back substitution H y = g on the leading j x j block */
        for (int i = j - 1; i >= 0; --i) {
            cplx s = gv[i];
            for (int q = i + 1; q < j; ++q) s -= H[i * m + q] * y[q];
            y[i] = s / H[i * m + i];
        }
        for (int i = 0; i < j; ++i)
            for (long q = 0; q < n; ++q) x[q] += y[i] * Z[(long)i * n + q];
    }
    {
        or_apply_global(c, 1, x, w);
        double rn = 0.0;
        for (long i = 0; i < n; ++i) { cplx d = f[i] - w[i]; rn += creal(d) * creal(d) + cimag(d) * cimag(d); }
        rel = sqrt(rn) / fn;
    }
done:
    if (iters_out) *iters_out = iters;
    if (relres_out) *relres_out = rel;
    free(V); free(Z); free(w); free(H); free(cs); free(sn); free(gv); free(y);
    return rel <= tol ? 0 : 1;
}
