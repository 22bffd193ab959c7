/*
 * oracle.c - plain FP64 CPU reference for finite element local assembly.
 *
 * TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
 * baseline). Shares no code with the GPU library.
 *
 * Paper anchors: the kernel structure of section 2 (Fig. 1: Jacobian, basis
 * functions, loop nest over quadrature points and test/trial functions), the
 * objects of Table 1 (det, K = inverse Jacobian, coords, fields w, weights W,
 * basis tables, element matrix A), Listing 1 (Helmholtz: the integrand is
 * multiplied by det * W[i] and summed over points i) and Listing 2 (Burgers:
 * coefficient values and gradients evaluated at each point before the j-k
 * loops). Algorithms used here, each chosen for being easy to check by eye:
 *   - Gauss-Jacobi nodes by Newton iteration with deflation on the
 *     three-term recurrence; weights from the classical closed formula;
 *   - Stroud's collapsed (Duffy) product rule on the simplex, or a fully
 *     symmetric rule from the moment equations (symrule.c);
 *   - Lagrange basis by Silvester's product formula in barycentric
 *     coordinates, gradients by the product rule;
 *   - inverse Jacobian by Gauss-Jordan elimination with partial pivoting;
 *   - per-entry integrands written straight from the weak forms, summed over
 *     the points with Neumaier compensation;
 *   - gradients by the complex-step derivative (Squire and Trapp 1998).
 *
 * The per-cell code is compiled twice from element.inc: once on double and
 * once on double complex (for the complex step).
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXD 3
#define MAXP 4
#define MAXN 35         /* scalar P4 on a tetrahedron */
#define MAXQ 216        /* 6 points per direction, tetrahedron */

/* ------------------------------------------------------------------ */
/* One-dimensional Gauss-Jacobi rules                                  */
/* ------------------------------------------------------------------ */

/* P_n^{(a,b)}(x) by the three-term recurrence. */
static double jacobi_poly(int n, double a, double b, double x) {
    if (n == 0) return 1.0;
    double pm1 = 1.0;
    double p = 0.5 * (a - b + (a + b + 2.0) * x);
    for (int k = 2; k <= n; ++k) {
        double c = 2.0 * k + a + b;
        double a1 = 2.0 * k * (k + a + b) * (c - 2.0);
        double a2 = (c - 1.0) * (a * a - b * b);
        double a3 = (c - 2.0) * (c - 1.0) * c;
        double a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
        double pn = ((a2 + a3 * x) * p - a4 * pm1) / a1;
        pm1 = p;
        p = pn;
    }
    return p;
}

/* d/dx P_n^{(a,b)} = (n + a + b + 1)/2 * P_{n-1}^{(a+1,b+1)}. */
static double jacobi_dpoly(int n, double a, double b, double x) {
    if (n == 0) return 0.0;
    return 0.5 * (n + a + b + 1.0) * jacobi_poly(n - 1, a + 1.0, b + 1.0, x);
}

static int cmp_double(const void* p, const void* q) {
    double a = *(const double*)p, b = *(const double*)q;
    return (a > b) - (a < b);
}

/* m-point rule for the integral over [0,1] with weight (1-x)^alpha. */
int oracle_gauss_jacobi(int m, int alpha, double* xo, double* wo) {
    if (m < 1 || m > 16 || alpha < 0 || alpha > 4 || !xo || !wo) return OR_E_INVALID_ARG;
    const double a = alpha, b = 0.0;
    double r[16];
    for (int k = 0; k < m; ++k) {
        double x = -cos(M_PI * (k + 0.5) / m);
        for (int it = 0; it < 200; ++it) {
            double p = jacobi_poly(m, a, b, x);
            double dp = jacobi_dpoly(m, a, b, x);
            double defl = 0.0;
            for (int j = 0; j < k; ++j) defl += 1.0 / (x - r[j]);
            double delta = p / (dp - p * defl);
            x -= delta;
            if (fabs(delta) < 1e-16 * (1.0 + fabs(x))) break;
        }
        r[k] = x;
    }
    qsort(r, m, sizeof(double), cmp_double);
    /* classical weights on [-1,1]: C / ((1 - x^2) P_n'(x)^2) */
    double logC = (a + b + 1.0) * log(2.0) + lgamma(m + a + 1.0) + lgamma(m + b + 1.0)
                  - lgamma(m + a + b + 1.0) - lgamma(m + 1.0);
    double C = exp(logC);
    for (int k = 0; k < m; ++k) {
        double x = r[k];
        if (!(x > -1.0 && x < 1.0)) return OR_E_INVALID_ARG;
        if (k > 0 && !(x > r[k - 1])) return OR_E_INVALID_ARG;
        double dp = jacobi_dpoly(m, a, b, x);
        double wx = C / ((1.0 - x * x) * dp * dp);
        /* x = 2u - 1: (1-x)^a dx = 2^(a+1) (1-u)^a du */
        xo[k] = 0.5 * (1.0 + x);
        wo[k] = wx / pow(2.0, a + 1.0);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Collapsed product rule on the reference simplex                     */
/* ------------------------------------------------------------------ */

static int rule_points_per_dir(int q) { return (q + 2) / 2; }   /* ceil((q+1)/2) */

/* Points X[nq][dim], weights W[nq]; lexicographic, first direction outermost.
 * Triangle: X = (u, (1-u) v), u ~ (1-u)^1, v ~ 1.
 * Tetrahedron: X = (u, (1-u) v, (1-u)(1-v) w), u ~ (1-u)^2, v ~ (1-v)^1, w ~ 1. */
static int simplex_rule(int dim, int quad, int* nq, double* X, double* W) {
    /* quad = q + 16 * rule: rule 1 is the fully symmetric rule (symrule.c) */
    int q = quad & 15, rule = quad >> 4;
    if (rule == 1) return oracle_symmetric_rule(dim, q, nq, X, W);
    if (rule != 0 || q > 10) return OR_E_INVALID_ARG;
    int m = rule_points_per_dir(q);
    double xu[16], wu[16], xv[16], wv[16], xw[16], ww[16];
    if (dim == 2) {
        if (oracle_gauss_jacobi(m, 1, xu, wu) || oracle_gauss_jacobi(m, 0, xv, wv)) return OR_E_INVALID_ARG;
        int k = 0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j, ++k) {
                if (X) { X[2 * k] = xu[i]; X[2 * k + 1] = (1.0 - xu[i]) * xv[j]; }
                if (W) W[k] = wu[i] * wv[j];
            }
        *nq = m * m;
    } else {
        if (oracle_gauss_jacobi(m, 2, xu, wu) || oracle_gauss_jacobi(m, 1, xv, wv) ||
            oracle_gauss_jacobi(m, 0, xw, ww)) return OR_E_INVALID_ARG;
        int k = 0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                for (int l = 0; l < m; ++l, ++k) {
                    if (X) {
                        X[3 * k] = xu[i];
                        X[3 * k + 1] = (1.0 - xu[i]) * xv[j];
                        X[3 * k + 2] = (1.0 - xu[i]) * (1.0 - xv[j]) * xw[l];
                    }
                    if (W) W[k] = wu[i] * wv[j] * ww[l];
                }
        *nq = m * m * m;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Lagrange basis: Silvester's formula on lattice multi-indices          */
/* ------------------------------------------------------------------ */

static const int TRI_EDGE[3][2] = {{1, 2}, {0, 2}, {0, 1}};
static const int TET_EDGE[6][2] = {{2, 3}, {1, 3}, {1, 2}, {0, 3}, {0, 2}, {0, 1}};

/* Barycentric multi-indices alpha[n][dim+1] of the degree-p nodes, in the
 * order: vertices, edges (points from the lower to the higher vertex),
 * faces (face f opposite vertex f; points (i,j) with j outermost), interior. */
static int lattice_nodes(int dim, int p, int alpha[][4]) {
    int n = 0;
    if (p == 0) { memset(alpha[0], 0, sizeof alpha[0]); return 1; }
    for (int v = 0; v <= dim; ++v) {
        memset(alpha[n], 0, sizeof alpha[n]);
        alpha[n++][v] = p;
    }
    int ne = dim == 2 ? 3 : 6;
    for (int e = 0; e < ne; ++e) {
        int a = dim == 2 ? TRI_EDGE[e][0] : TET_EDGE[e][0];
        int b = dim == 2 ? TRI_EDGE[e][1] : TET_EDGE[e][1];
        for (int k = 1; k < p; ++k) {
            memset(alpha[n], 0, sizeof alpha[n]);
            alpha[n][a] = p - k;
            alpha[n][b] = k;
            ++n;
        }
    }
    int nf = dim == 2 ? 1 : 4;
    for (int f = 0; f < nf; ++f) {
        int vv[3], c = 0;
        for (int v = 0; v <= dim; ++v)
            if (dim == 2 || v != f) vv[c++] = v;
        for (int j = 1; j < p; ++j)
            for (int i = 1; i + j < p; ++i) {
                memset(alpha[n], 0, sizeof alpha[n]);
                alpha[n][vv[0]] = p - i - j;
                alpha[n][vv[1]] = i;
                alpha[n][vv[2]] = j;
                ++n;
            }
    }
    if (dim == 3)
        for (int k = 1; k < p; ++k)
            for (int j = 1; j + k < p; ++j)
                for (int i = 1; i + j + k < p; ++i) {
                    alpha[n][0] = p - i - j - k;
                    alpha[n][1] = i;
                    alpha[n][2] = j;
                    alpha[n][3] = k;
                    ++n;
                }
    return n;
}

/* s_m(t) = prod_{k<m} (p t - k)/(k+1) and its derivative. */
static void silvester_factor(int p, int m, double t, double* s, double* ds) {
    double val = 1.0, der = 0.0;
    for (int k = 0; k < m; ++k) {
        double f = (p * t - k) / (k + 1.0);
        der = der * f + val * p / (k + 1.0);
        val *= f;
    }
    *s = val;
    *ds = der;
}

/* phi[n] and reference gradients dphi[dim][n] at reference point X. */
static void silvester_eval(int dim, int p, int n, int alpha[][4], const double* X,
                           double* phi, double* dphi) {
    double lam[4];
    lam[0] = 1.0;
    for (int j = 0; j < dim; ++j) { lam[j + 1] = X[j]; lam[0] -= X[j]; }
    for (int a = 0; a < n; ++a) {
        double s[4], ds[4];
        for (int i = 0; i <= dim; ++i) silvester_factor(p, alpha[a][i], lam[i], &s[i], &ds[i]);
        double val = 1.0;
        for (int i = 0; i <= dim; ++i) val *= s[i];
        phi[a] = val;
        /* d phi / d lam_i */
        double dl[4];
        for (int i = 0; i <= dim; ++i) {
            double t = ds[i];
            for (int k = 0; k <= dim; ++k)
                if (k != i) t *= s[k];
            dl[i] = t;
        }
        /* lam_0 = 1 - sum X_j, lam_{j+1} = X_j */
        for (int j = 0; j < dim; ++j) dphi[j * n + a] = dl[j + 1] - dl[0];
    }
}

static int nscalar(int dim, int p) {
    return dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
}

int oracle_tabulate(int dim, int degree, int quad_degree, int* nq, int* ndof,
                    double* points, double* weights, double* basis, double* dbasis) {
    if (dim == OR_PRISM) return prism_tabulate(degree, quad_degree, nq, ndof, points, weights, basis, dbasis);
    if ((dim != 2 && dim != 3) || degree < 0 || degree > MAXP || !nq || !ndof) return OR_E_INVALID_ARG;
    if (quad_degree < 0) return OR_E_INVALID_ARG;
    int alpha[MAXN][4];
    int n = lattice_nodes(dim, degree, alpha);
    double X[MAXQ * 3], W[MAXQ];
    int q;
    int st = simplex_rule(dim, quad_degree, &q, X, W);
    if (st) return st;
    *nq = q;
    *ndof = n;
    if (points) memcpy(points, X, sizeof(double) * q * dim);
    if (weights) memcpy(weights, W, sizeof(double) * q);
    if (basis || dbasis) {
        double phi[MAXN], dphi[3 * MAXN];
        for (int k = 0; k < q; ++k) {
            silvester_eval(dim, degree, n, alpha, X + k * dim, phi, dphi);
            if (basis) memcpy(basis + (size_t)k * n, phi, sizeof(double) * n);
            if (dbasis)
                for (int j = 0; j < dim; ++j)
                    memcpy(dbasis + ((size_t)j * q + k) * n, dphi + j * n, sizeof(double) * n);
        }
    }
    return OR_OK;
}

/* Basis values phi[npts][ndof] and reference gradients dphi[dim][npts][ndof]
 * of the degree-p element at arbitrary reference points X[npts][dim]. */
int oracle_basis_at(int dim, int degree, int npts, const double* X, double* phi, double* dphi) {
    if (dim == OR_PRISM) return prism_basis_at(degree, npts, X, phi, dphi);
    if ((dim != 2 && dim != 3) || degree < 0 || degree > MAXP || npts < 0 || (npts && (!X || !phi)))
        return OR_E_INVALID_ARG;
    int alpha[MAXN][4];
    int n = lattice_nodes(dim, degree, alpha);
    double ph[MAXN], dph[3 * MAXN];
    for (int k = 0; k < npts; ++k) {
        silvester_eval(dim, degree, n, alpha, X + (size_t)k * dim, ph, dph);
        memcpy(phi + (size_t)k * n, ph, sizeof(double) * n);
        if (dphi)
            for (int j = 0; j < dim; ++j)
                memcpy(dphi + ((size_t)j * npts + k) * n, dph + j * n, sizeof(double) * n);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Tables of one assembly call                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    int nq, n;              /* points, dofs of the degree-p element */
    double* W;              /* [nq] */
    double* phi;            /* [nq][n] */
    double* dphi;           /* [dim][nq][n] */
} table;

typedef struct {
    int form, dim, p, N, out_len, ncomp_space, nfield;
    table sp;                       /* space of the test/trial functions */
    table fl[4];                    /* one per coefficient field */
    int fncomp[4], fnloc[4];
    double cst[2];
} ctx;

static void free_table(table* t) {
    free(t->W); free(t->phi); free(t->dphi);
    t->W = t->phi = t->dphi = NULL;
}

static int make_table(int dim, int p, int q, table* t) {
    int nq, n;
    int st = oracle_tabulate(dim, p, q, &nq, &n, NULL, NULL, NULL, NULL);
    if (st) return st;
    t->nq = nq; t->n = n;
    t->W = malloc(sizeof(double) * nq);
    t->phi = malloc(sizeof(double) * nq * n);
    t->dphi = malloc(sizeof(double) * dim * nq * n);
    if (!t->W || !t->phi || !t->dphi) { free_table(t); return OR_E_NOMEM; }
    return oracle_tabulate(dim, p, q, &nq, &n, NULL, t->W, t->phi, t->dphi);
}

int oracle_tensor_dim(int form, int dim, int degree) {
    if (dim == OR_PRISM)
        return (form == OR_MASS || form == OR_HELMHOLTZ || form == OR_DIFFUSION) ? prism_ndofs(degree) : -1;
    int n = nscalar(dim, degree);
    switch (form) {
        case OR_MASS: case OR_HELMHOLTZ: case OR_DIFFUSION: return n;
        case OR_ELASTICITY: case OR_BURGERS: case OR_SVK_RESIDUAL: case OR_SVK_JACOBIAN: return dim * n;
        case OR_SVK_ENERGY: return 0;
        default: return -1;
    }
}

static void free_ctx(ctx* c) {
    free_table(&c->sp);
    for (int i = 0; i < 4; ++i) free_table(&c->fl[i]);
}

static int make_ctx(int form, int dim, int degree, int quad_degree, const oracle_field* fields,
                    int nfield, const double* constants, int nconst, ctx* c) {
    memset(c, 0, sizeof *c);
    if (dim != 2 && dim != 3) return OR_E_INVALID_ARG;
    if (form < OR_MASS || form > OR_DIFFUSION) return OR_E_INVALID_ARG;
    if (degree < 1 || degree > MAXP) return OR_E_UNSUPPORTED;
    if (nfield < 0 || nfield > 4 || (nfield > 0 && !fields) || nconst < 0) return OR_E_INVALID_ARG;
    if (nconst > 0 && !constants) return OR_E_INVALID_ARG;
    int q = quad_degree >= 0 ? quad_degree : (form == OR_BURGERS ? 2 * degree + 1 : 2 * degree);
    c->form = form; c->dim = dim; c->p = degree; c->nfield = nfield;
    int N = oracle_tensor_dim(form, dim, degree);
    c->N = N;
    c->ncomp_space = (form == OR_MASS || form == OR_HELMHOLTZ || form == OR_DIFFUSION) ? 1 : dim;
    c->out_len = form == OR_SVK_ENERGY ? 1 : (form == OR_SVK_RESIDUAL ? N : N * N);
    /* field count and shape per form */
    int need_vec = 0;
    switch (form) {
        case OR_MASS: case OR_HELMHOLTZ:
            if (nfield > 1) return OR_E_INVALID_ARG;
            break;
        case OR_DIFFUSION:
            if (nfield != 0) return OR_E_INVALID_ARG;
            break;
        case OR_ELASTICITY:
            if (!(nfield == 2 || (nfield == 0 && nconst >= 2))) return OR_E_INVALID_ARG;
            break;
        default:
            if (nfield != 1) return OR_E_INVALID_ARG;
            need_vec = 1;
    }
    for (int i = 0; i < nfield; ++i) {
        if (!fields[i].values || fields[i].degree < 0 || fields[i].degree > MAXP) return OR_E_INVALID_ARG;
        int want = need_vec ? dim : 1;
        if (fields[i].ncomp != want) return OR_E_INVALID_ARG;
        c->fncomp[i] = fields[i].ncomp;
        c->fnloc[i] = fields[i].degree == 0 ? 1 : nscalar(dim, fields[i].degree);
    }
    c->cst[0] = 1.0; c->cst[1] = 1.0;
    for (int i = 0; i < nconst && i < 2; ++i) c->cst[i] = constants[i];
    int st = make_table(dim, degree, q, &c->sp);
    for (int i = 0; !st && i < nfield; ++i) st = make_table(dim, fields[i].degree, q, &c->fl[i]);
    if (st) free_ctx(c);
    return st;
}

/* ------------------------------------------------------------------ */
/* Per-cell evaluation on double and on double complex                  */
/* ------------------------------------------------------------------ */

#define SC double
#define FN(x) x##_r
#define SC_REAL 1
#include "element.inc"
#undef SC
#undef FN
#undef SC_REAL

#define SC double complex
#define FN(x) x##_c
#define SC_REAL 0
#include "element.inc"
#undef SC
#undef FN
#undef SC_REAL

static int nthreads_or_default(int nthreads) {
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

static int check_mesh_args(const double* coords, int64_t nvert, const int32_t* c2v, int64_t ncells) {
    if (ncells < 0 || nvert < 0) return OR_E_INVALID_ARG;
    if (ncells > 0 && (!coords || !c2v)) return OR_E_INVALID_ARG;
    return OR_OK;
}

/* local vertex coordinates and coefficient dofs of cell e */
static int gather_cell(const ctx* c, const double* coords, int64_t nvert, const int32_t* c2v,
                       int64_t e, const oracle_field* fields, double* xs, double* cf[4]) {
    int d = c->dim;
    for (int v = 0; v <= d; ++v) {
        int32_t g = c2v[e * (d + 1) + v];
        if (g < 0 || g >= nvert) return OR_E_INVALID_ARG;
        for (int i = 0; i < d; ++i) xs[v * d + i] = coords[(int64_t)g * d + i];
    }
    for (int f = 0; f < c->nfield; ++f) {
        int nl = c->fnloc[f], nc = c->fncomp[f];
        for (int r = 0; r < nl; ++r)
            for (int k = 0; k < nc; ++k) {
                int64_t src = fields[f].cell_to_dof
                    ? (int64_t)fields[f].cell_to_dof[e * nl + r] * nc + k
                    : (e * nl + r) * nc + k;
                cf[f][r * nc + k] = fields[f].values[src];
            }
    }
    return OR_OK;
}

int oracle_assemble(int form, int dim, int degree, int quad_degree,
                    const double* coords, int64_t nvert, const int32_t* c2v, int64_t ncells,
                    const oracle_field* fields, int nfield, const double* constants, int nconst,
                    const int64_t* cells, int64_t nsel, double* out, int nthreads) {
    if (dim == OR_PRISM)
        return prism_assemble(form, degree, quad_degree, coords, nvert, c2v, ncells, fields, nfield, constants,
                              nconst, cells, nsel, out, nthreads);
    int st = check_mesh_args(coords, nvert, c2v, ncells);
    if (st) return st;
    if (!cells && nsel != ncells) return OR_E_INVALID_ARG;
    if (nsel > 0 && !out) return OR_E_INVALID_ARG;
    ctx c;
    st = make_ctx(form, dim, degree, quad_degree, fields, nfield, constants, nconst, &c);
    if (st) return st;
    int status = OR_OK;
    int nt = nthreads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
    {
        double xs[12], cfb[4][MAXN * 3];
        double* cf[4] = {cfb[0], cfb[1], cfb[2], cfb[3]};
        double* work = malloc(sizeof(double) * 2 * (size_t)c.out_len);
        int my = work ? OR_OK : OR_E_NOMEM;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < nsel; ++k) {
            if (my) continue;
            int64_t e = cells ? cells[k] : k;
            if (e < 0 || e >= ncells) { my = OR_E_INVALID_ARG; continue; }
            int s = gather_cell(&c, coords, nvert, c2v, e, fields, xs, cf);
            if (!s) s = element_r(&c, xs, (const double* const*)cf, out + k * c.out_len, work);
            if (s) my = s;
        }
        free(work);
        if (my) {
#pragma omp critical
            { if (!status) status = my; }
        }
    }
    free_ctx(&c);
    return status;
}

/* S_e for complex-valued inputs: lam^T A u, lam^T b or Pi. */
static double complex cell_functional(const ctx* c, const double complex* A, const double* lam,
                                      const double* u) {
    double complex s = 0.0;
    if (c->form == OR_SVK_ENERGY) return A[0];
    if (c->form == OR_SVK_RESIDUAL) {
        for (int i = 0; i < c->N; ++i) s += lam[i] * A[i];
        return s;
    }
    for (int i = 0; i < c->N; ++i) {
        double complex r = 0.0;
        for (int j = 0; j < c->N; ++j) r += A[i * c->N + j] * u[j];
        s += lam[i] * r;
    }
    return s;
}

int oracle_adjoint(int form, int dim, int degree, int quad_degree,
                   const double* coords, int64_t nvert, const int32_t* c2v, int64_t ncells,
                   const oracle_field* fields, int nfield, const double* constants, int nconst,
                   const double* lam, const double* u, double seed,
                   double* grad_coords, double* const* grad_fields, double* value, int nthreads) {
    int st = check_mesh_args(coords, nvert, c2v, ncells);
    if (st) return st;
    ctx c;
    st = make_ctx(form, dim, degree, quad_degree, fields, nfield, constants, nconst, &c);
    if (st) return st;
    if (form != OR_SVK_ENERGY && (!lam || (form != OR_SVK_RESIDUAL && !u))) { free_ctx(&c); return OR_E_INVALID_ARG; }
    const int d = dim;
    int nloc = (d + 1) * d;
    for (int f = 0; f < nfield; ++f) nloc += c.fnloc[f] * c.fncomp[f];
    double* g = calloc((size_t)(ncells > 0 ? ncells : 1) * nloc, sizeof(double));
    double* sv = calloc((size_t)(ncells > 0 ? ncells : 1), sizeof(double));
    if (!g || !sv) { free(g); free(sv); free_ctx(&c); return OR_E_NOMEM; }
    const double h = 1e-30;
    int status = OR_OK;
    int nt = nthreads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
    {
        double xs[12], cfb[4][MAXN * 3];
        double* cf[4] = {cfb[0], cfb[1], cfb[2], cfb[3]};
        double complex xz[12], cfz[4][MAXN * 3];
        double complex* cz[4] = {cfz[0], cfz[1], cfz[2], cfz[3]};
        double complex* A = malloc(sizeof(double complex) * (size_t)c.out_len);
        double complex* work = malloc(sizeof(double complex) * 2 * (size_t)c.out_len);
        int my = (A && work) ? OR_OK : OR_E_NOMEM;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < ncells; ++e) {
            if (my) continue;
            int s = gather_cell(&c, coords, nvert, c2v, e, fields, xs, cf);
            if (s) { my = s; continue; }
            const double* le = lam ? lam + e * (c.form == OR_SVK_ENERGY ? 0 : c.N) : NULL;
            const double* ue = u ? u + e * c.N : NULL;
            int k = 0;
            for (int pass = 0; pass < nloc && !my; ++pass) {
                for (int i = 0; i < (d + 1) * d; ++i) xz[i] = xs[i];
                for (int f = 0; f < c.nfield; ++f)
                    for (int r = 0; r < c.fnloc[f] * c.fncomp[f]; ++r) cz[f][r] = cf[f][r];
                /* perturb input number `pass` by i*h */
                if (pass < (d + 1) * d) xz[pass] += I * h;
                else {
                    int rem = pass - (d + 1) * d;
                    for (int f = 0; f < c.nfield; ++f) {
                        int len = c.fnloc[f] * c.fncomp[f];
                        if (rem < len) { cz[f][rem] += I * h; break; }
                        rem -= len;
                    }
                }
                s = element_c(&c, xz, (const double complex* const*)cz, A, work);
                if (s) { my = s; break; }
                double complex S = cell_functional(&c, A, le, ue);
                g[e * nloc + k++] = cimag(S) / h;
                if (pass == 0) sv[e] = creal(S);
            }
        }
        free(A);
        free(work);
        if (my) {
#pragma omp critical
            { if (!status) status = my; }
        }
    }
    if (!status) {
        /* sequential scatter-add: deterministic */
        double total = 0.0;
        for (int64_t e = 0; e < ncells; ++e) {
            const double* ge = g + e * nloc;
            total += sv[e];
            for (int v = 0; v <= d; ++v) {
                int32_t gv = c2v[e * (d + 1) + v];
                if (grad_coords)
                    for (int i = 0; i < d; ++i) grad_coords[(int64_t)gv * d + i] += seed * ge[v * d + i];
            }
            int off = (d + 1) * d;
            for (int f = 0; f < nfield; ++f) {
                int nl = c.fnloc[f], nc = c.fncomp[f];
                if (grad_fields && grad_fields[f])
                    for (int r = 0; r < nl; ++r)
                        for (int kk = 0; kk < nc; ++kk) {
                            int64_t dst = fields[f].cell_to_dof
                                ? (int64_t)fields[f].cell_to_dof[e * nl + r] * nc + kk
                                : (e * nl + r) * nc + kk;
                            grad_fields[f][dst] += seed * ge[off + r * nc + kk];
                        }
                off += nl * nc;
            }
        }
        if (value) *value = total;
    }
    free(g);
    free(sv);
    free_ctx(&c);
    return status;
}
