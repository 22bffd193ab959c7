/*
 * prism.c - plain FP64 CPU reference for prism cells (triangle x interval).
 *
 * TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
 * baseline). Shares no code with the GPU library.
 *
 * The paper's benchmarks run on triangles, tetrahedra and prisms with
 * Lagrange elements of degree 1..4 (section 5.2; for p = 1 the prism's j and
 * k loops have 6 iterations). A prism cell is the image of the reference
 * prism T x [0,1] (T the reference triangle (0,0),(1,0),(0,1)) under the map
 * spanned by the six degree-1 prism basis functions, so J depends on the
 * point: here J, det J and K = J^-1 are formed afresh at every quadrature
 * point, and every entry is summed straight from the weak form:
 *   MASS       f u v                  f a degree-1 prism field (1 if absent)
 *   HELMHOLTZ  grad u . grad v + f u v
 *   DIFFUSION  kappa dt grad u . grad v   (no mass term; constants kappa, dt)
 *
 * Element of degree p: the tensor product of the degree-p Lagrange triangle
 * (nodes and order of oracle.c) and the degree-p Lagrange interval with
 * equispaced nodes ordered 0, 1, then the interior ones ascending; local dof
 * (a, b) of the two factors has index a (p + 1) + b. So the six vertices of
 * a degree-1 prism are (t0,0), (t0,1), (t1,0), (t1,1), (t2,0), (t2,1): each
 * triangle vertex at the bottom, then at the top.
 *
 * Rule of degree q: the triangle rule of degree q (collapsed Gauss-Jacobi or,
 * for q + 16, the symmetric rule) times Gauss-Legendre with
 * m = ceil((q + 1) / 2) points on [0,1]; triangle point outermost.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

#define PMAXP 4
#define PMAXN 75     /* (4+1)(4+2)/2 * (4+1) */
#define PMAXQ 576    /* 24 symmetric or 25 Gauss-Jacobi triangle points x 5, bounded */

/* Degree-p Lagrange basis on [0,1] at z: nodes 0, 1, 1/p, ..., (p-1)/p;
 * values l[p+1], derivatives dl[p+1] by the product rule. */
static void lagrange_interval(int p, double z, double* l, double* dl) {
    double t[PMAXP + 1];
    t[0] = 0.0;
    if (p >= 1) t[1] = 1.0;
    for (int k = 1; k < p; ++k) t[k + 1] = (double)k / p;
    for (int i = 0; i <= p; ++i) {
        double val = 1.0, der = 0.0;
        for (int j = 0; j <= p; ++j) {
            if (j == i) continue;
            double f = (z - t[j]) / (t[i] - t[j]);
            der = der * f + val / (t[i] - t[j]);
            val *= f;
        }
        l[i] = val;
        dl[i] = der;
    }
}

static int tri_count(int p) { return (p + 1) * (p + 2) / 2; }

int prism_ndofs(int p) { return tri_count(p) * (p + 1); }

/* The rule: X[nq][3], W[nq]. */
static int prism_rule(int quad, int* nq, double* X, double* W) {
    int q = quad & 15;
    int m = (q + 2) / 2;
    int nt = 0, nd = 0;
    if (oracle_tabulate(2, 1, quad, &nt, &nd, NULL, NULL, NULL, NULL)) return OR_E_INVALID_ARG;
    double* Xt = malloc(sizeof(double) * 2 * (size_t)nt);
    double* Wt = malloc(sizeof(double) * (size_t)nt);
    double z[16], wz[16];
    int st = (!Xt || !Wt) ? OR_E_NOMEM : OR_OK;
    if (!st) st = oracle_tabulate(2, 1, quad, &nt, &nd, Xt, Wt, NULL, NULL);
    if (!st && (m > 16 || oracle_gauss_jacobi(m, 0, z, wz))) st = OR_E_INVALID_ARG;
    if (!st && nt * m > PMAXQ) st = OR_E_UNSUPPORTED;
    if (!st) {
        int k = 0;
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < m; ++j, ++k) {
                if (X) {
                    X[3 * k] = Xt[2 * i];
                    X[3 * k + 1] = Xt[2 * i + 1];
                    X[3 * k + 2] = z[j];
                }
                if (W) W[k] = Wt[i] * wz[j];
            }
        *nq = nt * m;
    }
    free(Xt);
    free(Wt);
    return st;
}

/* Basis values phi[n] and reference gradients dphi[3][n] at one point. */
static int prism_basis(int p, const double* X, double* phi, double* dphi) {
    const int nt = tri_count(p), n = nt * (p + 1);
    double tp[15], tdp[2 * 15], l[PMAXP + 1], dl[PMAXP + 1];
    if (oracle_basis_at(2, p, 1, X, tp, tdp)) return OR_E_INVALID_ARG;
    lagrange_interval(p, X[2], l, dl);
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b <= p; ++b) {
            int i = a * (p + 1) + b;
            phi[i] = tp[a] * l[b];
            dphi[i] = tdp[a] * l[b];
            dphi[n + i] = tdp[nt + a] * l[b];
            dphi[2 * n + i] = tp[a] * dl[b];
        }
    return OR_OK;
}

int prism_tabulate(int degree, int quad_degree, int* nq, int* ndof, double* points, double* weights,
                   double* basis, double* dbasis) {
    if (degree < 0 || degree > PMAXP || quad_degree < 0 || !nq || !ndof) return OR_E_INVALID_ARG;
    int q = 0;
    double* Xl = malloc(sizeof(double) * PMAXQ * 3);
    double* Wl = malloc(sizeof(double) * PMAXQ);
    if (!Xl || !Wl) { free(Xl); free(Wl); return OR_E_NOMEM; }
    int st = prism_rule(quad_degree, &q, Xl, Wl);
    if (st) { free(Xl); free(Wl); return st; }
    int n = prism_ndofs(degree);
    *nq = q;
    *ndof = n;
    if (points) memcpy(points, Xl, sizeof(double) * 3 * q);
    if (weights) memcpy(weights, Wl, sizeof(double) * q);
    if (basis || dbasis) {
        double phi[PMAXN], dphi[3 * PMAXN];
        for (int k = 0; k < q && !st; ++k) {
            st = prism_basis(degree, Xl + 3 * k, phi, dphi);
            if (basis) memcpy(basis + (size_t)k * n, phi, sizeof(double) * n);
            if (dbasis)
                for (int j = 0; j < 3; ++j) memcpy(dbasis + ((size_t)j * q + k) * n, dphi + j * n, sizeof(double) * n);
        }
    }
    free(Xl);
    free(Wl);
    return st;
}

int prism_basis_at(int degree, int npts, const double* X, double* phi, double* dphi) {
    if (degree < 0 || degree > PMAXP || npts < 0 || (npts && (!X || !phi))) return OR_E_INVALID_ARG;
    const int n = prism_ndofs(degree);
    double ph[PMAXN], dph[3 * PMAXN];
    for (int k = 0; k < npts; ++k) {
        if (prism_basis(degree, X + 3 * (size_t)k, ph, dph)) return OR_E_INVALID_ARG;
        memcpy(phi + (size_t)k * n, ph, sizeof(double) * n);
        if (dphi)
            for (int j = 0; j < 3; ++j) memcpy(dphi + ((size_t)j * npts + k) * n, dph + j * n, sizeof(double) * n);
    }
    return OR_OK;
}

/* Neumaier-compensated s + c += x. */
static void nadd(double* s, double* c, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

/* K = J^-1 by cofactors and |det J|; J[i][a] = d x_i / d X_a. */
static int invert3(const double J[3][3], double K[3][3], double* adet) {
    double C[3][3];
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    if (!(det != 0.0) || !isfinite(det)) return OR_E_DEGENERATE;
    /* adj(J) = C^T; K = adj(J) / det */
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < 3; ++i) K[a][i] = C[i][a] / det;
    *adet = fabs(det);
    return OR_OK;
}

typedef struct {
    int form, p, n, nq, nfield;
    double* X;     /* [nq][3] */
    double* W;     /* [nq] */
    double* phi;   /* [nq][n] */
    double* dphi;  /* [3][nq][n] */
    double* gphi;  /* degree-1 geometry basis [nq][6] */
    double* gdphi; /* [3][nq][6] */
    double kdt;
} pctx;

static void pctx_free(pctx* c) {
    free(c->X); free(c->W); free(c->phi); free(c->dphi); free(c->gphi); free(c->gdphi);
}

/* Element tensor of one prism: x[6][3] vertex coordinates, f[6] the field's
 * vertex values (NULL: f = 1), out[n][n]. */
static int prism_element(const pctx* c, const double x[6][3], const double* f, double* out, double* comp) {
    const int n = c->n, nq = c->nq;
    for (int v = 0; v < 6; ++v)
        for (int i = 0; i < 3; ++i)
            if (!isfinite(x[v][i])) return OR_E_DEGENERATE;
    for (int i = 0; i < n * n; ++i) out[i] = comp[i] = 0.0;
    double g[PMAXN][3];
    for (int q = 0; q < nq; ++q) {
        double J[3][3], K[3][3], adet;
        for (int i = 0; i < 3; ++i)
            for (int a = 0; a < 3; ++a) {
                double t = 0.0;
                for (int v = 0; v < 6; ++v) t += x[v][i] * c->gdphi[((size_t)a * nq + q) * 6 + v];
                J[i][a] = t;
            }
        int st = invert3(J, K, &adet);
        if (st) return st;
        const double wq = c->W[q] * adet;
        for (int b = 0; b < n; ++b)
            for (int i = 0; i < 3; ++i) {
                double t = 0.0;
                for (int a = 0; a < 3; ++a) t += K[a][i] * c->dphi[((size_t)a * nq + q) * n + b];
                g[b][i] = t;
            }
        double fq = 1.0;
        if (f) {
            fq = 0.0;
            for (int v = 0; v < 6; ++v) fq += f[v] * c->gphi[(size_t)q * 6 + v];
        }
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                const double pa = c->phi[(size_t)q * n + a], pb = c->phi[(size_t)q * n + b];
                const double gg = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
                double val;
                if (c->form == OR_MASS) val = fq * pa * pb;
                else if (c->form == OR_HELMHOLTZ) val = gg + fq * pa * pb;
                else val = c->kdt * gg;
                nadd(&out[a * n + b], &comp[a * n + b], wq * val);
            }
    }
    for (int i = 0; i < n * n; ++i) out[i] += comp[i];
    return OR_OK;
}

int prism_assemble(int form, int degree, int quad_degree, const double* coords, int64_t nvert,
                   const int32_t* c2v, int64_t ncells, const oracle_field* fields, int nfield,
                   const double* constants, int nconst, const int64_t* cells, int64_t nsel, double* out,
                   int nthreads) {
    if (form != OR_MASS && form != OR_HELMHOLTZ && form != OR_DIFFUSION) return OR_E_UNSUPPORTED;
    if (degree < 1 || degree > PMAXP) return OR_E_UNSUPPORTED;
    if (ncells < 0 || nvert < 0 || (ncells > 0 && (!coords || !c2v))) return OR_E_INVALID_ARG;
    if (!cells && nsel != ncells) return OR_E_INVALID_ARG;
    if (nsel > 0 && !out) return OR_E_INVALID_ARG;
    if (nfield < 0 || nfield > 1 || (nfield && !fields) || nconst < 0 || (nconst && !constants))
        return OR_E_INVALID_ARG;
    if (form == OR_DIFFUSION && nfield) return OR_E_INVALID_ARG;
    if (nfield && (fields[0].degree != 1 || fields[0].ncomp != 1 || !fields[0].values)) return OR_E_UNSUPPORTED;
    pctx c;
    memset(&c, 0, sizeof c);
    c.form = form;
    c.p = degree;
    c.nfield = nfield;
    c.kdt = (nconst > 0 ? constants[0] : 1.0) * (nconst > 1 ? constants[1] : 1.0);
    int q = quad_degree >= 0 ? quad_degree : 2 * degree;
    int nq = 0, n = 0;
    int st = prism_tabulate(degree, q, &nq, &n, NULL, NULL, NULL, NULL);
    if (st) return st;
    c.nq = nq;
    c.n = n;
    c.X = malloc(sizeof(double) * 3 * nq);
    c.W = malloc(sizeof(double) * nq);
    c.phi = malloc(sizeof(double) * (size_t)nq * n);
    c.dphi = malloc(sizeof(double) * 3 * (size_t)nq * n);
    c.gphi = malloc(sizeof(double) * (size_t)nq * 6);
    c.gdphi = malloc(sizeof(double) * 3 * (size_t)nq * 6);
    if (!c.X || !c.W || !c.phi || !c.dphi || !c.gphi || !c.gdphi) { pctx_free(&c); return OR_E_NOMEM; }
    st = prism_tabulate(degree, q, &nq, &n, c.X, c.W, c.phi, c.dphi);
    if (!st) st = prism_basis_at(1, nq, c.X, c.gphi, c.gdphi);
    if (st) { pctx_free(&c); return st; }
    int status = OR_OK;
    const int nt = nthreads > 0 ? nthreads :
#ifdef _OPENMP
        omp_get_max_threads();
#else
        1;
#endif
#pragma omp parallel num_threads(nt)
    {
        double* comp = malloc(sizeof(double) * (size_t)n * n);
        int my = comp ? OR_OK : OR_E_NOMEM;
#pragma omp for schedule(static)
        for (int64_t k = 0; k < nsel; ++k) {
            if (my) continue;
            const int64_t e = cells ? cells[k] : k;
            if (e < 0 || e >= ncells) { my = OR_E_INVALID_ARG; continue; }
            double x[6][3], fv[6];
            for (int v = 0; v < 6 && !my; ++v) {
                const int32_t gv = c2v[e * 6 + v];
                if (gv < 0 || gv >= nvert) { my = OR_E_INVALID_ARG; break; }
                for (int i = 0; i < 3; ++i) x[v][i] = coords[(int64_t)gv * 3 + i];
                if (nfield) {
                    const int64_t src = fields[0].cell_to_dof ? fields[0].cell_to_dof[e * 6 + v] : e * 6 + v;
                    fv[v] = fields[0].values[src];
                    if (!isfinite(fv[v])) my = OR_E_DEGENERATE;
                }
            }
            if (my) continue;
            int s = prism_element(&c, x, nfield ? fv : NULL, out + k * (int64_t)n * n, comp);
            if (s) my = s;
        }
        free(comp);
        if (my) {
#pragma omp critical
            { if (!status) status = my; }
        }
    }
    pctx_free(&c);
    return status;
}
