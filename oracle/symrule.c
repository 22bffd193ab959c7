/*
 * symrule.c - fully symmetric quadrature rules for the oracle.
 *
 * TEST INFRASTRUCTURE ONLY (part of liboracle.so). Shares no code with the
 * GPU library.
 *
 * The paper's kernels use small symmetric rules (3 points in Listing 1,
 * 5 points in Listing 2) without printing them. A fully symmetric rule is a
 * union of orbits of the simplex's symmetry group acting on barycentric
 * coordinates, with one weight per orbit. Its points and weights are fixed by
 * requiring exact integration of every barycentric monomial
 * lambda^alpha, |alpha| <= degree, whose integral over the unit simplex of
 * dimension d is alpha! / (|alpha| + d)! (the Dirichlet integral). This file
 * solves those equations by Gauss-Newton with a backtracking line search
 * (forward-difference Jacobian) from a deterministic grid of starting
 * points, in long double (the search abandons starts that do not converge).
 *
 * Structures (orbits, exact degree) for q = 0..6:
 *   triangle  1: centroid; 2: (a,a,1-2a); 3-4: two (a,a,1-2a);
 *             5: centroid + two (a,a,1-2a); 6: two (a,a,1-2a) + (a,b,1-a-b)
 *   tetra     1: centroid; 2: (a,a,a,1-3a); 3: centroid + (a,a,a,1-3a)
 *             (negative centroid weight allowed); 4-5: two (a,a,a,1-3a) +
 *             (a,a,1/2-a,1/2-a) (exact to degree 5); 6: three (a,a,a,1-3a)
 *             + (a,a,b,1-2a-b).
 * Solutions must have every point strictly inside the simplex and (except
 * the tetrahedral degree-3 structure) positive weights. When several exist,
 * the rule kept is the one whose orbit parameters, each orbit reduced to one
 * representative ((a,a,1/2-a,1/2-a): a <= 1/4; (a,b,1-a-b): sorted;
 * (a,a,b,c): b <= c) and orbits of one kind sorted, come first in
 * lexicographic order (parameters, then weight, per orbit; kinds in the
 * order listed above).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { K_CENTROID = 0, K_TRI2 = 1, K_TRI3 = 2, K_TET31 = 3, K_TET22 = 4, K_TET211 = 5 };

typedef struct {
    int dim, exact, norb, kind[4], negative_ok;
} sym_structure;

static int structure(int dim, int q, sym_structure* s) {
    memset(s, 0, sizeof *s);
    s->dim = dim;
    if (dim == 2) {
        if (q <= 1) { s->exact = 1; s->norb = 1; s->kind[0] = K_CENTROID; }
        else if (q == 2) { s->exact = 2; s->norb = 1; s->kind[0] = K_TRI2; }
        else if (q <= 4) { s->exact = 4; s->norb = 2; s->kind[0] = s->kind[1] = K_TRI2; }
        else if (q == 5) { s->exact = 5; s->norb = 3; s->kind[0] = K_CENTROID; s->kind[1] = s->kind[2] = K_TRI2; }
        else if (q == 6) { s->exact = 6; s->norb = 3; s->kind[0] = s->kind[1] = K_TRI2; s->kind[2] = K_TRI3; }
        else return 0;
        return 1;
    }
    if (q <= 1) { s->exact = 1; s->norb = 1; s->kind[0] = K_CENTROID; }
    else if (q == 2) { s->exact = 2; s->norb = 1; s->kind[0] = K_TET31; }
    else if (q == 3) { s->exact = 3; s->norb = 2; s->kind[0] = K_CENTROID; s->kind[1] = K_TET31; s->negative_ok = 1; }
    else if (q <= 5) { s->exact = 5; s->norb = 3; s->kind[0] = s->kind[1] = K_TET31; s->kind[2] = K_TET22; }
    else if (q == 6) {
        s->exact = 6; s->norb = 4;
        s->kind[0] = s->kind[1] = s->kind[2] = K_TET31; s->kind[3] = K_TET211;
    } else return 0;
    return 1;
}

static int kind_params(int k) { return k == K_CENTROID ? 0 : (k == K_TRI3 || k == K_TET211) ? 2 : 1; }

/* Base tuple of an orbit (d+1 barycentric coordinates). */
static void base_tuple(int dim, int kind, const long double* p, long double* t) {
    switch (kind) {
        case K_CENTROID: for (int i = 0; i <= dim; ++i) t[i] = 1.0L / (dim + 1); break;
        case K_TRI2: t[0] = p[0]; t[1] = p[0]; t[2] = 1 - 2 * p[0]; break;
        case K_TRI3: t[0] = p[0]; t[1] = p[1]; t[2] = 1 - p[0] - p[1]; break;
        case K_TET31: t[0] = t[1] = t[2] = p[0]; t[3] = 1 - 3 * p[0]; break;
        case K_TET22: t[0] = t[1] = p[0]; t[2] = t[3] = 0.5L - p[0]; break;
        case K_TET211: t[0] = t[1] = p[0]; t[2] = p[1]; t[3] = 1 - 2 * p[0] - p[1]; break;
    }
}

/* All distinct rearrangements of t (n = d+1 <= 4 entries), written to out;
 * returns their count. Rearrangements are enumerated as permutations of the
 * positions in lexicographic order and duplicates are dropped. */
static int rearrangements(int n, const long double* t, long double out[][4]) {
    int perm[4] = {0, 1, 2, 3}, cnt = 0;
    int total = 1;
    for (int i = 2; i <= n; ++i) total *= i;
    for (int r = 0; r < total; ++r) {
        /* r-th permutation by the factorial number system */
        int avail[4] = {0, 1, 2, 3}, na = n, x = r;
        int f = total;
        for (int i = 0; i < n; ++i) {
            f /= (n - i);
            int k = x / f;
            x %= f;
            perm[i] = avail[k];
            for (int j = k; j < na - 1; ++j) avail[j] = avail[j + 1];
            --na;
        }
        long double v[4];
        for (int i = 0; i < n; ++i) v[i] = t[perm[i]];
        int dup = 0;
        for (int c = 0; c < cnt && !dup; ++c) {
            int same = 1;
            for (int i = 0; i < n; ++i) if (out[c][i] != v[i]) same = 0;
            dup = same;
        }
        if (!dup) { for (int i = 0; i < n; ++i) out[cnt][i] = v[i]; ++cnt; }
    }
    return cnt;
}

typedef struct {
    sym_structure s;
    int nunk, neq, nexp[4096][4];
    long double rhs[4096];
} problem;

static long double fact(int n) { long double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

static void problem_init(problem* P, const sym_structure* s) {
    P->s = *s;
    P->nunk = 0;
    for (int o = 0; o < s->norb; ++o) P->nunk += kind_params(s->kind[o]) + 1;
    P->neq = 0;
    int d = s->dim, e = s->exact;
    for (int a = 0; a <= e; ++a)
        for (int b = 0; a + b <= e; ++b)
            for (int c = 0; a + b + c <= e; ++c)
                for (int g = 0; a + b + c + g <= e; ++g) {
                    if (d == 2 && g > 0) break;
                    int* x = P->nexp[P->neq];
                    x[0] = a; x[1] = b; x[2] = c; x[3] = g;
                    P->rhs[P->neq] = fact(a) * fact(b) * fact(c) * fact(g) / fact(a + b + c + g + d);
                    ++P->neq;
                }
}

/* Barycentric points (rows of 4) and weights of the unknown vector u. */
static int expand(const problem* P, const long double* u, long double pts[][4], long double* w) {
    int np = 0, k = 0, d = P->s.dim;
    for (int o = 0; o < P->s.norb; ++o) {
        int kind = P->s.kind[o], npar = kind_params(kind);
        long double t[4], rr[24][4];
        base_tuple(d, kind, u + k, t);
        int c = rearrangements(d + 1, t, rr);
        for (int i = 0; i < c; ++i) {
            memcpy(pts[np], rr[i], sizeof rr[i]);
            w[np] = u[k + npar];
            ++np;
        }
        k += npar + 1;
    }
    return np;
}

/* Relative residuals of the moment equations. */
static void residual(const problem* P, const long double* u, long double* r) {
    long double pts[64][4], w[64];
    int np = expand(P, u, pts, w), d = P->s.dim;
    for (int m = 0; m < P->neq; ++m) {
        long double acc = 0;
        for (int p = 0; p < np; ++p) {
            long double t = w[p];
            for (int i = 0; i <= d; ++i)
                for (int e = 0; e < P->nexp[m][i]; ++e) t *= pts[p][i];
            acc += t;
        }
        r[m] = acc / P->rhs[m] - 1;
    }
}

static long double sumsq(const long double* r, int n) { long double s = 0; for (int i = 0; i < n; ++i) s += r[i] * r[i]; return s; }

/* Gauss-Newton with backtracking; step h for the forward differences.
 * Returns the final sum of squared residuals. */
static long double gauss_newton(const problem* P, long double* u, long double h, int iters, int give_up) {
    int n = P->nunk, m = P->neq;
    long double* r = malloc(sizeof(long double) * m);
    long double* r2 = malloc(sizeof(long double) * m);
    long double* J = malloc(sizeof(long double) * m * n);
    residual(P, u, r);
    long double f = sumsq(r, m);
    for (int it = 0; it < iters && f > 1e-34L; ++it) {
        if (give_up && it == 15 && f > 1e-6L) break;  /* not converging: abandon this start */
        for (int j = 0; j < n; ++j) {
            long double uj = u[j];
            u[j] = uj + h;
            residual(P, u, r2);
            u[j] = uj;
            for (int i = 0; i < m; ++i) J[i * n + j] = (r2[i] - r[i]) / h;
        }
        /* normal equations N du = -J^T r, solved by Gauss-Jordan */
        long double N[12][13];
        for (int a = 0; a < n; ++a) {
            for (int b = 0; b < n; ++b) {
                long double s = 0;
                for (int i = 0; i < m; ++i) s += J[i * n + a] * J[i * n + b];
                N[a][b] = s + (a == b ? 1e-24L : 0);
            }
            long double s = 0;
            for (int i = 0; i < m; ++i) s += J[i * n + a] * r[i];
            N[a][n] = -s;
        }
        int singular = 0;
        for (int c = 0; c < n && !singular; ++c) {
            int pr = c;
            for (int i = c + 1; i < n; ++i) if (fabsl(N[i][c]) > fabsl(N[pr][c])) pr = i;
            if (fabsl(N[pr][c]) == 0) { singular = 1; break; }
            for (int k = 0; k <= n; ++k) { long double t = N[c][k]; N[c][k] = N[pr][k]; N[pr][k] = t; }
            for (int i = 0; i < n; ++i) {
                if (i == c) continue;
                long double fct = N[i][c] / N[c][c];
                for (int k = c; k <= n; ++k) N[i][k] -= fct * N[c][k];
            }
        }
        if (singular) break;
        long double step = 1, un[12];
        int moved = 0;
        for (int ls = 0; ls < 30; ++ls, step *= 0.5L) {
            for (int j = 0; j < n; ++j) un[j] = u[j] + step * N[j][n] / N[j][j];
            residual(P, un, r2);
            long double fn = sumsq(r2, m);
            if (isfinite((double)fn) && fn < f) {
                memcpy(u, un, sizeof(long double) * n);
                memcpy(r, r2, sizeof(long double) * m);
                f = fn;
                moved = 1;
                break;
            }
        }
        if (!moved) break;
    }
    free(r); free(r2); free(J);
    return f;
}

static int inside(const problem* P, const long double* u) {
    long double pts[64][4], w[64];
    int np = expand(P, u, pts, w);
    for (int p = 0; p < np; ++p) {
        for (int i = 0; i <= P->s.dim; ++i) if (!(pts[p][i] > 1e-12L)) return 0;
        if (!P->s.negative_ok && !(w[p] > 0)) return 0;
    }
    return 1;
}

/* Canonical parameter vector (see the header comment) into c; returns length. */
static int canonical(const problem* P, const long double* u, long double* c) {
    long double orb[4][3];
    int kinds[4], len[4], k = 0;
    for (int o = 0; o < P->s.norb; ++o) {
        int kind = P->s.kind[o], np = kind_params(kind);
        for (int j = 0; j <= np; ++j) orb[o][j] = u[k + j];
        if (kind == K_TET22 && orb[o][0] > 0.25L) orb[o][0] = 0.5L - orb[o][0];
        if (kind == K_TRI3) {
            long double t[3] = {orb[o][0], orb[o][1], 1 - orb[o][0] - orb[o][1]};
            for (int i = 0; i < 3; ++i)
                for (int j = i + 1; j < 3; ++j) if (t[j] < t[i]) { long double x = t[i]; t[i] = t[j]; t[j] = x; }
            orb[o][0] = t[0]; orb[o][1] = t[1];
        }
        if (kind == K_TET211) {
            long double cc = 1 - 2 * orb[o][0] - orb[o][1];
            if (cc < orb[o][1]) orb[o][1] = cc;
        }
        kinds[o] = kind;
        len[o] = np + 1;
        k += np + 1;
    }
    /* order orbits by kind, then by parameters (insertion sort) */
    int idx[4] = {0, 1, 2, 3};
    for (int i = 1; i < P->s.norb; ++i)
        for (int j = i; j > 0; --j) {
            int a = idx[j - 1], b = idx[j], swap = 0;
            if (kinds[b] < kinds[a]) swap = 1;
            else if (kinds[b] == kinds[a]) {
                for (int t = 0; t < len[a]; ++t) {
                    if (orb[b][t] < orb[a][t]) { swap = 1; break; }
                    if (orb[b][t] > orb[a][t]) break;
                }
            }
            if (!swap) break;
            idx[j - 1] = b; idx[j] = a;
        }
    int n = 0;
    for (int i = 0; i < P->s.norb; ++i)
        for (int t = 0; t < len[idx[i]]; ++t) c[n++] = orb[idx[i]][t];
    return n;
}

/* -1, 0, 1: lexicographic comparison with a tolerance for equal entries. */
static int lexcmp(const long double* a, const long double* b, int n) {
    for (int i = 0; i < n; ++i) {
        if (fabsl(a[i] - b[i]) < 1e-9L) continue;
        return a[i] < b[i] ? -1 : 1;
    }
    return 0;
}

/* Rules already solved, per (dim, q). */
static struct { int done, np; double X[64 * 3], W[64]; } cache[2][7];

static int solve_rule(int dim, int q, int* nq, double* X, double* W);

int oracle_symmetric_rule(int dim, int q, int* nq, double* X, double* W) {
    if ((dim != 2 && dim != 3) || q < 0 || q > 6 || !nq) return OR_E_INVALID_ARG;
    int qq = q < 1 ? 1 : q;
    if (!cache[dim - 2][qq].done) {
        int st = solve_rule(dim, qq, &cache[dim - 2][qq].np, cache[dim - 2][qq].X, cache[dim - 2][qq].W);
        if (st) return st;
        cache[dim - 2][qq].done = 1;
    }
    *nq = cache[dim - 2][qq].np;
    if (X) memcpy(X, cache[dim - 2][qq].X, sizeof(double) * dim * *nq);
    if (W) memcpy(W, cache[dim - 2][qq].W, sizeof(double) * *nq);
    return OR_OK;
}

static int solve_rule(int dim, int q, int* nq, double* X, double* W) {
    sym_structure s;
    if (!structure(dim, q, &s)) return OR_E_INVALID_ARG;
    problem* P = malloc(sizeof(problem));
    if (!P) return OR_E_NOMEM;
    problem_init(P, &s);
    /* number of points and parameters */
    int npar = 0, npts;
    {
        long double u[12], pts[64][4], w[64];
        for (int i = 0; i < 12; ++i) u[i] = 0.1L + 0.01L * i;
        npts = expand(P, u, pts, w);
    }
    for (int o = 0; o < s.norb; ++o) npar += kind_params(s.kind[o]);
    const long double vol = dim == 2 ? 0.5L : 1.0L / 6;
    /* starting grid: G values per parameter, spread over its range */
    const int G = npar <= 2 ? 9 : (npar <= 4 ? 5 : 4);
    long total = 1;
    for (int i = 0; i < npar; ++i) total *= G;
    int have = 0;
    long double best[12], bestc[12];
    int nc = 0;
    for (long g = 0; g < total; ++g) {
        long double u[12];
        long gg = g;
        int k = 0, ordered = 1;
        long double prev_f0 = -1;
        for (int o = 0; o < s.norb; ++o) {
            int kind = s.kind[o];
            long double f0 = 0, f1 = 0;
            if (kind_params(kind) >= 1) { f0 = (gg % G + 0.5L) / G; gg /= G; }
            if (kind_params(kind) >= 2) { f1 = (gg % G + 0.5L) / G; gg /= G; }
            /* orbits of one kind are interchangeable: start them in increasing order */
            if (o > 0 && s.kind[o - 1] == kind && f0 < prev_f0) ordered = 0;
            prev_f0 = f0;
            switch (kind) {
                case K_TRI2: u[k++] = 0.5L * f0; break;
                case K_TRI3: u[k++] = 0.5L * f0; u[k++] = (1 - 0.5L * f0) * f1 * 0.5L; break;
                case K_TET31: u[k++] = f0 / 3; break;
                case K_TET22: u[k++] = 0.25L * f0; break;
                case K_TET211: u[k++] = 0.5L * f0; u[k++] = (1 - f0) * f1; break;
                default: break;
            }
            u[k++] = vol / npts;
        }
        if (!ordered) continue;
        if (gauss_newton(P, u, 1e-7L, 60, 1) > 1e-20L) continue;
        if (!inside(P, u)) continue;
        long double c[12];
        nc = canonical(P, u, c);
        if (!have || lexcmp(c, bestc, nc) < 0) {
            memcpy(best, u, sizeof best);
            memcpy(bestc, c, sizeof bestc);
            have = 1;
        }
    }
    if (!have) { free(P); return OR_E_UNSUPPORTED; }
    gauss_newton(P, best, 1e-10L, 40, 0);  /* refine */
    long double pts[64][4], w[64];
    int np = expand(P, best, pts, w);
    *nq = np;
    for (int p = 0; p < np; ++p) {
        if (X) for (int i = 0; i < dim; ++i) X[p * dim + i] = (double)pts[p][i + 1];
        if (W) W[p] = (double)w[p];
    }
    free(P);
    return OR_OK;
}
