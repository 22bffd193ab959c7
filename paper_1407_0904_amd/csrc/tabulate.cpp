// Host tabulation of reference quadrature rules and Lagrange bases.
//
// The paper's kernels carry these as constant tables (section 2; Listings 1-2:
// W, X_D10, X_D01, Y; Table 1). Here they are
// computed once per key on the host, in extended precision:
//   - Gauss-Jacobi rules by the Golub-Welsch method: eigen-decomposition of the
//     symmetric tridiagonal Jacobi matrix by implicit QL iteration, tracking the
//     first eigenvector components for the weights;
//   - the collapsed (Stroud conical product) rule on the simplex;
//   - the nodal Lagrange basis by inverting the monomial Vandermonde matrix at
//     the lattice nodes (LU with partial pivoting).
#include "tables.h"

#include <cmath>
#include <cstring>

namespace coffee {

using ld = long double;

static bool tridiag_ql(int n, ld* d, ld* e, ld* z) {
    // d: diagonal, e[i]: coupling of i and i+1 (e[n-1] = 0), z: first row of
    // the eigenvector matrix (starts as e_0).
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        int m;
        do {
            for (m = l; m < n - 1; ++m) {
                ld dd = fabsl(d[m]) + fabsl(d[m + 1]);
                if (fabsl(e[m]) <= 1e-19L * dd) break;
            }
            if (m != l) {
                if (iter++ == 100) return false;
                ld g = (d[l + 1] - d[l]) / (2.0L * e[l]);
                ld r = hypotl(g, 1.0L);
                g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
                ld s = 1.0L, c = 1.0L, p = 0.0L;
                int i;
                bool early = false;
                for (i = m - 1; i >= l; --i) {
                    ld f = s * e[i], b = c * e[i];
                    r = hypotl(f, g);
                    e[i + 1] = r;
                    if (r == 0.0L) {
                        d[i + 1] -= p;
                        e[m] = 0.0L;
                        early = true;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0L * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                    ld zf = z[i + 1];
                    z[i + 1] = s * z[i] + c * zf;
                    z[i] = c * z[i] - s * zf;
                }
                if (early) continue;
                d[l] -= p;
                e[l] = g;
                e[m] = 0.0L;
            }
        } while (m != l);
    }
    return true;
}

// m-point Gauss-Jacobi rule on [0,1] for the weight (1-x)^alpha.
bool gauss_jacobi01(int m, int alpha, ld* x, ld* w) {
    if (m < 1 || m > 16) return false;
    const ld a = alpha, b = 0.0L;
    ld d[16], e[16], z[16];
    for (int k = 0; k < m; ++k) {
        ld s = 2.0L * k + a + b;
        if (k == 0) d[k] = (b - a) / (a + b + 2.0L);
        else d[k] = (b * b - a * a) / (s * (s + 2.0L));
        if (k + 1 < m) {
            ld kk = k + 1, t = 2.0L * kk + a + b;
            ld beta = 4.0L * kk * (kk + a) * (kk + b) * (kk + a + b) / (t * t * (t + 1.0L) * (t - 1.0L));
            e[k] = sqrtl(beta);
        } else {
            e[k] = 0.0L;
        }
        z[k] = (k == 0) ? 1.0L : 0.0L;
    }
    if (!tridiag_ql(m, d, e, z)) return false;
    // mu0 = int_{-1}^{1} (1-x)^a (1+x)^b dx; on [0,1] divide by 2^(a+b+1)
    ld mu0 = powl(2.0L, a + b + 1.0L) * tgammal(a + 1.0L) * tgammal(b + 1.0L) / tgammal(a + b + 2.0L);
    // sort ascending (selection sort, m <= 16)
    int idx[16];
    for (int i = 0; i < m; ++i) idx[i] = i;
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j)
            if (d[idx[j]] < d[idx[i]]) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; }
    for (int i = 0; i < m; ++i) {
        x[i] = 0.5L * (1.0L + d[idx[i]]);
        w[i] = mu0 * z[idx[i]] * z[idx[i]] / powl(2.0L, a + b + 1.0L);
    }
    return true;
}

int n_scalar(int dim, int p) {
    if (p < 0) return 0;
    return dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
}

int rule_size(int dim, int quad) {
    const int q = quad & 15, rule = quad >> 4;
    if (rule == COFFEE_RULE_SYMMETRIC) return symmetric_rule_size(dim, q);
    if (rule != COFFEE_RULE_GAUSS_JACOBI || q > 10) return -1;
    int m = (q + 2) / 2;
    return dim == 2 ? m * m : m * m * m;
}

bool simplex_rule(int dim, int quad, ld* X, ld* W) {
    const int q = quad & 15, rule = quad >> 4;
    if (rule == COFFEE_RULE_SYMMETRIC) return symmetric_rule(dim, q, X, W);
    if (rule != COFFEE_RULE_GAUSS_JACOBI || q > 10) return false;
    int m = (q + 2) / 2;
    ld xa[16], wa[16], xb[16], wb[16], xc[16], wc[16];
    if (dim == 2) {
        if (!gauss_jacobi01(m, 1, xa, wa) || !gauss_jacobi01(m, 0, xb, wb)) return false;
        int k = 0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j, ++k) {
                X[2 * k] = xa[i];
                X[2 * k + 1] = (1.0L - xa[i]) * xb[j];
                W[k] = wa[i] * wb[j];
            }
        return true;
    }
    if (!gauss_jacobi01(m, 2, xa, wa) || !gauss_jacobi01(m, 1, xb, wb) || !gauss_jacobi01(m, 0, xc, wc))
        return false;
    int k = 0;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            for (int l = 0; l < m; ++l, ++k) {
                X[3 * k] = xa[i];
                X[3 * k + 1] = (1.0L - xa[i]) * xb[j];
                X[3 * k + 2] = (1.0L - xa[i]) * (1.0L - xb[j]) * xc[l];
                W[k] = wa[i] * wb[j] * wc[l];
            }
    return true;
}

// Reference coordinates of the degree-p Lagrange nodes, in dof order.
int lagrange_nodes(int dim, int p, ld* pts) {
    static const int tri_e[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    static const int tet_e[6][2] = {{2, 3}, {1, 3}, {1, 2}, {0, 3}, {0, 2}, {0, 1}};
    ld V[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int n = 0;
    auto put = [&](const ld* x) {
        for (int j = 0; j < dim; ++j) pts[n * dim + j] = x[j];
        ++n;
    };
    if (p == 0) {
        ld c[3] = {0, 0, 0};
        for (int v = 0; v <= dim; ++v)
            for (int j = 0; j < dim; ++j) c[j] += V[v][j] / (dim + 1);
        put(c);
        return n;
    }
    for (int v = 0; v <= dim; ++v) put(V[v]);
    int ne = dim == 2 ? 3 : 6;
    for (int e = 0; e < ne; ++e) {
        int a = dim == 2 ? tri_e[e][0] : tet_e[e][0];
        int b = dim == 2 ? tri_e[e][1] : tet_e[e][1];
        for (int k = 1; k < p; ++k) {
            ld x[3];
            for (int j = 0; j < 3; ++j) x[j] = V[a][j] + (ld)k / p * (V[b][j] - V[a][j]);
            put(x);
        }
    }
    int nf = dim == 2 ? 1 : 4;
    for (int f = 0; f < nf; ++f) {
        int vv[3], c = 0;
        for (int v = 0; v <= dim; ++v)
            if (dim == 2 || v != f) vv[c++] = v;
        for (int j = 1; j < p; ++j)
            for (int i = 1; i + j < p; ++i) {
                ld x[3];
                for (int t = 0; t < 3; ++t)
                    x[t] = V[vv[0]][t] + (ld)i / p * (V[vv[1]][t] - V[vv[0]][t]) +
                           (ld)j / p * (V[vv[2]][t] - V[vv[0]][t]);
                put(x);
            }
    }
    if (dim == 3)
        for (int k = 1; k < p; ++k)
            for (int j = 1; j + k < p; ++j)
                for (int i = 1; i + j + k < p; ++i) {
                    ld x[3] = {(ld)i / p, (ld)j / p, (ld)k / p};
                    put(x);
                }
    return n;
}

// exponents of the monomials of total degree <= p
static int monomial_list(int dim, int p, int (*e)[3]) {
    int n = 0;
    for (int i = 0; i <= p; ++i)
        for (int j = 0; i + j <= p; ++j)
            if (dim == 2) { e[n][0] = i; e[n][1] = j; e[n][2] = 0; ++n; }
            else
                for (int k = 0; i + j + k <= p; ++k) { e[n][0] = i; e[n][1] = j; e[n][2] = k; ++n; }
    return n;
}

bool Basis::init(int dim_, int p_) {
    dim = dim_;
    p = p_;
    ld nodes[kMaxN * 3];
    n = lagrange_nodes(dim, p, nodes);
    int nm = monomial_list(dim, p, exps);
    if (nm != n) return false;
    // V[b][m] = X_b^{e_m}; solve V C = I
    ld A[kMaxN][2 * kMaxN];
    for (int b = 0; b < n; ++b) {
        for (int m = 0; m < n; ++m) {
            ld v = 1.0L;
            for (int j = 0; j < dim; ++j) v *= powl(nodes[b * dim + j], exps[m][j]);
            A[b][m] = v;
        }
        for (int m = 0; m < n; ++m) A[b][n + m] = (b == m) ? 1.0L : 0.0L;
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0L) return false;
        if (piv != col)
            for (int j = 0; j < 2 * n; ++j) { ld t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
        ld pv = A[col][col];
        for (int j = 0; j < 2 * n; ++j) A[col][j] /= pv;
        for (int r = 0; r < n; ++r) {
            if (r == col || A[r][col] == 0.0L) continue;
            ld f = A[r][col];
            for (int j = 0; j < 2 * n; ++j) A[r][j] -= f * A[col][j];
        }
    }
    // inverse: coef[m][a] = (V^{-1})[m][a]
    for (int m = 0; m < n; ++m)
        for (int a = 0; a < n; ++a) coef[m][a] = A[m][n + a];
    return true;
}

void Basis::eval(const ld* X, ld* phi, ld* dphi /* [dim][n] */) const {
    ld pw[3][kMaxP + 1];
    for (int j = 0; j < dim; ++j) {
        pw[j][0] = 1.0L;
        for (int k = 1; k <= p; ++k) pw[j][k] = pw[j][k - 1] * X[j];
    }
    for (int a = 0; a < n; ++a) {
        phi[a] = 0.0L;
        for (int j = 0; j < dim; ++j) dphi[j * n + a] = 0.0L;
    }
    for (int m = 0; m < n; ++m) {
        ld mono = 1.0L;
        for (int j = 0; j < dim; ++j) mono *= pw[j][exps[m][j]];
        ld dmono[3];
        for (int j = 0; j < dim; ++j) {
            if (exps[m][j] == 0) { dmono[j] = 0.0L; continue; }
            ld t = exps[m][j];
            for (int i = 0; i < dim; ++i) t *= (i == j) ? pw[i][exps[m][i] - 1] : pw[i][exps[m][i]];
            dmono[j] = t;
        }
        for (int a = 0; a < n; ++a) {
            phi[a] += coef[m][a] * mono;
            for (int j = 0; j < dim; ++j) dphi[j * n + a] += coef[m][a] * dmono[j];
        }
    }
}

bool Tables::init(int dim_, int p_, int q_) {
    dim = dim_;
    p = p_;
    q = q_;
    if (!basis.init(dim, p)) return false;
    n = basis.n;
    nq = rule_size(dim, q);
    if (nq <= 0) return false;
    X.assign(nq * dim, 0.0L);
    W.assign(nq, 0.0L);
    if (!simplex_rule(dim, q, X.data(), W.data())) return false;
    phi.assign((size_t)nq * n, 0.0L);
    dphi.assign((size_t)dim * nq * n, 0.0L);
    ld ph[kMaxN], dph[3 * kMaxN];
    for (int k = 0; k < nq; ++k) {
        basis.eval(&X[k * dim], ph, dph);
        for (int a = 0; a < n; ++a) {
            phi[(size_t)k * n + a] = ph[a];
            for (int j = 0; j < dim; ++j) dphi[((size_t)j * nq + k) * n + a] = dph[j * n + a];
        }
    }
    return true;
}

int n_prism(int p) { return (p + 1) * (p + 2) / 2 * (p + 1); }

int prism_rule_size(int quad) {
    const int nt = rule_size(2, quad);
    return nt <= 0 ? -1 : nt * (((quad & 15) + 2) / 2);
}

// Degree-p Lagrange basis on [0,1] with nodes 0, 1, 1/p, ..., (p-1)/p, as
// monomial coefficients from the inverse Vandermonde matrix (as for Basis).
static bool interval_basis(int p, ld (*coef)[kMaxP + 1]) {
    const int n = p + 1;
    ld nodes[kMaxP + 1];
    nodes[0] = 0.0L;
    if (p >= 1) nodes[1] = 1.0L;
    for (int k = 1; k < p; ++k) nodes[k + 1] = (ld)k / p;
    ld A[kMaxP + 1][2 * (kMaxP + 1)];
    for (int b = 0; b < n; ++b) {
        ld v = 1.0L;
        for (int m = 0; m < n; ++m) { A[b][m] = v; v *= nodes[b]; }
        for (int m = 0; m < n; ++m) A[b][n + m] = (b == m) ? 1.0L : 0.0L;
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0L) return false;
        if (piv != col)
            for (int j = 0; j < 2 * n; ++j) { ld t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
        const ld pv = A[col][col];
        for (int j = 0; j < 2 * n; ++j) A[col][j] /= pv;
        for (int r = 0; r < n; ++r) {
            if (r == col || A[r][col] == 0.0L) continue;
            const ld f = A[r][col];
            for (int j = 0; j < 2 * n; ++j) A[r][j] -= f * A[col][j];
        }
    }
    for (int m = 0; m < n; ++m)
        for (int b = 0; b < n; ++b) coef[m][b] = A[m][n + b];
    return true;
}

bool PrismTables::init(int p_, int quad) {
    p = p_;
    Basis tb;
    if (p < 0 || p > kMaxP || !tb.init(2, p)) return false;
    const int nt = rule_size(2, quad);
    if (nt <= 0) return false;
    const int m = ((quad & 15) + 2) / 2;
    std::vector<ld> Xt(2 * nt), Wt(nt);
    ld z[16], wz[16];
    if (!simplex_rule(2, quad, Xt.data(), Wt.data()) || !gauss_jacobi01(m, 0, z, wz)) return false;
    ld coef[kMaxP + 1][kMaxP + 1];
    if (!interval_basis(p, coef)) return false;
    const int nt_dofs = tb.n;
    n = nt_dofs * (p + 1);
    nq = nt * m;
    X.assign(3 * nq, 0.0L);
    W.assign(nq, 0.0L);
    phi.assign((size_t)nq * n, 0.0L);
    dphi.assign((size_t)3 * nq * n, 0.0L);
    ld tph[kMaxN], tdph[2 * kMaxN];
    for (int i = 0; i < nt; ++i) {
        tb.eval(&Xt[2 * i], tph, tdph);
        for (int j = 0; j < m; ++j) {
            const int k = i * m + j;
            X[3 * k] = Xt[2 * i];
            X[3 * k + 1] = Xt[2 * i + 1];
            X[3 * k + 2] = z[j];
            W[k] = Wt[i] * wz[j];
            ld l[kMaxP + 1], dl[kMaxP + 1];
            for (int b = 0; b <= p; ++b) {
                ld v = 0.0L, dv = 0.0L, pw = 1.0L;
                for (int e = 0; e <= p; ++e) {
                    v += coef[e][b] * pw;
                    if (e + 1 <= p) dv += coef[e + 1][b] * (e + 1) * pw;
                    pw *= z[j];
                }
                l[b] = v;
                dl[b] = dv;
            }
            for (int a = 0; a < nt_dofs; ++a)
                for (int b = 0; b <= p; ++b) {
                    const int r = a * (p + 1) + b;
                    phi[(size_t)k * n + r] = tph[a] * l[b];
                    dphi[((size_t)0 * nq + k) * n + r] = tdph[a] * l[b];
                    dphi[((size_t)1 * nq + k) * n + r] = tdph[nt_dofs + a] * l[b];
                    dphi[((size_t)2 * nq + k) * n + r] = tph[a] * dl[b];
                }
        }
    }
    return true;
}

}  // namespace coffee

extern "C" coffee_status coffee_tabulate(int cell, int degree, int quad_degree, int* nq, int* ndof,
                                         double* points, double* weights, double* basis, double* dbasis) {
    if ((cell != COFFEE_TRIANGLE && cell != COFFEE_TETRAHEDRON && cell != COFFEE_PRISM) || !nq || !ndof)
        return COFFEE_E_INVALID_ARG;
    if (degree < 0 || degree > coffee::kMaxP || quad_degree < 0) return COFFEE_E_INVALID_ARG;
    if (cell == COFFEE_PRISM) {
        const int nqp = coffee::prism_rule_size(quad_degree);
        if (nqp <= 0) return COFFEE_E_INVALID_ARG;
        *nq = nqp;
        *ndof = coffee::n_prism(degree);
        if (!points && !weights && !basis && !dbasis) return COFFEE_OK;
        coffee::PrismTables t;
        if (!t.init(degree, quad_degree)) return COFFEE_E_INVALID_ARG;
        for (int k = 0; k < t.nq; ++k) {
            if (points)
                for (int j = 0; j < 3; ++j) points[k * 3 + j] = (double)t.X[k * 3 + j];
            if (weights) weights[k] = (double)t.W[k];
            if (basis)
                for (int a = 0; a < t.n; ++a) basis[(size_t)k * t.n + a] = (double)t.phi[(size_t)k * t.n + a];
        }
        if (dbasis)
            for (size_t i = 0; i < t.dphi.size(); ++i) dbasis[i] = (double)t.dphi[i];
        return COFFEE_OK;
    }
    const int dim = cell;
    if (coffee::rule_size(dim, quad_degree) <= 0) return COFFEE_E_INVALID_ARG;
    *nq = coffee::rule_size(dim, quad_degree);
    *ndof = coffee::n_scalar(dim, degree);
    if (!points && !weights && !basis && !dbasis) return COFFEE_OK;
    coffee::Tables t;
    if (!t.init(dim, degree, quad_degree)) return COFFEE_E_INVALID_ARG;
    for (int k = 0; k < t.nq; ++k) {
        if (points)
            for (int j = 0; j < dim; ++j) points[k * dim + j] = (double)t.X[k * dim + j];
        if (weights) weights[k] = (double)t.W[k];
        if (basis)
            for (int a = 0; a < t.n; ++a) basis[(size_t)k * t.n + a] = (double)t.phi[(size_t)k * t.n + a];
    }
    if (dbasis)
        for (size_t i = 0; i < t.dphi.size(); ++i) dbasis[i] = (double)t.dphi[i];
    return COFFEE_OK;
}
