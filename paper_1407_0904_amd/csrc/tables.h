// Host-side tables of libcoffee: quadrature rules, Lagrange bases and the
// reference tensors of the contraction (internal header).
#pragma once
#include <cstdint>
#include <vector>

#include "../../include/coffee.h"

namespace coffee {

constexpr int kMaxP = 4;
constexpr int kMaxN = 35;  // scalar P4 on a tetrahedron

bool gauss_jacobi01(int m, int alpha, long double* x, long double* w);
// Quadrature degree arguments below are encoded as COFFEE_QUAD(q, rule):
// q = quad & 15, rule = quad >> 4 (0 collapsed Gauss-Jacobi, 1 symmetric).
bool simplex_rule(int dim, int quad, long double* X, long double* W);
int rule_size(int dim, int quad);  // -1 if the rule does not exist
// Fully symmetric rules (symrule.cpp), q <= 6.
int symmetric_rule_size(int dim, int q);
bool symmetric_rule(int dim, int q, long double* X, long double* W);
int n_scalar(int dim, int p);
int lagrange_nodes(int dim, int p, long double* pts);

// Nodal Lagrange basis of degree p as monomial coefficients.
struct Basis {
    int dim = 0, p = 0, n = 0;
    int exps[kMaxN][3];
    long double coef[kMaxN][kMaxN];  // phi_a = sum_m coef[m][a] X^{exps[m]}
    bool init(int dim, int p);
    void eval(const long double* X, long double* phi, long double* dphi) const;
};

// A quadrature rule and one basis tabulated on it.
struct Tables {
    int dim = 0, p = 0, q = 0, n = 0, nq = 0;
    Basis basis;
    std::vector<long double> X, W, phi, dphi;  // [nq][dim], [nq], [nq][n], [dim][nq][n]
    bool init(int dim, int p, int q);
};

// A rule and a basis on the reference prism T x [0,1] (T the reference
// triangle): the triangle rule of `quad` times Gauss-Legendre with
// m = ceil((q + 1) / 2) points on [0,1], triangle point outermost; the degree-p
// tensor-product Lagrange basis, local dof a (p + 1) + b for triangle dof a and
// interval dof b (interval nodes 0, 1, then interior ascending).
struct PrismTables {
    int p = 0, n = 0, nq = 0;
    std::vector<long double> X, W, phi, dphi;  // [nq][3], [nq], [nq][n], [3][nq][n]
    bool init(int p, int quad);
};
int prism_rule_size(int quad);  // -1 if the rule does not exist
int n_prism(int p);

// Reference tensors of a linear form: the element tensor of every affine cell
// is A[blk][ab] = sum_k G[blk][k](cell) R[k][ab], exactly (up to rounding) the
// quadrature sum, because the geometry and the coefficient fields are
// polynomial in the reference coordinates.
struct RefTensor {
    int KR = 0;                  // number of reference tensors
    int NS = 0;                  // scalar dofs
    std::vector<long double> R;  // [KR][NS*NS]
};

// fdeg: degree of the coefficient field (0 = no field / constants).
bool build_reference(int form, int dim, int p, int q, int fdeg, RefTensor& out);

}  // namespace coffee
