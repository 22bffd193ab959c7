// Reference tensors of the linear forms.
//
// On an affine cell the Jacobian is constant, so every integrand of a linear
// form is a sum of (cell-dependent factor) x (product of reference basis
// functions and reference derivatives). Moving the cell factors out of the
// quadrature sum (the paper's generalized loop-invariant code motion, section
// 3.2, taken to the whole i loop, and the expansion used by FFC, section 5.8)
// turns the element tensor into A[ab] = sum_k G[k] R[k][ab] with
// R[k][ab] = sum_q W_q (reference products at point q). The sum runs over
// the same quadrature points, so the result equals the quadrature sum up to
// rounding; the contraction is the outer-product form of the paper's
// equation (section 3.3), with G as the left factor.
//
// Tensor order per form (the device builds G in the same order):
//   MASS        [r]                       r over field dofs (one tensor if no field)
//   HELMHOLTZ   [(a,b) a<=b] + mass part  stiffness pairs, symmetric sum for a<b
//   DIFFUSION   [(a,b) a<=b]              the Helmholtz stiffness pairs alone
//   ELASTICITY  [(r, a, b)]               r over Lame dofs (one if constants)
//   BURGERS     [M] [(a,b) a<=b] [C(r,a)] [E(r,a)]
//       M = W phi_a phi_b, C(r,a) = W psi_r phi_a d_a phi_b, E(r,a) = W d_a psi_r phi_a phi_b
#include <cmath>

#include "tables.h"

namespace coffee {

using ld = long double;

static int sym_pairs(int dim, int (*pr)[2]) {
    int k = 0;
    for (int a = 0; a < dim; ++a)
        for (int b = a; b < dim; ++b) { pr[k][0] = a; pr[k][1] = b; ++k; }
    return k;
}

bool build_reference(int form, int dim, int p, int q, int fdeg, RefTensor& out) {
    Tables sp;
    if (!sp.init(dim, p, q)) return false;
    Tables fl;
    const bool has_field = fdeg > 0;
    if (has_field && !fl.init(dim, fdeg, q)) return false;
    const int n = sp.n, nq = sp.nq, NN = n * n;
    const int nf = has_field ? fl.n : 1;
    auto psi = [&](int k, int r) -> ld { return has_field ? fl.phi[(size_t)k * nf + r] : 1.0L; };
    auto dpsi = [&](int a, int k, int r) -> ld { return has_field ? fl.dphi[((size_t)a * nq + k) * nf + r] : 0.0L; };
    auto phi = [&](int k, int a) -> ld { return sp.phi[(size_t)k * n + a]; };
    auto dphi = [&](int al, int k, int a) -> ld { return sp.dphi[((size_t)al * nq + k) * n + a]; };
    int pr[6][2];
    const int npair = sym_pairs(dim, pr);

    out.NS = n;
    int KR = 0;
    switch (form) {
        case COFFEE_MASS: KR = nf; break;
        case COFFEE_HELMHOLTZ: KR = npair + nf; break;
        case COFFEE_DIFFUSION: KR = npair; break;
        case COFFEE_ELASTICITY: KR = nf * dim * dim; break;
        case COFFEE_BURGERS: KR = 1 + npair + 2 * nf * dim; break;
        default: return false;
    }
    out.KR = KR;
    out.R.assign((size_t)KR * NN, 0.0L);
    auto R = [&](int k, int a, int b) -> ld& { return out.R[(size_t)k * NN + a * n + b]; };

    for (int k = 0; k < nq; ++k) {
        const ld w = sp.W[k];
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                const ld pp = phi(k, a) * phi(k, b);
                int t = 0;
                if (form == COFFEE_HELMHOLTZ || form == COFFEE_BURGERS || form == COFFEE_DIFFUSION) {
                    if (form == COFFEE_BURGERS) R(t++, a, b) += w * pp;
                    for (int s = 0; s < npair; ++s) {
                        int al = pr[s][0], be = pr[s][1];
                        ld v = dphi(al, k, a) * dphi(be, k, b);
                        if (al != be) v += dphi(be, k, a) * dphi(al, k, b);
                        R(t++, a, b) += w * v;
                    }
                }
                if (form == COFFEE_MASS || form == COFFEE_HELMHOLTZ) {
                    for (int r = 0; r < nf; ++r) R(t++, a, b) += w * psi(k, r) * pp;
                } else if (form == COFFEE_ELASTICITY) {
                    for (int r = 0; r < nf; ++r)
                        for (int al = 0; al < dim; ++al)
                            for (int be = 0; be < dim; ++be)
                                R(t++, a, b) += w * psi(k, r) * dphi(al, k, a) * dphi(be, k, b);
                } else if (form == COFFEE_BURGERS) {
                    for (int r = 0; r < nf; ++r)
                        for (int al = 0; al < dim; ++al) R(t++, a, b) += w * psi(k, r) * phi(k, a) * dphi(al, k, b);
                    for (int r = 0; r < nf; ++r)
                        for (int al = 0; al < dim; ++al) R(t++, a, b) += w * dpsi(al, k, r) * pp;
                }
            }
    }
    return true;
}

}  // namespace coffee
