// St Venant-Kirchhoff hyperelasticity: energy, residual and Jacobian.
#include "library.h"

namespace coffee {

coffee_status assemble_svk(int, int, int, int, int, const double*, int64_t, const int32_t*, int64_t,
                           const coffee_field*, const double*, int, void*, void*) {
    return COFFEE_E_UNSUPPORTED;
}

}  // namespace coffee

extern "C" coffee_status coffee_assemble_adjoint(int form, int cell, int degree, int quad_degree,
                                                 const double* coords, int64_t nvert, const int32_t* c2v,
                                                 int64_t ncells, const coffee_field* coeffs, int ncoeff,
                                                 const double* constants, int nconst, const double* lam,
                                                 const double* u, double seed, double* grad_coords,
                                                 double* const* grad_coeff_values, double* cell_value,
                                                 int deterministic, void* workspace, int64_t workspace_bytes,
                                                 void* hip_stream) {
    using namespace coffee;
    int q = 0, fd = 0;
    coffee_status st = validate_common(form, cell, degree, quad_degree, coords, nvert, c2v, ncells, coeffs, ncoeff,
                                       constants, nconst, &q, &fd);
    if (st != COFFEE_OK) return st;
    if (deterministic != 0 && deterministic != 1) return COFFEE_E_INVALID_ARG;
    if (deterministic) return COFFEE_E_UNSUPPORTED;
    (void)workspace;
    (void)workspace_bytes;
    if (form >= COFFEE_SVK_ENERGY) return COFFEE_E_UNSUPPORTED;
    return adjoint_linear(form, cell, degree, q, fd, coords, nvert, c2v, ncells, coeffs, ncoeff, constants, nconst,
                          lam, u, seed, grad_coords, grad_coeff_values, cell_value, hip_stream);
}

extern "C" int64_t coffee_adjoint_workspace_size(int, int, int, int64_t, int64_t, const coffee_field*, int) {
    return 0;
}
