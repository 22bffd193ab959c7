// St Venant-Kirchhoff hyperelasticity: energy, residual and Jacobian.
#include "library.h"

namespace coffee {

coffee_status assemble_svk(int, int, int, int, int, const double*, int64_t, const int32_t*, int64_t,
                           const coffee_field*, const double*, int, void*, void*) {
    return COFFEE_E_UNSUPPORTED;
}

}  // namespace coffee

extern "C" coffee_status coffee_assemble_adjoint(int, int, int, int, const double*, int64_t, const int32_t*,
                                                 int64_t, const coffee_field*, int, const double*, int,
                                                 const double*, const double*, double, double*,
                                                 double* const*, double*, int, void*, int64_t, void*) {
    return COFFEE_E_UNSUPPORTED;
}

extern "C" int64_t coffee_adjoint_workspace_size(int, int, int, int64_t, int64_t, const coffee_field*, int) {
    return 0;
}
