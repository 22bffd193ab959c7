// Compiled instances of the linear-form engine: Burgers Jacobian on triangles
// (P1-P3) and tetrahedra (P1-P2), state field in the trial space (FD = P).
#include "registry.h"

namespace coffee {

void register_burgers(std::vector<LinEntry>& v) {
    using namespace dev;
    add_all_prec<F_BURG, 2, 1, 1>(v);
    add_all_prec<F_BURG, 2, 2, 2>(v);
    add_all_prec<F_BURG, 2, 3, 3>(v);
    add_all_prec<F_BURG, 3, 1, 1>(v);
    add_all_prec<F_BURG, 3, 2, 2>(v);
}

}  // namespace coffee
