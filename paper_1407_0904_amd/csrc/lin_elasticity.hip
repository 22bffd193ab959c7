// Compiled instances of the linear-form engine: elasticity on triangles and
// tetrahedra, P1-P3, Lame parameters as constants (FD = 0) or P1 fields.
#include "registry.h"

namespace coffee {

void register_elasticity(std::vector<LinEntry>& v) {
    using namespace dev;
    add_all_prec<F_ELAST, 2, 1, 0>(v);
    add_all_prec<F_ELAST, 2, 1, 1>(v);
    add_all_prec<F_ELAST, 2, 2, 0>(v);
    add_all_prec<F_ELAST, 2, 2, 1>(v);
    add_all_prec<F_ELAST, 2, 3, 0>(v);
    add_all_prec<F_ELAST, 2, 3, 1>(v);
    add_all_prec<F_ELAST, 3, 1, 0>(v);
    add_all_prec<F_ELAST, 3, 1, 1>(v);
    add_all_prec<F_ELAST, 3, 2, 0>(v);
    add_all_prec<F_ELAST, 3, 2, 1>(v);
    add_all_prec<F_ELAST, 3, 3, 0>(v);
    add_all_prec<F_ELAST, 3, 3, 1>(v);
}

}  // namespace coffee
