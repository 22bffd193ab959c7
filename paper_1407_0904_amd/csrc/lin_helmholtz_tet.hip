// Compiled instances of the linear-form engine: helmholtz, tet, P1-P4,
// coefficient field absent (FD = 0), P1 or P2; FP64, FP32 and BF16X3.
#include "registry.h"

namespace coffee {

void register_helmholtz_tet(std::vector<LinEntry>& v) {
    using namespace dev;
    add_all_prec<F_HELM, 3, 1, 0>(v);
    add_all_prec<F_HELM, 3, 1, 1>(v);
    add_all_prec<F_HELM, 3, 1, 2>(v);
    add_all_prec<F_HELM, 3, 2, 0>(v);
    add_all_prec<F_HELM, 3, 2, 1>(v);
    add_all_prec<F_HELM, 3, 2, 2>(v);
    add_all_prec<F_HELM, 3, 3, 0>(v);
    add_all_prec<F_HELM, 3, 3, 1>(v);
    add_all_prec<F_HELM, 3, 3, 2>(v);
    add_all_prec<F_HELM, 3, 4, 0>(v);
    add_all_prec<F_HELM, 3, 4, 1>(v);
    add_all_prec<F_HELM, 3, 4, 2>(v);
}

}  // namespace coffee
