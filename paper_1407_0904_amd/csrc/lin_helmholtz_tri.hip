// Compiled instances of the linear-form engine: helmholtz, tri, P1-P4,
// coefficient field absent (FD = 0), P1 or P2; FP64, FP32 and BF16X3.
#include "registry.h"

namespace coffee {

void register_helmholtz_tri(std::vector<LinEntry>& v) {
    using namespace dev;
    add_all_prec<F_HELM, 2, 1, 0>(v);
    add_all_prec<F_HELM, 2, 1, 1>(v);
    add_all_prec<F_HELM, 2, 1, 2>(v);
    add_all_prec<F_HELM, 2, 2, 0>(v);
    add_all_prec<F_HELM, 2, 2, 1>(v);
    add_all_prec<F_HELM, 2, 2, 2>(v);
    add_all_prec<F_HELM, 2, 3, 0>(v);
    add_all_prec<F_HELM, 2, 3, 1>(v);
    add_all_prec<F_HELM, 2, 3, 2>(v);
    add_all_prec<F_HELM, 2, 4, 0>(v);
    add_all_prec<F_HELM, 2, 4, 1>(v);
    add_all_prec<F_HELM, 2, 4, 2>(v);
}

}  // namespace coffee
