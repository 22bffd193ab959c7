// Instances of the symmetric engine for the diffusion form (no field).
#include "registry.h"

namespace coffee {

void register_diffusion(std::vector<LinEntry>& v) {
    using namespace dev;
    add_all_prec<F_DIFF, 2, 1, 0>(v);
    add_all_prec<F_DIFF, 2, 2, 0>(v);
    add_all_prec<F_DIFF, 2, 3, 0>(v);
    add_all_prec<F_DIFF, 2, 4, 0>(v);
    add_all_prec<F_DIFF, 3, 1, 0>(v);
    add_all_prec<F_DIFF, 3, 2, 0>(v);
    add_all_prec<F_DIFF, 3, 3, 0>(v);
    add_all_prec<F_DIFF, 3, 4, 0>(v);
}

}  // namespace coffee
