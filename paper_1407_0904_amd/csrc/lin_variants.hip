// Compiled tile-shape variants 1 and 2 of the symmetric engine (scalar.hpp)
// for the keys the autotuner searches: Helmholtz and mass on P2 tetrahedra
// with a P1 or P2 field, Helmholtz on P3 and P4 triangles with a P1 field;
// FP64, FP32 and BF16X3. Every other key runs variant 0 (at two waves per
// SIMD the P3 tetrahedron's tiles spill registers).
#include "registry.h"

namespace coffee {

void register_variants(std::vector<LinEntry>& v) {
    using namespace dev;
    add_variants<F_HELM, 3, 2, 2>(v);
    add_variants<F_HELM, 3, 2, 1>(v);
    add_variants<F_MASS, 3, 2, 2>(v);
    add_variants<F_MASS, 3, 2, 1>(v);
    add_variants<F_HELM, 2, 3, 1>(v);
    add_variants<F_HELM, 2, 4, 1>(v);
}

}  // namespace coffee
