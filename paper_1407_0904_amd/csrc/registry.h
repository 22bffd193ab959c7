// Kernel registry of libcoffee (internal header): every compiled (form, cell,
// degree, field degree, precision) instance of the device engines.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "elast.hpp"
#include "linear.hpp"
#include "scalar.hpp"
#include "vector.hpp"

namespace coffee {

typedef hipError_t (*LinLaunch)(const dev::LinArgs&, hipStream_t, int grid);

struct LinEntry {
    int form, dim, p, fd, prec;
    int variant;          // tile-shape variant of the engine (scalar.hpp)
    LinLaunch launch;
    const void* kernel;
    int threads;          // workgroup size
    int lds_bytes;        // dynamic LDS per workgroup
    int cells_per_chunk;  // LinArgs::nchunks = ceil(ncells / cells_per_chunk)
};

// Mass, Helmholtz and diffusion are symmetric single-block forms and use the symmetric
// engine (scalar.hpp); elasticity uses the cell-row engine (elast.hpp) where its
// ring of cell slots fits the LDS, the panel engine (vector.hpp) otherwise, and
// Burgers the panel engine.
constexpr bool uses_scalar_engine(int form) {
    return form == dev::F_MASS || form == dev::F_HELM || form == dev::F_DIFF;
}
constexpr bool uses_elast_engine(int form, int d, int p, int fd, int prec) {
    return form == dev::F_ELAST && dev::el_sizes(d, p, fd, prec).fits;
}

template <int FORM, int D, int P, int FD, int PREC, int VAR = 0>
const void* kernel_of() {
    if constexpr (uses_scalar_engine(FORM))
        return reinterpret_cast<const void*>(&dev::k_scalar<FORM, D, P, FD, PREC, VAR>);
    else if constexpr (uses_elast_engine(FORM, D, P, FD, PREC))
        return reinterpret_cast<const void*>(&dev::k_elast<D, P, FD, PREC>);
    else
        return reinterpret_cast<const void*>(&dev::k_vector<FORM, D, P, FD, PREC>);
}

// The vector engine takes its LDS dynamically (it can exceed the 64 KiB of
// static allocations); the attribute is set once per kernel.
template <int FORM, int D, int P, int FD, int PREC, int VAR = 0>
hipError_t launch_linear(const dev::LinArgs& a, hipStream_t s, int grid) {
    if constexpr (uses_scalar_engine(FORM)) {
        hipLaunchKernelGGL((dev::k_scalar<FORM, D, P, FD, PREC, VAR>), dim3(grid), dim3(256), 0, s, a);
    } else if constexpr (uses_elast_engine(FORM, D, P, FD, PREC)) {
        using C = dev::ElCfg<D, P, FD, PREC>;
        static const hipError_t attr = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&dev::k_elast<D, P, FD, PREC>),
            hipFuncAttributeMaxDynamicSharedMemorySize, C::S.lds_bytes);
        if (attr != hipSuccess) return attr;
        hipLaunchKernelGGL((dev::k_elast<D, P, FD, PREC>), dim3(grid), dim3(C::WAVES * 64), C::S.lds_bytes, s, a);
    } else {
        using C = dev::VecCfg<FORM, D, P, FD, PREC>;
        static const hipError_t attr = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&dev::k_vector<FORM, D, P, FD, PREC>),
            hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_BYTES);
        if (attr != hipSuccess) return attr;
        hipLaunchKernelGGL((dev::k_vector<FORM, D, P, FD, PREC>), dim3(grid), dim3(C::WAVES * 64), C::LDS_BYTES, s,
                           a);
    }
    return hipGetLastError();
}

template <int FORM, int D, int P, int FD, int PREC, int VAR = 0>
LinEntry lin_entry() {
    if constexpr (uses_scalar_engine(FORM)) {
        return LinEntry{FORM, D, P, FD, PREC, VAR, &launch_linear<FORM, D, P, FD, PREC, VAR>,
                        kernel_of<FORM, D, P, FD, PREC, VAR>(), 256, 0, 256};
    } else if constexpr (uses_elast_engine(FORM, D, P, FD, PREC)) {
        using C = dev::ElCfg<D, P, FD, PREC>;
        return LinEntry{FORM, D, P, FD, PREC, 0, &launch_linear<FORM, D, P, FD, PREC>, kernel_of<FORM, D, P, FD, PREC>(),
                        C::WAVES * 64, C::S.lds_bytes, C::WAVES * 16};
    } else {
        using C = dev::VecCfg<FORM, D, P, FD, PREC>;
        return LinEntry{FORM, D, P, FD, PREC, 0, &launch_linear<FORM, D, P, FD, PREC>, kernel_of<FORM, D, P, FD, PREC>(),
                        C::WAVES * 64, C::LDS_BYTES, C::WAVES * 16};
    }
}

// one instance for each precision
template <int FORM, int D, int P, int FD>
void add_all_prec(std::vector<LinEntry>& v) {
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_F64>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_F32>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_BF16X3>());
}

// the symmetric engine's other tile-shape variants (1, 2, 3) for each precision
template <int FORM, int D, int P, int FD>
void add_variants(std::vector<LinEntry>& v) {
    static_assert(uses_scalar_engine(FORM), "tile-shape variants of the symmetric engine");
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_F64, 1>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_F32, 1>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_BF16X3, 1>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_F64, 2>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_F32, 2>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_BF16X3, 2>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_F64, 3>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_F32, 3>());
    v.push_back(lin_entry<FORM, D, P, FD, dev::PREC_BF16X3, 3>());
}

void register_mass_tri(std::vector<LinEntry>& v);
void register_mass_tet(std::vector<LinEntry>& v);
void register_helmholtz_tri(std::vector<LinEntry>& v);
void register_helmholtz_tet(std::vector<LinEntry>& v);
void register_elasticity(std::vector<LinEntry>& v);
void register_burgers(std::vector<LinEntry>& v);
void register_diffusion(std::vector<LinEntry>& v);
void register_variants(std::vector<LinEntry>& v);

}  // namespace coffee
