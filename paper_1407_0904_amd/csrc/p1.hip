// Degree-1 mass, Helmholtz and diffusion: one thread per cell, FMA arithmetic (the
// per-cell arithmetic is in p1.hpp). Each lane gathers its cell, forms J,
// |det J|, K = J^-1 and the G row in FP64 registers and writes its tensor to
// an LDS row; the wave's 64 tensors then leave as stores whose 64 lanes cover
// consecutive elements of the wave's contiguous output range.
#include <hip/hip_runtime.h>

#include <cstring>

#include "library.h"
#include "p1.hpp"

namespace coffee {
namespace dev {

template <int FORM, int D, int FD, typename OT>
__global__ __launch_bounds__(256) void k_p1(LinArgs A, const double* __restrict__ R) {
    constexpr int NN = (D + 1) * (D + 1), KR = kref(FORM, D, FD);
    constexpr int SR = p1_row<D>();
    __shared__ OT stage[4][64 * SR];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    OT* st = stage[wave];
    OT* out = reinterpret_cast<OT*>(A.out);
    const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64;
    if (base >= A.ncells) return;  // wave-uniform; no workgroup barrier follows
    const int64_t last = A.ncells - 1;
    const int64_t cell = base + lane <= last ? base + lane : last;
    CellData<FORM, D, FD> cd;
    load_cell<FORM, D, FD>(A, cell, cd);
    double G[KR];
    build_G<FORM, D, FD, 0, 0>(cd, A, G);
    p1_tensor<FORM, D, FD, OT>(G, R, st + lane * SR);
    wave_sync();
    const int n = A.ncells - base < 64 ? (int)(A.ncells - base) : 64;
    OT* dst = out + base * NN;
#pragma unroll
    for (int i0 = 0; i0 < 64 * NN; i0 += 64) {
        const int i = i0 + lane;
        const int c = i / NN, e = i - (i / NN) * NN;
        if (c < n) dst[i] = st[c * SR + e];
    }
}

}  // namespace dev

template <int FORM, int D, int FD>
static hipError_t launch_p1(const dev::LinArgs& a, const double* R, int prec, hipStream_t s) {
    const int64_t waves = (a.ncells + 63) / 64;
    const int grid = (int)((waves + 3) / 4);
    if (prec == COFFEE_FP64)
        hipLaunchKernelGGL((dev::k_p1<FORM, D, FD, double>), dim3(grid), dim3(256), 0, s, a, R);
    else
        hipLaunchKernelGGL((dev::k_p1<FORM, D, FD, float>), dim3(grid), dim3(256), 0, s, a, R);
    return hipGetLastError();
}

// Mass, Helmholtz or diffusion at degree 1 with no field or a P1 field, FP64 or FP32
// (BF16X3 and every other case take the MFMA engines).
coffee_status assemble_p1(int form, int cell, int fd, int q, int precision, const double* coords, const int32_t* c2v,
                          int64_t ncells, const coffee_field* coeffs, int ncoeff, const double* constants, int nconst,
                          void* out, void* hip_stream) {
    if (ncells == 0) return COFFEE_OK;
    if (ncells > (int64_t)INT32_MAX * 64) return COFFEE_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return COFFEE_E_HIP;
    const double* R = nullptr;
    coffee_status st = reference_table_f64(dev, form, cell, 1, q, fd, &R);
    if (st != COFFEE_OK) return st;
    dev::LinArgs a;
    std::memset(&a, 0, sizeof a);
    a.coords = coords;
    a.c2v = c2v;
    a.ncells = ncells;
    if (ncoeff >= 1) a.f0 = dev::FieldArg{coeffs[0].values, coeffs[0].cell_to_dof};
    a.out = out;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e;
    const bool helm = form == COFFEE_HELMHOLTZ;
    if (form == COFFEE_DIFFUSION) {
        a.c0 = (nconst > 0 ? constants[0] : 1.0) * (nconst > 1 ? constants[1] : 1.0);  // kappa dt
        e = cell == 2 ? launch_p1<dev::F_DIFF, 2, 0>(a, R, precision, s) : launch_p1<dev::F_DIFF, 3, 0>(a, R, precision, s);
    } else if (cell == 2) {
        if (fd == 0) e = helm ? launch_p1<dev::F_HELM, 2, 0>(a, R, precision, s) : launch_p1<dev::F_MASS, 2, 0>(a, R, precision, s);
        else e = helm ? launch_p1<dev::F_HELM, 2, 1>(a, R, precision, s) : launch_p1<dev::F_MASS, 2, 1>(a, R, precision, s);
    } else {
        if (fd == 0) e = helm ? launch_p1<dev::F_HELM, 3, 0>(a, R, precision, s) : launch_p1<dev::F_MASS, 3, 0>(a, R, precision, s);
        else e = helm ? launch_p1<dev::F_HELM, 3, 1>(a, R, precision, s) : launch_p1<dev::F_MASS, 3, 1>(a, R, precision, s);
    }
    return e == hipSuccess ? COFFEE_OK : COFFEE_E_HIP;
}

}  // namespace coffee
