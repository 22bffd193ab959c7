// Degree-1 mass and Helmholtz arithmetic for one cell, shared by the
// single-form kernel (p1.hip) and the degree-1 bins of the mixed batch, so
// that both give the same bits.
//
// At p = 1 the element tensor is 3 x 3 (triangle) or 4 x 4 (tetrahedron) and
// the collapsed contraction A[a][b] = sum_k G[k] R[k][a][b] (section 2, Fig. 1;
// the quadrature sum folded into R as in linear.hpp) is a few dozen multiply-
// adds: far too small to fill an MFMA tile. One lane owns one cell; R is read
// at wave-uniform addresses (scalar loads). Only a <= b is formed and the
// value is mirrored (the symmetric iteration space of the paper's j, k loops).
#pragma once

#include "linear.hpp"

namespace coffee {
namespace dev {

// LDS row of one cell's tensor: NN elements padded to an odd count, so that
// 64 lanes writing their own rows hit distinct banks.
template <int D>
constexpr int p1_row() {
    return ((D + 1) * (D + 1)) | 1;
}

// G -> the cell's full tensor (row-major a, b) in `row`. R must be the same
// pointer in every lane (it is read through the scalar path).
template <int FORM, int D, int FD, typename OT>
__device__ inline void p1_tensor(const double* G, const double* __restrict__ R, OT* row) {
    constexpr int NS = D + 1, NN = NS * NS, KR = kref(FORM, D, FD);
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int b = a; b < NS; ++b) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < KR; ++k) s += G[k] * cload(R + k * NN + a * NS + b);
            row[a * NS + b] = (OT)s;
            row[b * NS + a] = (OT)s;
        }
}

}  // namespace dev
}  // namespace coffee
