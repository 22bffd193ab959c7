// Shared device pieces of the assembly engines (mass, Helmholtz, elasticity,
// Burgers Jacobian).
//
// Per cell (paper, section 2, Fig. 1): the Jacobian, its determinant and
// inverse from the vertex coordinates; coefficient dofs; then the element
// tensor. Here the element tensor of block (c, c') is the contraction
//     A[e][c n + a][c' n + b] = sum_k G[e][k] R[k][a n + b]
// of a per-cell geometry tensor G (built in FP64 from K = J^-1, |det J| and the
// coefficient dofs) with the reference tensors R (tables.h). Over a tile of 16
// cells this is a 16 x K by K x 16 matrix product, which runs on MFMA:
//     FP64   v_mfma_f64_16x16x4f64
//     FP32   v_mfma_f32_16x16x4f32
//     BF16X3 v_mfma_f32_16x16x32_bf16 on [G_hi | G_hi | G_lo] x [R_hi ; R_lo ; R_hi]
// The reference tensors are pre-packed on the host in MFMA B-fragment order
// so that each fragment load is one coalesced 512-byte (or 1 KiB) read.
// This file holds the gathers, the FP64 geometry, the G builders and their
// transposes (used by the adjoint), and the MFMA helpers; the engines are
// scalar.hpp (symmetric single-block forms) and vector.hpp (vector forms).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace coffee {
namespace dev {

// ---------------------------------------------------------------- address spaces
// Memory accesses that name their address space. A kernel infers the global
// space for pointers that come from its arguments, but code compiled as a
// separate (non-inlined) function sees only generic pointers and would use
// flat instructions, which are slower for LDS and make every wait on an LDS
// or scalar result also wait for outstanding global loads and stores. The
// casts are no-ops for pointers that already are global (or LDS).
template <typename T>
using global_ptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ inline T gload(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ inline T gload_nt(const T* p) {
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}
template <typename T>
__device__ inline void gstore(T* p, T v) {
    *(__attribute__((address_space(1))) T*)p = v;
}
template <typename T>
__device__ inline void gstore_nt(T* p, T v) {
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) T*)p);
}
// Load through the scalar (constant) path: for data no kernel writes, at an
// address that is the same in every lane.
template <typename T>
__device__ inline T cload(const T* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}
// A wave-uniform pointer held in scalar registers (its value in the first
// active lane; callers pass one that is the same in every lane).
template <typename T>
__device__ inline T* uniform_ptr(T* p) {
    const uint64_t u = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}
__device__ inline int64_t uniform_i64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
// A generic pointer known to address LDS: the result is generic again, but
// derived from an LDS pointer, so accesses through it compile to LDS
// instructions.
template <typename T>
__device__ inline T* as_lds(T* p) {
    return (T*)(__attribute__((address_space(3))) T*)p;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2 };
// same values as the public coffee_form enum
enum { F_MASS = 0, F_HELM = 1, F_ELAST = 2, F_BURG = 3, F_DIFF = 7 };

constexpr int nsc(int d, int p) { return d == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6; }
constexpr int npair(int d) { return d * (d + 1) / 2; }
constexpr int nfield(int d, int fd) { return fd > 0 ? nsc(d, fd) : 1; }
constexpr int ncomp_space(int form, int d) { return (form == F_ELAST || form == F_BURG) ? d : 1; }
constexpr int kref(int form, int d, int fd) {
    return form == F_MASS   ? nfield(d, fd)
         : form == F_HELM   ? npair(d) + nfield(d, fd)
         : form == F_DIFF   ? npair(d)
         : form == F_ELAST  ? nfield(d, fd) * d * d
                            : 1 + npair(d) + 2 * nfield(d, fd) * d;
}
constexpr int kstep(int prec) { return prec == PREC_BF16X3 ? 32 : 4; }
constexpr int keff(int form, int d, int fd, int prec) { return prec == PREC_BF16X3 ? 3 * kref(form, d, fd) : kref(form, d, fd); }
constexpr int ksteps(int form, int d, int fd, int prec) { return (keff(form, d, fd, prec) + kstep(prec) - 1) / kstep(prec); }
constexpr int ntiles(int d, int p) { return (nsc(d, p) * nsc(d, p) + 15) / 16; }

struct FieldArg {
    const double* values;
    const int32_t* map;  // NULL: cell-major values
};

struct LinArgs {
    const double* coords;
    const int32_t* c2v;
    int64_t ncells;
    FieldArg f0, f1;
    double c0, c1;          // elasticity (mu, lambda) if no fields; Burgers (nu, 1/dt); diffusion c0 = kappa dt
    const void* rfrag;      // packed reference fragments
    void* out;
    int64_t nchunks;        // ceil(ncells / 256)
};

// ---------------------------------------------------------------- geometry

template <int D, typename T = double>
struct Geom {
    T K[D][D];
    T adet;
};

// ---------------------------------------------------------------- split gathers
// The gathers of one cell in two dependent stages, so that a persistent loop
// can issue them for a later chunk while the current chunk is contracted.

template <int FORM, int D, int FD>
struct CellIdx {
    static constexpr int NF = nfield(D, FD);
    int v[D + 1];
    int f0[FD > 0 ? NF : 1];
    int f1[(FORM == F_ELAST && FD > 0) ? NF : 1];
};

template <int FORM, int D, int FD>
struct CellRaw {
    static constexpr int NF = nfield(D, FD);
    static constexpr int WC = (FORM == F_BURG) ? D : 1;
    double x[D + 1][D];
    double f0[FD > 0 ? NF * WC : 1];
    double f1[(FORM == F_ELAST && FD > 0) ? NF : 1];
};

// MAPF: -1 tests at run time whether the first field has a dof map, 1 and 0
// state that it has one or not (no branch: a branch around a load makes the
// next wait for outstanding loads drain every earlier load and store).
template <int FORM, int D, int FD, int MAPF = -1>
__device__ inline void load_idx(const LinArgs& A, int64_t cell, CellIdx<FORM, D, FD>& ix) {
    constexpr int NF = nfield(D, FD);
    const int32_t* cv = A.c2v + cell * (D + 1);
#pragma unroll
    for (int v = 0; v <= D; ++v) ix.v[v] = gload_nt(cv + v);
    if constexpr (FD > 0) {
        if (MAPF == 1 || (MAPF < 0 && A.f0.map)) {
            const int32_t* m = A.f0.map + cell * NF;
#pragma unroll
            for (int r = 0; r < NF; ++r) ix.f0[r] = gload_nt(m + r);
        }
        if constexpr (FORM == F_ELAST) {
            if (A.f1.map) {
                const int32_t* m = A.f1.map + cell * NF;
#pragma unroll
                for (int r = 0; r < NF; ++r) ix.f1[r] = gload_nt(m + r);
            }
        }
    }
}

template <int NL, int NCOMP, int MAPF = -1>
__device__ inline void load_field_vals(const FieldArg& f, int64_t cell, const int* idx, double* v) {
#pragma unroll
    for (int r = 0; r < NL; ++r) {
        const bool mapped = MAPF == 1 || (MAPF < 0 && f.map);
        const int64_t base = mapped ? (int64_t)idx[r] * NCOMP : (cell * NL + r) * NCOMP;
#pragma unroll
        for (int c = 0; c < NCOMP; ++c) v[r * NCOMP + c] = gload(f.values + base + c);
    }
}

template <int FORM, int D, int FD, int MAPF = -1>
__device__ inline void load_raw(const LinArgs& A, int64_t cell, const CellIdx<FORM, D, FD>& ix,
                                CellRaw<FORM, D, FD>& rw) {
    constexpr int NF = nfield(D, FD);
#pragma unroll
    for (int v = 0; v <= D; ++v)
#pragma unroll
        for (int i = 0; i < D; ++i) rw.x[v][i] = gload(A.coords + (int64_t)ix.v[v] * D + i);
    if constexpr (FD > 0) {
        load_field_vals<NF, CellRaw<FORM, D, FD>::WC, MAPF>(A.f0, cell, ix.f0, rw.f0);
        if constexpr (FORM == F_ELAST) load_field_vals<NF, 1>(A.f1, cell, ix.f1, rw.f1);
    }
}

template <int D, typename T = double>
__host__ __device__ inline void geometry_from_coords(const T (&x)[D + 1][D], Geom<D, T>& g) {
    T J[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) J[i][j] = x[j + 1][i] - x[0][i];
    if constexpr (D == 2) {
        const T det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const T r = 1.0 / det;
        g.K[0][0] = J[1][1] * r;
        g.K[0][1] = -J[0][1] * r;
        g.K[1][0] = -J[1][0] * r;
        g.K[1][1] = J[0][0] * r;
        g.adet = fabs(det);
    } else {
        const T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const T c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const T c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const T det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        const T r = 1.0 / det;
        g.K[0][0] = c00 * r;
        g.K[1][0] = c01 * r;
        g.K[2][0] = c02 * r;
        g.K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
        g.K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
        g.K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
        g.K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
        g.K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
        g.K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
        g.adet = fabs(det);
    }
}

// ---------------------------------------------------------------- G per form

// Cell data needed by the G builders.
template <int FORM, int D, int FD, typename T = double>
struct CellData {
    static constexpr int NF = nfield(D, FD);
    static constexpr int WC = (FORM == F_BURG) ? D : 1;
    Geom<D, T> g;
    T f0[FD > 0 ? NF * WC : 1];
    T f1[(FORM == F_ELAST && FD > 0) ? NF : 1];
};

template <int FORM, int D, int FD>
__device__ inline void cell_from_raw(const CellRaw<FORM, D, FD>& rw, CellData<FORM, D, FD>& cd) {
    geometry_from_coords<D>(rw.x, cd.g);
    if constexpr (FD > 0) {
#pragma unroll
        for (int i = 0; i < (int)(sizeof(cd.f0) / sizeof(double)); ++i) cd.f0[i] = rw.f0[i];
        if constexpr (FORM == F_ELAST) {
#pragma unroll
            for (int i = 0; i < (int)(sizeof(cd.f1) / sizeof(double)); ++i) cd.f1[i] = rw.f1[i];
        }
    }
}

template <int FORM, int D, int FD>
__device__ inline void load_cell(const LinArgs& A, int64_t cell, CellData<FORM, D, FD>& cd) {
    CellIdx<FORM, D, FD> ix;
    CellRaw<FORM, D, FD> rw;
    load_idx<FORM, D, FD>(A, cell, ix);
    load_raw<FORM, D, FD>(A, cell, ix, rw);
    cell_from_raw<FORM, D, FD>(rw, cd);
}

// G[k] of block (c1, c2) in the tensor order of reference.cpp.
template <int FORM, int D, int FD, int C1, int C2, typename T = double>
__host__ __device__ inline void build_G(const CellData<FORM, D, FD, T>& cd, const LinArgs& A, T* G) {
    constexpr int NF = nfield(D, FD);
    const auto& K = cd.g.K;
    const T ad = cd.g.adet;
    int t = 0;
    if constexpr (FORM == F_HELM || FORM == F_BURG || FORM == F_DIFF) {
        // nu for Burgers, kappa dt for diffusion
        const T sc = (FORM == F_BURG || FORM == F_DIFF) ? T(ad * A.c0) : ad;
        if constexpr (FORM == F_BURG) G[t++] = (C1 == C2) ? ad * A.c1 : T(0.0);
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b) {
                T s = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) s += K[a][i] * K[b][i];
                G[t++] = (C1 == C2) ? sc * s : T(0.0);
            }
    }
    if constexpr (FORM == F_MASS || FORM == F_HELM) {
#pragma unroll
        for (int r = 0; r < NF; ++r) G[t++] = (FD > 0) ? ad * cd.f0[r] : ad;
    } else if constexpr (FORM == F_ELAST) {
#pragma unroll
        for (int r = 0; r < NF; ++r) {
            const T mu = (FD > 0) ? cd.f0[r] : T(A.c0);
            const T lm = (FD > 0) ? cd.f1[r] : T(A.c1);
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    T kk = 0.0;
                    if constexpr (C1 == C2) {
#pragma unroll
                        for (int i = 0; i < D; ++i) kk += K[a][i] * K[b][i];
                    }
                    G[t++] = ad * (mu * (kk + K[a][C2] * K[b][C1]) + lm * K[a][C1] * K[b][C2]);
                }
        }
    } else if constexpr (FORM == F_BURG) {
        // C(r, a): delta_c1c2 |det J| sum_i w_{r,i} K[a][i]
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int a = 0; a < D; ++a) {
                T s = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) s += cd.f0[r * D + i] * K[a][i];
                G[t++] = (C1 == C2) ? ad * s : T(0.0);
            }
        // E(r, a): |det J| w_{r,c1} K[a][c2]
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int a = 0; a < D; ++a) G[t++] = ad * cd.f0[r * D + C1] * K[a][C2];
    }
}

// Transpose of build_G: with gbar(k) = dS/dG[k] for block (c1, c2), add the
// block's value sum_k G[k] gbar(k) to S, dS/dK to Kbar and dS/d(coefficient
// dofs) to f0bar / f1bar. gbar is evaluated once per k. Every term of G has
// exactly one factor |det J|, so dS/d|det J| = S / |det J| follows from S.
template <int FORM, int D, int FD, int C1, int C2, typename GB>
__host__ __device__ inline void reverse_G(const CellData<FORM, D, FD>& cd, const LinArgs& A, GB&& gbar, double& S,
                                          double (&Kbar)[D][D], double* f0bar, double* f1bar) {
    constexpr int NF = nfield(D, FD);
    const auto& K = cd.g.K;
    const double ad = cd.g.adet;
    int t = 0;
    if constexpr (FORM == F_HELM || FORM == F_BURG || FORM == F_DIFF) {
        const double sc = (FORM == F_BURG || FORM == F_DIFF) ? ad * A.c0 : ad;
        if constexpr (FORM == F_BURG) {
            // (1/dt) |det J|: no K or coefficient dependence
            if (C1 == C2) S += ad * A.c1 * gbar(t);
            ++t;
        }
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = a; b < D; ++b) {
                // G = sc sum_i K[a][i] K[b][i]
                if (C1 == C2) {
                    const double g = sc * gbar(t);
                    double kk = 0.0;
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        kk += K[a][i] * K[b][i];
                        Kbar[a][i] += g * K[b][i];
                        Kbar[b][i] += g * K[a][i];
                    }
                    S += g * kk;
                }
                ++t;
            }
    }
    if constexpr (FORM == F_MASS || FORM == F_HELM) {
#pragma unroll
        for (int r = 0; r < NF; ++r) {
            const double g = ad * gbar(t + r);
            if constexpr (FD > 0) {
                f0bar[r] += g;
                S += g * cd.f0[r];
            } else {
                S += g;
            }
        }
    } else if constexpr (FORM == F_ELAST) {
#pragma unroll
        for (int r = 0; r < NF; ++r) {
            const double mu = (FD > 0) ? cd.f0[r] : A.c0;
            const double lm = (FD > 0) ? cd.f1[r] : A.c1;
            double mubar = 0.0, lmbar = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    // G = ad (mu (delta KK^T_ab + K[a][C2] K[b][C1]) + lm K[a][C1] K[b][C2])
                    const double gb = ad * gbar(t++);
                    double kk = 0.0;
                    if constexpr (C1 == C2) {
#pragma unroll
                        for (int i = 0; i < D; ++i) kk += K[a][i] * K[b][i];
                    }
                    mubar += gb * (kk + K[a][C2] * K[b][C1]);
                    lmbar += gb * K[a][C1] * K[b][C2];
                    const double gm = gb * mu, gl = gb * lm;
                    if constexpr (C1 == C2) {
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            Kbar[a][i] += gm * K[b][i];
                            Kbar[b][i] += gm * K[a][i];
                        }
                    }
                    Kbar[a][C2] += gm * K[b][C1];
                    Kbar[b][C1] += gm * K[a][C2];
                    Kbar[a][C1] += gl * K[b][C2];
                    Kbar[b][C2] += gl * K[a][C1];
                }
            S += mu * mubar + lm * lmbar;
            if constexpr (FD > 0) {
                f0bar[r] += mubar;
                f1bar[r] += lmbar;
            }
        }
    } else if constexpr (FORM == F_BURG) {
        // C(r, a) = delta ad sum_i w_{r,i} K[a][i]
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int a = 0; a < D; ++a) {
                if (C1 == C2) {
                    const double g = ad * gbar(t);
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        s += cd.f0[r * D + i] * K[a][i];
                        Kbar[a][i] += g * cd.f0[r * D + i];
                        f0bar[r * D + i] += g * K[a][i];
                    }
                    S += g * s;
                }
                ++t;
            }
        // E(r, a) = ad w_{r,c1} K[a][c2]
#pragma unroll
        for (int r = 0; r < NF; ++r)
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double g = ad * gbar(t++);
                Kbar[a][C2] += g * cd.f0[r * D + C1];
                f0bar[r * D + C1] += g * K[a][C2];
                S += g * cd.f0[r * D + C1] * K[a][C2];
            }
    }
}

// ---------------------------------------------------------------- precision helpers

// bf16(x), rounded to nearest even: one v_cvt_pk_bf16_f32 on gfx950.
__device__ inline u16 bf16_bits_rne(float x) { return __builtin_bit_cast(u16, (__bf16)x); }
__device__ inline float bf16_to_float(u16 h) { return __uint_as_float(((uint32_t)h) << 16); }

template <int PREC> struct PrecT;
template <> struct PrecT<PREC_F64> { typedef double gtype; typedef double otype; typedef double frag; typedef d4 acc; };
template <> struct PrecT<PREC_F32> { typedef float gtype; typedef float otype; typedef float frag; typedef f4 acc; };
template <> struct PrecT<PREC_BF16X3> { typedef u16 gtype; typedef float otype; typedef bf8 frag; typedef f4 acc; };

template <int PREC>
__device__ inline typename PrecT<PREC>::acc mfma(typename PrecT<PREC>::frag a, typename PrecT<PREC>::frag b,
                                                 typename PrecT<PREC>::acc c) {
    if constexpr (PREC == PREC_F64) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else if constexpr (PREC == PREC_F32) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Row (within the 16-row tile) of accumulator element v held by `lane`.
// Measured on gfx950: FP64 16x16x4 holds rows lane/16 + 4 v; the FP32 and
// BF16 variants hold rows 4 (lane/16) + v. Columns are lane % 16 for all.
template <int PREC>
__device__ inline int acc_row(int lane, int v) {
    return PREC == PREC_F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}

template <int FORM, int D, int FD, int PREC>
struct GLayout {
    static constexpr int KR = kref(FORM, D, FD);
    static constexpr int KS = ksteps(FORM, D, FD, PREC);
    // row length in elements: odd (FP64/FP32) so that the 16 rows of a
    // fragment hit different banks; BF16 rows stay 16-byte aligned and are
    // shifted by 16 bytes.
    static constexpr int ROW = PREC == PREC_BF16X3 ? KS * 32 + 8 : KS * 4 + 1;
};

// Write one cell's G row to LDS (with the hi/lo split for BF16X3).
template <int FORM, int D, int FD, int PREC>
__device__ inline void put_G_row(typename PrecT<PREC>::gtype* row, const double* G) {
    constexpr int KR = kref(FORM, D, FD);
    constexpr int KS = ksteps(FORM, D, FD, PREC);
    if constexpr (PREC == PREC_F64) {
#pragma unroll
        for (int k = 0; k < KS * 4; ++k) row[k] = k < KR ? G[k < KR ? k : 0] : 0.0;
    } else if constexpr (PREC == PREC_F32) {
#pragma unroll
        for (int k = 0; k < KS * 4; ++k) row[k] = k < KR ? (float)G[k < KR ? k : 0] : 0.0f;
    } else {
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const float x = (float)G[k];
            const u16 hi = bf16_bits_rne(x);
            const u16 lo = bf16_bits_rne(x - bf16_to_float(hi));
            row[k] = hi;
            row[KR + k] = hi;
            row[2 * KR + k] = lo;
        }
#pragma unroll
        for (int k = 3 * KR; k < KS * 32; ++k) row[k] = 0;
    }
}

template <int PREC>
__device__ inline typename PrecT<PREC>::frag load_afrag(const typename PrecT<PREC>::gtype* tile, int row_len,
                                                        int lane, int s) {
    const int r = lane & 15, g = lane >> 4;
    if constexpr (PREC == PREC_BF16X3) {
        return *reinterpret_cast<const bf8*>(tile + r * row_len + 32 * s + 8 * g);
    } else {
        return tile[r * row_len + 4 * s + g];
    }
}

// Orders the LDS accesses of one wave around a point where its lanes exchange
// data through LDS.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave combining of scatter-adds of NV values per key: the lanes insert
// (key, values) into an open-addressing table in LDS, equal keys are summed
// there, and each distinct key then goes to global memory as one atomic add
// per value (cells that share a dof are neighbours, so a wave's 64 cells hold
// far fewer distinct dofs than dof references). A key that finds no slot
// within the probe limit is added to global memory directly.
constexpr unsigned long long kEmptyKey = ~0ull;

template <int NV, int TS>
__device__ inline void combine_clear(unsigned long long* keys, double* vals, int lane) {
    for (int i = lane; i < TS; i += 64) {
        keys[i] = kEmptyKey;
#pragma unroll
        for (int c = 0; c < NV; ++c) vals[i * NV + c] = 0.0;
    }
}

template <int NV, int TS>
__device__ inline void combine_add(unsigned long long* keys, double* vals, unsigned long long key, const double* v,
                                   double* global_base) {
    unsigned h = (unsigned)((key * 0x9E3779B97F4A7C15ull) >> 40) & (TS - 1);
    for (int t = 0; t < 32; ++t) {
        const unsigned long long old = atomicCAS(&keys[h], kEmptyKey, key);
        if (old == kEmptyKey || old == key) {
#pragma unroll
            for (int c = 0; c < NV; ++c) atomicAdd(&vals[h * NV + c], v[c]);
            return;
        }
        h = (h + 1) & (TS - 1);
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) atomicAdd(global_base + key * NV + c, v[c]);
}

template <int NV, int TS>
__device__ inline void combine_flush(const unsigned long long* keys, const double* vals, double* global_base,
                                     int lane) {
    for (int i = lane; i < TS; i += 64) {
        const unsigned long long key = keys[i];
        if (key == kEmptyKey) continue;
#pragma unroll
        for (int c = 0; c < NV; ++c) atomicAdd(global_base + key * NV + c, vals[i * NV + c]);
    }
}


}  // namespace dev
}  // namespace coffee
