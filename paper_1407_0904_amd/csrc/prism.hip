// Prism cells (triangle x interval): mass, Helmholtz and diffusion.
//
// The paper's benchmarks run on prisms as well as on simplices (section 5.2;
// at p = 1 a prism's j and k loops have 6 iterations). A prism is the image
// of the reference prism under the map spanned by its six degree-1 basis
// functions; that map is not affine, so J, det J and K = J^-1 change from
// quadrature point to point and the quadrature sum cannot be folded into
// point-free reference tensors as on simplices (the point loop carries the
// geometry). It stays the contraction of section 3.3's outer-product form,
// with the point index inside K:
//     A[e][a][b] = sum_{q, j} G[e][q, j] R[q, j][a][b]
//     G[e][q, j] = W_q |det J_q| (K_q K_q^T)_{al be}   (j over al <= be; kappa dt for diffusion)
//                  W_q |det J_q| f(X_q)                 (mass term; f = 1 without a field)
//     R[q, j][a][b] = d_al phi_a d_be phi_b (+ d_be phi_a d_al phi_b for al != be), phi_a phi_b at X_q
// so K = nq x (6 + 1) for Helmholtz, nq x 6 for diffusion, nq for mass. Over
// 16 cells this is a 16 x K by K x 16 product per 16 unique entries (a <= b;
// the matrices are symmetric), on the same MFMA instructions as the simplex
// engines (linear.hpp).
//
// Degree 1 (k_prism), per wave: one tile of 16 cells at a time. The 64
// lanes are 16 cells x 4 groups of quadrature points: each lane gathers its
// cell (all four lanes of a cell read the same lines), forms J, K and |det J|
// in FP64 at its points and writes those G entries to the tile's LDS rows.
// The MFMA loop then runs over all n-tiles at once, and the 16 element
// matrices leave through LDS as contiguous 16-byte stores (the staging area
// reuses the G rows). Degrees 2 and 3 (k_prism_big): the waves of a
// workgroup share 32 cells, each wave taking a share of the n-tiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "library.h"
#include "linear.hpp"
#include "tables.h"

namespace coffee {
namespace dev {

typedef unsigned int u32x4p __attribute__((ext_vector_type(4)));

constexpr int prism_ns(int p) { return (p + 1) * (p + 2) / 2 * (p + 1); }
// G entries per point: the six pairs al <= be, then the mass term
constexpr int prism_jq(int form) { return form == F_MASS ? 1 : (form == F_HELM ? 7 : 6); }

template <int FORM, int P, int FD, int PREC, int NQ>
struct PrismCfg {
    using g_t = typename PrecT<PREC>::gtype;
    using frag_t = typename PrecT<PREC>::frag;
    using acc_t = typename PrecT<PREC>::acc;
    using out_t = typename PrecT<PREC>::otype;
    static constexpr int NS = prism_ns(P);
    static constexpr int NN = NS * NS;
    static constexpr int NU = NS * (NS + 1) / 2;
    static constexpr int NT = (NU + 15) / 16;
    static constexpr int JQ = prism_jq(FORM);
    static constexpr int KR = NQ * JQ;
    static constexpr int KE = PREC == PREC_BF16X3 ? 3 * KR : KR;
    static constexpr int KS = (KE + kstep(PREC) - 1) / kstep(PREC);
    // odd FP64/FP32 rows spread a fragment's 16 rows over the banks; BF16
    // rows stay 16-byte aligned
    static constexpr int ROW = PREC == PREC_BF16X3 ? KS * 32 + 8 : KS * 4 + 1;
    static constexpr int GT_BYTES = 16 * ROW * (int)sizeof(g_t);
    static constexpr int ST_BYTES = 8 * NN * (int)sizeof(out_t);
    static constexpr int WAVE_BYTES = ((GT_BYTES > ST_BYTES ? GT_BYTES : ST_BYTES) + 15) / 16 * 16;
    // two waves per workgroup when four would take more than half the LDS
    static constexpr int WAVES = 4 * WAVE_BYTES <= 80 * 1024 ? 4 : 2;
    static constexpr int LDS_BYTES = WAVES * WAVE_BYTES;
    static constexpr int REGB = NT * KS * (PREC == PREC_F64 ? 2 : (PREC == PREC_F32 ? 1 : 4));
    static constexpr bool RREG = REGB <= 64;  // reference fragments held in registers
};

// Word 3 of a raw buffer resource on gfx9-family chips: 32-bit data format
// (a zero format would make untyped buffer accesses read zeros).
constexpr int kBufferWord3 = 0x00020000;

// One MFMA fragment (8, 4 or 16 bytes) from a raw buffer.
template <typename F>
__device__ inline F buffer_frag(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    if constexpr (sizeof(F) == 4) {
        return __builtin_bit_cast(F, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    } else if constexpr (sizeof(F) == 8) {
        return __builtin_bit_cast(F, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    } else {
        static_assert(sizeof(F) == 16, "fragment of 4, 8 or 16 bytes");
        return __builtin_bit_cast(F, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    }
}

struct PrismArgs {
    const double* coords;  // [nvert][3]
    const int32_t* c2v;    // [ncells][6]
    int64_t ncells;
    FieldArg f;            // degree-1 prism field (6 dofs per cell); values NULL: none
    double kdt;            // kappa dt (diffusion)
    const double* qtab;    // [NQ][4]: X, Y, Z, W
    const void* rfrag;     // packed reference fragments
    void* out;
    int64_t ntiles;        // ceil(ncells / 16)
};

// K = J^-1 (K[a][i] = d X_a / d x_i, J[i][a] = d x_i / d X_a) and |det J|.
__device__ inline void prism_inverse(const double (&J)[3][3], double (&K)[3][3], double& adet) {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double r = 1.0 / det;
    K[0][0] = c00 * r;
    K[1][0] = c01 * r;
    K[2][0] = c02 * r;
    K[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
    K[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
    K[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
    K[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
    K[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
    K[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
    adet = fabs(det);
}

// One G value into LDS column k (with the hi/lo split for BF16X3: columns k,
// KR + k hold the high part, 2 KR + k the low part, against R's (hi, lo, hi)).
template <int PREC, int KR>
__device__ inline void put_g(typename PrecT<PREC>::gtype* row, int k, double g) {
    if constexpr (PREC == PREC_F64) {
        row[k] = g;
    } else if constexpr (PREC == PREC_F32) {
        row[k] = (float)g;
    } else {
        const float x = (float)g;
        const u16 hi = bf16_bits_rne(x);
        row[k] = hi;
        row[KR + k] = hi;
        row[2 * KR + k] = bf16_bits_rne(x - bf16_to_float(hi));
    }
}

// The gathers of one cell in two dependent stages (indices, then values), so
// that the tile loop can issue them ahead of use.
struct PrismIdx {
    int v[6];
    int fm[6];
};
template <int FD>
struct PrismRaw {
    double x[6][3];
    double f[FD > 0 ? 6 : 1];
};

template <int FD>
__device__ inline void prism_idx(const PrismArgs& A, int64_t cell, PrismIdx& ix) {
#pragma unroll
    for (int v = 0; v < 6; ++v) ix.v[v] = gload_nt(A.c2v + cell * 6 + v);
    if constexpr (FD > 0) {
        if (A.f.map) {
#pragma unroll
            for (int v = 0; v < 6; ++v) ix.fm[v] = gload_nt(A.f.map + cell * 6 + v);
        }
    }
}

template <int FD>
__device__ inline void prism_raw(const PrismArgs& A, int64_t cell, const PrismIdx& ix, PrismRaw<FD>& r) {
#pragma unroll
    for (int v = 0; v < 6; ++v)
#pragma unroll
        for (int i = 0; i < 3; ++i) r.x[v][i] = gload(A.coords + (int64_t)ix.v[v] * 3 + i);
    if constexpr (FD > 0) {
#pragma unroll
        for (int v = 0; v < 6; ++v) r.f[v] = gload(A.f.values + (A.f.map ? (int64_t)ix.fm[v] : cell * 6 + v));
    }
}

template <int FORM, int P, int FD, int PREC, int NQ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_prism(PrismArgs A) {
    using C = PrismCfg<FORM, P, FD, PREC, NQ>;
    using g_t = typename C::g_t;
    using frag_t = typename C::frag_t;
    using acc_t = typename C::acc_t;
    using out_t = typename C::out_t;
    constexpr int NS = C::NS, NN = C::NN, NU = C::NU, NT = C::NT, KS = C::KS, ROW = C::ROW, JQ = C::JQ,
                  KR = C::KR;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;
    g_t* gt = reinterpret_cast<g_t*>(lds + wave * C::WAVE_BYTES);
    out_t* st = reinterpret_cast<out_t*>(lds + wave * C::WAVE_BYTES);
    const frag_t* rf = reinterpret_cast<const frag_t*>(A.rfrag);
    out_t* out = reinterpret_cast<out_t*>(A.out);

    // (a, b) of the unique entry u = 16 t + col, a <= b, row-major over the upper triangle
    int ua[NT], ub[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        int u = t * 16 + col, a = 0;
        while (a < NS - 1 && u >= NS - a) { u -= NS - a; ++a; }
        ua[t] = a;
        ub[t] = a + u;
    }
    constexpr unsigned FB = sizeof(frag_t);
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<frag_t*>(rf), (short)0, NT * KS * 64 * (int)FB, kBufferWord3);
    const unsigned vlane = lane * FB;
    frag_t rreg[C::RREG ? NT : 1][C::RREG ? KS : 1];
    if constexpr (C::RREG) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int s = 0; s < KS; ++s) rreg[t][s] = gload(rf + (t * KS + s) * 64 + lane);
    }

    // the rule's points and weights, once per workgroup
    __shared__ double sq[NQ * 4];
    for (int i = threadIdx.x; i < NQ * 4; i += blockDim.x) sq[i] = gload(A.qtab + i);
    __syncthreads();

    // Persistent loop over 16-cell tiles, software-pipelined at degree 1:
    // while tile i is contracted and stored, the vertices and field values of
    // tile i + 1 and the indices of tile i + 2 are in flight (issued before
    // this tile's stores, which share the in-order memory counter with them).
    const int64_t stride = (int64_t)gridDim.x * C::WAVES;
    int64_t tile = (int64_t)blockIdx.x * C::WAVES + wave;
    if (tile >= A.ntiles) return;  // wave-uniform; no workgroup barrier follows
    auto clamp = [&](int64_t t) -> int64_t {
        const int64_t c = (t < A.ntiles ? t : tile) * 16 + col;
        return c < A.ncells ? c : A.ncells - 1;
    };
    // degree 1 prefetches (short contraction, gather latency dominates); at
    // degree 2 the contraction hides it and the registers go to occupancy
    constexpr bool PIPE = P == 1;
    PrismIdx ix;
    PrismRaw<FD> raw;
    if constexpr (PIPE) {
        prism_idx<FD>(A, clamp(tile), ix);
        prism_raw<FD>(A, clamp(tile), ix, raw);
        prism_idx<FD>(A, clamp(tile + stride), ix);
        // Complete the prologue's loads here (no store is outstanding yet):
        // the loop's first wait then merges with an empty queue, and the
        // waits inside the loop can leave this tile's stores in flight.
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            asm volatile("" ::"v"(ix.v[v]));
            if constexpr (FD > 0) asm volatile("" ::"v"(ix.fm[v]), "v"(raw.f[v]));
#pragma unroll
            for (int i = 0; i < 3; ++i) asm volatile("" ::"v"(raw.x[v][i]));
        }
    }
    // One tile. FULL: all 16 cells exist, so the stores have compile-time counts
    // and the next tile's waits need not drain them.
    auto tile_body = [&](auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        const int64_t base = tile * 16;
        const bool valid = FULL || base + col < A.ncells;
        if constexpr (!PIPE) {
            prism_idx<FD>(A, clamp(tile), ix);
            prism_raw<FD>(A, clamp(tile), ix, raw);
        }

        // per-cell edge vectors of the map (bottom and top triangle edges from
        // vertex t0, vertical edges)
        double e[7][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            e[0][i] = raw.x[2][i] - raw.x[0][i];
            e[1][i] = raw.x[3][i] - raw.x[1][i];
            e[2][i] = raw.x[4][i] - raw.x[0][i];
            e[3][i] = raw.x[5][i] - raw.x[1][i];
            e[4][i] = raw.x[1][i] - raw.x[0][i];
            e[5][i] = raw.x[3][i] - raw.x[2][i];
            e[6][i] = raw.x[5][i] - raw.x[4][i];
        }
        double f[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) f[v] = FD > 0 ? raw.f[v] : 0.0;
        if constexpr (PIPE) {
            // next tile's values (indices loaded one tile ago), then the indices two ahead
            prism_raw<FD>(A, clamp(tile + stride), ix, raw);
            prism_idx<FD>(A, clamp(tile + 2 * stride), ix);
        }

        // G entries of this lane's points q = grp, grp + 4, ...
        g_t* row = gt + col * ROW;
#pragma unroll
        for (int it = 0; it < (NQ + 3) / 4; ++it) {
            const int q = grp + 4 * it;
            if (q >= NQ) break;
            const double X = sq[4 * q], Y = sq[4 * q + 1], Z = sq[4 * q + 2], W = sq[4 * q + 3];
            const double zb = 1.0 - Z, l0 = 1.0 - X - Y;
            double J[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                J[i][0] = zb * e[0][i] + Z * e[1][i];
                J[i][1] = zb * e[2][i] + Z * e[3][i];
                J[i][2] = l0 * e[4][i] + X * e[5][i] + Y * e[6][i];
            }
            double K[3][3], adet;
            prism_inverse(J, K, adet);
            const double w = valid ? W * adet : 0.0;
            int j = q * JQ;
            if constexpr (FORM != F_MASS) {
                const double sc = FORM == F_DIFF ? w * A.kdt : w;
#pragma unroll
                for (int al = 0; al < 3; ++al)
#pragma unroll
                    for (int be = al; be < 3; ++be) {
                        const double s = K[al][0] * K[be][0] + K[al][1] * K[be][1] + K[al][2] * K[be][2];
                        put_g<PREC, KR>(row, j++, sc * s);
                    }
            }
            if constexpr (FORM != F_DIFF) {
                double fq = 1.0;
                if constexpr (FD > 0) {
                    // degree-1 prism basis lambda_t(X, Y) l_s(Z) at the point
                    fq = (l0 * f[0] + X * f[2] + Y * f[4]) * zb + (l0 * f[1] + X * f[3] + Y * f[5]) * Z;
                }
                put_g<PREC, KR>(row, j, w * fq);
            }
        }
        // zero K padding up to a whole number of k-steps
        constexpr int KFILL = PREC == PREC_BF16X3 ? 3 * KR : KR;
#pragma unroll 1
        for (int k = KFILL + grp; k < KS * kstep(PREC); k += 4) row[k] = g_t(0);
        wave_sync();

        acc_t acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
        if constexpr (C::RREG) {
            // fragments in registers: straight-line code (constant indices);
            // every G fragment is read from LDS before the first product, so
            // the reads overlap one another instead of each MFMA pair waiting
            // for its own read
            frag_t afr[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) afr[s] = load_afrag<PREC>(gt, ROW, lane, s);
#pragma unroll
            for (int s = 0; s < KS; ++s) asm volatile("" ::"v"(afr[s]));  // one wait for all reads
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma<PREC>(afr[s], rreg[t][s], acc[t]);
        } else {
            // fragments through the caches as buffer loads (the lane's offset
            // in one register, each n-tile's a constant), the next k-step's
            // loads in flight during this k-step's products
            frag_t b[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) b[t] = buffer_frag<frag_t>(rsrc, vlane, t * KS * 64 * FB);
#pragma unroll 1
            for (int s = 0; s < KS; ++s) {
                const frag_t a = load_afrag<PREC>(gt, ROW, lane, s);
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[t] = mfma<PREC>(a, b[t], acc[t]);
                if (s + 1 < KS) {
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        b[t] = buffer_frag<frag_t>(rsrc, vlane + (s + 1) * 64 * FB, t * KS * 64 * FB);
                }
            }
        }
        wave_sync();  // every G read is done: the staging area reuses the rows

        // two halves of 8 cells, each written to LDS in full (both triangles)
        // and copied out as contiguous 16-byte stores
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t c0 = base + 8 * h;
            if (!FULL && c0 >= A.ncells) break;  // wave-uniform
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (t * 16 + col >= NU) continue;
                const int oab = ua[t] * NS + ub[t], oba = ub[t] * NS + ua[t];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = acc_row<PREC>(lane, v);
                    if ((r >> 3) != h) continue;
                    const out_t xv = (out_t)acc[t][v];
                    st[(r & 7) * NN + oab] = xv;
                    st[(r & 7) * NN + oba] = xv;
                }
            }
            wave_sync();
            constexpr int PER16 = 16 / (int)sizeof(out_t);
            const u32x4p* s4 = reinterpret_cast<const u32x4p*>(st);
            out_t* dst = out + c0 * NN;
            u32x4p* d4 = reinterpret_cast<u32x4p*>(dst);
            if constexpr (FULL) {
                // 8 NN is a multiple of PER16; groups of four LDS reads, then
                // their four nontemporal stores. Every lane stores (lanes past
                // the end repeat the last vector, same address and value), so
                // no branch hides the store count from the wait counters.
                constexpr int NV = 8 * NN / PER16;
                constexpr int PL = (NV + 63) / 64;
#pragma unroll
                for (int i0 = 0; i0 < PL; i0 += 4) {
                    u32x4p tmp[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int k = (i0 + i) * 64 + lane < NV ? (i0 + i) * 64 + lane : NV - 1;
                        if (i0 + i < PL) tmp[i] = s4[k];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int k = (i0 + i) * 64 + lane < NV ? (i0 + i) * 64 + lane : NV - 1;
                        if (i0 + i < PL) gstore_nt(&d4[k], tmp[i]);
                    }
                }
            } else {
                const int nc = A.ncells - c0 < 8 ? (int)(A.ncells - c0) : 8;
                const int nelem = nc * NN;
                const int nvec = nelem / PER16;
                for (int i = lane; i < nvec; i += 64) gstore_nt(&d4[i], s4[i]);
                for (int i = nvec * PER16 + lane; i < nelem; i += 64) gstore(&dst[i], st[i]);
            }
            wave_sync();
        }
    };
    const int64_t nfull = A.ncells / 16;  // tiles whose 16 cells all exist
    for (; tile < nfull; tile += stride) tile_body(std::integral_constant<bool, true>());
    if (tile < A.ntiles) tile_body(std::integral_constant<bool, false>());
}

// ---------------------------------------------------------------- degrees 2, 3
// At degree 3 (40 dofs, 820 unique entries in 52 n-tiles, 64 points, K = 448
// for Helmholtz) one wave cannot hold the accumulators of all n-tiles, and 16
// cells' matrices (205 KB in FP64) are larger than the LDS. A cell's matrix
// written a few entries at a time over a long contraction leaves partial lines
// that the L2 evicts before they are complete, so the matrices go out through
// a staging area, a few whole cells at a time.
//
// A workgroup takes two 16-cell tiles (32 cells): all its threads form the
// 32 cells' G rows in LDS once (each thread one cell and a share of the
// points), and each wave contracts both tiles' rows with its share of the
// n-tiles, so that every R fragment loaded from L2 serves two products (one
// fragment per product would ask the L2 for about 64 bytes per clock per CU
// at the FP64 matrix-core rate, its whole bandwidth). Degree 3 runs eight
// waves (6 or 7 of the 52 n-tiles each), degree 2 four (2 or 3 of 11). The
// fragments of step s + 1 load during the products of step s. Then, in passes
// of as many cells as fit in the G rows' LDS (four at degree 3, sixteen at
// degree 2), the waves write their accumulators (both mirrored entries) into
// that staging area, and the workgroup copies those cells out as contiguous
// 16-byte stores.
template <int FORM, int P, int FD, int PREC, int NQ>
struct PrismBigCfg {
    using C = PrismCfg<FORM, P, FD, PREC, NQ>;
    static constexpr int CT = 2;  // 16-cell tiles per workgroup
    // eight waves at degree 3 (52 n-tiles); four at degree 2 (11 n-tiles:
    // three per wave, so that each G fragment read feeds six products)
    static constexpr int WAVES = P >= 3 ? 8 : 4;
    // n-tiles per wave. FP64/FP32: the first NT % WAVES waves take one more
    // (waves w and w + 4 share a SIMD, so each SIMD gets an equal share when
    // NT % WAVES <= 4), with no tile computed twice. BF16X3 (short products,
    // where the per-tile branches cost more than they save): TCH tiles on
    // every wave, tiles past NT repeating the last one, their products never
    // stored.
    static constexpr bool BAL = PREC != PREC_BF16X3;
    static constexpr int TB = BAL ? C::NT / WAVES : (C::NT + WAVES - 1) / WAVES;
    static constexpr int TR = BAL ? C::NT % WAVES : 0;
    static constexpr int TCH = TB + (TR ? 1 : 0);
    static constexpr int GT_BYTES = 16 * CT * C::ROW * (int)sizeof(typename C::g_t);
    // cells per staging pass: the most (4, 8, 16 or 32) whose matrices fit in
    // the G rows' LDS, at least four
    static constexpr int CB = C::NN * (int)sizeof(typename C::out_t);
    static constexpr int PC = 32 * CB <= GT_BYTES && CT == 2   ? 32
                              : 16 * CB <= GT_BYTES             ? 16
                              : 8 * CB <= GT_BYTES              ? 8
                                                                : 4;
    static constexpr int ST_BYTES = PC * CB;
    static constexpr int LDS_BYTES = ((GT_BYTES > ST_BYTES ? GT_BYTES : ST_BYTES) + 15) / 16 * 16;
    static_assert(LDS_BYTES + NQ * 32 <= 160 * 1024, "G rows, staging and the rule fit the LDS");
    static_assert(C::NN * (int)sizeof(typename C::out_t) % 16 == 0, "cell matrices of whole 16-byte vectors");
};

template <int FORM, int P, int FD, int PREC, int NQ>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_prism_big(PrismArgs A) {
    using C = PrismCfg<FORM, P, FD, PREC, NQ>;
    using B = PrismBigCfg<FORM, P, FD, PREC, NQ>;
    using g_t = typename C::g_t;
    using frag_t = typename C::frag_t;
    using acc_t = typename C::acc_t;
    using out_t = typename C::out_t;
    constexpr int NS = C::NS, NN = C::NN, NU = C::NU, NT = C::NT, KS = C::KS, JQ = C::JQ, KR = C::KR,
                  ROW = C::ROW, TCH = B::TCH, CT = B::CT;
    constexpr int CELLS = 16 * CT;  // cells per workgroup tile
    extern __shared__ __attribute__((aligned(16))) char lds[];
    __shared__ double sq[NQ * 4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    g_t* gt = reinterpret_cast<g_t*>(lds);
    out_t* st = reinterpret_cast<out_t*>(lds);
    const frag_t* rf = reinterpret_cast<const frag_t*>(A.rfrag);
    out_t* out = reinterpret_cast<out_t*>(A.out);
    // this wave's n-tiles t0 .. t0 + ntw - 1 (scalars)
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int t0 = wv * B::TB + (wv < B::TR ? wv : B::TR);
    const int ntw = B::TB + (wv < B::TR ? 1 : 0);

    // staging offsets of this lane's unique entries u = 16 t + (lane & 15):
    // (a, b), a <= b, row-major over the upper triangle (low half), and its
    // mirror (b, a) (high half)
    static_assert(NN <= 65536, "offsets in 16 bits");
    unsigned off[TCH];
#pragma unroll
    for (int i = 0; i < TCH; ++i) {
        int u = 16 * (t0 + i) + (lane & 15), a = 0;
        while (a < NS - 1 && u >= NS - a) {
            u -= NS - a;
            ++a;
        }
        off[i] = (unsigned)(a * NS + a + u) | (unsigned)((a + u) * NS + a) << 16;
    }
    for (int i = tid; i < NQ * 4; i += blockDim.x) sq[i] = gload(A.qtab + i);
    // the R fragments of this wave's n-tiles at k-step g, as buffer loads: the
    // lane's offset in one register, each tile's offset a scalar
    constexpr unsigned FB = sizeof(frag_t);
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<frag_t*>(rf), (short)0, NT * KS * 64 * (int)FB, kBufferWord3);
    auto load_b = [&](frag_t* b, int g) {
        const unsigned vo = ((unsigned)(t0 * KS + g) * 64 + lane) * FB;
#pragma unroll
        for (int i = 0; i < TCH; ++i)
            if (i < ntw)
                b[i] = buffer_frag<frag_t>(rsrc, vo, (unsigned)((B::BAL || t0 + i < NT ? i : NT - 1 - t0) * KS * 64) * FB);
    };

    const int64_t ngroups = (A.ncells + CELLS - 1) / CELLS;
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int64_t base = grp * CELLS;
        __syncthreads();  // the previous tile's staging reads are done (and sq is loaded)

        // G rows: thread (cell r, point group pg) forms points pg, pg + 16, ...
        {
            const int r = tid % CELLS, pg = tid / CELLS;
            constexpr int PG = 64 * B::WAVES / CELLS;  // point groups
            const bool valid = base + r < A.ncells;
            const int64_t cell = valid ? base + r : A.ncells - 1;
            PrismIdx ix;
            PrismRaw<FD> raw;
            prism_idx<FD>(A, cell, ix);
            prism_raw<FD>(A, cell, ix, raw);
            double e[7][3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                e[0][i] = raw.x[2][i] - raw.x[0][i];
                e[1][i] = raw.x[3][i] - raw.x[1][i];
                e[2][i] = raw.x[4][i] - raw.x[0][i];
                e[3][i] = raw.x[5][i] - raw.x[1][i];
                e[4][i] = raw.x[1][i] - raw.x[0][i];
                e[5][i] = raw.x[3][i] - raw.x[2][i];
                e[6][i] = raw.x[5][i] - raw.x[4][i];
            }
            g_t* row = gt + r * ROW;
            // k padding past the G entries (the staging area overwrote it)
            constexpr int KFILL = PREC == PREC_BF16X3 ? 3 * KR : KR;
            for (int k = KFILL + pg; k < KS * kstep(PREC); k += PG) row[k] = g_t(0);
#pragma unroll 1
            for (int q = pg; q < NQ; q += PG) {
                const double X = sq[4 * q], Y = sq[4 * q + 1], Z = sq[4 * q + 2], W = sq[4 * q + 3];
                const double zb = 1.0 - Z, l0 = 1.0 - X - Y;
                double J[3][3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    J[i][0] = zb * e[0][i] + Z * e[1][i];
                    J[i][1] = zb * e[2][i] + Z * e[3][i];
                    J[i][2] = l0 * e[4][i] + X * e[5][i] + Y * e[6][i];
                }
                double K[3][3], adet;
                prism_inverse(J, K, adet);
                const double w = valid ? W * adet : 0.0;
                int j = q * JQ;
                if constexpr (FORM != F_MASS) {
                    const double sc = FORM == F_DIFF ? w * A.kdt : w;
#pragma unroll
                    for (int al = 0; al < 3; ++al)
#pragma unroll
                        for (int be = al; be < 3; ++be) {
                            const double sv = K[al][0] * K[be][0] + K[al][1] * K[be][1] + K[al][2] * K[be][2];
                            put_g<PREC, KR>(row, j++, sc * sv);
                        }
                }
                if constexpr (FORM != F_DIFF) {
                    double fq = 1.0;
                    if constexpr (FD > 0)
                        fq = (l0 * raw.f[0] + X * raw.f[2] + Y * raw.f[4]) * zb +
                             (l0 * raw.f[1] + X * raw.f[3] + Y * raw.f[5]) * Z;
                    put_g<PREC, KR>(row, j, w * fq);
                }
            }
        }
        frag_t b[TCH];
        load_b(b, 0);
        __syncthreads();

        // contraction of the two tiles' G rows with this wave's n-tiles (the G
        // fragments of step s + 1 are read during the products of step s)
        acc_t acc[CT][TCH];
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int i = 0; i < TCH; ++i) acc[c][i] = acc_t{0, 0, 0, 0};
        frag_t a[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) a[c] = load_afrag<PREC>(gt + 16 * c * ROW, ROW, lane, 0);
        // one k-step: the products of step s with R fragments bc, the G
        // fragments of step s + 1 read meanwhile; R fragments of step s + 1
        // into bn (issued before the products when bn is a second buffer,
        // after them when it is bc itself)
        auto step = [&](int s, frag_t* bc, frag_t* bn) {
            if (bn != bc && s + 1 < KS) load_b(bn, s + 1);
            frag_t an[CT];
#pragma unroll
            for (int c = 0; c < CT; ++c) an[c] = load_afrag<PREC>(gt + 16 * c * ROW, ROW, lane, s + 1 < KS ? s + 1 : s);
#pragma unroll
            for (int i = 0; i < TCH; ++i)
                if (i < ntw) {
#pragma unroll
                    for (int c = 0; c < CT; ++c) acc[c][i] = mfma<PREC>(a[c], bc[i], acc[c][i]);
                }
            if (bn == bc && s + 1 < KS) load_b(bc, s + 1);
#pragma unroll
            for (int c = 0; c < CT; ++c) a[c] = an[c];
        };
        if constexpr (B::BAL) {
            // FP64/FP32: two R buffers (BF16X3's short products were slower so)
            frag_t b1[TCH];
#pragma unroll 1
            for (int s = 0; s < KS; s += 2) {
                step(s, b, b1);
                if (s + 1 < KS) step(s + 1, b1, b);
            }
        } else {
#pragma unroll 1
            for (int s = 0; s < KS; ++s) step(s, b, b);
        }

        // 4 CT / NVP passes. Pass p holds the NVP (tile c, accumulator element
        // v) pairs j = p NVP .. p NVP + NVP - 1, c = j / 4, v = j % 4; staging
        // slot 4 jj + lane / 16 is the cell of pair jj held by lane group
        // lane / 16.
        constexpr int NVP = B::PC / 4;
        constexpr int NV1 = NN * (int)sizeof(out_t) / 16;  // 16-byte vectors per cell
        const u32x4p* s4 = reinterpret_cast<const u32x4p*>(st);
#pragma unroll
        for (int p = 0; p < 4 * CT / NVP; ++p) {
            __syncthreads();  // G reads (first pass) or the previous pass's copies are done
#pragma unroll
            for (int jj = 0; jj < NVP; ++jj) {
                const int c = (p * NVP + jj) / 4, v = (p * NVP + jj) % 4;
#pragma unroll
                for (int i = 0; i < TCH; ++i) {
                    if (i >= ntw || 16 * (t0 + i) + (lane & 15) >= NU) continue;
                    const out_t x = (out_t)acc[c][i][v];
                    st[(4 * jj + (lane >> 4)) * NN + (off[i] & 0xffff)] = x;
                    st[(4 * jj + (lane >> 4)) * NN + (off[i] >> 16)] = x;
                }
            }
            __syncthreads();
            if constexpr (NVP >= 4) {
                // whole tiles: the pass's cells are contiguous, copied in
                // memory order (lines shared by neighbouring cells are then
                // written together); cell r of a tile sits in the slot of
                // its (lane group, v)
                const int64_t c0 = base + 16 * (p * NVP / 4);
                for (int k = tid; k < B::PC * NV1; k += blockDim.x) {
                    const int lc = k / NV1, r = lc % 16;
                    const int g = PREC == PREC_F64 ? r % 4 : r / 4, v = PREC == PREC_F64 ? r / 4 : r % 4;
                    const int slot = 4 * (4 * (lc / 16) + v) + g;
                    if (c0 + lc < A.ncells)
                        gstore_nt(reinterpret_cast<u32x4p*>(out + (c0 + lc) * NN) + (k - lc * NV1),
                                  s4[slot * NV1 + (k - lc * NV1)]);
                }
            } else {
                for (int k = tid; k < B::PC * NV1; k += blockDim.x) {
                    const int slot = k / NV1, j = p * NVP + slot / 4;
                    const int64_t cl = base + 16 * (j / 4) + acc_row<PREC>(16 * (slot % 4), j % 4);
                    if (cl < A.ncells)
                        gstore_nt(reinterpret_cast<u32x4p*>(out + cl * NN) + (k - slot * NV1), s4[k]);
                }
            }
        }
    }
}

}  // namespace dev

namespace {

using ld = long double;

// Reference products per point (no weights; the weights are in G), in the
// device's column order k = q JQ + j.
bool prism_reference(int form, int p, int quad, RefTensor& R, std::vector<double>& qtab) {
    PrismTables t;
    if (!t.init(p, quad)) return false;
    const int n = t.n, nq = t.nq, NN = n * n;
    const int JQ = dev::prism_jq(form == COFFEE_MASS ? dev::F_MASS : (form == COFFEE_HELMHOLTZ ? dev::F_HELM
                                                                                                : dev::F_DIFF));
    R.NS = n;
    R.KR = nq * JQ;
    R.R.assign((size_t)R.KR * NN, 0.0L);
    auto ph = [&](int k, int a) -> ld { return t.phi[(size_t)k * n + a]; };
    auto dph = [&](int al, int k, int a) -> ld { return t.dphi[((size_t)al * nq + k) * n + a]; };
    for (int k = 0; k < nq; ++k) {
        int j = k * JQ;
        if (form != COFFEE_MASS) {
            for (int al = 0; al < 3; ++al)
                for (int be = al; be < 3; ++be, ++j)
                    for (int a = 0; a < n; ++a)
                        for (int b = 0; b < n; ++b) {
                            ld v = dph(al, k, a) * dph(be, k, b);
                            if (al != be) v += dph(be, k, a) * dph(al, k, b);
                            R.R[(size_t)j * NN + a * n + b] = v;
                        }
        }
        if (form != COFFEE_DIFFUSION)
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) R.R[(size_t)j * NN + a * n + b] = ph(k, a) * ph(k, b);
    }
    qtab.resize(4 * (size_t)nq);
    for (int k = 0; k < nq; ++k) {
        for (int i = 0; i < 3; ++i) qtab[4 * k + i] = (double)t.X[3 * k + i];
        qtab[4 * k + 3] = (double)t.W[k];
    }
    return true;
}

struct PrismTable {
    void* frag = nullptr;
    double* qtab = nullptr;
};

std::mutex g_prism_mu;
std::map<std::tuple<int, int, int, int, int>, PrismTable> g_prism_tabs;  // (dev, form, p, quad, prec)

coffee_status prism_table(int dev, int form, int p, int quad, int prec, PrismTable* out) {
    std::lock_guard<std::mutex> lk(g_prism_mu);
    auto key = std::make_tuple(dev, form, p, quad, prec);
    auto it = g_prism_tabs.find(key);
    if (it != g_prism_tabs.end()) {
        *out = it->second;
        return COFFEE_OK;
    }
    RefTensor R;
    std::vector<double> qtab;
    if (!prism_reference(form, p, quad, R, qtab)) return COFFEE_E_INVALID_ARG;
    const std::vector<char> frag = pack_fragments(R, prec, true, 0);
    PrismTable t;
    if (hipMalloc(&t.frag, frag.size()) != hipSuccess) return COFFEE_E_NOMEM;
    if (hipMalloc((void**)&t.qtab, qtab.size() * sizeof(double)) != hipSuccess) {
        (void)hipFree(t.frag);
        return COFFEE_E_NOMEM;
    }
    if (hipMemcpy(t.frag, frag.data(), frag.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t.qtab, qtab.data(), qtab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(t.frag);
        (void)hipFree(t.qtab);
        return COFFEE_E_HIP;
    }
    g_prism_tabs[key] = t;
    *out = t;
    return COFFEE_OK;
}

template <int FORM, int P, int FD, int PREC, int NQ>
hipError_t launch_prism(const dev::PrismArgs& a, hipStream_t s, int dev_id) {
    using C = dev::PrismCfg<FORM, P, FD, PREC, NQ>;
    const void* kern = reinterpret_cast<const void*>(&dev::k_prism<FORM, P, FD, PREC, NQ>);
    static const hipError_t attr =
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_BYTES);
    if (attr != hipSuccess) return attr;
    const int64_t wgs_needed = (a.ntiles + C::WAVES - 1) / C::WAVES;
    // grid multiplier from the tuning cache (prism keys: cell COFFEE_PRISM)
    int tuned_variant = 0;
    const int tuned = tuned_linear(FORM, COFFEE_PRISM, P, FD, PREC, &tuned_variant);
    const int grid = grid_for(dev_id, kern, C::WAVES * 64, C::LDS_BYTES, wgs_needed, tuned > 0 ? tuned : 1);
    hipLaunchKernelGGL((dev::k_prism<FORM, P, FD, PREC, NQ>), dim3(grid), dim3(C::WAVES * 64), C::LDS_BYTES, s, a);
    return hipGetLastError();
}

template <int FORM, int P, int FD, int PREC, int NQ>
hipError_t launch_prism_big(const dev::PrismArgs& a, hipStream_t s, int dev_id) {
    using B = dev::PrismBigCfg<FORM, P, FD, PREC, NQ>;
    const void* kern = reinterpret_cast<const void*>(&dev::k_prism_big<FORM, P, FD, PREC, NQ>);
    static const hipError_t attr =
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, B::LDS_BYTES);
    if (attr != hipSuccess) return attr;
    const int64_t wgs_needed = (a.ncells + 16 * B::CT - 1) / (16 * B::CT);  // one tile group per workgroup at a time
    int tuned_variant = 0;
    const int tuned = tuned_linear(FORM, COFFEE_PRISM, P, FD, PREC, &tuned_variant);
    const int grid = grid_for(dev_id, kern, B::WAVES * 64, B::LDS_BYTES, wgs_needed, tuned > 0 ? tuned : 1);
    hipLaunchKernelGGL((dev::k_prism_big<FORM, P, FD, PREC, NQ>), dim3(grid), dim3(B::WAVES * 64), B::LDS_BYTES, s,
                       a);
    return hipGetLastError();
}

template <int FORM, int P, int FD, int NQ>
hipError_t launch_prism_prec(int prec, const dev::PrismArgs& a, hipStream_t s, int dev_id) {
    if constexpr (P >= 2) {
        if (prec == COFFEE_FP64) return launch_prism_big<FORM, P, FD, dev::PREC_F64, NQ>(a, s, dev_id);
        if (prec == COFFEE_FP32) return launch_prism_big<FORM, P, FD, dev::PREC_F32, NQ>(a, s, dev_id);
        return launch_prism_big<FORM, P, FD, dev::PREC_BF16X3, NQ>(a, s, dev_id);
    } else {
        if (prec == COFFEE_FP64) return launch_prism<FORM, P, FD, dev::PREC_F64, NQ>(a, s, dev_id);
        if (prec == COFFEE_FP32) return launch_prism<FORM, P, FD, dev::PREC_F32, NQ>(a, s, dev_id);
        return launch_prism<FORM, P, FD, dev::PREC_BF16X3, NQ>(a, s, dev_id);
    }
}

template <int P, int NQ>
hipError_t launch_prism_form(int form, int fd, int prec, const dev::PrismArgs& a, hipStream_t s, int dev_id) {
    using namespace dev;
    if (form == COFFEE_DIFFUSION) return launch_prism_prec<F_DIFF, P, 0, NQ>(prec, a, s, dev_id);
    if (form == COFFEE_MASS)
        return fd ? launch_prism_prec<F_MASS, P, 1, NQ>(prec, a, s, dev_id)
                  : launch_prism_prec<F_MASS, P, 0, NQ>(prec, a, s, dev_id);
    return fd ? launch_prism_prec<F_HELM, P, 1, NQ>(prec, a, s, dev_id)
              : launch_prism_prec<F_HELM, P, 0, NQ>(prec, a, s, dev_id);
}

}  // namespace

// Prism entry of coffee_assemble: arguments already validated (form mass,
// Helmholtz or diffusion; field none or degree 1 scalar).
coffee_status assemble_prism(int form, int degree, int quad, int precision, const double* coords,
                             const int32_t* c2v, int64_t ncells, const coffee_field* coeffs, int ncoeff,
                             const double* constants, int nconst, void* out, void* hip_stream) {
    // compiled: the default rule (q = 2p) at degree 1 (8 points), 2 (27 points) and 3 (64 points)
    if (degree < 1 || degree > 3 || quad != 2 * degree) return COFFEE_E_UNSUPPORTED;
    if (ncells == 0) return COFFEE_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return COFFEE_E_HIP;
    PrismTable t;
    coffee_status st = prism_table(dev, form, degree, quad, precision, &t);
    if (st != COFFEE_OK) return st;
    dev::PrismArgs a;
    std::memset(&a, 0, sizeof a);
    a.coords = coords;
    a.c2v = c2v;
    a.ncells = ncells;
    if (ncoeff >= 1) a.f = dev::FieldArg{coeffs[0].values, coeffs[0].cell_to_dof};
    a.kdt = (nconst > 0 ? constants[0] : 1.0) * (nconst > 1 ? constants[1] : 1.0);
    a.qtab = t.qtab;
    a.rfrag = t.frag;
    a.out = out;
    a.ntiles = (ncells + 15) / 16;
    const int fd = ncoeff >= 1 ? 1 : 0;
    hipStream_t s = (hipStream_t)hip_stream;
    const hipError_t e = degree == 1   ? launch_prism_form<1, 8>(form, fd, precision, a, s, dev)
                         : degree == 2 ? launch_prism_form<2, 27>(form, fd, precision, a, s, dev)
                                       : launch_prism_form<3, 64>(form, fd, precision, a, s, dev);
    return e == hipSuccess ? COFFEE_OK : COFFEE_E_HIP;
}

void free_prism_tables() {
    std::lock_guard<std::mutex> lk(g_prism_mu);
    for (auto& kv : g_prism_tabs) {
        (void)hipSetDevice(std::get<0>(kv.first));
        (void)hipFree(kv.second.frag);
        (void)hipFree(kv.second.qtab);
    }
    g_prism_tabs.clear();
}

}  // namespace coffee
