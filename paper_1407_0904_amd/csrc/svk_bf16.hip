// St Venant-Kirchhoff energy, residual and Jacobian in BF16X3: every dense
// contraction of the per-point evaluation runs on the bf16 matrix cores with
// the hi + lo split of both operands (x_hi = bf16(x), x_lo = bf16(x - x_hi);
// products hi*hi + hi*lo + lo*hi accumulated in FP32); the geometry (J,
// det J, K = J^-1) is FP64, the point arithmetic FP32.
//
// Per point q of the rule the kernels of section 2 evaluate the coefficient
// at the point (Listing 2's F values): here the displacement gradient in
// reference coordinates, U[c][al] = sum_r u_(c,r) dphi_r/dX_al(q). Over a
// 16-cell tile this is, per component c, the product of the tile's dof rows
// (16 x NS) with the reference table [NS x (q, al)] -- one MFMA k-step, since
// the split operand [u_hi | u_hi | u_lo] is 3 NS <= 32 wide. Then per (cell,
// point), in FP32: F = I + U K, E = (H + H^T + H^T H)/2 with H = U K,
// S = lambda tr(E) I + 2 mu E, and
//   energy    w psi(E), summed over the points;
//   residual  Q = w P K^T (P = F S), contracted with the reference gradients:
//             b[(c,a)] = sum_(q,al) Q[c][(q,al)] dphi_a/dX_al(q), a 16 x (3 NQ D)
//             by (3 NQ D) x NS product per component on MFMA;
//   Jacobian  block (c1, c2), c1 <= c2, of the element matrix as the
//             contraction of the per-point tensor
//             H_ab = w (delta S^_ab + lambda k1_a k2_b + mu k2_a k1_b + mu (F_c1.F_c2) M_ab)
//             (S^ = K S K^T, k_c = K F_c, M = K K^T) with the reference tensor
//             R[(q,a,b)][(i,j)] = dphi_i/dX_a(q) dphi_j/dX_b(q): the outer-product
//             form of the element matrix (section 3.3) with G = H on the left,
//             16 cells x (NQ D^2) by (NQ D^2) x NS^2 per block, on MFMA.
// The point data live in LDS between the phases; the Jacobian's reference
// fragments are read from global memory (L2-resident), the element matrices
// staged in LDS and written as contiguous 16-byte stores.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "library.h"
#include "linear.hpp"
#include "tables.h"

namespace coffee {
namespace dev {

typedef unsigned short svkb_u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int svkb_u32x4 __attribute__((ext_vector_type(4)));

struct SvkBArgs {
    const double* coords;
    const int32_t* c2v;
    int64_t ncells;
    FieldArg u;
    float mu, lambda;
    const bf8* tabI;  // interpolation fragments [NTU][64]
    const bf8* tabR;  // residual fragments [KSR][64]
    const bf8* tabJ;  // Jacobian fragments [KSJ][NTJ][2][64] (hi, lo)
    const float* W;   // weights [NQ]
    void* out;
    int64_t ntiles;   // ceil(ncells / 16)
};

template <int D, int P, int NQ>
struct SvkBCfg {
    static constexpr int NS = nsc(D, P), N = D * NS, DD = D * D, NP = D * (D + 1) / 2, NB = NP;
    static constexpr int NQA = NQ * D;               // (point, direction) pairs
    static constexpr int NTU = (NQA + 15) / 16;      // interpolation n-tiles
    static constexpr int KSR = (3 * NQA + 31) / 32;  // residual k-steps
    static constexpr int KJ = NQ * DD;               // Jacobian contraction length
    static constexpr int KSJ = (KJ + 31) / 32;
    static constexpr int NTJ = (NS * NS + 15) / 16;
    static constexpr int PDN = 2 * DD + NP + 1;      // Jacobian point data: S^, k, F.F (sym), w
    static constexpr int UE = 16 * NQ * DD;          // LDS floats per wave: U
    static constexpr int CKE = 16 * (2 * DD + 1);    // K, M, |det J| per cell
    static_assert(3 * NS <= 32, "the split dof row must fit one k-step");
    static_assert(NS <= 16, "one residual n-tile");
    template <int MODE>
    static constexpr int pde() { return MODE == 0 ? 16 * NQ : MODE == 1 ? 16 * NQ * DD : 16 * NQ * PDN; }
    template <int MODE>
    static constexpr int wave_floats() { return (UE + CKE + pde<MODE>() + 3) / 4 * 4; }
    // cells staged per round in the Jacobian's output
    static constexpr int CR = wave_floats<2>() / (N * N) < 16 ? wave_floats<2>() / (N * N) : 16;
    static_assert(CR >= 1, "staging area");
};

__device__ inline bf8 svkb_split(const float (&x)[8], bool lo) {
    svkb_u16x8 h;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const u16 hi = bf16_bits_rne(x[j]);
        h[j] = lo ? bf16_bits_rne(x[j] - bf16_to_float(hi)) : hi;
    }
    return __builtin_bit_cast(bf8, h);
}

extern __shared__ __attribute__((aligned(16))) float svkb_lds[];

// MODE 0 energy, 1 residual, 2 Jacobian. One wave per 16-cell tile at a time.
template <int D, int P, int NQ, int MODE>
__global__ __launch_bounds__(256, 1) void k_svk_bf16(SvkBArgs A) {
    using C = SvkBCfg<D, P, NQ>;
    constexpr int NS = C::NS, N = C::N, DD = C::DD, NP = C::NP, NQA = C::NQA, PDN = C::PDN;
    constexpr int WA = C::template wave_floats<MODE>();
    constexpr int CKS = 2 * DD + 1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = lane & 15, grp = lane >> 4;
    float* U = svkb_lds + wave * WA;  // U[cell][q][c][al]
    float* CK = U + C::UE;            // per cell: K (row-major), M = K K^T, |det J|
    float* PD = CK + C::CKE;          // point data
    const float mu = A.mu, lm = A.lambda;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < A.ntiles; tile += nw) {
        const int64_t cell0 = tile * 16;
        const int64_t cell = cell0 + row < A.ncells ? cell0 + row : A.ncells - 1;
        // FP64 geometry and the cell's displacement dofs (every lane of the cell)
        double x[D + 1][D];
        int vid[D + 1];
#pragma unroll
        for (int v = 0; v <= D; ++v) vid[v] = A.c2v[cell * (D + 1) + v];
#pragma unroll
        for (int v = 0; v <= D; ++v)
#pragma unroll
            for (int i = 0; i < D; ++i) x[v][i] = A.coords[(int64_t)vid[v] * D + i];
        Geom<D> g;
        geometry_from_coords<D>(x, g);
        if (grp == 0) {
            float* ck = CK + row * CKS;
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    double m = 0.0;
#pragma unroll
                    for (int i = 0; i < D; ++i) m += g.K[a][i] * g.K[b][i];
                    ck[a * D + b] = (float)g.K[a][b];
                    ck[DD + a * D + b] = (float)m;
                }
            ck[2 * DD] = (float)g.adet;
        }
        // Phase 0: U[c][(q, al)] = sum_r u_(c,r) dphi_r/dX_al(q) on MFMA, one
        // k-step per component: A = [u_hi | u_hi | u_lo], B = [D_hi; D_lo; D_hi]
#pragma unroll
        for (int c = 0; c < D; ++c) {
            float xs[8];
            bool lo[8];
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                const int k = 8 * grp + jj;
                const int part = k / NS, r = k - part * NS;
                double v = 0.0;
                if (k < 3 * NS) {
                    const int64_t base = A.u.map ? (int64_t)A.u.map[cell * NS + r] * D : (cell * NS + r) * D;
                    v = A.u.values[base + c];
                }
                xs[jj] = (float)v;
                lo[jj] = part == 2;
            }
            // the lane's eight entries mix hi and lo parts: split each by its part
            svkb_u16x8 h;
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                const u16 hi = bf16_bits_rne(xs[jj]);
                h[jj] = lo[jj] ? bf16_bits_rne(xs[jj] - bf16_to_float(hi)) : hi;
            }
            const bf8 a = __builtin_bit_cast(bf8, h);
#pragma unroll
            for (int t = 0; t < C::NTU; ++t) {
                const f4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, A.tabI[t * 64 + lane], f4{0, 0, 0, 0}, 0, 0, 0);
                const int j = 16 * t + row;  // (q, al) column
                if (j < NQA) {
                    const int q = j / D, al = j - (j / D) * D;
#pragma unroll
                    for (int v = 0; v < 4; ++v) U[(((4 * grp + v) * NQ + q) * D + c) * D + al] = acc[v];
                }
            }
        }
        wave_sync();
        // Phase 1: per (cell, point) in FP32
        for (int pi = lane; pi < 16 * NQ; pi += 64) {
            const int rc = pi / NQ, q = pi - (pi / NQ) * NQ;
            const float* ck = CK + rc * CKS;
            const float* uq = U + (rc * NQ + q) * DD;
            float K[D][D], Hm[D][D], F[D][D], E[D][D], S[D][D], trE = 0.f;
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) K[a][b] = ck[a * D + b];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    float h = 0.f;
#pragma unroll
                    for (int a = 0; a < D; ++a) h += uq[i * D + a] * K[a][j];
                    Hm[i][j] = h;
                    F[i][j] = (i == j ? 1.f : 0.f) + h;
                }
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    float t = Hm[i][j] + Hm[j][i];
#pragma unroll
                    for (int k = 0; k < D; ++k) t += Hm[k][i] * Hm[k][j];
                    E[i][j] = 0.5f * t;
                }
#pragma unroll
            for (int i = 0; i < D; ++i) trE += E[i][i];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) S[i][j] = (i == j ? lm * trE : 0.f) + 2.f * mu * E[i][j];
            const float w = A.W[q];
            if constexpr (MODE == 0) {
                float EE = 0.f;
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int j = 0; j < D; ++j) EE += E[i][j] * E[i][j];
                PD[rc * NQ + q] = w * (0.5f * lm * trE * trE + mu * EE);
            } else if constexpr (MODE == 1) {
                float Pm[D][D];
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        float t = 0.f;
#pragma unroll
                        for (int k = 0; k < D; ++k) t += F[i][k] * S[k][j];
                        Pm[i][j] = t;
                    }
                float* qd = PD + (rc * NQ + q) * DD;
#pragma unroll
                for (int c = 0; c < D; ++c)
#pragma unroll
                    for (int al = 0; al < D; ++al) {
                        float t = 0.f;
#pragma unroll
                        for (int j = 0; j < D; ++j) t += Pm[c][j] * K[al][j];
                        qd[c * D + al] = w * t;
                    }
            } else {
                float* pd = PD + (rc * NQ + q) * PDN;
                float KS[D][D];
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int l = 0; l < D; ++l) {
                        float t = 0.f;
#pragma unroll
                        for (int j = 0; j < D; ++j) t += K[a][j] * S[j][l];
                        KS[a][l] = t;
                    }
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int b = 0; b < D; ++b) {
                        float t = 0.f;
#pragma unroll
                        for (int l = 0; l < D; ++l) t += KS[a][l] * K[b][l];
                        pd[a * D + b] = t;  // S^ = K S K^T
                    }
#pragma unroll
                for (int c = 0; c < D; ++c)
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        float t = 0.f;
#pragma unroll
                        for (int j = 0; j < D; ++j) t += K[a][j] * F[c][j];
                        pd[DD + c * D + a] = t;  // k_c = K F_c
                    }
                int s = 0;
#pragma unroll
                for (int c1 = 0; c1 < D; ++c1)
#pragma unroll
                    for (int c2 = c1; c2 < D; ++c2, ++s) {
                        float t = 0.f;
#pragma unroll
                        for (int j = 0; j < D; ++j) t += F[c1][j] * F[c2][j];
                        pd[2 * DD + s] = t;  // F_c1 . F_c2
                    }
                pd[PDN - 1] = w;
            }
        }
        wave_sync();
        if constexpr (MODE == 0) {
            if (lane < 16 && cell0 + lane < A.ncells) {
                float e = 0.f;
#pragma unroll
                for (int q = 0; q < NQ; ++q) e += PD[lane * NQ + q];
                reinterpret_cast<float*>(A.out)[cell0 + lane] = CK[lane * CKS + 2 * DD] * e;
            }
        } else if constexpr (MODE == 1) {
            // b[(c, a)] = sum_(q,al) Q[c][(q,al)] dphi_a/dX_al(q): A = [Q_hi | Q_hi | Q_lo]
            float* o = reinterpret_cast<float*>(A.out);
#pragma unroll
            for (int c = 0; c < D; ++c) {
                f4 acc = {0, 0, 0, 0};
#pragma unroll
                for (int s = 0; s < C::KSR; ++s) {
                    float xs[8];
                    bool lo[8];
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        const int k = 32 * s + 8 * grp + jj;
                        const int part = k / NQA, j = k - part * NQA;
                        const int q = j / D, al = j - (j / D) * D;
                        xs[jj] = k < 3 * NQA ? PD[((row * NQ + q) * D + c) * D + al] : 0.f;
                        lo[jj] = part == 2;
                    }
                    svkb_u16x8 h;
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        const u16 hi = bf16_bits_rne(xs[jj]);
                        h[jj] = lo[jj] ? bf16_bits_rne(xs[jj] - bf16_to_float(hi)) : hi;
                    }
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, h), A.tabR[s * 64 + lane],
                                                                   acc, 0, 0, 0);
                }
                if (row < NS) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int rc = 4 * grp + v;
                        if (cell0 + rc < A.ncells) o[(cell0 + rc) * N + c * NS + row] = CK[rc * CKS + 2 * DD] * acc[v];
                    }
                }
            }
        } else {
            f4 acc[NP][C::NTJ];
#pragma unroll
            for (int b = 0; b < NP; ++b)
#pragma unroll
                for (int t = 0; t < C::NTJ; ++t) acc[b][t] = f4{0, 0, 0, 0};
            const float* ckr = CK + row * CKS;
#pragma unroll 1
            for (int s = 0; s < C::KSJ; ++s) {
                bf8 rh[C::NTJ], rl[C::NTJ];
#pragma unroll
                for (int t = 0; t < C::NTJ; ++t) {
                    rh[t] = A.tabJ[((s * C::NTJ + t) * 2 + 0) * 64 + lane];
                    rl[t] = A.tabJ[((s * C::NTJ + t) * 2 + 1) * 64 + lane];
                }
                float hv[NP][8];
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    const int k = 32 * s + 8 * grp + jj;
                    if (k < C::KJ) {
                        const int q = k / DD, ab = k - (k / DD) * DD, a = ab / D, b = ab - (ab / D) * D;
                        const float* pd = PD + (row * NQ + q) * PDN;
                        const float sh = pd[a * D + b], w = pd[PDN - 1], m = ckr[DD + a * D + b];
                        float ka[D], kb[D];
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            ka[c] = pd[DD + c * D + a];
                            kb[c] = pd[DD + c * D + b];
                        }
                        int t = 0;
#pragma unroll
                        for (int c1 = 0; c1 < D; ++c1)
#pragma unroll
                            for (int c2 = c1; c2 < D; ++c2, ++t)
                                hv[t][jj] = w * ((c1 == c2 ? sh : 0.f) + lm * ka[c1] * kb[c2] + mu * ka[c2] * kb[c1] +
                                                 mu * pd[2 * DD + t] * m);
                    } else {
#pragma unroll
                        for (int t = 0; t < NP; ++t) hv[t][jj] = 0.f;
                    }
                }
#pragma unroll
                for (int b = 0; b < NP; ++b) {
                    const bf8 ah = svkb_split(hv[b], false), al = svkb_split(hv[b], true);
#pragma unroll
                    for (int t = 0; t < C::NTJ; ++t) {
                        acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, rh[t], acc[b][t], 0, 0, 0);
                        acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, rl[t], acc[b][t], 0, 0, 0);
                        acc[b][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, rh[t], acc[b][t], 0, 0, 0);
                    }
                }
            }
            // |det J| of this lane's four rows, read before the staging
            // overwrites the cell constants
            float adv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) adv[v] = CK[(4 * grp + v) * CKS + 2 * DD];
            wave_sync();  // the point data are dead: the wave's area stages the tensors
            float* stg = U;
            float* out = reinterpret_cast<float*>(A.out);
            constexpr int CR = C::CR;
#pragma unroll 1
            for (int r0 = 0; r0 < 16; r0 += CR) {
                if (cell0 + r0 >= A.ncells) break;  // wave-uniform
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rc = 4 * grp + v;
                    if (rc < r0 || rc >= r0 + CR) continue;
                    const float ad = adv[v];
                    float* sc = stg + (rc - r0) * N * N;
                    int bi = 0;
#pragma unroll
                    for (int c1 = 0; c1 < D; ++c1)
#pragma unroll
                        for (int c2 = c1; c2 < D; ++c2, ++bi)
#pragma unroll
                            for (int t = 0; t < C::NTJ; ++t) {
                                const int n = 16 * t + row;
                                if (n >= NS * NS) continue;
                                const int a = n / NS, b = n - (n / NS) * NS;
                                const float val = ad * acc[bi][t][v];
                                sc[(c1 * NS + a) * N + c2 * NS + b] = val;
                                if (c1 != c2) sc[(c2 * NS + b) * N + c1 * NS + a] = val;
                            }
                }
                wave_sync();
                const int nc = CR < 16 - r0 ? CR : 16 - r0;
                const int nr = (int)(A.ncells - (cell0 + r0) < nc ? A.ncells - (cell0 + r0) : nc);
                const int nvec = nr * N * N / 4;
                const svkb_u32x4* s4 = reinterpret_cast<const svkb_u32x4*>(stg);
                svkb_u32x4* o4 = reinterpret_cast<svkb_u32x4*>(out + (cell0 + r0) * (int64_t)N * N);
                for (int i = lane; i < nvec; i += 64) __builtin_nontemporal_store(s4[i], &o4[i]);
                wave_sync();
            }
        }
        wave_sync();  // the next tile rewrites the wave's LDS
    }
}

}  // namespace dev

namespace {

uint16_t host_bf16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float host_bf16_float(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
uint16_t split_part(long double x, int part) {  // part 0 hi, 1 lo
    const float f = (float)x;
    const uint16_t hi = host_bf16(f);
    return part == 0 ? hi : host_bf16(f - host_bf16_float(hi));
}

struct SvkBTables {
    void* ptr = nullptr;
    const dev::bf8 *I = nullptr, *R = nullptr, *J = nullptr;
    const float* W = nullptr;
};

std::mutex g_mu;
std::map<std::tuple<int, int, int, int>, SvkBTables> g_tabs;  // (dev, dim, p, q)

// Tables of one (dim, p, q): the rule is the one the FP64 kernels use (P1: one
// point with the summed weight; P2: the fully symmetric rule of degree q).
coffee_status svkb_tables(int devid, int dim, int p, int q, SvkBTables* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    const auto key = std::make_tuple(devid, dim, p, q);
    auto it = g_tabs.find(key);
    if (it != g_tabs.end()) {
        *out = it->second;
        return COFFEE_OK;
    }
    Tables t;
    if (!t.init(dim, p, p == 2 ? COFFEE_QUAD(q & 15, COFFEE_RULE_SYMMETRIC) : q)) return COFFEE_E_INVALID_ARG;
    const int NS = t.n, D = dim, DD = D * D;
    const int NQ = p == 1 ? 1 : t.nq;
    std::vector<long double> W(NQ), dphi((size_t)D * NQ * NS);  // dphi[al][q][r]
    if (p == 1) {
        long double s = 0;
        for (int k = 0; k < t.nq; ++k) s += t.W[k];
        W[0] = s;
    } else {
        for (int k = 0; k < NQ; ++k) W[k] = t.W[k];
    }
    for (int al = 0; al < D; ++al)
        for (int k = 0; k < NQ; ++k)
            for (int r = 0; r < NS; ++r) dphi[((size_t)al * NQ + k) * NS + r] = t.dphi[((size_t)al * t.nq + k) * NS + r];
    auto dp = [&](int al, int k, int r) { return dphi[((size_t)al * NQ + k) * NS + r]; };
    const int NQA = NQ * D, NTU = (NQA + 15) / 16, KSR = (3 * NQA + 31) / 32;
    const int KJ = NQ * DD, KSJ = (KJ + 31) / 32, NTJ = (NS * NS + 15) / 16;
    // interpolation: B rows k = part NS + r (parts D_hi, D_lo, D_hi), column (q, al)
    std::vector<uint16_t> tI((size_t)NTU * 64 * 8, 0);
    for (int tt = 0; tt < NTU; ++tt)
        for (int l = 0; l < 64; ++l)
            for (int jj = 0; jj < 8; ++jj) {
                const int k = 8 * (l / 16) + jj, j = 16 * tt + l % 16;
                if (k >= 3 * NS || j >= NQA) continue;
                const int part = k / NS, r = k % NS;
                tI[((size_t)tt * 64 + l) * 8 + jj] = split_part(dp(j % D, j / D, r), part == 1 ? 1 : 0);
            }
    // residual: B rows k = part NQA + (q, al), column a
    std::vector<uint16_t> tR((size_t)KSR * 64 * 8, 0);
    for (int s = 0; s < KSR; ++s)
        for (int l = 0; l < 64; ++l)
            for (int jj = 0; jj < 8; ++jj) {
                const int k = 32 * s + 8 * (l / 16) + jj, a = l % 16;
                if (k >= 3 * NQA || a >= NS) continue;
                const int part = k / NQA, j = k % NQA;
                tR[((size_t)s * 64 + l) * 8 + jj] = split_part(dp(j % D, j / D, a), part == 1 ? 1 : 0);
            }
    // Jacobian: R[(q, al, be)][(i, j)] = dphi_i/dX_al(q) dphi_j/dX_be(q), hi and lo
    std::vector<uint16_t> tJ((size_t)KSJ * NTJ * 2 * 64 * 8, 0);
    for (int s = 0; s < KSJ; ++s)
        for (int tt = 0; tt < NTJ; ++tt)
            for (int part = 0; part < 2; ++part)
                for (int l = 0; l < 64; ++l)
                    for (int jj = 0; jj < 8; ++jj) {
                        const int k = 32 * s + 8 * (l / 16) + jj, n = 16 * tt + l % 16;
                        if (k >= KJ || n >= NS * NS) continue;
                        const int q = k / DD, ab = k % DD, al = ab / D, be = ab % D, i = n / NS, j = n % NS;
                        tJ[((((size_t)s * NTJ + tt) * 2 + part) * 64 + l) * 8 + jj] =
                            split_part(dp(al, q, i) * dp(be, q, j), part);
                    }
    std::vector<float> tW(NQ);
    for (int k = 0; k < NQ; ++k) tW[k] = (float)W[k];
    const size_t bI = tI.size() * 2, bR = tR.size() * 2, bJ = tJ.size() * 2, bW = tW.size() * 4;
    const size_t oR = (bI + 255) / 256 * 256, oJ = oR + (bR + 255) / 256 * 256, oW = oJ + (bJ + 255) / 256 * 256;
    std::vector<char> buf(oW + bW);
    std::memcpy(buf.data(), tI.data(), bI);
    std::memcpy(buf.data() + oR, tR.data(), bR);
    std::memcpy(buf.data() + oJ, tJ.data(), bJ);
    std::memcpy(buf.data() + oW, tW.data(), bW);
    void* d = nullptr;
    if (hipMalloc(&d, buf.size()) != hipSuccess) return COFFEE_E_NOMEM;
    if (hipMemcpy(d, buf.data(), buf.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return COFFEE_E_HIP;
    }
    SvkBTables T;
    T.ptr = d;
    T.I = reinterpret_cast<const dev::bf8*>(d);
    T.R = reinterpret_cast<const dev::bf8*>((char*)d + oR);
    T.J = reinterpret_cast<const dev::bf8*>((char*)d + oJ);
    T.W = reinterpret_cast<const float*>((char*)d + oW);
    g_tabs[key] = T;
    *out = T;
    return COFFEE_OK;
}

template <int D, int P, int NQ, int MODE>
hipError_t launch_svkb(const dev::SvkBArgs& a, hipStream_t s, int ncu) {
    using C = dev::SvkBCfg<D, P, NQ>;
    const int lds = 4 * C::template wave_floats<MODE>() * (int)sizeof(float);
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::k_svk_bf16<D, P, NQ, MODE>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (attr != hipSuccess) return attr;
    const int64_t wgs = (a.ntiles + 3) / 4;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(wgs, (int64_t)ncu * (lds <= 80 * 1024 ? 2 : 1)));
    hipLaunchKernelGGL((dev::k_svk_bf16<D, P, NQ, MODE>), dim3(grid), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <int D, int P, int NQ>
hipError_t launch_svkb_form(int form, const dev::SvkBArgs& a, hipStream_t s, int ncu) {
    if (form == COFFEE_SVK_ENERGY) return launch_svkb<D, P, NQ, 0>(a, s, ncu);
    if (form == COFFEE_SVK_RESIDUAL) return launch_svkb<D, P, NQ, 1>(a, s, ncu);
    return launch_svkb<D, P, NQ, 2>(a, s, ncu);
}

}  // namespace

coffee_status assemble_svk_bf16(int form, int cell, int degree, int q, const double* coords, const int32_t* c2v,
                                int64_t ncells, const coffee_field* coeffs, const double* constants, int nconst,
                                void* out, void* hip_stream) {
    if (coeffs[0].degree != degree) return COFFEE_E_UNSUPPORTED;
    const int qd = q & 15;
    const bool known = (degree == 1 && qd == 2) || (degree == 2 && qd == 4);
    if (!known) return COFFEE_E_UNSUPPORTED;
    if (ncells == 0) return COFFEE_OK;
    int devid = 0;
    if (hipGetDevice(&devid) != hipSuccess) return COFFEE_E_HIP;
    SvkBTables T;
    coffee_status st = svkb_tables(devid, cell, degree, q, &T);
    if (st != COFFEE_OK) return st;
    dev::SvkBArgs a;
    std::memset(&a, 0, sizeof a);
    a.coords = coords;
    a.c2v = c2v;
    a.ncells = ncells;
    a.u = dev::FieldArg{coeffs[0].values, coeffs[0].cell_to_dof};
    a.mu = (float)(nconst > 0 ? constants[0] : 1.0);
    a.lambda = (float)(nconst > 1 ? constants[1] : 1.0);
    a.tabI = T.I;
    a.tabR = T.R;
    a.tabJ = T.J;
    a.W = T.W;
    a.out = out;
    a.ntiles = (ncells + 15) / 16;
    const hipStream_t s = (hipStream_t)hip_stream;
    const int ncu = num_cu(devid);
    hipError_t e = hipSuccess;
    if (cell == 2 && degree == 1) e = launch_svkb_form<2, 1, 1>(form, a, s, ncu);
    else if (cell == 2) e = launch_svkb_form<2, 2, 6>(form, a, s, ncu);
    else if (degree == 1) e = launch_svkb_form<3, 1, 1>(form, a, s, ncu);
    else e = launch_svkb_form<3, 2, 14>(form, a, s, ncu);
    return e == hipSuccess ? COFFEE_OK : COFFEE_E_HIP;
}

void free_svkb_tables() {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_tabs) {
        (void)hipSetDevice(std::get<0>(kv.first));
        (void)hipFree(kv.second.ptr);
    }
    g_tabs.clear();
}

}  // namespace coffee
