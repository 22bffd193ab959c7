// Reverse mode of the linear-form assembly.
//
// For a bilinear form the per-cell functional S_e = lam_e^T A_e u_e equals
// sum_blk sum_k G^blk_k T^blk_k with T^blk_k = lam_{c1}^T R_k u_{c2}: the
// reference tensors are contracted with the test and trial vectors once, and
// the geometry tensor G carries every dependence on the cell. The transpose of
// the G builder (reverse_G, beside build_G in linear.hpp) maps Gbar = T to
// Kbar = dS/dK and to the bars of the local coefficient dofs; every term of G
// is linear in |det J|, so dS/d|det J| = S / |det J|. The chain to the vertex
// coordinates is analytic:
//     dK = -K dJ K  ->  Jbar = -K^T Kbar K^T,
//     d|det J| = |det J| tr(K dJ)  ->  Jbar += Sbar_adet |det J| K^T,
//     J = [x1 - x0, ..., xd - x0]  ->  xbar_{j+1} = Jbar[:, j], xbar_0 = -sum_j Jbar[:, j].
// One thread per cell; gradients are scatter-added with FP64 atomics.
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

struct AdjArgs {
    LinArgs L;               // mesh, fields, constants (rfrag/out unused)
    const double* R;         // reference tensors [KR][NS * NS]
    const double* lam;       // [E][N]
    const double* u;         // [E][N]
    double seed;
    double* grad_coords;     // [V][D]
    double* grad_f0;         // shaped like f0 values, or NULL
    double* grad_f1;
    double* cell_value;      // [E] or NULL
    // deterministic mode: per-cell contributions written here instead of
    // scatter-added (scatter.hip sums them in a fixed order); NULL otherwise
    double* det_x;           // [E][D+1][D]
    double* det_f0;          // [E][nloc][ncomp of field 0]
    double* det_f1;          // [E][nloc]
};

template <int FORM, int D, int FD>
struct AdjDirs {
    static constexpr int NF = nfield(D, FD);
    static constexpr int WC = (FORM == F_BURG) ? D : 1;
    static constexpr int N0 = FD > 0 ? NF * WC : 0;                      // field 0 dofs
    static constexpr int N1 = (FORM == F_ELAST && FD > 0) ? NF : 0;      // field 1 dofs
};

// Accumulate the contribution of block B: value, Kbar and coefficient bars.
template <int FORM, int D, int P, int FD, int B>
__device__ inline void adjoint_block(const AdjArgs& A, const double* Rs, const CellData<FORM, D, FD, double>& cd,
                                     const double* lam_e,
                                     const double* u_e, double& S, double (&Kbar)[D][D], double* f0bar,
                                     double* f1bar) {
    constexpr int NS = nsc(D, P), NN = NS * NS;
    constexpr int NC = ncomp_space(FORM, D);
    constexpr int C1 = B / NC, C2 = B % NC;
    // the block's rows of lam_e and u_e (re-read per block from the L1 cache)
    double lam[NS], u[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        lam[i] = lam_e[C1 * NS + i];
        u[i] = u_e[C2 * NS + i];
    }
    // gbar(k) = T_k = lam_c1^T R_k u_c2 (R_k read with wave-uniform addresses)
    auto gbar = [&](int k) -> double {
        // keeps the compiler from hoisting every R_k load of the block into
        // registers at once
        asm volatile("" ::: "memory");
        const double* Rk = Rs + (size_t)k * NN;
        double t = 0.0;
#pragma unroll 1
        for (int a = 0; a < NS; ++a) {
            double r = 0.0;
#pragma unroll
            for (int b = 0; b < NS; ++b) r += Rk[a * NS + b] * u[b];
            t += lam[a] * r;
        }
        return t;
    };
    reverse_G<FORM, D, FD, C1, C2>(cd, A.L, gbar, S, Kbar, f0bar, f1bar);
}

// One block per iteration of a runtime loop, so that the compiler keeps one
// block's temporaries live at a time.
template <int FORM, int D, int P, int FD, int B, int NB>
__device__ inline void adjoint_block_switch(int b, const AdjArgs& A, const double* Rs,
                                            const CellData<FORM, D, FD, double>& cd, const double* lam,
                                            const double* u, double& S, double (&Kbar)[D][D], double* f0bar,
                                            double* f1bar) {
    if constexpr (B < NB) {
        if (b == B) adjoint_block<FORM, D, P, FD, B>(A, Rs, cd, lam, u, S, Kbar, f0bar, f1bar);
        else adjoint_block_switch<FORM, D, P, FD, B + 1, NB>(b, A, Rs, cd, lam, u, S, Kbar, f0bar, f1bar);
    }
}

template <int FORM, int D, int P, int FD, int NB>
__device__ inline void adjoint_blocks(const AdjArgs& A, const double* Rs, const CellData<FORM, D, FD, double>& cd,
                                      const double* lam, const double* u, double& S, double (&Kbar)[D][D],
                                      double* f0bar, double* f1bar) {
#pragma unroll 1
    for (int b = 0; b < NB; ++b)
        adjoint_block_switch<FORM, D, P, FD, 0, NB>(b, A, Rs, cd, lam, u, S, Kbar, f0bar, f1bar);
}

// Reference tensors of the adjoint kernels live in LDS when they fit.
template <int FORM, int D, int P, int FD>
constexpr int adj_r_elems() { return kref(FORM, D, FD) * nsc(D, P) * nsc(D, P); }
template <int FORM, int D, int P, int FD>
constexpr bool adj_r_in_lds() { return adj_r_elems<FORM, D, P, FD>() * 8 <= 56 * 1024; }

template <int FORM, int D, int P, int FD>
__global__ __launch_bounds__(256) void k_adjoint_linear(AdjArgs A) {
    constexpr int NS = nsc(D, P);
    constexpr int NC = ncomp_space(FORM, D);
    constexpr int N = NC * NS;
    using Dirs = AdjDirs<FORM, D, FD>;
    constexpr bool LDSR = adj_r_in_lds<FORM, D, P, FD>();
    constexpr int RE = adj_r_elems<FORM, D, P, FD>();
    __shared__ double sR[LDSR ? RE : 1];
    const double* Rs = A.R;
    if constexpr (LDSR) {
        for (int i = threadIdx.x; i < RE; i += blockDim.x) sR[i] = A.R[i];
        __syncthreads();
        Rs = sR;
    }
    // per-wave combining of the gradient scatter-adds (vertex coordinates and
    // the fields' dofs)
    constexpr int TS = 128;
    constexpr int W0 = Dirs::N0 > 0 ? Dirs::WC : 1;
    __shared__ unsigned long long ckx[4][TS], ck0[4][TS], ck1[4][TS];
    __shared__ double cvx[4][TS * D], cv0[4][TS * W0], cv1[4][TS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // wave-uniform loop: every lane takes part in the tables' clear and flush
    for (int64_t wbase = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) - lane; wbase < A.L.ncells;
         wbase += (int64_t)gridDim.x * blockDim.x) {
        const bool valid = wbase + lane < A.L.ncells;
        const int64_t cell = valid ? wbase + lane : A.L.ncells - 1;
        const bool det = A.det_x != nullptr;  // same in every lane
        if (!det) {
            combine_clear<D, TS>(ckx[wave], cvx[wave], lane);
            if constexpr (Dirs::N0 > 0) combine_clear<W0, TS>(ck0[wave], cv0[wave], lane);
            if constexpr (Dirs::N1 > 0) combine_clear<1, TS>(ck1[wave], cv1[wave], lane);
            wave_sync();
        }
        CellIdx<FORM, D, FD> ix;
        CellRaw<FORM, D, FD> raw;
        load_idx<FORM, D, FD>(A.L, cell, ix);
        load_raw<FORM, D, FD>(A.L, cell, ix, raw);
        CellData<FORM, D, FD, double> cd;
        cell_from_raw<FORM, D, FD>(raw, cd);
        const double* lam = A.lam + cell * N;
        const double* u = A.u + cell * N;
        double S = 0.0, Kbar[D][D];
        double f0bar[Dirs::N0 > 0 ? Dirs::N0 : 1], f1bar[Dirs::N1 > 0 ? Dirs::N1 : 1];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) Kbar[i][j] = 0.0;
#pragma unroll
        for (int r = 0; r < (Dirs::N0 > 0 ? Dirs::N0 : 1); ++r) f0bar[r] = 0.0;
#pragma unroll
        for (int r = 0; r < (Dirs::N1 > 0 ? Dirs::N1 : 1); ++r) f1bar[r] = 0.0;
        adjoint_blocks<FORM, D, P, FD, NC * NC>(A, Rs, cd, lam, u, S, Kbar, f0bar, f1bar);
        if (A.cell_value && valid) A.cell_value[cell] = S;

        // chain to the coordinates
        const auto& K = cd.g.K;
        const double adbar_ad = S;  // d S / d|det J| * |det J|
        double Jbar[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                // -(K^T Kbar K^T)_ij = -sum_ab K[a][i] Kbar[a][b] K[j][b]
                double s = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int b = 0; b < D; ++b) s += K[a][i] * Kbar[a][b] * K[j][b];
                Jbar[i][j] = -s + adbar_ad * K[j][i];
            }
        const double sd = A.seed;
        if (valid) {
            double vx[D + 1][D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double x0 = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    vx[j + 1][i] = sd * Jbar[i][j];
                    x0 -= Jbar[i][j];
                }
                vx[0][i] = sd * x0;
            }
            if (det) {
#pragma unroll
                for (int v = 0; v <= D; ++v)
#pragma unroll
                    for (int i = 0; i < D; ++i) A.det_x[(cell * (D + 1) + v) * D + i] = vx[v][i];
                if constexpr (Dirs::N0 > 0) {
#pragma unroll
                    for (int r = 0; r < Dirs::N0; ++r) A.det_f0[cell * Dirs::N0 + r] = sd * f0bar[r];
                }
                if constexpr (Dirs::N1 > 0) {
#pragma unroll
                    for (int r = 0; r < Dirs::N1; ++r) A.det_f1[cell * Dirs::N1 + r] = sd * f1bar[r];
                }
            } else {
                if (A.grad_coords) {
#pragma unroll
                    for (int v = 0; v <= D; ++v)
                        combine_add<D, TS>(ckx[wave], cvx[wave], (unsigned long long)ix.v[v], vx[v], A.grad_coords);
                }
                if constexpr (Dirs::N0 > 0) {
                    if (A.grad_f0) {
                        constexpr int NF = Dirs::NF;
#pragma unroll
                        for (int r = 0; r < NF; ++r) {
                            const int64_t key = A.L.f0.map ? (int64_t)ix.f0[r] : cell * NF + r;
                            double v[W0];
#pragma unroll
                            for (int c = 0; c < W0; ++c) v[c] = sd * f0bar[r * W0 + c];
                            combine_add<W0, TS>(ck0[wave], cv0[wave], (unsigned long long)key, v, A.grad_f0);
                        }
                    }
                }
                if constexpr (Dirs::N1 > 0) {
                    if (A.grad_f1) {
                        constexpr int NF = Dirs::NF;
#pragma unroll
                        for (int r = 0; r < NF; ++r) {
                            const int64_t key = A.L.f1.map ? (int64_t)ix.f1[r] : cell * NF + r;
                            const double v = sd * f1bar[r];
                            combine_add<1, TS>(ck1[wave], cv1[wave], (unsigned long long)key, &v, A.grad_f1);
                        }
                    }
                }
            }
        }
        if (!det) {
            wave_sync();
            if (A.grad_coords) combine_flush<D, TS>(ckx[wave], cvx[wave], A.grad_coords, lane);
            if constexpr (Dirs::N0 > 0) {
                if (A.grad_f0) combine_flush<W0, TS>(ck0[wave], cv0[wave], A.grad_f0, lane);
            }
            if constexpr (Dirs::N1 > 0) {
                if (A.grad_f1) combine_flush<1, TS>(ck1[wave], cv1[wave], A.grad_f1, lane);
            }
            wave_sync();
        }
    }
}

// Elasticity: the contraction T = lam_c1^T R_k u_c2 factored as
// V_k = R_k u_c2 (shared by the NC test components c1) and T = lam_c1 . V_k,
// consumed entry by entry: for k = (r, alpha, beta) and every block (c1, c2)
// the transpose of G's entry
//     G = |det J| (mu_r (delta_c1c2 (K K^T)_ab + K[a][c2] K[b][c1]) + lambda_r K[a][c1] K[b][c2])
// (the same arithmetic as reverse_G in linear.hpp, per entry instead of per
// block). lam_e stays in registers, u_e rows are re-read per dof r (L1), R is
// read through the scalar path (its addresses are the same in every lane; from
// LDS each wave-wide read of one value would cost as much LDS bandwidth as a
// read of 64 different values). Per cell: NF D^2 NC (NS^2 +
// NC NS) multiply-adds for the values (14k for P2 tetrahedra, against 32k for
// the per-block contraction), and the dof r's coefficient bars are added to
// the global gradients as soon as its loop ends.
template <int D, typename T>
__device__ inline T sel_rt(const T* x, int n, int r) {
    T v = T(0);
    for (int j = 0; j < n; ++j) v += (r == j ? T(1) : T(0)) * x[j];
    return v;
}

template <int D, int P, int FD>
__global__ __launch_bounds__(256, 2) void k_adjoint_elast(AdjArgs A) {
    constexpr int NS = nsc(D, P), NN = NS * NS, NC = D, N = NC * NS;
    constexpr int NF = nfield(D, FD), KR = NF * D * D;
    (void)KR;
    // per-wave combining of the gradient scatter-adds (vertex coordinates,
    // then the two fields' dofs)
    constexpr int TS = 256;
    __shared__ unsigned long long ckx[4][TS], ckf[4][2][TS];
    __shared__ double cvx[4][TS * D], cvf[4][2][TS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // wave-uniform loop: every lane takes part in the tables' clear and flush
    for (int64_t base = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) - lane; base < A.L.ncells;
         base += (int64_t)gridDim.x * blockDim.x) {
        const bool valid = base + lane < A.L.ncells;
        const int64_t cell = valid ? base + lane : A.L.ncells - 1;
        const bool det = A.det_x != nullptr;  // same in every lane
        if (!det) {
            combine_clear<D, TS>(ckx[wave], cvx[wave], lane);
            combine_clear<1, TS>(ckf[wave][0], cvf[wave][0], lane);
            combine_clear<1, TS>(ckf[wave][1], cvf[wave][1], lane);
            wave_sync();
        }
        CellIdx<F_ELAST, D, FD> ix;
        CellRaw<F_ELAST, D, FD> raw;
        load_idx<F_ELAST, D, FD>(A.L, cell, ix);
        load_raw<F_ELAST, D, FD>(A.L, cell, ix, raw);
        CellData<F_ELAST, D, FD, double> cd;
        cell_from_raw<F_ELAST, D, FD>(raw, cd);
        const auto& K = cd.g.K;
        const double ad = cd.g.adet;
        const double* lam_e = A.lam + cell * N;
        const double* u_e = A.u + cell * N;
        double lam[N];
#pragma unroll
        for (int i = 0; i < N; ++i) lam[i] = lam_e[i];
        double S = 0.0, Kbar[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) Kbar[i][j] = 0.0;
#pragma unroll 1
        for (int r = 0; r < NF; ++r) {
            const double mu = FD > 0 ? sel_rt<D>(cd.f0, NF, r) : A.L.c0;
            const double lm = FD > 0 ? sel_rt<D>(cd.f1, NF, r) : A.L.c1;
            double mub = 0.0, lmb = 0.0;
#pragma unroll
            for (int c2 = 0; c2 < NC; ++c2) {
                double u[NS];
#pragma unroll
                for (int b = 0; b < NS; ++b) u[b] = u_e[c2 * NS + b];
                // (alpha, beta) in a rolled loop; the rows K[alpha][.] and
                // K[beta][.] are picked arithmetically and the Kbar updates of
                // the two rows collected in xa, xb and added back the same way
#pragma unroll 1
                for (int ab = 0; ab < D * D; ++ab) {
                    const int al = ab / D, be = ab - (ab / D) * D;
                    double Ka[D], Kb[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) {
                        double x = 0.0, y = 0.0;
#pragma unroll
                        for (int row = 0; row < D; ++row) {
                            x += (row == al ? 1.0 : 0.0) * K[row][i];
                            y += (row == be ? 1.0 : 0.0) * K[row][i];
                        }
                        Ka[i] = x;
                        Kb[i] = y;
                    }
                    const double* Rk = A.R + (r * D * D + ab) * NN;
                    double V[NS];
#pragma unroll
                    for (int a = 0; a < NS; ++a) {
                        double v = 0.0;
#pragma unroll
                        for (int b = 0; b < NS; ++b) v += cload(Rk + a * NS + b) * u[b];
                        V[a] = v;
                    }
                    double kk = 0.0;  // (K K^T)_{alpha beta}
#pragma unroll
                    for (int i = 0; i < D; ++i) kk += Ka[i] * Kb[i];
                    double xa[D], xb[D];
#pragma unroll
                    for (int i = 0; i < D; ++i) xa[i] = xb[i] = 0.0;
#pragma unroll
                    for (int c1 = 0; c1 < NC; ++c1) {
                        double g = 0.0;
#pragma unroll
                        for (int a = 0; a < NS; ++a) g += lam[c1 * NS + a] * V[a];
                        const double gb = ad * g;
                        mub += gb * ((c1 == c2 ? kk : 0.0) + Ka[c2] * Kb[c1]);
                        lmb += gb * Ka[c1] * Kb[c2];
                        const double gm = gb * mu, gl = gb * lm;
                        if (c1 == c2) {
#pragma unroll
                            for (int i = 0; i < D; ++i) {
                                xa[i] += gm * Kb[i];
                                xb[i] += gm * Ka[i];
                            }
                        }
                        xa[c2] += gm * Kb[c1];
                        xb[c1] += gm * Ka[c2];
                        xa[c1] += gl * Kb[c2];
                        xb[c2] += gl * Ka[c1];
                    }
#pragma unroll
                    for (int row = 0; row < D; ++row) {
                        const double wa = row == al ? 1.0 : 0.0, wb = row == be ? 1.0 : 0.0;
#pragma unroll
                        for (int i = 0; i < D; ++i) Kbar[row][i] += wa * xa[i] + wb * xb[i];
                    }
                }
            }
            S += mu * mub + lm * lmb;
            if constexpr (FD > 0) {
                if (det) {
                    if (valid) {
                        A.det_f0[cell * NF + r] = A.seed * mub;
                        A.det_f1[cell * NF + r] = A.seed * lmb;
                    }
                } else if (A.grad_f0 && valid) {
                    const int64_t i0 = A.L.f0.map ? (int64_t)A.L.f0.map[cell * NF + r] : cell * NF + r;
                    const double x = A.seed * mub;
                    combine_add<1, TS>(ckf[wave][0], cvf[wave][0], (unsigned long long)i0, &x, A.grad_f0);
                }
                if (!det && A.grad_f1 && valid) {
                    const int64_t i1 = A.L.f1.map ? (int64_t)A.L.f1.map[cell * NF + r] : cell * NF + r;
                    const double x = A.seed * lmb;
                    combine_add<1, TS>(ckf[wave][1], cvf[wave][1], (unsigned long long)i1, &x, A.grad_f1);
                }
            }
        }
        if (A.cell_value && valid) A.cell_value[cell] = S;
        // chain to the coordinates (as in k_adjoint_linear)
        double Jbar[D][D];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                double t = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int b = 0; b < D; ++b) t += K[a][i] * Kbar[a][b] * K[j][b];
                Jbar[i][j] = -t + S * K[j][i];
            }
        const double sd = A.seed;
        if (valid) {
            double vx[D + 1][D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double x0 = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    vx[j + 1][i] = sd * Jbar[i][j];
                    x0 -= Jbar[i][j];
                }
                vx[0][i] = sd * x0;
            }
            if (det) {
#pragma unroll
                for (int v = 0; v <= D; ++v)
#pragma unroll
                    for (int i = 0; i < D; ++i) A.det_x[(cell * (D + 1) + v) * D + i] = vx[v][i];
            } else if (A.grad_coords) {
#pragma unroll
                for (int v = 0; v <= D; ++v)
                    combine_add<D, TS>(ckx[wave], cvx[wave], (unsigned long long)ix.v[v], vx[v], A.grad_coords);
            }
        }
        if (!det) {
            wave_sync();
            if (A.grad_coords) combine_flush<D, TS>(ckx[wave], cvx[wave], A.grad_coords, lane);
            if (A.grad_f0) combine_flush<1, TS>(ckf[wave][0], cvf[wave][0], A.grad_f0, lane);
            if (A.grad_f1) combine_flush<1, TS>(ckf[wave][1], cvf[wave][1], A.grad_f1, lane);
            wave_sync();
        }
    }
}

}  // namespace dev

typedef hipError_t (*AdjLaunch)(const dev::AdjArgs&, hipStream_t, int grid);
struct AdjEntry {
    int form, dim, p, fd;
    AdjLaunch launch;
};

// Elasticity uses the factored kernel when its reference tensor fits in LDS.
template <int FORM, int D, int P, int FD>
hipError_t launch_adjoint(const dev::AdjArgs& a, hipStream_t s, int grid) {
    if constexpr (FORM == dev::F_ELAST && dev::adj_r_in_lds<FORM, D, P, FD>())
        hipLaunchKernelGGL((dev::k_adjoint_elast<D, P, FD>), dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((dev::k_adjoint_linear<FORM, D, P, FD>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

static const std::vector<AdjEntry>& adj_registry() {
    using namespace dev;
    static const std::vector<AdjEntry> reg = {
        {F_MASS, 2, 1, 1, &launch_adjoint<F_MASS, 2, 1, 1>},
        {F_MASS, 3, 1, 1, &launch_adjoint<F_MASS, 3, 1, 1>},
        {F_MASS, 3, 2, 2, &launch_adjoint<F_MASS, 3, 2, 2>},
        {F_HELM, 2, 1, 1, &launch_adjoint<F_HELM, 2, 1, 1>},
        {F_HELM, 2, 2, 1, &launch_adjoint<F_HELM, 2, 2, 1>},
        {F_HELM, 3, 1, 1, &launch_adjoint<F_HELM, 3, 1, 1>},
        {F_HELM, 3, 2, 2, &launch_adjoint<F_HELM, 3, 2, 2>},
        {F_ELAST, 2, 1, 1, &launch_adjoint<F_ELAST, 2, 1, 1>},
        {F_ELAST, 2, 2, 1, &launch_adjoint<F_ELAST, 2, 2, 1>},
        {F_ELAST, 3, 1, 1, &launch_adjoint<F_ELAST, 3, 1, 1>},
        {F_ELAST, 3, 2, 1, &launch_adjoint<F_ELAST, 3, 2, 1>},
        {F_BURG, 2, 1, 1, &launch_adjoint<F_BURG, 2, 1, 1>},
        {F_BURG, 3, 1, 1, &launch_adjoint<F_BURG, 3, 1, 1>},
        {F_BURG, 3, 2, 2, &launch_adjoint<F_BURG, 3, 2, 2>},
        {F_DIFF, 2, 1, 0, &launch_adjoint<F_DIFF, 2, 1, 0>},
        {F_DIFF, 2, 2, 0, &launch_adjoint<F_DIFF, 2, 2, 0>},
        {F_DIFF, 3, 1, 0, &launch_adjoint<F_DIFF, 3, 1, 0>},
        {F_DIFF, 3, 2, 0, &launch_adjoint<F_DIFF, 3, 2, 0>},
    };
    return reg;
}

static std::mutex g_adj_mu;
static std::map<std::tuple<int, int, int, int, int, int>, void*> g_adj_tables;  // (dev, form, dim, p, q, fd)

// FP64 reference tensors [KR][NS * NS] (unpacked), host values.
bool r64_table(int form, int dim, int p, int q, int fd, std::vector<double>& h) {
    RefTensor R;
    if (!build_reference(form, dim, p, q, fd, R)) return false;
    h.resize(R.R.size());
    for (size_t i = 0; i < h.size(); ++i) h[i] = (double)R.R[i];
    return true;
}

// FP64 reference tensors [KR][NS * NS] (unpacked), built and uploaded on first
// use; shared by the adjoint kernels and the degree-1 FMA kernels.
coffee_status reference_table_f64(int dev, int form, int dim, int p, int q, int fd, const double** out) {
    std::lock_guard<std::mutex> lk(g_adj_mu);
    auto key = std::make_tuple(dev, form, dim, p, q, fd);
    auto it = g_adj_tables.find(key);
    if (it != g_adj_tables.end()) {
        *out = (const double*)it->second;
        return COFFEE_OK;
    }
    std::vector<double> h;
    if (!r64_table(form, dim, p, q, fd, h)) return COFFEE_E_INVALID_ARG;
    void* d = nullptr;
    if (hipMalloc(&d, h.size() * sizeof(double)) != hipSuccess) return COFFEE_E_NOMEM;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return COFFEE_E_HIP;
    }
    g_adj_tables[key] = d;
    *out = (const double*)d;
    return COFFEE_OK;
}

void free_adjoint_tables() {
    std::lock_guard<std::mutex> lk(g_adj_mu);
    for (auto& kv : g_adj_tables) {
        (void)hipSetDevice(std::get<0>(kv.first));
        (void)hipFree(kv.second);
    }
    g_adj_tables.clear();
}

coffee_status adjoint_linear(int form, int cell, int degree, int q, int fd, const double* coords, int64_t nvert,
                             const int32_t* c2v, int64_t ncells, const coffee_field* coeffs, int ncoeff,
                             const double* constants, int nconst, const double* lam, const double* u,
                             double seed, double* grad_coords, double* const* grad_coeff_values,
                             double* cell_value, const DetTarget* det, void* hip_stream) {
    const AdjEntry* e = nullptr;
    for (const AdjEntry& x : adj_registry())
        if (x.form == form && x.dim == cell && x.p == degree && x.fd == fd) e = &x;
    if (!e) return COFFEE_E_UNSUPPORTED;
    if (ncells > 0 && (!lam || !u)) return COFFEE_E_INVALID_ARG;
    if (ncells == 0) return COFFEE_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return COFFEE_E_HIP;
    const double* R = nullptr;
    coffee_status st = reference_table_f64(dev, form, cell, degree, q, fd, &R);
    if (st != COFFEE_OK) return st;
    dev::AdjArgs a;
    std::memset(&a, 0, sizeof a);
    a.L.coords = coords;
    a.L.c2v = c2v;
    a.L.ncells = ncells;
    if (ncoeff >= 1) a.L.f0 = dev::FieldArg{coeffs[0].values, coeffs[0].cell_to_dof};
    if (ncoeff >= 2) a.L.f1 = dev::FieldArg{coeffs[1].values, coeffs[1].cell_to_dof};
    if (form == COFFEE_BURGERS) {
        a.L.c0 = nconst > 0 ? constants[0] : 1.0;
        a.L.c1 = nconst > 1 ? constants[1] : 1.0;
    } else if (form == COFFEE_ELASTICITY && ncoeff == 0) {
        a.L.c0 = constants[0];
        a.L.c1 = constants[1];
    } else if (form == COFFEE_DIFFUSION) {
        a.L.c0 = (nconst > 0 ? constants[0] : 1.0) * (nconst > 1 ? constants[1] : 1.0);  // kappa dt
    }
    a.R = R;
    a.lam = lam;
    a.u = u;
    a.seed = seed;
    a.grad_coords = grad_coords;
    a.grad_f0 = (grad_coeff_values && ncoeff >= 1) ? grad_coeff_values[0] : nullptr;
    a.grad_f1 = (grad_coeff_values && ncoeff >= 2) ? grad_coeff_values[1] : nullptr;
    a.cell_value = cell_value;
    if (det) {
        a.det_x = det[0].local;
        a.det_f0 = ncoeff >= 1 ? det[1].local : nullptr;
        a.det_f1 = ncoeff >= 2 ? det[2].local : nullptr;
    }
    const int64_t blocks = (ncells + 255) / 256;
    const int grid = (int)std::min<int64_t>(blocks, (int64_t)num_cu(dev) * 8);
    if (e->launch(a, (hipStream_t)hip_stream, grid) != hipSuccess) return COFFEE_E_HIP;
    return COFFEE_OK;
}

}  // namespace coffee
