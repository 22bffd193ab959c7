// St Venant-Kirchhoff hyperelasticity: energy, residual and Jacobian, and the
// reverse pass of the energy.
//
// Per quadrature point (the paper's section 2 kernel structure, with the
// coefficient evaluated at the point as in Listing 2): the displacement
// gradient grad u = U K (U[i][a] = sum_r u_{r,i} dphi_r/dX_a in reference
// coordinates), F = I + grad u, E = (F^T F - I)/2, S = lambda tr(E) I + 2 mu E,
// P = F S, psi = lambda/2 tr(E)^2 + mu E:E. Then
//   energy   Pi_e = sum_q w_q |det J| psi
//   residual b_(c,a) = sum_q w_q |det J| sum_j P_cj dphi_a/dx_j
//   Jacobian A_(c,a),(c',b) = sum_q w_q |det J| sum_jl dphi_a/dx_j C_cjc'l dphi_b/dx_l,
// with the tangent C_cjc'l = delta_cc' S_lj + lambda F_cj F_c'l + mu F_cl F_c'j
// + mu delta_lj (F F^T)_cc' (the derivative of P along e_c' (x) e_l). In
// reference coordinates the Jacobian block is sum_q sum_ab dphi_a/dX_a H_ab
// dphi_b/dX_b with H = w |det J| K C K^T, accumulated as two rank-structured
// updates per point and reference direction.
//
// Work layout: energy, residual and the energy's reverse pass one thread per
// cell (the reverse pass also scatters the residual into the displacement
// gradient, and combines its scatter-adds per wave in LDS). Jacobian: a wave
// takes a few consecutive cells; F and K S K^T at each (cell, point) are formed
// once into LDS, then each lane accumulates a slice of rows of one block
// c <= c' (the mirrored block comes from the same values: the Jacobian is
// symmetric), and the cells' tensors are staged in LDS and written as
// contiguous 16-byte stores. Reference gradients and weights are read at
// wave-uniform addresses through the scalar path (staged in LDS where the
// Jacobian's lanes read different rows).
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

struct SvkArgs {
    const double* coords;
    const int32_t* c2v;
    int64_t ncells;
    FieldArg u;          // displacement, ncomp = D
    double mu, lambda;
    const double* tab;   // W[nq] then dphi[D][nq][NS]
    void* out;
    // reverse passes (energy; residual against lam)
    double seed;
    double* grad_coords;
    double* grad_u;
    double* cell_value;
    const double* lam;   // residual reverse pass: [E][D * NS] component-blocked
    // deterministic mode: per-cell contributions written here instead of
    // scatter-added (scatter.hip sums them in a fixed order); NULL otherwise
    double* det_x;       // [E][D+1][D]
    double* det_u;       // [E][NS][D]
};

// Reference-table read: through the scalar path when the address is the same
// in every lane (SC), else a plain (LDS) read.
template <bool SC>
__device__ inline double tread(const double* p) {
    if constexpr (SC) return cload(p);
    else return *p;
}

// F = I + U K at point q from the reference displacement gradient.
template <int D, int NS, bool SC = false>
__device__ inline void svk_F(const double (&uv)[NS * D], const double (&K)[D][D], const double* dphi_q, int nq,
                             double (&F)[D][D]) {
    double U[D][D];  // U[i][a] = sum_r u_{r,i} dphi_r/dX_a
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < NS; ++r) s += uv[r * D + i] * tread<SC>(dphi_q + (size_t)a * nq * NS + r);
            U[i][a] = s;
        }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double g = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) g += U[i][a] * K[a][j];
            F[i][j] = (i == j ? 1.0 : 0.0) + g;
        }
}

// S = lambda tr(E) I + 2 mu E with E = (F^T F - I) / 2.
template <int D>
__device__ inline void svk_S(const double (&F)[D][D], double mu, double lm, double (&S)[D][D]) {
    double E[D][D], trE = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) t += F[k][i] * F[k][j];
            E[i][j] = 0.5 * (t - (i == j ? 1.0 : 0.0));
        }
#pragma unroll
    for (int i = 0; i < D; ++i) trE += E[i][i];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) S[i][j] = (i == j ? lm * trE : 0.0) + 2.0 * mu * E[i][j];
}

// F, S, psi and P at point q from the reference displacement gradient, in
// the arithmetic type T (FP64, or FP32 for the FP32 energy and residual).
// E is formed from the displacement gradient H = grad u as (H + H^T + H^T H)/2,
// which equals (F^T F - I)/2 without the cancellation of F^T F against I.
template <int D, int NS, bool SC = false, typename T = double>
__device__ inline void svk_point(const T (&uv)[NS * D], const T (&K)[D][D], const double* dphi_q, int nq, T mu,
                                 T lm, T (&F)[D][D], T* psi, T (&Pout)[D][D]) {
    T U[D][D];  // U[i][a] = sum_r u_{r,i} dphi_r/dX_a
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T s = T(0);
#pragma unroll
            for (int r = 0; r < NS; ++r) s += uv[r * D + i] * (T)tread<SC>(dphi_q + (size_t)a * nq * NS + r);
            U[i][a] = s;
        }
    T H[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T g = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) g += U[i][a] * K[a][j];
            H[i][j] = g;
            F[i][j] = (i == j ? T(1) : T(0)) + g;
        }
    T E[D][D], trE = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T t = H[i][j] + H[j][i];
#pragma unroll
            for (int k = 0; k < D; ++k) t += H[k][i] * H[k][j];
            E[i][j] = T(0.5) * t;
        }
#pragma unroll
    for (int i = 0; i < D; ++i) trE += E[i][i];
    T S[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) S[i][j] = (i == j ? lm * trE : T(0)) + T(2) * mu * E[i][j];
    if (psi) {
        T EE = T(0);
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) EE += E[i][j] * E[i][j];
        *psi = T(0.5) * lm * trE * trE + mu * EE;
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T t = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) t += F[i][k] * S[k][j];
            Pout[i][j] = t;
        }
}

template <int D, int NS>
__device__ inline void svk_load(const SvkArgs& A, int64_t cell, Geom<D>& g, double (&uv)[NS * D],
                                int (&vid)[D + 1], int (&uid)[NS]) {
    double x[D + 1][D];
#pragma unroll
    for (int v = 0; v <= D; ++v) vid[v] = A.c2v[cell * (D + 1) + v];
#pragma unroll
    for (int v = 0; v <= D; ++v)
#pragma unroll
        for (int i = 0; i < D; ++i) x[v][i] = A.coords[(int64_t)vid[v] * D + i];
    geometry_from_coords<D>(x, g);
    if (A.u.map) {
#pragma unroll
        for (int r = 0; r < NS; ++r) uid[r] = A.u.map[cell * NS + r];
    }
#pragma unroll
    for (int r = 0; r < NS; ++r) {
        const int64_t base = A.u.map ? (int64_t)uid[r] * D : (cell * NS + r) * D;
#pragma unroll
        for (int i = 0; i < D; ++i) uv[r * D + i] = A.u.values[base + i];
    }
}

typedef unsigned int svk_u32x4 __attribute__((ext_vector_type(4)));

template <int D, int P>
constexpr int svk_tab_elems(int nq) { return nq + D * nq * nsc(D, P); }

// The per-cell results of a reverse pass: the vertex-coordinate gradients vx
// (seed already applied) and, if U, the displacement-dof gradients
// f * g[c * NS + r] (component-blocked). Deterministic mode writes them to
// the cell's slots of the workspace; otherwise they are scatter-added through
// the wave's combining tables.
template <int D, int NS, int TS, int TU, bool U, typename GT>
__device__ inline void svk_scatter_cell(const SvkArgs& A, bool det, int64_t cell, const int (&vid)[D + 1],
                                        const int (&uid)[NS], const double (&vx)[D + 1][D], const GT* g, double f,
                                        unsigned long long* ckeys, double* cvals, unsigned long long* ukeys,
                                        double* uvals) {
    if (det) {
#pragma unroll
        for (int v = 0; v <= D; ++v)
#pragma unroll
            for (int i = 0; i < D; ++i) A.det_x[(cell * (D + 1) + v) * D + i] = vx[v][i];
        if constexpr (U) {
#pragma unroll
            for (int r = 0; r < NS; ++r)
#pragma unroll
                for (int c = 0; c < D; ++c) A.det_u[(cell * NS + r) * D + c] = f * (double)g[c * NS + r];
        }
        return;
    }
    if (A.grad_coords) {
#pragma unroll
        for (int v = 0; v <= D; ++v)
            combine_add<D, TS>(ckeys, cvals, (unsigned long long)vid[v], vx[v], A.grad_coords);
    }
    if constexpr (U) {
#pragma unroll
        for (int r = 0; r < NS; ++r) {
            const unsigned long long key = A.u.map ? (unsigned long long)uid[r] : (unsigned long long)(cell * NS + r);
            double v[D];
#pragma unroll
            for (int c = 0; c < D; ++c) v[c] = f * (double)g[c * NS + r];
            combine_add<D, TU>(ukeys, uvals, key, v, A.grad_u);
        }
    }
}

// Vertex-coordinate gradients of a cell from Kbar = dS/dK (already scaled by
// |det J|) and S (every term is linear in |det J|):
//   Jbar = -K^T Kbar K^T + S K^T,  xbar_{j+1} = Jbar[:, j],  xbar_0 = -sum_j Jbar[:, j].
template <int D>
__device__ inline void svk_coord_bars(const double (&K)[D][D], const double (&Kbar)[D][D], double S, double sd,
                                      double (&vx)[D + 1][D]) {
    double Jbar[D][D];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b) s += K[a][i] * Kbar[a][b] * K[j][b];
            Jbar[i][j] = -s + S * K[j][i];
        }
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
}

// MODE 0: energy, 1: residual, 2: reverse pass of the energy (coordinates),
// 3: the reverse pass with the displacement gradient (the residual) too.
template <int D, int P, int NQ, int MODE, typename OT>
__global__ __launch_bounds__(256) void k_svk_vec(SvkArgs A) {
    constexpr int NS = nsc(D, P);
    // arithmetic type of the point loop: the output type for the forward
    // energy and residual (FP32 mode computes them in FP32 from the FP64
    // geometry), FP64 for the reverse pass
    using T = std::conditional_t<(MODE <= 1), OT, double>;
    // every table read below has the same address in all lanes: scalar path
    const double* W = A.tab;
    const double* dphi = A.tab + NQ;
    // reverse pass: the scatter-adds (vertex coordinates; MODE 3 also the
    // displacement dofs) are combined per wave
    constexpr bool REV = MODE >= 2;                 // reverse pass
    constexpr bool RES = MODE == 1 || MODE == 3;    // residual (MODE 3: scattered into grad_u)
    constexpr int TS = REV ? 256 : 1;
    constexpr int TU = MODE == 3 ? 256 : 1;
    __shared__ unsigned long long ckeys[4][TS], ukeys[4][TU];
    __shared__ double cvals[4][TS * D], uvals[4][TU * D];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // wave-uniform loop (every lane takes part in the table's clear and flush)
    for (int64_t base = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) - lane; base < A.ncells;
         base += (int64_t)gridDim.x * blockDim.x) {
        const bool valid = base + lane < A.ncells;
        const int64_t cell = valid ? base + lane : A.ncells - 1;
        const bool det = A.det_x != nullptr;  // same in every lane
        if (REV && !det) {
            combine_clear<D, TS>(ckeys[wave], cvals[wave], lane);
            if constexpr (MODE == 3) combine_clear<D, TU>(ukeys[wave], uvals[wave], lane);
            wave_sync();
        }
        Geom<D> g;
        double uvd[NS * D];
        int vid[D + 1], uid[NS];
        svk_load<D, NS>(A, cell, g, uvd, vid, uid);
        T uv[NS * D], K[D][D];
#pragma unroll
        for (int i = 0; i < NS * D; ++i) uv[i] = (T)uvd[i];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) K[i][j] = (T)g.K[i][j];
        T energy = T(0);
        T res[RES ? D * NS : 1];
        double Kbar[D][D];  // reverse pass: d Pi / d K
        if constexpr (RES) {
#pragma unroll
            for (int i = 0; i < D * NS; ++i) res[i] = T(0);
        }
        if constexpr (REV) {
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) Kbar[i][j] = 0.0;
        }
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
            T Fm[D][D], psi, Pm[D][D];
            svk_point<D, NS, true, T>(uv, K, dphi + q * NS, NQ, (T)A.mu, (T)A.lambda, Fm, &psi, Pm);
            const T wq = (T)cload(W + q);
            energy += wq * psi;
            if constexpr (RES) {
                // b_(c,a) += w sum_al (P K^T)_c,al dphi_a/dX_al
                T Q[D][D];
#pragma unroll
                for (int c = 0; c < D; ++c)
#pragma unroll
                    for (int al = 0; al < D; ++al) {
                        T t = T(0);
#pragma unroll
                        for (int j = 0; j < D; ++j) t += Pm[c][j] * K[al][j];
                        Q[c][al] = wq * t;
                    }
#pragma unroll
                for (int a = 0; a < NS; ++a) {
                    T dp[D];
#pragma unroll
                    for (int al = 0; al < D; ++al) dp[al] = (T)cload(dphi + (size_t)al * NQ * NS + q * NS + a);
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        T t = T(0);
#pragma unroll
                        for (int al = 0; al < D; ++al) t += Q[c][al] * dp[al];
                        res[c * NS + a] += t;
                    }
                }
            }
            if constexpr (REV) {
                // d Pi / d K[al][j] = |det J| sum_q w sum_i P_ij U_i,al
                double U[D][D];
#pragma unroll
                for (int i = 0; i < D; ++i)
#pragma unroll
                    for (int al = 0; al < D; ++al) {
                        double s = 0.0;
#pragma unroll
                        for (int r = 0; r < NS; ++r) s += uvd[r * D + i] * cload(dphi + (size_t)al * NQ * NS + q * NS + r);
                        U[i][al] = s;
                    }
#pragma unroll
                for (int al = 0; al < D; ++al)
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        double s = 0.0;
#pragma unroll
                        for (int i = 0; i < D; ++i) s += Pm[i][j] * U[i][al];
                        Kbar[al][j] += wq * s;
                    }
            }
        }
        const double ad = g.adet;
        if constexpr (MODE == 0) {
            if (valid) reinterpret_cast<OT*>(A.out)[cell] = (OT)((T)ad * energy);
        } else if constexpr (MODE == 1) {
            OT* o = reinterpret_cast<OT*>(A.out) + cell * (D * NS);
            if (valid) {
#pragma unroll
                for (int i = 0; i < D * NS; ++i) o[i] = (OT)((T)ad * res[i]);
            }
        } else {
            const double Pi = ad * energy;
            if (A.cell_value && valid) A.cell_value[cell] = Pi;
            // Kbar scaled by |det J|; d Pi/d|det J| |det J| = Pi
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) Kbar[i][j] *= ad;
            const double sd = A.seed;
            if (valid) {
                double vx[D + 1][D];
                svk_coord_bars<D>(g.K, Kbar, Pi, sd, vx);
                svk_scatter_cell<D, NS, TS, TU, MODE == 3>(A, det, cell, vid, uid, vx, res, sd * ad, ckeys[wave],
                                                           cvals[wave], ukeys[wave], uvals[wave]);
            }
            if (!det) {
                wave_sync();
                if (A.grad_coords) combine_flush<D, TS>(ckeys[wave], cvals[wave], A.grad_coords, lane);
                if constexpr (MODE == 3) combine_flush<D, TU>(ukeys[wave], uvals[wave], A.grad_u, lane);
                wave_sync();
            }
        }
    }
}

// Reverse pass of the residual: S_e = lam_e^T b_e with b_(c,a) = sum_q w |det J|
// P(F) : grad phi_a e_c, i.e. S_e = sum_q w |det J| P : L with L = Lam K the
// physical gradient of the field lam_e (Lam[c][al] = sum_a lam_(c,a) dphi_a/dX_al).
// Per point, with Pbar = w L and Lbar = w P (|det J| applied at the end):
//   P = F S(F):  Fbar = Pbar S + F sym(Z),  M = F^T Pbar,  Z = lambda tr(M) I + 2 mu M
//                (S symmetric; dS = lambda tr(dE) I + 2 mu dE, dE = (dF^T F + F^T dF)/2)
//   F = I + U K: Ubar = Fbar K^T -> u-dof bars Ubar dphi_r;  Kbar += U^T Fbar
//   L = Lam K:   Kbar += Lam^T Lbar
// so the displacement gradient is (db/du)^T lam = A_e lam_e (the Jacobian is
// symmetric). One thread per cell, FP64.
template <int D, int P, int NQ>
__global__ __launch_bounds__(256) void k_svk_res_adj(SvkArgs A) {
    constexpr int NS = nsc(D, P), N = D * NS;
    const double* W = A.tab;
    const double* dphi = A.tab + NQ;
    constexpr int TS = 256;
    __shared__ unsigned long long ckeys[4][TS], ukeys[4][TS];
    __shared__ double cvals[4][TS * D], uvals[4][TS * D];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double mu = A.mu, lm = A.lambda;
    for (int64_t base = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) - lane; base < A.ncells;
         base += (int64_t)gridDim.x * blockDim.x) {
        const bool valid = base + lane < A.ncells;
        const int64_t cell = valid ? base + lane : A.ncells - 1;
        const bool det = A.det_x != nullptr;
        if (!det) {
            combine_clear<D, TS>(ckeys[wave], cvals[wave], lane);
            combine_clear<D, TS>(ukeys[wave], uvals[wave], lane);
            wave_sync();
        }
        Geom<D> g;
        double uv[NS * D];
        int vid[D + 1], uid[NS];
        svk_load<D, NS>(A, cell, g, uv, vid, uid);
        const auto& K = g.K;
        const double* lam = A.lam + cell * N;
        double val = 0.0, Kbar[D][D], gu[N];
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) Kbar[i][j] = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) gu[i] = 0.0;
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
            const double* dq = dphi + q * NS;
            double U[D][D], Lm[D][D];  // reference gradients of u and of lam
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int al = 0; al < D; ++al) {
                    double s = 0.0, t = 0.0;
#pragma unroll
                    for (int r = 0; r < NS; ++r) {
                        const double dp = cload(dq + (size_t)al * NQ * NS + r);
                        s += uv[r * D + i] * dp;
                        t += lam[i * NS + r] * dp;
                    }
                    U[i][al] = s;
                    Lm[i][al] = t;
                }
            double H[D][D], F[D][D], L[D][D];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    double h = 0.0, l = 0.0;
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        h += U[i][a] * K[a][j];
                        l += Lm[i][a] * K[a][j];
                    }
                    H[i][j] = h;
                    F[i][j] = (i == j ? 1.0 : 0.0) + h;
                    L[i][j] = l;
                }
            double E[D][D], trE = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    double t = H[i][j] + H[j][i];
#pragma unroll
                    for (int k = 0; k < D; ++k) t += H[k][i] * H[k][j];
                    E[i][j] = 0.5 * t;
                }
#pragma unroll
            for (int i = 0; i < D; ++i) trE += E[i][i];
            double S[D][D], Pm[D][D];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) S[i][j] = (i == j ? lm * trE : 0.0) + 2.0 * mu * E[i][j];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    double t = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k) t += F[i][k] * S[k][j];
                    Pm[i][j] = t;
                }
            const double wq = cload(W + q);
            double pl = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) pl += Pm[i][j] * L[i][j];
            val += wq * pl;
            // M = F^T Pbar with Pbar = w L; Z = lambda tr(M) I + 2 mu M
            double M[D][D], trM = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    double t = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k) t += F[k][i] * L[k][j];
                    M[i][j] = wq * t;
                }
#pragma unroll
            for (int i = 0; i < D; ++i) trM += M[i][i];
            // Fbar = Pbar S + F sym(Z), sym(Z) = lambda tr(M) I + mu (M + M^T)
            double Fb[D][D];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    double t = 0.0, z = 0.0;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        t += L[i][k] * S[k][j];
                        z += F[i][k] * ((k == j ? lm * trM : 0.0) + mu * (M[k][j] + M[j][k]));
                    }
                    Fb[i][j] = wq * t + z;
                }
            // Kbar += U^T Fbar + Lam^T (w P); Ubar = Fbar K^T -> u-dof bars
#pragma unroll
            for (int al = 0; al < D; ++al)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    double t = 0.0;
#pragma unroll
                    for (int i = 0; i < D; ++i) t += U[i][al] * Fb[i][j] + Lm[i][al] * wq * Pm[i][j];
                    Kbar[al][j] += t;
                }
            double Ub[D][D];
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int al = 0; al < D; ++al) {
                    double t = 0.0;
#pragma unroll
                    for (int j = 0; j < D; ++j) t += Fb[i][j] * K[al][j];
                    Ub[i][al] = t;
                }
#pragma unroll
            for (int r = 0; r < NS; ++r) {
                double dp[D];
#pragma unroll
                for (int al = 0; al < D; ++al) dp[al] = cload(dq + (size_t)al * NQ * NS + r);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double t = 0.0;
#pragma unroll
                    for (int al = 0; al < D; ++al) t += Ub[i][al] * dp[al];
                    gu[i * NS + r] += t;
                }
            }
        }
        const double ad = g.adet;
        const double Se = ad * val;
        if (A.cell_value && valid) A.cell_value[cell] = Se;
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) Kbar[i][j] *= ad;
        const double sd = A.seed;
        if (valid) {
            double vx[D + 1][D];
            svk_coord_bars<D>(K, Kbar, Se, sd, vx);
            svk_scatter_cell<D, NS, TS, TS, true>(A, det, cell, vid, uid, vx, gu, sd * ad, ckeys[wave], cvals[wave],
                                                  ukeys[wave], uvals[wave]);
        }
        if (!det) {
            wave_sync();
            if (A.grad_coords) combine_flush<D, TS>(ckeys[wave], cvals[wave], A.grad_coords, lane);
            if (A.grad_u) combine_flush<D, TS>(ukeys[wave], uvals[wave], A.grad_u, lane);
            wave_sync();
        }
    }
}

// Jacobian, shared-point layout: CPW cells per wave, lane (cell, block
// c1 <= c2, row slice h) accumulating rows h*NA .. h*NA + NA - 1 of that block.
// At every (cell, point), F and S^ = K S K^T are formed once, by the cell's
// lanes in turn, into LDS. Each lane forms its block's H = w K C K^T for the
// tangent above, with k_c = K F_c (row c of F mapped by K), as
//   H = w (delta_c1c2 S^ + lambda k_c1 k_c2^T + mu k_c2 k_c1^T + mu (F_c1 . F_c2) K K^T)
// and accumulates its rows as A[a][b] += sum_be (sum_al dphi_al,a H[al][be])
// dphi_be,b.
template <int D, int P, int NQ, typename AT, int AH>
__global__ __launch_bounds__(256, 2) void k_svk_jac(SvkArgs A) {
    constexpr int NS = nsc(D, P);
    constexpr int N = D * NS;
    constexpr int NB = D * (D + 1) / 2;
    constexpr int LPC = NB * AH;  // lanes per cell
    constexpr int CPW = 64 / LPC;  // cells per wave
    constexpr int NA = (NS + AH - 1) / AH;
    constexpr int TE = NQ + D * NQ * NS;
    // per wave: F and S (upper) at the group's points, later one cell's
    // staged tensor
    constexpr int PEQ = D * D + NB;
    constexpr int FE = CPW * NQ * PEQ;
    constexpr int SE = (N * N * (int)sizeof(AT) + 7) / 8;  // one staged cell, in doubles
    // cells staged per round: as many as the point data's area holds, or as
    // fit in 6 KiB
    constexpr int CR0 = FE / SE > 6144 / (SE * 8) ? FE / SE : 6144 / (SE * 8);
    constexpr int CR = CR0 < 1 ? 1 : (CR0 > CPW ? CPW : CR0);
    __shared__ double tab[TE];
    constexpr int WE = ((FE > CR * SE ? FE : CR * SE) + 1) / 2 * 2;  // 16-byte multiple
    __shared__ __attribute__((aligned(16))) double fbuf[4][WE];
    for (int i = threadIdx.x; i < TE; i += blockDim.x) tab[i] = A.tab[i];
    __syncthreads();
    const double* W = tab;
    const double* dphi = tab + NQ;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int k = lane % LPC, cl = lane / LPC;
    const int blk = k % NB, h = k / NB;
    int c1 = 0, c2 = 0;
    {
        int t = blk;
        while (t >= D - c1) { t -= D - c1; ++c1; }
        c2 = c1 + t;
    }
    const int a0 = h * NA;
    const double diag = c1 == c2 ? 1.0 : 0.0;
    double* Fw = fbuf[wave];
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t w0 = (int64_t)blockIdx.x * 4 + wave; w0 * CPW < A.ncells; w0 += nwaves) {
        const int64_t cell = w0 * CPW + cl;
        const bool active = cl < CPW && cell < A.ncells;
        // lanes without a cell work on the group's last one and store nothing
        const int64_t lcell = active ? cell : (w0 * CPW + CPW - 1 < A.ncells ? w0 * CPW + CPW - 1 : A.ncells - 1);
        Geom<D> g;
        double uv[NS * D];
        int vid[D + 1], uid[NS];
        svk_load<D, NS>(A, lcell, g, uv, vid, uid);
        double M[D][D];  // K K^T
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int b = 0; b < D; ++b) {
                double x = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) x += g.K[a][i] * g.K[b][i];
                M[a][b] = x;
            }
        double* Fc = Fw + (cl < CPW ? cl : CPW - 1) * NQ * PEQ;
        // F at the cell's points, LPC points at a time
#pragma unroll 1
        for (int q = k; q < NQ; q += LPC) {
            if (!active) break;
            double F[D][D], S[D][D], KS[D][D];
            svk_F<D, NS>(uv, g.K, dphi + q * NS, NQ, F);
            svk_S<D>(F, A.mu, A.lambda, S);
            double* pq = Fc + q * PEQ;
#pragma unroll
            for (int c = 0; c < D; ++c)
#pragma unroll
                for (int a = 0; a < D; ++a) pq[c * D + a] = F[c][a];
            // S^ = K S K^T (upper)
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int l = 0; l < D; ++l) {
                    double x = 0.0;
#pragma unroll
                    for (int j = 0; j < D; ++j) x += g.K[a][j] * S[j][l];
                    KS[a][l] = x;
                }
            int t = 0;
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = a; b < D; ++b, ++t) {
                    double x = 0.0;
#pragma unroll
                    for (int l = 0; l < D; ++l) x += KS[a][l] * g.K[b][l];
                    pq[D * D + t] = x;
                }

        }
        wave_sync();
        AT acc[NA][NS];
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NS; ++b) acc[a][b] = (AT)0;
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
            const double* Fq = Fc + q * PEQ;
            // rows c1, c2 of F; k_c = K F_c
            double F1[D], F2[D], k1[D], k2[D], Sh[D][D];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                F1[j] = Fq[c1 * D + j];
                F2[j] = Fq[c2 * D + j];
            }
#pragma unroll
            for (int a = 0; a < D; ++a) {
                double x = 0.0, y = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    x += g.K[a][j] * F1[j];
                    y += g.K[a][j] * F2[j];
                }
                k1[a] = x;
                k2[a] = y;
            }
            // S^ enters the diagonal blocks only
            {
                int t = 0;
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int b = a; b < D; ++b, ++t) {
                        Sh[a][b] = diag * Fq[D * D + t];
                        Sh[b][a] = Sh[a][b];
                    }
            }
            double FF = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) FF += F1[j] * F2[j];
            // H = w K C K^T = w (delta S^ + lambda k1 k2^T + mu k2 k1^T + mu FF K K^T)
            double H[D][D];
            const double wq = W[q];
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = 0; b < D; ++b)
                    H[a][b] = wq * (Sh[a][b] + A.lambda * k1[a] * k2[b] + A.mu * k2[a] * k1[b] + A.mu * FF * M[a][b]);
            // this lane's rows: wv[i][be] = sum_al dphi_al,a H[al][be], then
            // A[a][b] += sum_be wv[i][be] dphi_be,b
            AT wv[NA][D];
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int a = a0 + i < NS ? a0 + i : NS - 1;
#pragma unroll
                for (int be = 0; be < D; ++be) {
                    double s = 0.0;
#pragma unroll
                    for (int al = 0; al < D; ++al) s += dphi[(size_t)al * NQ * NS + q * NS + a] * H[al][be];
                    wv[i][be] = (AT)s;
                }
            }
#pragma unroll
            for (int be = 0; be < D; ++be)
#pragma unroll
                for (int b = 0; b < NS; ++b) {
                    // wave-uniform: through the scalar path, not an LDS broadcast
                    const AT db = (AT)cload(A.tab + NQ + (size_t)be * NQ * NS + q * NS + b);
#pragma unroll
                    for (int i = 0; i < NA; ++i) acc[i][b] += wv[i][be] * db;
                }
        }
        wave_sync();  // the next cell's F overwrites this one's
        const AT ad = (AT)g.adet;
        // the wave's cells are consecutive: stage CR cells' tensors at a time in
        // LDS (over the point data, no longer needed) and write them as
        // contiguous 16-byte stores
        AT* stg = reinterpret_cast<AT*>(Fw);
        AT* out = reinterpret_cast<AT*>(A.out);
        wave_sync();
#pragma unroll 1
        for (int r0 = 0; r0 < CPW; r0 += CR) {
            const int64_t rc = w0 * CPW + r0;
            if (rc >= A.ncells) break;  // wave-uniform
            // cells of this round: CR, fewer in the group's last round and at
            // the end of the mesh
            const int nc = CPW - r0 < CR ? CPW - r0 : CR;
            const int nr = (int)(A.ncells - rc < nc ? A.ncells - rc : nc);
            if (active && cl >= r0 && cl < r0 + CR) {
                AT* sc = stg + (cl - r0) * N * N;
#pragma unroll
                for (int i = 0; i < NA; ++i) {
                    const int a = a0 + i;
                    if (a >= NS) continue;
#pragma unroll
                    for (int b = 0; b < NS; ++b) {
                        const AT x = ad * acc[i][b];
                        sc[(c1 * NS + a) * N + c2 * NS + b] = x;
                        if (c1 != c2) sc[(c2 * NS + b) * N + c1 * NS + a] = x;
                    }
                }
            }
            wave_sync();
            AT* o = out + rc * (int64_t)N * N;
            if constexpr ((N * N * sizeof(AT)) % 16 == 0) {
                constexpr int NV = (int)(N * N * sizeof(AT) / 16);
                const int nv = nr * NV;
                const svk_u32x4* s4 = reinterpret_cast<const svk_u32x4*>(stg);
                svk_u32x4* o4 = reinterpret_cast<svk_u32x4*>(o);
#pragma unroll
                for (int e0 = 0; e0 < CR * NV; e0 += 64)
                    if (e0 + lane < nv) __builtin_nontemporal_store(s4[e0 + lane], &o4[e0 + lane]);
            } else {
                const int ne = nr * N * N;
#pragma unroll
                for (int e0 = 0; e0 < CR * N * N; e0 += 64)
                    if (e0 + lane < ne) o[e0 + lane] = stg[e0 + lane];
            }
            wave_sync();
        }
    }
}

}  // namespace dev

// ---------------------------------------------------------------- host side

static std::mutex g_svk_mu;
static std::map<std::tuple<int, int, int, int>, void*> g_svk_tabs;  // (dev, dim, p, q)

static coffee_status svk_table(int dev, int dim, int p, int q, const double** out) {
    std::lock_guard<std::mutex> lk(g_svk_mu);
    auto key = std::make_tuple(dev, dim, p, q);
    auto it = g_svk_tabs.find(key);
    if (it != g_svk_tabs.end()) {
        *out = (const double*)it->second;
        return COFFEE_OK;
    }
    // The SVK integrands at q = 2p are polynomials of degree exactly 2p on an
    // affine cell (F is of degree p - 1), so every rule exact to degree q
    // gives the same integral up to rounding: P2 uses the fully symmetric
    // rule (6 points on triangles, 14 on tetrahedra, against 9 and 27 for the
    // collapsed Gauss-Jacobi rule of that degree).
    Tables t;
    if (!t.init(dim, p, p == 2 ? COFFEE_QUAD(q & 15, COFFEE_RULE_SYMMETRIC) : q)) return COFFEE_E_INVALID_ARG;
    std::vector<double> h;
    if (p == 1) {
        // P1 on an affine cell: the displacement gradient, hence the whole
        // integrand, is the same at every point, so the point loop is
        // invariant (section 3.2's loop-invariant code motion applied to the
        // whole loop): one point carrying the summed weight.
        long double w = 0.0L;
        for (int k = 0; k < t.nq; ++k) w += t.W[k];
        h.push_back((double)w);
        for (int al = 0; al < dim; ++al)
            for (int a = 0; a < t.n; ++a) h.push_back((double)t.dphi[((size_t)al * t.nq + 0) * t.n + a]);
    } else {
        for (int k = 0; k < t.nq; ++k) h.push_back((double)t.W[k]);
        for (size_t i = 0; i < t.dphi.size(); ++i) h.push_back((double)t.dphi[i]);
    }
    void* d = nullptr;
    if (hipMalloc(&d, h.size() * sizeof(double)) != hipSuccess) return COFFEE_E_NOMEM;
    if (hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return COFFEE_E_HIP;
    }
    g_svk_tabs[key] = d;
    *out = (const double*)d;
    return COFFEE_OK;
}

void free_svk_tables() {
    std::lock_guard<std::mutex> lk(g_svk_mu);
    for (auto& kv : g_svk_tabs) {
        (void)hipSetDevice(std::get<0>(kv.first));
        (void)hipFree(kv.second);
    }
    g_svk_tabs.clear();
}

namespace {

constexpr int svk_jac_slices(int, int p) { return p == 2 ? 2 : 1; }

// compiled set: triangles and tetrahedra, P1 (q = 2, evaluated at one point
// with the summed weight) and P2 (q = 4)
template <int D, int P, int NQ>
hipError_t launch_svk(int form, int precision, const dev::SvkArgs& a, hipStream_t s, int ncu, bool reverse) {
    const int64_t blocks = (a.ncells + 255) / 256;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(blocks, (int64_t)ncu * 8));
    if (reverse) {
        if (form == COFFEE_SVK_RESIDUAL)
            hipLaunchKernelGGL((dev::k_svk_res_adj<D, P, NQ>), dim3(grid), dim3(256), 0, s, a);
        else if (a.grad_u || a.det_u)
            hipLaunchKernelGGL((dev::k_svk_vec<D, P, NQ, 3, double>), dim3(grid), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((dev::k_svk_vec<D, P, NQ, 2, double>), dim3(grid), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const bool f64 = precision == COFFEE_FP64;
    if (form == COFFEE_SVK_ENERGY) {
        if (f64) hipLaunchKernelGGL((dev::k_svk_vec<D, P, NQ, 0, double>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((dev::k_svk_vec<D, P, NQ, 0, float>), dim3(grid), dim3(256), 0, s, a);
    } else if (form == COFFEE_SVK_RESIDUAL) {
        if (f64) hipLaunchKernelGGL((dev::k_svk_vec<D, P, NQ, 1, double>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((dev::k_svk_vec<D, P, NQ, 1, float>), dim3(grid), dim3(256), 0, s, a);
    } else {
        // row slices per block: enough to keep the accumulators of a P2
        // tetrahedron block well under the register file of 2 waves per SIMD
        constexpr int AH = svk_jac_slices(D, P);
        constexpr int CPW = 64 / (D * (D + 1) / 2 * AH);
        const int64_t waves = (a.ncells + CPW - 1) / CPW;
        const int g2 = (int)std::max<int64_t>(1, std::min<int64_t>((waves + 3) / 4, (int64_t)ncu * 16));
        if (f64) hipLaunchKernelGGL((dev::k_svk_jac<D, P, NQ, double, AH>), dim3(g2), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((dev::k_svk_jac<D, P, NQ, float, AH>), dim3(g2), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t dispatch_svk(int form, int dim, int p, int q, int precision, const dev::SvkArgs& a, hipStream_t s,
                        int ncu, bool reverse, bool* found) {
    *found = true;
    q &= 15;  // either rule family: the integrands are integrated exactly (svk_table)
    if (dim == 2 && p == 1 && q == 2) return launch_svk<2, 1, 1>(form, precision, a, s, ncu, reverse);
    if (dim == 2 && p == 2 && q == 4) return launch_svk<2, 2, 6>(form, precision, a, s, ncu, reverse);
    if (dim == 3 && p == 1 && q == 2) return launch_svk<3, 1, 1>(form, precision, a, s, ncu, reverse);
    if (dim == 3 && p == 2 && q == 4) return launch_svk<3, 2, 14>(form, precision, a, s, ncu, reverse);
    *found = false;
    return hipSuccess;
}

coffee_status svk_common(int cell, int degree, int q, const double* coords, const int32_t* c2v, int64_t ncells,
                         const coffee_field* coeffs, const double* constants, int nconst, dev::SvkArgs& a,
                         const double** tab, int* dev_out) {
    if (coeffs[0].degree != degree) return COFFEE_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return COFFEE_E_HIP;
    coffee_status st = svk_table(dev, cell, degree, q, tab);
    if (st != COFFEE_OK) return st;
    std::memset(&a, 0, sizeof a);
    a.coords = coords;
    a.c2v = c2v;
    a.ncells = ncells;
    a.u = dev::FieldArg{coeffs[0].values, coeffs[0].cell_to_dof};
    a.mu = nconst > 0 ? constants[0] : 1.0;
    a.lambda = nconst > 1 ? constants[1] : 1.0;
    a.tab = *tab;
    *dev_out = dev;
    return COFFEE_OK;
}

}  // namespace

coffee_status assemble_svk(int form, int cell, int degree, int q, int precision, const double* coords, int64_t nvert,
                           const int32_t* c2v, int64_t ncells, const coffee_field* coeffs, const double* constants,
                           int nconst, void* out, void* hip_stream) {
    (void)nvert;
    if (precision == COFFEE_BF16X3)
        return assemble_svk_bf16(form, cell, degree, q, coords, c2v, ncells, coeffs, constants, nconst, out,
                                 hip_stream);
    if (ncells == 0) return COFFEE_OK;
    dev::SvkArgs a;
    const double* tab = nullptr;
    int dev = 0;
    coffee_status st = svk_common(cell, degree, q, coords, c2v, ncells, coeffs, constants, nconst, a, &tab, &dev);
    if (st != COFFEE_OK) return st;
    a.out = out;
    bool found = false;
    hipError_t e = dispatch_svk(form, cell, degree, q, precision, a, (hipStream_t)hip_stream, num_cu(dev), false, &found);
    if (!found) return COFFEE_E_UNSUPPORTED;
    return e == hipSuccess ? COFFEE_OK : COFFEE_E_HIP;
}

coffee_status adjoint_svk(int form, int cell, int degree, int q, const double* coords, const int32_t* c2v,
                          int64_t ncells, const coffee_field* coeffs, const double* constants, int nconst,
                          const double* lam, double seed, double* grad_coords, double* const* grad_coeff_values,
                          double* cell_value, const DetTarget* det, void* hip_stream) {
    if (form == COFFEE_SVK_RESIDUAL && ncells > 0 && !lam) return COFFEE_E_INVALID_ARG;
    if (ncells == 0) return COFFEE_OK;
    dev::SvkArgs a;
    const double* tab = nullptr;
    int dev = 0;
    coffee_status st = svk_common(cell, degree, q, coords, c2v, ncells, coeffs, constants, nconst, a, &tab, &dev);
    if (st != COFFEE_OK) return st;
    a.seed = seed;
    a.grad_coords = grad_coords;
    a.grad_u = grad_coeff_values ? grad_coeff_values[0] : nullptr;
    a.cell_value = cell_value;
    a.lam = lam;
    if (det) {
        a.det_x = det[0].local;
        a.det_u = det[1].local;
    }
    bool found = false;
    hipError_t e = dispatch_svk(form, cell, degree, q, COFFEE_FP64, a, (hipStream_t)hip_stream, num_cu(dev), true,
                                &found);
    if (!found) return COFFEE_E_UNSUPPORTED;
    return e == hipSuccess ? COFFEE_OK : COFFEE_E_HIP;
}

// The gradient arrays of a reverse pass as deterministic-scatter targets:
// vertex coordinates (entries: cells x vertices, keys cell_to_vertex), then
// each coefficient field (entries: cells x local dofs, keys its dof map, or
// one entry per value for a cell-major field).
int adjoint_det_targets(int cell, int64_t nvert, const int32_t* c2v, int64_t ncells, const coffee_field* coeffs,
                        int ncoeff, double* grad_coords, double* const* grad_coeff_values, DetTarget* t) {
    const int d = cell;
    t[0] = DetTarget{c2v, 1, ncells * (d + 1), d, nvert, nullptr, grad_coords};
    for (int i = 0; i < ncoeff; ++i) {
        const int64_t n = ncells * n_scalar(d, coeffs[i].degree);
        const int32_t* keys = coeffs[i].cell_to_dof;
        // the field's dof count is not passed: its keys are sorted over 31 bits
        t[1 + i] = DetTarget{keys, keys ? 1 : 0, n, coeffs[i].ncomp, keys ? ((int64_t)1 << 31) : n, nullptr,
                             grad_coeff_values ? grad_coeff_values[i] : nullptr};
    }
    return 1 + ncoeff;
}

}  // namespace coffee

extern "C" coffee_status coffee_assemble_adjoint(int form, int cell, int degree, int quad_degree,
                                                 const double* coords, int64_t nvert, const int32_t* c2v,
                                                 int64_t ncells, const coffee_field* coeffs, int ncoeff,
                                                 const double* constants, int nconst, const double* lam,
                                                 const double* u, double seed, double* grad_coords,
                                                 double* const* grad_coeff_values, double* cell_value,
                                                 int deterministic, void* workspace, int64_t workspace_bytes,
                                                 void* hip_stream) {
    using namespace coffee;
    int q = 0, fd = 0;
    coffee_status st = validate_common(form, cell, degree, quad_degree, coords, nvert, c2v, ncells, coeffs, ncoeff,
                                       constants, nconst, &q, &fd);
    if (st != COFFEE_OK) return st;
    if (deterministic != 0 && deterministic != 1) return COFFEE_E_INVALID_ARG;
    if (form == COFFEE_SVK_JACOBIAN || cell == COFFEE_PRISM) return COFFEE_E_UNSUPPORTED;
    if (!is_svk_form(form) && ncells > 0 && (!lam || !u)) return COFFEE_E_INVALID_ARG;
    for (int i = 0; i < ncoeff; ++i)
        if (coeffs[i].ncomp > 3) return COFFEE_E_UNSUPPORTED;
    DetTarget det[3];
    int ndet = 0;
    if (deterministic) {
        ndet = adjoint_det_targets(cell, nvert, c2v, ncells, coeffs, ncoeff, grad_coords, grad_coeff_values, det);
        st = det_carve(workspace, workspace_bytes, det, ndet);
        if (st != COFFEE_OK) return st;
    }
    if (is_svk_form(form))
        st = adjoint_svk(form, cell, degree, q, coords, c2v, ncells, coeffs, constants, nconst, lam, seed,
                         grad_coords, grad_coeff_values, cell_value, deterministic ? det : nullptr, hip_stream);
    else
        st = adjoint_linear(form, cell, degree, q, fd, coords, nvert, c2v, ncells, coeffs, ncoeff, constants, nconst,
                            lam, u, seed, grad_coords, grad_coeff_values, cell_value, deterministic ? det : nullptr,
                            hip_stream);
    if (st != COFFEE_OK || !deterministic || ncells == 0) return st;
    return det_scatter(det, ndet, workspace, (hipStream_t)hip_stream);
}

extern "C" int64_t coffee_adjoint_workspace_size(int form, int cell, int degree, int64_t nvert, int64_t ncells,
                                                 const coffee_field* coeffs, int ncoeff) {
    using namespace coffee;
    if (form < COFFEE_MASS || form > COFFEE_DIFFUSION || form == COFFEE_SVK_JACOBIAN) return -1;
    if ((cell != COFFEE_TRIANGLE && cell != COFFEE_TETRAHEDRON) || degree < 1 || degree > kMaxP) return -1;
    if (nvert < 0 || ncells < 0 || ncoeff < 0 || ncoeff > 2 || (ncoeff > 0 && !coeffs)) return -1;
    for (int i = 0; i < ncoeff; ++i)
        if (coeffs[i].degree < 1 || coeffs[i].degree > kMaxP || coeffs[i].ncomp < 1 || coeffs[i].ncomp > 3) return -1;
    DetTarget det[3];
    const int ndet = adjoint_det_targets(cell, nvert, nullptr, ncells, coeffs, ncoeff, nullptr, nullptr, det);
    return det_workspace_bytes(det, ndet);
}
