// Device engine for the elasticity form (cell-row engine).
//
// The element tensor of a cell is D x D blocks A_cc' (n x n each), and the
// blocks are symmetric in pairs: A_c'c = A_cc'^T. The G row of block (c', c)
// is the row of (c, c') with its geometry indices swapped, and the reference
// tensor satisfies R^{be al}[b][a] = R^{al be}[a][b] (the bilinear form is
// symmetric, paper section 2: the j and k loops have the same extent and the
// integrand is symmetric under the swap of trial and test functions), so only
// the NB = D (D + 1) / 2 upper blocks are contracted. Each lower block is
// written from the same accumulator values at the transposed place.
//
// The rows of the MFMA products are (cell, upper block) pairs in cell-major
// order: row NB e + b is block b of cell e. A wave takes a unit of 16 cells
// (16 NB rows, NB 16-row tiles) and runs its row tiles in order, so the cells
// of the unit complete one after another: after row tile m, cells
// [16 m / NB, 16 (m + 1) / NB) are complete. The blocks of a cell are staged
// in LDS (a ring of cell slots, each a whole cell tensor), and every completed
// cell leaves as part of one contiguous range of 16-byte stores. Writing whole
// cells in order keeps the write stream sequential per wave: writing the same
// bytes as row pieces of 16 cells at a time (one panel of rows for every cell
// of a tile) reached only about 60% of the write bandwidth of whole cells.
//
// Per row tile: lane (row i, group g) builds the G entries of the coefficient
// dofs r = g, g + 4, ... of row i's (cell, block) into LDS. The cell's
// geometry (K, K K^T, |det J|) and coefficient values are computed once per
// unit by lane (cell, g), as in the panel engine (vector.hpp), and fetched
// for the row tile with cross-lane permutes.
#pragma once
#include "vector.hpp"

namespace coffee {
namespace dev {

// Upper block b = 0 .. NB-1 of a D x D block matrix, row-major over c <= c'.
template <int D>
__device__ __forceinline__ void el_block(int b, int& c, int& c2) {
    if constexpr (D == 2) {
        c = b < 2 ? 0 : 1;
        c2 = b - (c == 0 ? 0 : 1);
    } else {
        c = b < 3 ? 0 : (b < 5 ? 1 : 2);
        c2 = c == 0 ? b : (c == 1 ? b - 2 : 2);
    }
}

// Sizes of the cell-row engine for (D, P, FD, PREC); `fits` is false where a
// ring of cell slots does not fit the LDS of four waves (the panel engine
// takes those instances).
struct ElSizes {
    int ns, nn, n, cellv, nb, kr, ks, row, nt, ring;
    int g_bytes, ring_bytes, wave_bytes, tile_bytes;
    int waves;
    int rlt;  // n-tiles of reference fragments staged in LDS (the rest read through the caches)
    bool rreg, fits;
    int lds_bytes;
};

__host__ __device__ constexpr ElSizes el_sizes(int d, int p, int fd, int prec) {
    ElSizes s{};
    s.ns = nsc(d, p);
    s.nn = s.ns * s.ns;
    s.n = d * s.ns;
    s.cellv = s.n * s.n;
    s.nb = npair(d);
    s.kr = kref(F_ELAST, d, fd);
    s.ks = vec_ksteps(F_ELAST, d, fd, prec);
    s.row = vec_row(F_ELAST, d, fd, prec);
    s.nt = (s.nn + 15) / 16;
    // cells a 16-row tile touches: at most ceil(15 / NB) + 1
    const int touch = (15 + s.nb - 1) / s.nb + 1;
    s.ring = touch <= 4 ? 4 : 8;
    const int gsz = prec == PREC_F64 ? 8 : (prec == PREC_F32 ? 4 : 2);
    const int osz = prec == PREC_F64 ? 8 : 4;
    const int fsz = prec == PREC_F64 ? 8 : (prec == PREC_F32 ? 4 : 16);
    s.g_bytes = (16 * s.row * gsz + 15) / 16 * 16;
    s.ring_bytes = s.ring * s.cellv * osz;
    s.wave_bytes = s.g_bytes + s.ring_bytes;
    s.tile_bytes = s.ks * 64 * fsz;  // fragments of one n-tile
    constexpr int L = 160 * 1024;
    // two waves per SIMD when their rings fit, else one; the reference
    // fragments in registers when few, or at one wave per SIMD (512 registers)
    // when they take at most 160, else as many n-tiles in LDS as the rest of
    // it holds
    s.waves = 8 * s.wave_bytes <= L ? 8 : 4;
    const int rregs = s.nt * s.ks * (fsz / 4);
    s.rreg = rregs <= 32 || (s.waves == 4 && rregs <= 160);
    const int spare = L - s.waves * s.wave_bytes;
    const int rl = spare > 0 ? spare / s.tile_bytes : 0;
    s.rlt = s.rreg ? 0 : (rl < s.nt ? rl : s.nt);
    s.fits = 4 * s.wave_bytes <= L && s.cellv * osz % 16 == 0;
    s.lds_bytes = s.rlt * s.tile_bytes + s.waves * s.wave_bytes;
    return s;
}

template <int D, int P, int FD, int PREC>
struct ElCfg {
    using g_t = typename PrecT<PREC>::gtype;
    using frag_t = typename PrecT<PREC>::frag;
    using acc_t = typename PrecT<PREC>::acc;
    using out_t = typename PrecT<PREC>::otype;
    static constexpr ElSizes S = el_sizes(D, P, FD, PREC);
    static constexpr int NS = S.ns, NN = S.nn, N = S.n, CELLV = S.cellv, NB = S.nb;
    static constexpr int KR = S.kr, KS = S.ks, ROW = S.row, NT = S.nt, RING = S.ring;
    // n-tiles per accumulator chunk (BF16X3 fragments take four registers)
    static constexpr int TMAX = PREC == PREC_BF16X3 ? 4 : 8;
    static constexpr int TCH = NT <= TMAX ? NT : TMAX;
    static constexpr int NCH = (NT + TCH - 1) / TCH;
    static constexpr int WAVES = S.waves;
    static constexpr int RLT = S.rlt;
    static constexpr bool RREG = S.rreg;
    static constexpr int CPC = CELLV * (int)sizeof(out_t) / 16;  // 16-byte chunks per cell
    static constexpr int NF = VLane<F_ELAST, D, FD>::NF;
    static constexpr int RPL = VLane<F_ELAST, D, FD>::RPL;
    static_assert(S.fits, "cell ring exceeds the LDS of four waves");
};

template <int D, int P, int FD, int PREC>
struct ElWave {
    using C = ElCfg<D, P, FD, PREC>;
    typename C::g_t* gbuf;    // 16 G rows
    typename C::out_t* ring;  // RING cell slots
    const typename C::frag_t* rlds;  // first RLT n-tiles of the reference fragments (LDS)
    const typename C::frag_t* rglb;  // all of them (global)
    typename C::frag_t rreg[C::RREG ? C::NT : 1][C::RREG ? C::KS : 1];
    int lane;
};

__device__ inline double lane_get(double v, int src) { return __shfl(v, src, 64); }

// G row of row i (cell ci, upper block b) of row tile m: lane (i, g) writes the
// entries of the coefficient dofs r = g + 4 j, fetching cell ci's data from
// lane (ci, g).
template <int D, int P, int FD, int PREC, bool FULL>
__device__ __forceinline__ void el_put_G(const LinArgs& A, const ElWave<D, P, FD, PREC>& W,
                                const VCell<F_ELAST, D, FD>& cd, int m, int64_t unit_base) {
    using C = ElCfg<D, P, FD, PREC>;
    constexpr int NB = C::NB, NF = C::NF, RPL = C::RPL, KR = C::KR, KS = C::KS;
    const int lane = W.lane, i = lane & 15, g = lane >> 4;
    const int row = 16 * m + i;
    const int ci = row / NB, b = row - (row / NB) * NB;
    const int src = ci + 16 * g;
    int c, c2;
    el_block<D>(b, c, c2);
    // K from the cell's lane; K K^T formed here (fewer permutes)
    double K[D][D], M[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int k = 0; k < D; ++k) K[a][k] = lane_get(cd.K[a][k], src);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int e = 0; e < D; ++e) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) t += K[a][k] * K[e][k];
            M[a][e] = t;
        }
    // every lane takes part in every permute (a permute reads nothing from a
    // lane that is switched off), then invalid rows are zeroed
    const double ad_src = lane_get(cd.ad, src);
    const bool valid = FULL || unit_base + ci < A.ncells;
    const double ad = valid ? ad_src : 0.0;
    double k1[D], k2[D];  // columns c and c2 of K
#pragma unroll
    for (int a = 0; a < D; ++a) {
        k1[a] = pick<D>(K[a], c);
        k2[a] = pick<D>(K[a], c2);
    }
    const double dg = c == c2 ? 1.0 : 0.0;
    typename C::g_t* rw = W.gbuf + i * C::ROW;
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
        const int r = g + 4 * j;
        double mu, lm;
        if constexpr (FD > 0) {
            mu = ad * lane_get(cd.f[0][j][0], src);
            lm = ad * lane_get(cd.f[1][j][0], src);
        } else {
            mu = ad * A.c0;
            lm = ad * A.c1;
        }
        if (NF % 4 == 0 || r < NF) {
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int e = 0; e < D; ++e)
                    put_g<PREC, KR>(rw, r * D * D + a * D + e, mu * (dg * M[a][e] + k2[a] * k1[e]) + lm * k1[a] * k2[e]);
        }
    }
    if (g == 0) {
        if constexpr (PREC == PREC_BF16X3) {
#pragma unroll
            for (int k = 4 * KR; k < KS * 32; ++k) rw[k] = 0;
        } else {
#pragma unroll
            for (int k = KR; k < KS * 4; ++k) rw[k] = 0;
        }
    }
}

// Row tile m of a unit: G rows, contraction chunk by chunk into the cell ring,
// then the cells completed by this tile leave as one contiguous store range.
template <int D, int P, int FD, int PREC, bool FULL, int m>
__device__ __forceinline__ void el_rowtile(const LinArgs& A, const ElWave<D, P, FD, PREC>& W,
                                  const VCell<F_ELAST, D, FD>& cd, int64_t unit_base) {
    using C = ElCfg<D, P, FD, PREC>;
    using acc_t = typename C::acc_t;
    using frag_t = typename C::frag_t;
    using out_t = typename C::out_t;
    constexpr int NB = C::NB, NS = C::NS, N = C::N, NN = C::NN, KS = C::KS, TCH = C::TCH;
    __builtin_amdgcn_sched_barrier(0);
    el_put_G<D, P, FD, PREC, FULL>(A, W, cd, m, unit_base);
    wave_sync();
    // the lane index re-read opaquely: the staging offsets below are then
    // formed per tile instead of being hoisted out of the unit loop (hundreds
    // of loop-invariant addresses would not fit the registers)
    int lane = W.lane;
    asm volatile("" : "+v"(lane));
    // per accumulator element v: the (cell slot, block) origins of its row's
    // upper block and of the transposed lower block
    int based[4], baset[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = 16 * m + acc_row<PREC>(lane, v);
        const int ci = row / NB, bk = row - (row / NB) * NB;
        int c, c2;
        el_block<D>(bk, c, c2);
        const int slot = (ci & (C::RING - 1)) * C::CELLV;
        based[v] = slot + c * NS * N + c2 * NS;
        baset[v] = slot + c2 * NS * N + c * NS;
    }
#pragma unroll
    for (int h = 0; h < C::NCH; ++h) {
        const int t0 = h * TCH;
        const int nt = (t0 + TCH <= C::NT) ? TCH : C::NT - t0;
        acc_t acc[TCH];
#pragma unroll
        for (int t = 0; t < TCH; ++t) acc[t] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const frag_t a = load_afrag<PREC>(W.gbuf, C::ROW, lane, s);
            frag_t b[TCH];
#pragma unroll
            for (int t = 0; t < TCH; ++t) {
                if (t < nt) {
                    const int tt = t0 + t;
                    if constexpr (C::RREG) b[t] = W.rreg[tt][s];
                    else if (tt < C::RLT) b[t] = W.rlds[(tt * KS + s) * 64 + lane];
                    else b[t] = W.rglb[(tt * KS + s) * 64 + lane];
                }
            }
#pragma unroll
            for (int t = 0; t < TCH; ++t)
                if (t < nt) acc[t] = mfma<PREC>(a, b[t], acc[t]);
        }
        // stage: accumulator (row, entry (a, b)) of upper block (c, c2) of a
        // cell goes to (c n + a, c2 n + b) and to (c2 n + b, c n + a) of the
        // cell's slot. On a diagonal block (c = c2) the second write lands on
        // (b, a) of the same block: every entry of it is written once from
        // (a, b) and once from (b, a), two roundings of the same sum of the
        // symmetric integrand, and the later write in program order stays
        // (no branch per row; the result is the same on every run).
#pragma unroll
        for (int t = 0; t < TCH; ++t) {
            if (t < nt) {
                // this lane's column of n-tile t0 + t is entry (a, b): at a N + b
                // in an upper block, at b N + a in the transposed lower block
                const int el = 16 * (t0 + t) + (lane & 15);
                const int ea = el / NS, eb = el - (el / NS) * NS;
                const int od = ea * N + eb, ot = eb * N + ea;
                const bool ok = 16 * (t0 + t) + 16 <= NN || el < NN;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const out_t x = (out_t)acc[t][v];
                    if (ok) {
                        W.ring[based[v] + od] = x;
                        W.ring[baset[v] + ot] = x;
                    }
                }
            }
        }
    }
    wave_sync();
    // cells [cd0, cd1) of the unit are complete: one contiguous range of
    // the output. Their slots are consecutive except where the ring wraps
    // (compile-time: chunk WQ of the range is the first one in slot 0).
    constexpr int cd0 = (16 * m) / NB, cd1 = (16 * (m + 1)) / NB;
    constexpr int CPC = C::CPC, NQ = (cd1 - cd0) * CPC;
    constexpr int s0 = cd0 & (C::RING - 1), WQ = (C::RING - s0) * CPC, WRAP = C::RING * CPC;
    if constexpr (NQ > 0) {
        const vu32x4* rb = reinterpret_cast<const vu32x4*>(W.ring) + s0 * CPC;
        // a wave-uniform base and 32-bit byte offsets: scalar base addressing
        char* dst = reinterpret_cast<char*>(uniform_ptr(reinterpret_cast<vu32x4*>(A.out) +
                                                        (unit_base + cd0) * (int64_t)CPC));
#pragma unroll
        for (int q0 = 0; q0 < NQ; q0 += 64) {
            const int q = q0 + lane;
            int li = q;
            if constexpr (WQ < NQ) {
                if (q0 >= WQ) li = q - WRAP;
                else if (q0 + 64 > WQ) li = q >= WQ ? q - WRAP : q;
            }
            bool ok = q0 + 64 <= NQ || q < NQ;
            if constexpr (!FULL) ok = ok && unit_base + cd0 + q / CPC < A.ncells;
            if (ok) gstore_nt(reinterpret_cast<vu32x4*>(dst + (uint32_t)(q * 16)), rb[li]);
        }
    }
    wave_sync();
}

template <int D, int P, int FD, int PREC, bool FULL, int m>
__device__ __forceinline__ void el_rowtiles(const LinArgs& A, const ElWave<D, P, FD, PREC>& W,
                                   const VCell<F_ELAST, D, FD>& cd, int64_t unit_base) {
    el_rowtile<D, P, FD, PREC, FULL, m>(A, W, cd, unit_base);
    if constexpr (m + 1 < ElCfg<D, P, FD, PREC>::NB) el_rowtiles<D, P, FD, PREC, FULL, m + 1>(A, W, cd, unit_base);
}

// Persistent kernel: units of 16 cells, WAVES units per chunk, XCD-aware chunk
// order and two-deep gather prefetch as in the panel engine (vector.hpp).
// LinArgs::nchunks = ceil(ncells / (16 WAVES)).
template <int D, int P, int FD, int PREC>
__global__ __launch_bounds__((ElCfg<D, P, FD, PREC>::WAVES * 64)) void k_elast(LinArgs A) {
    using C = ElCfg<D, P, FD, PREC>;
    using frag_t = typename C::frag_t;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    ElWave<D, P, FD, PREC> W;
    W.lane = threadIdx.x & 63;
    const int g = W.lane >> 4;
    unsigned char* mine = lds + C::RLT * C::S.tile_bytes + wave * C::S.wave_bytes;
    W.gbuf = reinterpret_cast<typename C::g_t*>(mine);
    W.ring = reinterpret_cast<typename C::out_t*>(mine + C::S.g_bytes);
    const frag_t* rg = reinterpret_cast<const frag_t*>(A.rfrag);
    W.rglb = rg;
    W.rlds = reinterpret_cast<const frag_t*>(lds);
    if constexpr (C::RLT > 0) {
        frag_t* sR = reinterpret_cast<frag_t*>(lds);
        for (int i = threadIdx.x; i < C::RLT * C::KS * 64; i += C::WAVES * 64) sR[i] = rg[i];
        __syncthreads();
    }
    if constexpr (C::RREG) {
#pragma unroll
        for (int t = 0; t < C::NT; ++t)
#pragma unroll
            for (int s = 0; s < C::KS; ++s) W.rreg[t][s] = rg[(t * C::KS + s) * 64 + W.lane];
    }
    const int64_t GS = gridDim.x;
    const int64_t b = blockIdx.x;
    int64_t chunk = (GS % 8 == 0) ? (b % 8) * (GS / 8) + b / 8 : b;
    const int64_t nfull = A.ncells / 16;  // units whose 16 cells all exist
    auto unit_of = [&](int64_t ch) -> int64_t { return ch * C::WAVES + wave; };
    auto cell_of = [&](int64_t unit) -> int64_t { return unit * 16 + (W.lane & 15); };
    int64_t unit = unit_of(chunk);
    VIdx<F_ELAST, D, FD> ix;
    VRaw<F_ELAST, D, FD> raw;
    VCell<F_ELAST, D, FD> cd;
    if (unit < nfull) {
        vload_idx<F_ELAST, D, FD>(A, cell_of(unit), g, ix);
        vload_raw<F_ELAST, D, FD>(A, cell_of(unit), g, ix, raw);
        vcell_from_raw<F_ELAST, D, FD>(raw, cd);
        const int64_t u1 = unit_of(chunk + GS) < nfull ? unit_of(chunk + GS) : unit;
        vload_idx<F_ELAST, D, FD>(A, cell_of(u1), g, ix);
#pragma unroll
        for (int v = 0; v <= D; ++v) asm volatile("" ::"v"(ix.v[v]));
        asm volatile("" ::"v"(cd.ad));
    }
    while (unit < nfull) {
        const int64_t next = unit_of(chunk + GS);
        const int64_t n1 = next < nfull ? next : unit;
        const int64_t n2 = unit_of(chunk + 2 * GS) < nfull ? unit_of(chunk + 2 * GS) : unit;
        vload_raw<F_ELAST, D, FD>(A, cell_of(n1), g, ix, raw);
        vload_idx<F_ELAST, D, FD>(A, cell_of(n2), g, ix);
        el_rowtiles<D, P, FD, PREC, true, 0>(A, W, cd, unit * 16);
        vcell_from_raw<F_ELAST, D, FD>(raw, cd);
        chunk += GS;
        unit = next;
    }
    if (unit * 16 < A.ncells) {
        // the one partial unit: clamped loads, bounds-checked stores
        const int64_t last = A.ncells - 1;
        const int64_t c = cell_of(unit) < last ? cell_of(unit) : last;
        VIdx<F_ELAST, D, FD> ix2;
        VRaw<F_ELAST, D, FD> raw2;
        vload_idx<F_ELAST, D, FD>(A, c, g, ix2);
        vload_raw<F_ELAST, D, FD>(A, c, g, ix2, raw2);
        vcell_from_raw<F_ELAST, D, FD>(raw2, cd);
        el_rowtiles<D, P, FD, PREC, false, 0>(A, W, cd, unit * 16);
    }
}

}  // namespace dev
}  // namespace coffee
