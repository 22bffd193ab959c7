// Device engine for the vector-valued bilinear forms (elasticity, Burgers
// Jacobian): the element tensor of a cell is NC x NC blocks,
//     A[e][c n + a][c' n + b] = sum_k G_cc'[e][k] R[k][a n + b],
// one shared reference tensor R and a per-cell, per-block geometry row G_cc'
// (section 2, Fig. 1; the quadrature sum collapsed into R as in linear.hpp).
//
// Work unit: one wave takes a tile of 16 consecutive cells (the M dimension of
// the MFMA products) and completes it before the next tile, panel by panel:
// panel c is rows c n .. c n + n - 1 of every cell's tensor, NC n values per
// row, so a panel is one contiguous range of each cell's tensor. A panel is
// computed in row groups (a few rows, so that the accumulators of all NC
// blocks of the group stay in registers; R is packed group by group): the wave
// builds G_cc' of its 16 cells in LDS (lane (cell, g) writes the entries of
// the coefficient dofs r = g, g + 4, ...), contracts it against R's column
// tiles of the group (all NC blocks in one k-loop that loads each R fragment
// once, when their G rows fit in LDS), then the group's rows are transposed
// through LDS and leave as 16-byte stores covering whole contiguous ranges of
// 4 (or 16) cells. Writing every output line completely, once, keeps the
// store traffic at the algorithmic bytes: partial lines written at different
// times reach HBM more than once. The whole tile is unrolled, so that the
// wait for the next tile's prefetched gathers does not wait for this tile's
// stores (one in-order counter covers loads and stores).
#pragma once
#include "linear.hpp"

namespace coffee {
namespace dev {

typedef unsigned int vu32x4 __attribute__((ext_vector_type(4)));

// Rows per group of a panel: at most tb column tiles of 16 entries per block,
// so that the accumulators of all blocks of a group stay in registers. The
// reference tensor is packed group by group (library.hip), each group's
// entries a n + b starting on a fresh column tile.
__host__ __device__ constexpr int vec_rows_per_group(int ns, int tb) {
    const int r = (16 * tb) / ns;
    return r < 1 ? 1 : (r > ns ? ns : r);
}

// Column tiles per row group: the FP64 Burgers kernel, whose lanes also hold
// three state vectors, gets fewer, so that two waves fit on a SIMD.
__host__ __device__ constexpr int vec_group_tiles(int form, int prec) {
    return (prec == PREC_F64 && form == F_BURG) ? 2 : 4;
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// K steps and G row length of the vector engine. BF16X3 uses four k slots per
// G entry, (G_hi, G_hi, G_lo, 0) against (R_hi, R_lo, R_hi, 0), so that an
// entry is one aligned 8-byte LDS store and the zero leading steps of the
// off-diagonal Burgers blocks can still be skipped.
__host__ __device__ constexpr int vec_ksteps(int form, int d, int fd, int prec) {
    return prec == PREC_BF16X3 ? (4 * kref(form, d, fd) + 31) / 32 : ksteps(form, d, fd, prec);
}
__host__ __device__ constexpr int vec_row(int form, int d, int fd, int prec) {
    return prec == PREC_BF16X3 ? vec_ksteps(form, d, fd, prec) * 32 + 8 : vec_ksteps(form, d, fd, prec) * 4 + 1;
}

// Coefficient dofs per lane group, fields per dof, components per field.
template <int FORM, int D, int FD>
struct VLane {
    static constexpr int NF = nfield(D, FD);
    static constexpr int RPL = FD > 0 ? (NF + 3) / 4 : 1;
    static constexpr int NFLD = FORM == F_ELAST ? 2 : 1;
    static constexpr int WC = FORM == F_BURG ? D : 1;
};

template <int FORM, int D, int P, int FD, int PREC>
struct VecCfg {
    using g_t = typename PrecT<PREC>::gtype;
    using frag_t = typename PrecT<PREC>::frag;
    using acc_t = typename PrecT<PREC>::acc;
    using out_t = typename PrecT<PREC>::otype;
    static constexpr int NS = nsc(D, P);
    static constexpr int NN = NS * NS;
    static constexpr int NC = D;
    static constexpr int N = NC * NS;
    static constexpr int KR = kref(FORM, D, FD);
    static constexpr int KS = vec_ksteps(FORM, D, FD, PREC);
    static constexpr int NT = ntiles(D, P);
    static constexpr int ROW = vec_row(FORM, D, FD, PREC);
    static constexpr int NF = VLane<FORM, D, FD>::NF;
    static constexpr int RPL = VLane<FORM, D, FD>::RPL;
    static constexpr int TB = vec_group_tiles(FORM, PREC);
    static constexpr int RGR = vec_rows_per_group(NS, TB);
    static constexpr int NG = (NS + RGR - 1) / RGR;
    static constexpr int row0(int g) { return g * RGR; }
    static constexpr int row1(int g) { return (g + 1) * RGR < NS ? (g + 1) * RGR : NS; }
    static constexpr int tiles_of(int g) { return ((row1(g) - row0(g)) * NS + 15) / 16; }
    static constexpr int tile_off(int g) { return g == 0 ? 0 : tile_off(g - 1) + tiles_of(g - 1); }
    static constexpr int NTP = tile_off(NG);  // packed column tiles of R
    static constexpr int RGMAX = RGR;
    // reference fragments: registers when few, else LDS (shared by the
    // workgroup) when they fit, else read through the caches
    static constexpr int NFRAG = NTP * KS * 64;
    static constexpr int RBYTES = NFRAG * (int)sizeof(frag_t);
    static constexpr bool RREG = NTP * KS * (int)(sizeof(frag_t) / 4) <= 32;
    static constexpr bool RLDS = !RREG && RBYTES <= 64 * 1024;
    // 8 waves: two per SIMD, which is what the registers allow
    static constexpr int WAVES = 8;
    // output staging: 16 cells per pass when that takes at most 8 KiB, else 4
    static constexpr int SLOT = RGMAX * N;  // values of one cell's row group
    static constexpr int CPP = 16 * SLOT * (int)sizeof(out_t) <= 8192 ? 16 : 4;
    static constexpr int STAGE_BYTES = CPP * SLOT * (int)sizeof(out_t);
    static constexpr int RLDS_BYTES = RLDS ? (RBYTES + 15) / 16 * 16 : 0;
    // merged blocks: the G rows of all NC blocks of a row group are built
    // together and contracted in one k-loop that loads each reference
    // fragment once for the NC blocks (a third of the fragment traffic, and NC
    // times the MFMAs per wait), when the NC G buffers fit the LDS budget
    static constexpr int GROW = ROW;  // G row length in LDS
    static constexpr int wave_bytes(int nblk) {
        return (cmax(STAGE_BYTES, nblk * 16 * GROW * (int)sizeof(g_t)) + 15) / 16 * 16;
    }
    static constexpr bool MERGED = RLDS_BYTES + WAVES * wave_bytes(NC) <= 160 * 1024;
    static constexpr int WAVE_BYTES = wave_bytes(MERGED ? NC : 1);
    static constexpr int LDS_BYTES = RLDS_BYTES + WAVES * WAVE_BYTES;
    // 16-byte stores need every group's range and the cell stride aligned
    static constexpr int PER16 = 16 / (int)sizeof(out_t);
    static constexpr bool groups_aligned() {
        for (int g = 0; g < NG; ++g)
            if ((row1(g) - row0(g)) * N % PER16 != 0 || row0(g) * N % PER16 != 0) return false;
        return true;
    }
    static constexpr bool VEC16 = (N * NS % PER16 == 0) && (N * N % PER16 == 0) && groups_aligned();
    static_assert(LDS_BYTES <= 160 * 1024, "LDS budget exceeded");
};

// First k-step that can hold a nonzero G entry of block (c1, c2): the
// off-diagonal blocks of the Burgers Jacobian carry only the E(r, a) terms,
// which come last in the tensor order, so their leading steps are skipped
// (structurally zero blocks of the reference products are never contracted).
template <int FORM, int D, int FD, int PREC>
__device__ constexpr int vec_kstep_begin(int c1, int c2) {
    constexpr int K0 = 1 + npair(D) + nfield(D, FD) * D;  // first E(r, a) entry
    return (FORM == F_BURG && c1 != c2) ? (PREC == PREC_BF16X3 ? (4 * K0) / 32 : K0 / kstep(PREC)) : 0;
}

// ---------------------------------------------------------------- per-lane cell data
// Lane (cell = lane % 16, g = lane / 16) holds the geometry of its cell and the
// coefficient values of the dofs r = g + 4 j it builds G entries for.

template <int FORM, int D, int FD>
struct VIdx {
    using C = VLane<FORM, D, FD>;
    int v[D + 1];
    int f[C::NFLD][C::RPL];
};

template <int FORM, int D, int FD>
struct VRaw {
    using C = VLane<FORM, D, FD>;
    double x[D + 1][D];
    double f[C::NFLD][C::RPL][C::WC];
};

template <int FORM, int D, int FD>
struct VCell {
    using C = VLane<FORM, D, FD>;
    double K[D][D];
    double M[D][D];  // K K^T
    double ad;
    double f[C::NFLD][C::RPL][C::WC];
};

template <int FORM, int D, int FD>
__device__ inline void vload_idx(const LinArgs& A, int64_t cell, int g, VIdx<FORM, D, FD>& ix) {
    using C = VLane<FORM, D, FD>;
    const int32_t* cv = A.c2v + cell * (D + 1);
#pragma unroll
    for (int v = 0; v <= D; ++v) ix.v[v] = __builtin_nontemporal_load(cv + v);
    if constexpr (FD > 0) {
#pragma unroll
        for (int fl = 0; fl < C::NFLD; ++fl) {
            const FieldArg& F = fl == 0 ? A.f0 : A.f1;
#pragma unroll
            for (int j = 0; j < C::RPL; ++j) {
                const int r = g + 4 * j;
                ix.f[fl][j] = 0;
                if (F.map && r < C::NF) ix.f[fl][j] = __builtin_nontemporal_load(F.map + cell * C::NF + r);
            }
        }
    }
}

template <int FORM, int D, int FD>
__device__ inline void vload_raw(const LinArgs& A, int64_t cell, int g, const VIdx<FORM, D, FD>& ix,
                                 VRaw<FORM, D, FD>& rw) {
    using C = VLane<FORM, D, FD>;
#pragma unroll
    for (int v = 0; v <= D; ++v)
#pragma unroll
        for (int i = 0; i < D; ++i) rw.x[v][i] = A.coords[(int64_t)ix.v[v] * D + i];
    if constexpr (FD > 0) {
#pragma unroll
        for (int fl = 0; fl < C::NFLD; ++fl) {
            const FieldArg& F = fl == 0 ? A.f0 : A.f1;
#pragma unroll
            for (int j = 0; j < C::RPL; ++j) {
                const int r = g + 4 * j;
                const int64_t base = F.map ? (int64_t)ix.f[fl][j] * C::WC : (cell * C::NF + r) * C::WC;
#pragma unroll
                for (int c = 0; c < C::WC; ++c) rw.f[fl][j][c] = r < C::NF ? F.values[base + c] : 0.0;
            }
        }
    }
}

template <int FORM, int D, int FD>
__device__ inline void vcell_from_raw(const VRaw<FORM, D, FD>& rw, VCell<FORM, D, FD>& cd) {
    Geom<D> g;
    geometry_from_coords<D>(rw.x, g);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) cd.K[i][j] = g.K[i][j];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) t += g.K[a][i] * g.K[b][i];
            cd.M[a][b] = t;
        }
    cd.ad = g.adet;
    if constexpr (FD > 0) {
#pragma unroll
        for (int fl = 0; fl < VCell<FORM, D, FD>::C::NFLD; ++fl)
#pragma unroll
            for (int j = 0; j < VCell<FORM, D, FD>::C::RPL; ++j)
#pragma unroll
                for (int c = 0; c < VCell<FORM, D, FD>::C::WC; ++c) cd.f[fl][j][c] = rw.f[fl][j][c];
    }
}

// ---------------------------------------------------------------- G rows

// Entry k of a G row in the precision's layout (BF16X3: slots 4k .. 4k + 3
// hold hi, hi, lo, 0).
template <int PREC, int KR>
__device__ inline void put_g(typename PrecT<PREC>::gtype* row, int k, double v) {
    if constexpr (PREC == PREC_F64) {
        row[k] = v;
    } else if constexpr (PREC == PREC_F32) {
        row[k] = (float)v;
    } else {
        const float x = (float)v;
        const u16 hi = bf16_bits_rne(x);
        const u16 lo = bf16_bits_rne(x - bf16_to_float(hi));
        const uint2 w = make_uint2((uint32_t)hi | ((uint32_t)hi << 16), (uint32_t)lo);
        *reinterpret_cast<uint2*>(row + 4 * k) = w;
    }
}

// x[c] for an index c that is not a compile-time constant, as a sum of
// products with 0/1 weights (a select chain or an indexed access would be
// turned into a stack load).
template <int D>
__device__ inline double pick(const double (&x)[D], int c) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) v += (c == j ? 1.0 : 0.0) * x[j];
    return v;
}

// Lane (cell row, group g) writes its share of G_{C1 C2} for its cell (same
// entries and order as build_G in linear.hpp). Invalid cells get zero rows.
template <int FORM, int D, int FD, int PREC, int C1, int C2>
__device__ inline void vec_put_G(const LinArgs& A, const VCell<FORM, D, FD>& cd, bool valid,
                                 typename PrecT<PREC>::gtype* row, int g) {
    using C = VLane<FORM, D, FD>;
    constexpr int KR = kref(FORM, D, FD), NF = C::NF, KS = vec_ksteps(FORM, D, FD, PREC);
    const auto& K = cd.K;
    const auto& M = cd.M;
    const double ad = valid ? cd.ad : 0.0;
    constexpr bool diag = C1 == C2;
    double k1[D];  // column C1 of K
#pragma unroll
    for (int a = 0; a < D; ++a) k1[a] = K[a][C1];
    if constexpr (FORM == F_ELAST) {
#pragma unroll
        for (int j = 0; j < C::RPL; ++j) {
            const int r = g + 4 * j;
            if (r < NF) {
                const double mu = ad * (FD > 0 ? cd.f[0][j][0] : A.c0);
                const double lm = ad * (FD > 0 ? cd.f[1][j][0] : A.c1);
#pragma unroll
                for (int a = 0; a < D; ++a)
#pragma unroll
                    for (int b = 0; b < D; ++b) {
                        const double kk = diag ? M[a][b] : 0.0;
                        put_g<PREC, KR>(row, r * D * D + a * D + b,
                                        mu * (kk + K[a][C2] * k1[b]) + lm * k1[a] * K[b][C2]);
                    }
            }
        }
    } else {  // F_BURG
        if (g == 0) {
            put_g<PREC, KR>(row, 0, diag ? ad * A.c1 : 0.0);
            int t = 1;
            const double sc = ad * A.c0;
#pragma unroll
            for (int a = 0; a < D; ++a)
#pragma unroll
                for (int b = a; b < D; ++b) put_g<PREC, KR>(row, t++, diag ? sc * M[a][b] : 0.0);
        }
        constexpr int OC = 1 + npair(D), OE = OC + NF * D;
#pragma unroll
        for (int j = 0; j < C::RPL; ++j) {
            const int r = g + 4 * j;
            if (r < NF) {
                const double* w = cd.f[0][j];
                const double wc = ad * cd.f[0][j][C1];
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    double t = 0.0;
#pragma unroll
                    for (int i = 0; i < D; ++i) t += w[i] * K[a][i];
                    put_g<PREC, KR>(row, OC + r * D + a, diag ? ad * t : 0.0);
                    put_g<PREC, KR>(row, OE + r * D + a, wc * K[a][C2]);
                }
            }
        }
    }
    // zero padding of the last k-step
    if (g == 0) {
        if constexpr (PREC == PREC_BF16X3) {
#pragma unroll
            for (int k = 4 * KR; k < KS * 32; ++k) row[k] = 0;
        } else {
#pragma unroll
            for (int k = KR; k < KS * 4; ++k) row[k] = 0;
        }
    }
}

// ---------------------------------------------------------------- one tile

template <int FORM, int D, int P, int FD, int PREC>
struct VecWave {
    using C = VecCfg<FORM, D, P, FD, PREC>;
    typename C::g_t* gbuf;     // 16 G rows (shares its LDS with the stage)
    typename C::out_t* stage;  // CPP cells x SLOT values
    const typename C::frag_t* rsrc;
    typename C::frag_t rreg[C::RREG ? C::NTP : 1][C::RREG ? C::KS : 1];
    int lane, g;
};

// Row (cell in the tile) of the staging slot s in pass v.
template <int PREC>
__device__ constexpr int slot_row(int s, int v) {
    return PREC == PREC_F64 ? s + 4 * v : 4 * s + v;
}

// Store the staged rows of the cells of one pass: slot s holds rows a0 .. a1-1
// of panel c (contiguous in the output) of cell tile_base + row(s).
template <int FORM, int D, int P, int FD, int PREC, bool FULL, int GI, int c>
__device__ inline void vec_store_pass(const LinArgs& A, const VecWave<FORM, D, P, FD, PREC>& W, int v,
                                      int64_t tile_base) {
    using C = VecCfg<FORM, D, P, FD, PREC>;
    using out_t = typename C::out_t;
    constexpr int NS = C::NS, N = C::N, CPP = C::CPP;
    constexpr int a0 = C::row0(GI), a1 = C::row1(GI);
    constexpr int L = (a1 - a0) * N;  // values per slot
    // tile_base and c are wave-uniform: one scalar base, 32-bit lane offsets;
    // the lane index is re-read opaquely so that the offsets are recomputed
    // here instead of being hoisted out of the tile loop into registers
    out_t* tb = reinterpret_cast<out_t*>(A.out) + tile_base * (int64_t)(N * N) + (int64_t)(c * NS + a0) * N;
    int lane = W.lane;
    asm volatile("" : "+v"(lane));
    // lanes 16 j .. 16 j + 15 take slot 4 sg + j (sg = slot quad), consecutive
    // 16-byte chunks (or values) of that slot's contiguous range
    const int sl = lane >> 4, ql = lane & 15;
    auto row_of = [&](int s) -> int { return CPP == 16 ? s : slot_row<PREC>(s, v); };
    constexpr int CH = C::VEC16 ? L / C::PER16 : L;  // chunks per slot
#pragma unroll
    for (int sg = 0; sg < CPP / 4; ++sg) {
        const int s = 4 * sg + sl;
        const int r = row_of(s);
        const bool ok = FULL || tile_base + r < A.ncells;
#pragma unroll
        for (int q0 = 0; q0 < CH; q0 += 16) {
            const int q = q0 + ql;
            if ((q0 + 16 <= CH || q < CH) && ok) {
                if constexpr (C::VEC16) {
                    const vu32x4 x = reinterpret_cast<const vu32x4*>(W.stage)[s * (C::SLOT / C::PER16) + q];
                    *reinterpret_cast<vu32x4*>(tb + (uint32_t)(r * (N * N) + q * C::PER16)) = x;
                } else {
                    tb[(uint32_t)(r * (N * N) + q)] = W.stage[s * C::SLOT + q];
                }
            }
        }
    }
}

// Contract block (c, C2) of row group GI into acc[C2], then the next block.
template <int FORM, int D, int P, int FD, int PREC, int GI, int c, int C2>
__device__ inline void vec_blocks(const LinArgs& A, const VecWave<FORM, D, P, FD, PREC>& W,
                                  const VCell<FORM, D, FD>& cd, bool valid, int lane,
                                  typename PrecT<PREC>::acc (&acc)[D][VecCfg<FORM, D, P, FD, PREC>::tiles_of(GI)]) {
    using C = VecCfg<FORM, D, P, FD, PREC>;
    using acc_t = typename C::acc_t;
    using frag_t = typename C::frag_t;
    constexpr int KS = C::KS, ROW = C::GROW;
    constexpr int t0 = C::tile_off(GI), NTG = C::tiles_of(GI);
    // keeps the scheduler from building the G rows of later blocks early
    __builtin_amdgcn_sched_barrier(0);
    vec_put_G<FORM, D, FD, PREC, c, C2>(A, cd, valid, W.gbuf + (lane & 15) * ROW, W.g);
    wave_sync();
#pragma unroll
    for (int t = 0; t < NTG; ++t) acc[C2][t] = acc_t{0, 0, 0, 0};
    constexpr int kb = vec_kstep_begin<FORM, D, FD, PREC>(c, C2);
    if constexpr (C::RREG) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s < kb) continue;
            const frag_t a = load_afrag<PREC>(W.gbuf, ROW, lane, s);
#pragma unroll
            for (int t = 0; t < NTG; ++t) acc[C2][t] = mfma<PREC>(a, W.rreg[t0 + t][s], acc[C2][t]);
        }
    } else {
        // a rolled loop: unrolled, the scheduler hoists every fragment load
        // of the block and runs out of registers
#pragma unroll 1
        for (int s = kb; s < KS; ++s) {
            const frag_t a = load_afrag<PREC>(W.gbuf, ROW, lane, s);
            frag_t b[NTG];
#pragma unroll
            for (int t = 0; t < NTG; ++t) b[t] = W.rsrc[((t0 + t) * KS + s) * 64 + lane];
#pragma unroll
            for (int t = 0; t < NTG; ++t) acc[C2][t] = mfma<PREC>(a, b[t], acc[C2][t]);
        }
    }
    wave_sync();
    if constexpr (C2 + 1 < D) vec_blocks<FORM, D, P, FD, PREC, GI, c, C2 + 1>(A, W, cd, valid, lane, acc);
}

// Build the G rows of block (c, C2) into its own buffer, then the next block.
template <int FORM, int D, int P, int FD, int PREC, int c, int C2>
__device__ inline void vec_put_G_all(const LinArgs& A, const VecWave<FORM, D, P, FD, PREC>& W,
                                     const VCell<FORM, D, FD>& cd, bool valid, int lane) {
    using C = VecCfg<FORM, D, P, FD, PREC>;
    vec_put_G<FORM, D, FD, PREC, c, C2>(A, cd, valid, W.gbuf + C2 * 16 * C::GROW + (lane & 15) * C::GROW, W.g);
    if constexpr (C2 + 1 < D) vec_put_G_all<FORM, D, P, FD, PREC, c, C2 + 1>(A, W, cd, valid, lane);
}

// All NC blocks (c, c2) of row group GI in one k-loop: each step loads the
// group's reference fragments once and the NC blocks' G fragments.
template <int FORM, int D, int P, int FD, int PREC, int GI, int c>
__device__ inline void vec_blocks_merged(const LinArgs& A, const VecWave<FORM, D, P, FD, PREC>& W,
                                         const VCell<FORM, D, FD>& cd, bool valid, int lane,
                                         typename PrecT<PREC>::acc (&acc)[D][VecCfg<FORM, D, P, FD, PREC>::tiles_of(GI)]) {
    using C = VecCfg<FORM, D, P, FD, PREC>;
    using acc_t = typename C::acc_t;
    using frag_t = typename C::frag_t;
    constexpr int KS = C::KS, ROW = C::GROW, NC = C::NC;
    constexpr int t0 = C::tile_off(GI), NTG = C::tiles_of(GI);
    __builtin_amdgcn_sched_barrier(0);
    vec_put_G_all<FORM, D, P, FD, PREC, c, 0>(A, W, cd, valid, lane);
    wave_sync();
#pragma unroll
    for (int c2 = 0; c2 < NC; ++c2)
#pragma unroll
        for (int t = 0; t < NTG; ++t) acc[c2][t] = acc_t{0, 0, 0, 0};
    // unrolled (immediate fragment offsets), one scheduling region per step
    // so that the loads of one step are not all hoisted to the top
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        frag_t b[NTG];
#pragma unroll
        for (int t = 0; t < NTG; ++t) {
            if constexpr (C::RREG) b[t] = W.rreg[t0 + t][s];
            else b[t] = W.rsrc[((t0 + t) * KS + s) * 64 + lane];
        }
#pragma unroll
        for (int c2 = 0; c2 < NC; ++c2) {
            if (s < vec_kstep_begin<FORM, D, FD, PREC>(c, c2)) continue;
            const frag_t a = load_afrag<PREC>(W.gbuf + c2 * 16 * ROW, ROW, lane, s);
#pragma unroll
            for (int t = 0; t < NTG; ++t) acc[c2][t] = mfma<PREC>(a, b[t], acc[c2][t]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    wave_sync();
}

// Panel c, row group GI of the tile at tile_base.
template <int FORM, int D, int P, int FD, int PREC, bool FULL, int GI, int c>
__device__ inline void vec_group(const LinArgs& A, const VecWave<FORM, D, P, FD, PREC>& W,
                                 const VCell<FORM, D, FD>& cd, bool valid, int64_t tile_base) {
    using C = VecCfg<FORM, D, P, FD, PREC>;
    using acc_t = typename C::acc_t;
    using frag_t = typename C::frag_t;
    using out_t = typename C::out_t;
    constexpr int NS = C::NS, NN = C::NN, N = C::N, NC = C::NC, KS = C::KS, ROW = C::GROW;
    constexpr int a0 = C::row0(GI), a1 = C::row1(GI);
    constexpr int t0 = C::tile_off(GI), NTG = C::tiles_of(GI), NE = (a1 - a0) * NS;
    int lane = W.lane;
    asm volatile("" : "+v"(lane));  // lane-derived offsets: recomputed per group, not hoisted
    const int col = lane & 15;
    acc_t acc[NC][NTG];
    if constexpr (C::MERGED) vec_blocks_merged<FORM, D, P, FD, PREC, GI, c>(A, W, cd, valid, lane, acc);
    else vec_blocks<FORM, D, P, FD, PREC, GI, c, 0>(A, W, cd, valid, lane, acc);
    // transpose through LDS: group entry 16 t + col of block (c, c2) is
    // (a, b) = (a0, 0) + divmod(16 t + col, n), row a, column c2 n + b of the panel
    constexpr int NPASS = C::CPP == 16 ? 1 : 4;
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
#pragma unroll
        for (int t = 0; t < NTG; ++t) {
            const int el = 16 * t + col;
            const int a = el / NS, b = el - (el / NS) * NS;  // a relative to a0
            if (el < NE) {
#pragma unroll
                for (int c2 = 0; c2 < NC; ++c2) {
                    const int e = a * N + c2 * NS + b;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (NPASS == 4 && v != pass) continue;
                        const int s = NPASS == 1 ? acc_row<PREC>(lane, v) : (lane >> 4);
                        W.stage[s * C::SLOT + e] = (out_t)acc[c2][t][v];
                    }
                }
            }
        }
        wave_sync();
        vec_store_pass<FORM, D, P, FD, PREC, FULL, GI, c>(A, W, pass, tile_base);
        wave_sync();
    }
}

// Panels c .. D-1 (row groups GI .. NG-1 of panel c first). Everything is
// unrolled, so the number of stores between a prefetch load and its use is a
// compile-time count and the wait for the load need not wait for the stores
// (loads and stores share one in-order counter).
template <int FORM, int D, int P, int FD, int PREC, bool FULL, int c, int GI>
__device__ inline void vec_panels(const LinArgs& A, const VecWave<FORM, D, P, FD, PREC>& W,
                                  const VCell<FORM, D, FD>& cd, bool valid, int64_t tile_base) {
    vec_group<FORM, D, P, FD, PREC, FULL, GI, c>(A, W, cd, valid, tile_base);
    if constexpr (GI + 1 < VecCfg<FORM, D, P, FD, PREC>::NG)
        vec_panels<FORM, D, P, FD, PREC, FULL, c, GI + 1>(A, W, cd, valid, tile_base);
    else if constexpr (c + 1 < D)
        vec_panels<FORM, D, P, FD, PREC, FULL, c + 1, 0>(A, W, cd, valid, tile_base);
}

template <int FORM, int D, int P, int FD, int PREC, bool FULL>
__device__ inline void vec_tile(const LinArgs& A, const VecWave<FORM, D, P, FD, PREC>& W,
                                const VCell<FORM, D, FD>& cd, int64_t tile_base) {
    const bool valid = FULL || tile_base + (W.lane & 15) < A.ncells;
    vec_panels<FORM, D, P, FD, PREC, FULL, 0, 0>(A, W, cd, valid, tile_base);
}

// Persistent kernel: each workgroup takes chunks of WAVES tiles (XCD-aware
// order: consecutive chunks of one XCD are consecutive ranges of cells); the
// gathers of a wave's next tile are issued before the current tile's stores
// (indices two tiles ahead, coordinates and coefficient values one ahead).
// LinArgs::nchunks = ceil(ncells / (16 WAVES)).
template <int FORM, int D, int P, int FD, int PREC>
__global__ __launch_bounds__((VecCfg<FORM, D, P, FD, PREC>::WAVES * 64)) void k_vector(LinArgs A) {
    using C = VecCfg<FORM, D, P, FD, PREC>;
    using frag_t = typename C::frag_t;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    VecWave<FORM, D, P, FD, PREC> W;
    W.lane = threadIdx.x & 63;
    W.g = W.lane >> 4;
    unsigned char* mine = lds + C::RLDS_BYTES + wave * C::WAVE_BYTES;
    W.gbuf = reinterpret_cast<typename C::g_t*>(mine);
    W.stage = reinterpret_cast<typename C::out_t*>(mine);
    const frag_t* rg = reinterpret_cast<const frag_t*>(A.rfrag);
    W.rsrc = rg;
    if constexpr (C::RLDS) {
        frag_t* sR = reinterpret_cast<frag_t*>(lds);
        for (int i = threadIdx.x; i < C::NFRAG; i += C::WAVES * 64) sR[i] = rg[i];
        __syncthreads();
        W.rsrc = sR;
    }
    if constexpr (C::RREG) {
#pragma unroll
        for (int t = 0; t < C::NTP; ++t)
#pragma unroll
            for (int s = 0; s < C::KS; ++s) W.rreg[t][s] = rg[(t * C::KS + s) * 64 + W.lane];
    }
    const int64_t GS = gridDim.x;
    const int64_t b = blockIdx.x;
    int64_t chunk = (GS % 8 == 0) ? (b % 8) * (GS / 8) + b / 8 : b;
    const int64_t nfull = A.ncells / 16;  // tiles whose 16 cells all exist
    auto tile_of = [&](int64_t ch) -> int64_t { return ch * C::WAVES + wave; };
    auto cell_of = [&](int64_t tile) -> int64_t { return tile * 16 + (W.lane & 15); };
    int64_t tile = tile_of(chunk);
    VIdx<FORM, D, FD> ix;
    VRaw<FORM, D, FD> raw;
    VCell<FORM, D, FD> cd;
    if (tile < nfull) {
        vload_idx<FORM, D, FD>(A, cell_of(tile), W.g, ix);
        vload_raw<FORM, D, FD>(A, cell_of(tile), W.g, ix, raw);
        vcell_from_raw<FORM, D, FD>(raw, cd);
        const int64_t t1 = tile_of(chunk + GS) < nfull ? tile_of(chunk + GS) : tile;
        vload_idx<FORM, D, FD>(A, cell_of(t1), W.g, ix);
#pragma unroll
        for (int v = 0; v <= D; ++v) asm volatile("" ::"v"(ix.v[v]));
        asm volatile("" ::"v"(cd.ad));
    }
    while (tile < nfull) {
        const int64_t next = tile_of(chunk + GS);
        const int64_t n1 = next < nfull ? next : tile;
        const int64_t n2 = tile_of(chunk + 2 * GS) < nfull ? tile_of(chunk + 2 * GS) : tile;
        vload_raw<FORM, D, FD>(A, cell_of(n1), W.g, ix, raw);
        vload_idx<FORM, D, FD>(A, cell_of(n2), W.g, ix);
        vec_tile<FORM, D, P, FD, PREC, true>(A, W, cd, tile * 16);
        vcell_from_raw<FORM, D, FD>(raw, cd);
        chunk += GS;
        tile = next;
    }
    if (tile * 16 < A.ncells) {
        // the one partial tile: clamped loads, bounds-checked stores
        const int64_t last = A.ncells - 1;
        const int64_t c = cell_of(tile) < last ? cell_of(tile) : last;
        VIdx<FORM, D, FD> ix2;
        VRaw<FORM, D, FD> raw2;
        vload_idx<FORM, D, FD>(A, c, W.g, ix2);
        vload_raw<FORM, D, FD>(A, c, W.g, ix2, raw2);
        vcell_from_raw<FORM, D, FD>(raw2, cd);
        vec_tile<FORM, D, P, FD, PREC, false>(A, W, cd, tile * 16);
    }
}

}  // namespace dev
}  // namespace coffee
