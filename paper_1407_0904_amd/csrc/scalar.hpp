// Device engine for the symmetric scalar forms (mass, Helmholtz).
//
// Same contraction as linear.hpp (A = G R on MFMA), specialised for one
// symmetric block: only the n(n+1)/2 entries with a <= b are contracted (the
// paper's observation that the j and k loops share one iteration space,
// section 2), and each 16-cell MFMA tile is written back through LDS so that
// the element tensors of consecutive cells leave the CU as contiguous 16-byte
// stores (cells are contiguous in the output, so 8 cells form one contiguous
// region of 8 n^2 values).
//
// Per wave: 64 cells per step, one cell per lane for the FP64 geometry and G;
// four 16-row MFMA tiles; G rows of the current tile and an 8-cell output
// staging area in LDS.
#pragma once
#include "linear.hpp"

namespace coffee {
namespace dev {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int nuniq(int d, int p) { return nsc(d, p) * (nsc(d, p) + 1) / 2; }
constexpr int ntiles_sym(int d, int p) { return (nuniq(d, p) + 15) / 16; }

template <int D, int P, int PREC>
struct StageCfg {
    static constexpr int NS = nsc(D, P);
    static constexpr int NN = NS * NS;
    static constexpr int ELEM = PREC == PREC_F64 ? 8 : 4;
    // stage 8 cells through LDS when that needs at most 16 KiB per wave
    static constexpr bool STAGE = 8 * NN * ELEM <= 16384;
    static constexpr int STAGE_ELEMS = STAGE ? 8 * NN : 1;
};

// Tile-shape variants of the symmetric engine, chosen per (form, cell,
// degree, field degree, precision) by the offline autotuner:
//   0  reference fragments held in registers when they fit (else read through
//      the L1/L2 caches), register budget of one wave per SIMD;
//   1  reference fragments staged in LDS once per workgroup, register budget
//      of two waves per SIMD;
//   2  reference fragments read through the L1/L2 caches at every use,
//      register budget of two waves per SIMD;
//   3  as 2 at three waves per SIMD, with no gather prefetch across chunks
//      (each chunk's gathers, contraction and stores in turn): launched with
//      one workgroup per chunk, the many short-lived waves keep more stores
//      in flight than a persistent grid does.
constexpr int kScalarVariants = 4;

template <int FORM, int D, int P, int FD, int PREC, int VAR = 0>
struct ScalarCfg {
    using g_t = typename PrecT<PREC>::gtype;
    using frag_t = typename PrecT<PREC>::frag;
    using acc_t = typename PrecT<PREC>::acc;
    using out_t = typename PrecT<PREC>::otype;
    static constexpr int NS = nsc(D, P);
    static constexpr int NN = NS * NS;
    static constexpr int KR = kref(FORM, D, FD);
    static constexpr int KS = ksteps(FORM, D, FD, PREC);
    static constexpr int NT = ntiles_sym(D, P);
    static constexpr int NU = nuniq(D, P);
    static constexpr int ROW = GLayout<FORM, D, FD, PREC>::ROW;
    static constexpr bool STAGE = StageCfg<D, P, PREC>::STAGE;
    static constexpr int SE = StageCfg<D, P, PREC>::STAGE_ELEMS;
    static constexpr int REGB = NT * KS * (PREC == PREC_F64 ? 2 : (PREC == PREC_F32 ? 1 : 4));
    static constexpr bool RREG = VAR == 0 && REGB <= 64;
    static constexpr bool RLDS = VAR == 1;
    static constexpr int NFRAG = NT * KS;  // reference fragments of 64 lanes
    // the staged path writes whole cells, so it needs every n-tile at once
    static constexpr int NTC = STAGE ? NT : (NT < 8 ? NT : 8);
};

// Per-lane state of the symmetric engine.
template <int FORM, int D, int P, int FD, int PREC, int VAR = 0>
struct ScalarWave {
    using C = ScalarCfg<FORM, D, P, FD, PREC, VAR>;
    typename C::g_t* gtile;
    typename C::out_t* stage;
    const typename C::frag_t* rf;  // global fragments, or the LDS copy (variant 1)
    typename C::out_t* out;
    int lane, col;
    int ua[C::NT], ub[C::NT];
    typename C::frag_t rreg[C::RREG ? C::NT : 1][C::RREG ? C::KS : 1];
};

// Accumulate n-tiles t0 .. t0 + NTC - 1 of the 16-cell tile whose G rows are
// in W.gtile.
template <int FORM, int D, int P, int FD, int PREC, int NTC, int VAR>
__device__ inline void scalar_contract(const ScalarWave<FORM, D, P, FD, PREC, VAR>& W, int t0,
                                       typename PrecT<PREC>::acc (&acc)[NTC]) {
    using C = ScalarCfg<FORM, D, P, FD, PREC, VAR>;
#pragma unroll
    for (int t = 0; t < NTC; ++t) acc[t] = typename C::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < C::KS; ++s) {
        const typename C::frag_t a = load_afrag<PREC>(W.gtile, C::ROW, W.lane, s);
#pragma unroll
        for (int t = 0; t < NTC; ++t) {
            if (t0 + t < C::NT) {
                typename C::frag_t bf;
                if constexpr (C::RREG) bf = W.rreg[t0 + t < C::NT ? t0 + t : 0][s];
                else if constexpr (C::RLDS) bf = as_lds(W.rf)[((t0 + t) * C::KS + s) * 64 + W.lane];
                else bf = gload(W.rf + ((t0 + t) * C::KS + s) * 64 + W.lane);
                acc[t] = mfma<PREC>(a, bf, acc[t]);
            }
        }
    }
}

// Contract and store one 16-cell tile. FULL: all 16 cells exist, so the code
// is straight-line with compile-time store counts (the compiler can then track
// outstanding memory operations exactly instead of draining the store queue
// before the next use of a prefetched load).
template <int FORM, int D, int P, int FD, int PREC, bool FULL, int VAR = 0>
__device__ inline void scalar_tile(const LinArgs& A, ScalarWave<FORM, D, P, FD, PREC, VAR>& W, const double* Gv,
                                   int j, int64_t tile_base) {
    using C = ScalarCfg<FORM, D, P, FD, PREC, VAR>;
    using acc_t = typename C::acc_t;
    using frag_t = typename C::frag_t;
    using out_t = typename C::out_t;
    constexpr int NS = C::NS, NN = C::NN, NT = C::NT, NU = C::NU, KS = C::KS, NTC = C::NTC, ROW = C::ROW;
    const int lane = W.lane, col = W.col;
    if ((lane >> 4) == j) put_G_row<FORM, D, FD, PREC>(W.gtile + col * ROW, Gv);
    wave_sync();
#pragma unroll
    for (int t0 = 0; t0 < NT; t0 += NTC) {
        acc_t acc[NTC];
        scalar_contract<FORM, D, P, FD, PREC, NTC, VAR>(W, t0, acc);
        if constexpr (C::STAGE) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                wave_sync();
#pragma unroll
                for (int t = 0; t < NTC; ++t) {
                    if (t * 16 + col >= NU) continue;
                    const int oab = W.ua[t] * NS + W.ub[t], oba = W.ub[t] * NS + W.ua[t];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = acc_row<PREC>(lane, v);
                        if ((row >> 3) != h) continue;
                        const out_t x = (out_t)acc[t][v];
                        W.stage[(row & 7) * NN + oab] = x;
                        W.stage[(row & 7) * NN + oba] = x;
                    }
                }
                wave_sync();
                const int64_t c0 = tile_base + 8 * h;
                constexpr int PER16 = 16 / sizeof(out_t);
                const u32x4* s4 = reinterpret_cast<const u32x4*>(W.stage);
                out_t* dst = W.out + c0 * NN;
                u32x4* d4p = reinterpret_cast<u32x4*>(dst);
                if constexpr (FULL) {
                    // all LDS reads first, then the stores (nontemporal: the
                    // element tensors are not read again by this kernel)
                    constexpr int NV = 8 * NN / PER16;
                    constexpr int PL = (NV + 63) / 64;
                    u32x4 tmp[PL];
#pragma unroll
                    for (int i = 0; i < PL; ++i)
                        if (i * 64 + lane < NV) tmp[i] = s4[i * 64 + lane];
#pragma unroll
                    for (int i = 0; i < PL; ++i)
                        if (i * 64 + lane < NV) {
                            gstore_nt(&d4p[i * 64 + lane], tmp[i]);
                        }
                    if constexpr (NV * PER16 != 8 * NN) {
                        constexpr int REM = 8 * NN - NV * PER16;  // < PER16 elements
                        if (lane < REM) gstore(&dst[NV * PER16 + lane], W.stage[NV * PER16 + lane]);
                    }
                } else {
                    const int64_t nc = A.ncells - c0 < 8 ? A.ncells - c0 : 8;
                    if (nc > 0) {
                        const int nelem = (int)nc * NN;
                        const int nvec = nelem / PER16;
                        for (int i = lane; i < nvec; i += 64) gstore(&d4p[i], s4[i]);
                        for (int i = nvec * PER16 + lane; i < nelem; i += 64) gstore(&dst[i], W.stage[i]);
                    }
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < NTC; ++t) {
                if (t0 + t >= NT || (t0 + t) * 16 + col >= NU) continue;
                int a = 0, bb = 0;
#pragma unroll
                for (int tt = 0; tt < NT; ++tt)
                    if (tt == t0 + t) { a = W.ua[tt]; bb = W.ub[tt]; }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t c = tile_base + acc_row<PREC>(lane, v);
                    if (FULL || c < A.ncells) {
                        out_t* base = W.out + c * NN;
                        const out_t x = (out_t)acc[t][v];
                        gstore(&base[a * NS + bb], x);
                        gstore(&base[bb * NS + a], x);
                    }
                }
            }
        }
    }
    wave_sync();
}

template <int FORM, int D, int FD>
__device__ inline void G_from_raw(const CellRaw<FORM, D, FD>& raw, const LinArgs& A, bool valid, double* Gv) {
    constexpr int KR = kref(FORM, D, FD);
    CellData<FORM, D, FD> cd;
    cell_from_raw<FORM, D, FD>(raw, cd);
    build_G<FORM, D, FD, 0, 0>(cd, A, Gv);
    if (!valid) {
#pragma unroll
        for (int k = 0; k < KR; ++k) Gv[k] = 0.0;
    }
}

constexpr int scalar_waves_per_eu(int var) { return var == 0 ? 1 : (var == 3 ? 3 : 2); }

template <int FORM, int D, int P, int FD, int PREC, int VAR = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(scalar_waves_per_eu(VAR))))
void k_scalar(LinArgs A) {
    using C = ScalarCfg<FORM, D, P, FD, PREC, VAR>;
    constexpr int KR = C::KR, NT = C::NT, KS = C::KS, NS = C::NS;
    __shared__ __attribute__((aligned(16))) typename C::g_t sG[4][16 * C::ROW];
    __shared__ __attribute__((aligned(16))) typename C::out_t sO[4][C::SE];
    __shared__ __attribute__((aligned(16))) typename C::frag_t sR[C::RLDS ? C::NFRAG * 64 : 1];
    const int wave = threadIdx.x >> 6;
    ScalarWave<FORM, D, P, FD, PREC, VAR> W;
    W.lane = threadIdx.x & 63;
    W.col = W.lane & 15;
    W.gtile = sG[wave];
    W.stage = sO[wave];
    W.rf = reinterpret_cast<const typename C::frag_t*>(A.rfrag);
    if constexpr (C::RLDS) {
        // variant 1: the workgroup copies the reference fragments to LDS once
        for (int i = threadIdx.x; i < C::NFRAG * 64; i += blockDim.x) sR[i] = gload(W.rf + i);
        __syncthreads();
        W.rf = sR;
    }
    W.out = reinterpret_cast<typename C::out_t*>(A.out);
    const int lane = W.lane;

    // (a, b) of the unique entry u = 16 t + col, a <= b, row-major over the upper triangle
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        int u = t * 16 + W.col, a = 0;
        while (a < NS - 1 && u >= NS - a) { u -= NS - a; ++a; }
        W.ua[t] = a;
        W.ub[t] = a + u;
    }
    if constexpr (C::RREG) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int s = 0; s < KS; ++s) W.rreg[t][s] = gload(W.rf + (t * KS + s) * 64 + lane);
    }

    // Persistent loop over 256-cell chunks, XCD-contiguous ranges of chunks per
    // XCD, software-pipelined two deep: while chunk i is contracted and stored,
    // the coordinates and coefficient dofs of chunk i+1 and the vertex/dof
    // indices of chunk i+2 are in flight.
    const int64_t GS = gridDim.x;
    const int64_t b = blockIdx.x;
    int64_t chunk = (GS % 8 == 0) ? (b % 8) * (GS / 8) + b / 8 : b;
    if (chunk >= A.nchunks) return;
    const int64_t nfull = A.ncells / 256;  // chunks whose 256 cells all exist
    auto cell_of = [&](int64_t ch) -> int64_t { return ch * 256 + wave * 64 + lane; };

    double Gv[KR];
    if constexpr (VAR == 3) {
        // no prefetch: gathers, G rows, contraction and stores of one chunk
        // at a time (the last chunk bounds-checked)
        for (; chunk < A.nchunks; chunk += GS) {
            const int64_t wave_base = chunk * 256 + wave * 64;
            if (wave_base >= A.ncells) break;  // wave-uniform
            const int64_t last = A.ncells - 1;
            const int64_t c = cell_of(chunk) < last ? cell_of(chunk) : last;
            {
                CellIdx<FORM, D, FD> ix;
                CellRaw<FORM, D, FD> raw;
                load_idx<FORM, D, FD>(A, c, ix);
                load_raw<FORM, D, FD>(A, c, ix, raw);
                G_from_raw<FORM, D, FD>(raw, A, cell_of(chunk) < A.ncells, Gv);
            }
            if (wave_base + 64 <= A.ncells) {
                scalar_tile<FORM, D, P, FD, PREC, true, VAR>(A, W, Gv, 0, wave_base);
                scalar_tile<FORM, D, P, FD, PREC, true, VAR>(A, W, Gv, 1, wave_base + 16);
                scalar_tile<FORM, D, P, FD, PREC, true, VAR>(A, W, Gv, 2, wave_base + 32);
                scalar_tile<FORM, D, P, FD, PREC, true, VAR>(A, W, Gv, 3, wave_base + 48);
            } else {
#pragma unroll 1
                for (int j = 0; j < 4; ++j) {
                    const int64_t tile_base = wave_base + 16 * j;
                    if (tile_base >= A.ncells) break;  // wave-uniform
                    scalar_tile<FORM, D, P, FD, PREC, false, VAR>(A, W, Gv, j, tile_base);
                }
            }
        }
        return;
    }
    CellIdx<FORM, D, FD> ix;  // indices of the chunk after next
    CellRaw<FORM, D, FD> raw;
    if (chunk < nfull) {
        load_idx<FORM, D, FD>(A, cell_of(chunk), ix);
        load_raw<FORM, D, FD>(A, cell_of(chunk), ix, raw);
        G_from_raw<FORM, D, FD>(raw, A, true, Gv);
        const int64_t n1 = chunk + GS < nfull ? chunk + GS : chunk;
        load_idx<FORM, D, FD>(A, cell_of(n1), ix);
    }
    // Complete every load issued so far (no store is outstanding yet), so that
    // the loop below starts with an empty load queue: loads and stores share
    // one in-order counter, and a pending prologue load would otherwise make
    // each iteration wait for all of its stores.
    if constexpr (C::RREG) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int s = 0; s < KS; ++s) asm volatile("" ::"v"(W.rreg[t][s]));
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) asm volatile("" ::"v"(Gv[k]));
#pragma unroll
    for (int v = 0; v <= D; ++v) asm volatile("" ::"v"(ix.v[v]));
    while (chunk < nfull) {
        const int64_t wave_base = chunk * 256 + wave * 64;
        const int64_t next = chunk + GS;
        // Straight-line body. Before any store of this chunk: the coordinates
        // and coefficient dofs of the next chunk (indices loaded one chunk ago)
        // and the indices of the chunk after it. Prefetches past the last full
        // chunk repeat the current one and are unused.
        const int64_t n1 = next < nfull ? next : chunk;
        const int64_t n2 = next + GS < nfull ? next + GS : chunk;
        load_raw<FORM, D, FD>(A, cell_of(n1), ix, raw);
        load_idx<FORM, D, FD>(A, cell_of(n2), ix);
        scalar_tile<FORM, D, P, FD, PREC, true, VAR>(A, W, Gv, 0, wave_base);
        scalar_tile<FORM, D, P, FD, PREC, true, VAR>(A, W, Gv, 1, wave_base + 16);
        scalar_tile<FORM, D, P, FD, PREC, true, VAR>(A, W, Gv, 2, wave_base + 32);
        scalar_tile<FORM, D, P, FD, PREC, true, VAR>(A, W, Gv, 3, wave_base + 48);
        G_from_raw<FORM, D, FD>(raw, A, true, Gv);
        chunk = next;
    }
    if (chunk < A.nchunks) {
        // the partial last chunk: bounds-checked loads and stores, no prefetch
        const int64_t wave_base = chunk * 256 + wave * 64;
        if (wave_base >= A.ncells) return;  // wave-uniform; no block barrier follows
        const int64_t last = A.ncells - 1;
        const int64_t c = cell_of(chunk) < last ? cell_of(chunk) : last;
        {
            CellIdx<FORM, D, FD> ix;
            CellRaw<FORM, D, FD> raw;
            load_idx<FORM, D, FD>(A, c, ix);
            load_raw<FORM, D, FD>(A, c, ix, raw);
            G_from_raw<FORM, D, FD>(raw, A, cell_of(chunk) < A.ncells, Gv);
        }
#pragma unroll 1
        for (int j = 0; j < 4; ++j) {
            const int64_t tile_base = wave_base + 16 * j;
            if (tile_base >= A.ncells) break;  // wave-uniform
            scalar_tile<FORM, D, P, FD, PREC, false, VAR>(A, W, Gv, j, tile_base);
        }
    }
}

}  // namespace dev
}  // namespace coffee
