// Mixed persistent batch: cells of different shape, degree and form in one
// launch (the paper's inter-kernel vectorization across cells, section 4,
// applied to a heterogeneous set of cells).
//
// 1. Binning on the device, stable: per-slice histograms of the entries'
//    segment ids, prefix sums over (bin, slice), and an in-order scatter of
//    each entry's cell index and output offset into its bin's contiguous range
//    of the workspace (ranks inside a slice from wave ballots), so that the
//    entries of a bin keep their input order.
// 2. One persistent kernel: every wave takes tasks (task_cells consecutive
//    binned entries of one bin) from a single atomic queue that lists the bins
//    in segment order, and runs the symmetric-form engine of that bin's
//    (form, shape, degree) on them 64 entries at a time, software-pipelined
//    three deep inside the task (while group g is contracted and stored, the
//    coordinates and coefficient dofs of group g+1, the vertex indices of
//    g+2 and the binned cell index and offset of g+3 are in flight). Element
//    tensors go to the entries' own offsets, either staged through LDS (8
//    tensors at a time) or stored straight from the accumulators; in the
//    packed layout the library places each bin's tensors contiguously, in
//    input order, and the tile code of the single-form engine writes them as
//    whole contiguous 16-byte stores. Degree-1 bins run the single-form
//    degree-1 arithmetic instead (one lane per entry, no MFMA).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "library.h"
#include "p1.hpp"
#include "registry.h"
#include "tables.h"

namespace coffee {
namespace dev {

constexpr int kMaxBins = 16;
constexpr int kMaxSlices = 4096;
constexpr int kScanThreads = 1024;  // k_bin_scan: kMaxSlices / kScanThreads slices per thread

struct BinDesc {
    const double* coords;
    const int32_t* c2v;
    int64_t ncells;     // cells of the bin's mesh (entries outside are skipped)
    FieldArg f0;
    const void* rfrag;
    const double* r64;  // degree-1 bins: the FP64 reference tensor [K][n*n]
    int type;        // 7 * form + shape, shape in tri P1..P4, tet P1..P3
    int variant;     // 0 staged stores, 1 direct stores, 2 packed (contiguous)
    int task_cells;  // multiple of 64
    int nn;          // elements of one element tensor
};

struct BatchArgs {
    BinDesc bins[kMaxBins];
    int nbins;
    int64_t nentries;
    const int32_t* seg_of;
    const int64_t* cell_of;
    const int64_t* out_offset;    // input offsets (caller's layout)
    int64_t* out_offset_w;        // packed layout: offsets written here
    int packed;
    void* out;
    int64_t slice;                // entries per binning slice
    int nslices;
    // workspace
    unsigned long long* counts;   // [kMaxBins] entries per bin
    unsigned long long* offs;     // [kMaxBins] first binned position of each bin
    unsigned long long* ebase;    // [kMaxBins] packed layout: first element of each bin
    unsigned long long* queue;    // [1]
    unsigned int* scnt;           // [kMaxSlices][kMaxBins] per-slice counts, then bases
    int64_t* boff;                // [nentries] output offsets in bin order
    int32_t* bcell;               // [nentries] cell indices in bin order
    BatchArgs* self;              // copy of these arguments in global memory
};

// ---------------------------------------------------------------- binning

// Bin of entry i, or -1 for an entry whose segment id or cell index is out of
// range (such entries are skipped: nothing is read or written for them).
__device__ inline int entry_bin(const BatchArgs& A, int64_t i) {
    const int s = A.seg_of[i];
    if (s < 0 || s >= A.nbins) return -1;
    const int64_t c = A.cell_of[i];
    return (c >= 0 && c < A.bins[s].ncells) ? s : -1;
}

__global__ __launch_bounds__(256) void k_bin_count(BatchArgs A) {
    __shared__ unsigned int h[kMaxBins];
    if (threadIdx.x < kMaxBins) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t s0 = blockIdx.x * A.slice;
    const int64_t s1 = s0 + A.slice < A.nentries ? s0 + A.slice : A.nentries;
    for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        const int b = entry_bin(A, i);
        if (b >= 0) atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kMaxBins) A.scnt[blockIdx.x * kMaxBins + threadIdx.x] = h[threadIdx.x];
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) A.queue[0] = 0;  // task queue of k_batch
        // k_batch reads its arguments from this copy through wave-uniform
        // pointers instead of a per-lane copy of the kernel argument
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&A);
        uint32_t* dst = reinterpret_cast<uint32_t*>(A.self);
        for (int i = threadIdx.x; i < (int)(sizeof(BatchArgs) / 4); i += blockDim.x) dst[i] = src[i];
    }
}

// One workgroup per bin: an exclusive scan of the bin's per-slice counts (each
// slice's first position inside its bin; every thread takes consecutive
// slices), and the bin's total.
__global__ __launch_bounds__(kScanThreads) void k_bin_scan(BatchArgs A) {
    constexpr int PER = kMaxSlices / kScanThreads;
    __shared__ unsigned int sc[kScanThreads];
    const int t = threadIdx.x, b = blockIdx.x;
    unsigned int v[PER], sum = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int sl = t * PER + j;
        v[j] = sl < A.nslices ? A.scnt[sl * kMaxBins + b] : 0u;
        sum += v[j];
    }
    sc[t] = sum;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const unsigned int x = t >= d ? sc[t - d] : 0u;
        __syncthreads();
        sc[t] += x;
        __syncthreads();
    }
    unsigned int run = sc[t] - sum;  // exclusive prefix of this thread's slices
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int sl = t * PER + j;
        if (sl < A.nslices) A.scnt[sl * kMaxBins + b] = run;
        run += v[j];
    }
    if (t == kScanThreads - 1) A.counts[b] = sc[t];
}

// Slice s, in input order, 256 entries at a time: an entry's position in its
// bin is the slice's base for the bin, plus the entries of that bin in earlier
// chunks and earlier waves of this chunk, plus its rank among the lanes of its
// wave with the same bin (ballot).
__global__ __launch_bounds__(256) void k_bin_scatter(BatchArgs A) {
    __shared__ unsigned long long cur[kMaxBins], offs[kMaxBins], ebase[kMaxBins];
    __shared__ unsigned int wtot[4][kMaxBins];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t s0 = blockIdx.x * A.slice;
    const int64_t s1 = s0 + A.slice < A.nentries ? s0 + A.slice : A.nentries;
    if (t == 0) {
        // bin totals -> first positions and (packed layout) first elements;
        // block 0 publishes them for k_batch
        unsigned long long p = 0, e = 0;
        for (int b = 0; b < A.nbins; ++b) {
            offs[b] = p;
            ebase[b] = e;
            p += A.counts[b];
            e += A.counts[b] * (unsigned long long)A.bins[b].nn;
            if (blockIdx.x == 0) {
                A.offs[b] = offs[b];
                A.ebase[b] = ebase[b];
            }
        }
    }
    __syncthreads();
    if (t < A.nbins) cur[t] = offs[t] + A.scnt[blockIdx.x * kMaxBins + t];
    __syncthreads();
    const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int64_t i0 = s0; i0 < s1; i0 += 256) {
        const int64_t i = i0 + t;
        const bool valid = i < s1;
        const int b = valid ? entry_bin(A, i) : -1;
        int rank = 0;
        for (int bb = 0; bb < A.nbins; ++bb) {
            const unsigned long long m = __ballot(b == bb);
            if (b == bb) rank = __popcll(m & below);
            if (lane == 0) wtot[w][bb] = (unsigned int)__popcll(m);
        }
        __syncthreads();
        if (valid && b < 0 && A.packed) A.out_offset_w[i] = -1;  // skipped entry
        if (b >= 0) {
            unsigned long long pos = cur[b] + rank;
            for (int ww = 0; ww < w; ++ww) pos += wtot[ww][b];
            A.bcell[pos] = (int32_t)A.cell_of[i];
            int64_t off;
            if (A.packed) {
                off = (int64_t)(ebase[b] + (pos - offs[b]) * (unsigned long long)A.bins[b].nn);
                A.out_offset_w[i] = off;
            } else {
                off = A.out_offset[i];
            }
            A.boff[pos] = off;
        }
        __syncthreads();
        if (t < A.nbins) cur[t] += wtot[0][t] + wtot[1][t] + wtot[2][t] + wtot[3][t];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- tasks

constexpr int kGtileRow = 16;  // >= any G row of the compiled bin types (KR <= 10)
constexpr int kSoffs = 64;     // output offsets per wave in LDS (one per lane)

// k_batch's dynamic LDS, named at file scope so that the (non-inlined) task
// functions address it as LDS. Per wave: G tile (16 x kGtileRow), output
// offsets (kSoffs), then the staging area.
extern __shared__ __attribute__((aligned(16))) unsigned char batch_lds[];

template <int PREC>
struct WaveLds {
    using g_t = typename PrecT<PREC>::gtype;
    using out_t = typename PrecT<PREC>::otype;
    static constexpr unsigned GT_BYTES = 16 * kGtileRow * sizeof(g_t);
    g_t* gtile;
    int64_t* soffs;
    out_t* stage;
    __device__ explicit WaveLds(unsigned wave_off)
        : gtile(reinterpret_cast<g_t*>(batch_lds + wave_off)),
          soffs(reinterpret_cast<int64_t*>(batch_lds + wave_off + GT_BYTES)),
          stage(reinterpret_cast<out_t*>(batch_lds + wave_off + GT_BYTES + kSoffs * sizeof(int64_t))) {}
};

// Contract one 16-entry tile (rows j of the current group) and store each
// entry's tensor at its own offset. FULL: all 64 entries of the group exist,
// so the store count is a compile-time constant.
template <int FORM, int D, int P, int FD, int PREC, int VARIANT, bool FULL>
__device__ inline void batch_tile(ScalarWave<FORM, D, P, FD, PREC>& W, const double* Gv, int j, int64_t myoff,
                                  bool valid, int64_t* soffs) {
    using C = ScalarCfg<FORM, D, P, FD, PREC>;
    using acc_t = typename C::acc_t;
    using out_t = typename C::out_t;
    constexpr int NS = C::NS, NN = C::NN, NT = C::NT, NU = C::NU, ROW = C::ROW;
    static_assert(ROW <= kGtileRow, "G row does not fit the batch tile");
    const int lane = W.lane, col = W.col;
    if ((lane >> 4) == j) put_G_row<FORM, D, FD, PREC>(W.gtile + col * ROW, Gv);
    wave_sync();
    acc_t acc[NT];
    scalar_contract<FORM, D, P, FD, PREC, NT>(W, 0, acc);
    if constexpr (VARIANT == 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            wave_sync();
            if ((lane >> 3) == 2 * j + h) soffs[lane & 7] = (FULL || valid) ? myoff : -1;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
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
            constexpr int TOT = 8 * NN, IT = (TOT + 63) / 64;
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const int k = i * 64 + lane;
                if (k < TOT) {
                    const int c = k / NN, e = k - (k / NN) * NN;
                    const int64_t o = soffs[c];
                    if (FULL || o >= 0) gstore(&W.out[o + e], W.stage[k]);
                }
            }
        }
    } else {
        // offsets of the 4 rows this lane holds, fetched with every lane active
        int64_t roff[4];
        bool rok[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int src = 16 * j + acc_row<PREC>(lane, v);
            roff[v] = __shfl(myoff, src);
            rok[v] = FULL || __shfl((int)valid, src) != 0;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t * 16 + col >= NU) continue;
            const int a = W.ua[t], bb = W.ub[t];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (rok[v]) {
                    const out_t x = (out_t)acc[t][v];
                    gstore(&W.out[roff[v] + a * NS + bb], x);
                    gstore(&W.out[roff[v] + bb * NS + a], x);
                }
            }
        }
    }
    wave_sync();
}

// What a task function reads of the batch arguments, loaded once through the
// scalar path (the arguments and descriptors are wave-uniform and no kernel of
// the batch writes them after k_bin_count).
struct TaskView {
    const int32_t* bcell;
    const int64_t* boff;
    void* out;
    int64_t offs, ebase, count;  // of this task's bin
    LinArgs L;                   // the bin's mesh and field
    const void* rfrag;
    const double* r64;
};

__device__ inline TaskView task_view(const BatchArgs* Ap, const BinDesc* bdp, int bin) {
    const BatchArgs* A = uniform_ptr(Ap);
    const BinDesc* bd = uniform_ptr(bdp);
    TaskView v;
    v.bcell = cload(&A->bcell);
    v.boff = cload(&A->boff);
    v.out = cload(&A->out);
    v.offs = (int64_t)gload(cload(&A->offs) + bin);
    v.ebase = (int64_t)gload(cload(&A->ebase) + bin);
    v.count = (int64_t)gload(cload(&A->counts) + bin);
    v.L.coords = cload(&bd->coords);
    v.L.c2v = cload(&bd->c2v);
    v.L.f0 = FieldArg{cload(&bd->f0.values), cload(&bd->f0.map)};
    v.L.f1 = FieldArg{nullptr, nullptr};
    v.L.c0 = 0.0;
    v.L.c1 = 0.0;
    v.L.ncells = 0;
    v.rfrag = cload(&bd->rfrag);
    v.r64 = cload(&bd->r64);
    return v;
}

// n binned entries first .. first + n - 1 of one bin, 64 per group. Not
// inlined: each bin type is then register-allocated on its own instead of
// as one body holding every type's live values (which spilled heavily). The
// arguments are wave-uniform; the LDS areas are re-derived as LDS pointers
// (a non-inlined function sees generic pointers).
template <int FORM, int D, int P, int FD, int PREC, int VARIANT>
__device__ __attribute__((noinline)) void batch_task(const BatchArgs* Ap, const BinDesc* bdp, int bin, int64_t first,
                                                     int n, int lane, unsigned wave_off) {
    using C = ScalarCfg<FORM, D, P, FD, PREC>;
    constexpr int KR = C::KR, NT = C::NT, KS = C::KS, NS = C::NS;
    bin = __builtin_amdgcn_readfirstlane(bin);
    n = __builtin_amdgcn_readfirstlane(n);
    first = uniform_i64(first);
    const WaveLds<PREC> M(__builtin_amdgcn_readfirstlane(wave_off));
    int64_t* soffs = M.soffs;
    const TaskView V = task_view(Ap, bdp, bin);
    ScalarWave<FORM, D, P, FD, PREC> W;
    W.lane = lane;
    W.col = lane & 15;
    W.gtile = M.gtile;
    W.stage = M.stage;
    W.rf = reinterpret_cast<const typename C::frag_t*>(V.rfrag);
    W.out = reinterpret_cast<typename C::out_t*>(V.out);
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
    LinArgs L = V.L;
    const int nfull = n >> 6, ng = (n + 63) >> 6;
    const int64_t last = first + n - 1;
    // binned position of this lane's entry in group g (clamped into the task)
    auto at = [&](int g) -> int64_t {
        const int gg = g < ng ? g : ng - 1;
        const int64_t p = first + 64 * (int64_t)gg + lane;
        return p < last ? p : last;
    };
    double Gv[KR];
    CellIdx<FORM, D, FD> ix;
    CellRaw<FORM, D, FD> raw;
    int c1, c2;
    int64_t o0, o1, o2;
    {
        const int64_t p0 = at(0);
        const int c0 = gload(V.bcell + p0);
        o0 = gload(V.boff + p0);
        load_idx<FORM, D, FD>(L, c0, ix);
        load_raw<FORM, D, FD>(L, c0, ix, raw);
        G_from_raw<FORM, D, FD>(raw, L, true, Gv);
        const int64_t p1 = at(1);
        c1 = gload(V.bcell + p1);
        o1 = gload(V.boff + p1);
        load_idx<FORM, D, FD>(L, c1, ix);
        const int64_t p2 = at(2);
        c2 = gload(V.bcell + p2);
        o2 = gload(V.boff + p2);
    }
    // Complete the prologue's loads before the first store (one in-order
    // counter covers loads and stores).
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
    asm volatile("" ::"v"(c2), "v"(o1), "v"(o2));
    // packed layout: the bin's tensors are contiguous from out + ebase[bin]
    // in binned order, so entry p of the bin is local cell p of that range
    const int64_t local0 = first - V.offs;
    if constexpr (VARIANT == 2) {
        W.out += V.ebase;
        L.ncells = V.count;
    }
    for (int g = 0; g < nfull; ++g) {
        load_raw<FORM, D, FD>(L, c1, ix, raw);  // group g + 1
        load_idx<FORM, D, FD>(L, c2, ix);       // group g + 2
        const int64_t p3 = at(g + 3);
        const int c3 = gload(V.bcell + p3);
        const int64_t o3 = gload(V.boff + p3);
        if constexpr (VARIANT == 2) {
            const int64_t tb = local0 + 64 * (int64_t)g;
            scalar_tile<FORM, D, P, FD, PREC, true>(L, W, Gv, 0, tb);
            scalar_tile<FORM, D, P, FD, PREC, true>(L, W, Gv, 1, tb + 16);
            scalar_tile<FORM, D, P, FD, PREC, true>(L, W, Gv, 2, tb + 32);
            scalar_tile<FORM, D, P, FD, PREC, true>(L, W, Gv, 3, tb + 48);
        } else {
            batch_tile<FORM, D, P, FD, PREC, VARIANT, true>(W, Gv, 0, o0, true, soffs);
            batch_tile<FORM, D, P, FD, PREC, VARIANT, true>(W, Gv, 1, o0, true, soffs);
            batch_tile<FORM, D, P, FD, PREC, VARIANT, true>(W, Gv, 2, o0, true, soffs);
            batch_tile<FORM, D, P, FD, PREC, VARIANT, true>(W, Gv, 3, o0, true, soffs);
        }
        G_from_raw<FORM, D, FD>(raw, L, true, Gv);
        o0 = o1;
        o1 = o2;
        o2 = o3;
        c1 = c2;
        c2 = c3;
    }
    if (nfull < ng) {
        // the partial last group (its data came with the pipeline)
        const int rem = n - 64 * nfull;
        const bool valid = lane < rem;
#pragma unroll 1
        for (int j = 0; j < 4; ++j) {
            if (16 * j >= rem) break;  // wave-uniform
            if constexpr (VARIANT == 2) {
                // bounds: the task's last entry (L.ncells counts the whole bin)
                L.ncells = local0 + n;
                scalar_tile<FORM, D, P, FD, PREC, false>(L, W, Gv, j, local0 + 64 * (int64_t)nfull + 16 * j);
            } else {
                batch_tile<FORM, D, P, FD, PREC, VARIANT, false>(W, Gv, j, o0, valid, soffs);
            }
        }
    }
}

// Degree-1 bins: one lane per entry with the arithmetic of the single-form
// degree-1 kernel (p1.hpp), 64 entries per group. The tensors go through an
// LDS row per lane and leave as stores whose lanes cover consecutive elements:
// of the bin's contiguous range (packed layout) or of each entry's own range
// (caller's layout, offsets in LDS). The gathers of the next groups are issued
// before the current group's stores, as in the symmetric tiles.
template <int FORM, int D, int PREC, int VARIANT, int MAPF>
__device__ __attribute__((noinline)) void batch_task_p1(const BatchArgs* Ap, const BinDesc* bdp, int bin, int64_t first,
                                                        int n, int lane, unsigned wave_off) {
    using out_t = typename PrecT<PREC>::otype;
    constexpr int FD = 1, NN = (D + 1) * (D + 1), KR = kref(FORM, D, FD), SR = p1_row<D>();
    bin = __builtin_amdgcn_readfirstlane(bin);
    n = __builtin_amdgcn_readfirstlane(n);
    first = uniform_i64(first);
    const WaveLds<PREC> M(__builtin_amdgcn_readfirstlane(wave_off));
    out_t* stage = M.stage;
    int64_t* soffs = M.soffs;
    const TaskView V = task_view(Ap, bdp, bin);
    const LinArgs L = V.L;
    const double* R = V.r64;
    out_t* out = reinterpret_cast<out_t*>(V.out);
    if constexpr (VARIANT == 2) out += V.ebase + (first - V.offs) * NN;
    const int ng = (n + 63) >> 6;
    const int64_t last = first + n - 1;
    auto at = [&](int g) -> int64_t {
        const int gg = g < ng ? g : ng - 1;
        const int64_t p = first + 64 * (int64_t)gg + lane;
        return p < last ? p : last;
    };
    auto off = [&](int64_t p) -> int64_t { return VARIANT == 2 ? 0 : gload(V.boff + p); };
    CellIdx<FORM, D, FD> ix;
    CellRaw<FORM, D, FD> raw;
    int64_t o0, o1, o2;
    int c1, c2;
    {
        const int64_t p0 = at(0);
        const int c0 = gload(V.bcell + p0);
        o0 = off(p0);
        load_idx<FORM, D, FD, MAPF>(L, c0, ix);
        load_raw<FORM, D, FD, MAPF>(L, c0, ix, raw);
        const int64_t p1 = at(1);
        c1 = gload(V.bcell + p1);
        o1 = off(p1);
        load_idx<FORM, D, FD, MAPF>(L, c1, ix);
        const int64_t p2 = at(2);
        c2 = gload(V.bcell + p2);
        o2 = off(p2);
    }
    // Complete the prologue's loads before the loop, so that the loop is
    // entered with nothing outstanding and its waits count only its own loads
    // and stores.
#pragma unroll
    for (int v = 0; v <= D; ++v)
#pragma unroll
        for (int i = 0; i < D; ++i) asm volatile("" ::"v"(raw.x[v][i]));
#pragma unroll
    for (int r = 0; r < CellRaw<FORM, D, FD>::NF; ++r) asm volatile("" ::"v"(raw.f0[r]));
#pragma unroll
    for (int v = 0; v <= D; ++v) asm volatile("" ::"v"(ix.v[v]));
#pragma unroll
    for (int r = 0; r < CellIdx<FORM, D, FD>::NF; ++r) asm volatile("" ::"v"(ix.f0[r]));
    asm volatile("" ::"v"(c1), "v"(c2), "v"(o0), "v"(o1), "v"(o2));
    // One group: the next groups' gathers, then G and the tensors of the
    // current group into LDS and this group's stores. FULL groups store a
    // compile-time number of elements with no per-element condition, so the
    // wait for the prefetched gathers does not have to drain the stores.
    auto step = [&](int g, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        CellData<FORM, D, FD> cd;
        cell_from_raw<FORM, D, FD>(raw, cd);          // group g
        load_raw<FORM, D, FD, MAPF>(L, c1, ix, raw);  // group g + 1
        load_idx<FORM, D, FD, MAPF>(L, c2, ix);       // group g + 2
        const int64_t p3 = at(g + 3);
        const int c3 = gload(V.bcell + p3);
        const int64_t o3 = off(p3);
        // the gathers are issued before this group's arithmetic and stores,
        // and nothing of the next group moves above them
        __builtin_amdgcn_sched_barrier(0);
        double G[KR];
        build_G<FORM, D, FD, 0, 0>(cd, L, G);
        p1_tensor<FORM, D, FD, out_t>(G, R, stage + lane * SR);
        if constexpr (VARIANT != 2) soffs[lane] = o0;
        wave_sync();
        const int m = FULL ? 64 : n - 64 * g;
        out_t* dst = out + (int64_t)64 * g * NN;
        out_t v[NN];
        int64_t dd[NN];
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            const int i = k * 64 + lane;
            const int c = i / NN, e = i - (i / NN) * NN;
            v[k] = stage[c * SR + e];
            dd[k] = VARIANT == 2 ? (int64_t)i : soffs[c] + e;
        }
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            if (FULL || (k * 64 + lane) / NN < m) {
                if constexpr (VARIANT == 2) gstore(&dst[dd[k]], v[k]);
                else gstore(&out[dd[k]], v[k]);
            }
        }
        wave_sync();
        __builtin_amdgcn_sched_barrier(0);
        o0 = o1;
        o1 = o2;
        o2 = o3;
        c1 = c2;
        c2 = c3;
    };
    const int nfull = n >> 6;
    for (int g = 0; g < nfull; ++g) step(g, std::true_type{});
    if (nfull < ng) step(nfull, std::false_type{});
}

template <int PREC, int VARIANT>
__device__ inline void batch_dispatch_v(const BatchArgs* A, const BinDesc* bd, int type, bool mapped, int bin,
                                        int64_t first, int n, int lane, unsigned wave_off) {
    switch (type) {
        case 0:
            if (mapped) batch_task_p1<F_MASS, 2, PREC, VARIANT, 1>(A, bd, bin, first, n, lane, wave_off);
            else batch_task_p1<F_MASS, 2, PREC, VARIANT, 0>(A, bd, bin, first, n, lane, wave_off);
            break;
        case 1: batch_task<F_MASS, 2, 2, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        case 2: batch_task<F_MASS, 2, 3, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        case 3: batch_task<F_MASS, 2, 4, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        case 4:
            if (mapped) batch_task_p1<F_MASS, 3, PREC, VARIANT, 1>(A, bd, bin, first, n, lane, wave_off);
            else batch_task_p1<F_MASS, 3, PREC, VARIANT, 0>(A, bd, bin, first, n, lane, wave_off);
            break;
        case 5: batch_task<F_MASS, 3, 2, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        case 6: batch_task<F_MASS, 3, 3, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        case 7:
            if (mapped) batch_task_p1<F_HELM, 2, PREC, VARIANT, 1>(A, bd, bin, first, n, lane, wave_off);
            else batch_task_p1<F_HELM, 2, PREC, VARIANT, 0>(A, bd, bin, first, n, lane, wave_off);
            break;
        case 8: batch_task<F_HELM, 2, 2, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        case 9: batch_task<F_HELM, 2, 3, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        case 10: batch_task<F_HELM, 2, 4, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        case 11:
            if (mapped) batch_task_p1<F_HELM, 3, PREC, VARIANT, 1>(A, bd, bin, first, n, lane, wave_off);
            else batch_task_p1<F_HELM, 3, PREC, VARIANT, 0>(A, bd, bin, first, n, lane, wave_off);
            break;
        case 12: batch_task<F_HELM, 3, 2, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        case 13: batch_task<F_HELM, 3, 3, 1, PREC, VARIANT>(A, bd, bin, first, n, lane, wave_off); break;
        default: break;
    }
}

// Dynamic LDS per wave: G tile (16 x kGtileRow), output offsets (kSoffs), and
// the staging area of `stage_elems` elements (8 tensors of the largest staged
// bin, or 64 padded degree-1 tensors).
template <int PREC>
__global__ __launch_bounds__(256) void k_batch(const BatchArgs* __restrict__ Ap, int stage_elems) {
    const BatchArgs& A = *Ap;
    using out_t = typename PrecT<PREC>::otype;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned per_wave = WaveLds<PREC>::GT_BYTES + kSoffs * sizeof(int64_t) + (unsigned)stage_elems * sizeof(out_t);
    const unsigned wave_off = wave * per_wave;
    // tasks per bin from the device counts
    int64_t tstart[kMaxBins + 1];
    tstart[0] = 0;
#pragma unroll
    for (int b = 0; b < kMaxBins; ++b) {
        const int64_t c = b < A.nbins ? (int64_t)A.counts[b] : 0;
        const int tc = b < A.nbins ? A.bins[b].task_cells : 64;
        tstart[b + 1] = tstart[b] + (c + tc - 1) / tc;
    }
    const int64_t total = tstart[kMaxBins];
    for (;;) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(A.queue, 1ull);
        t = (unsigned long long)uniform_i64((int64_t)__shfl(t, 0));
        if ((int64_t)t >= total) break;
        int b = 0;
        int64_t tb = 0;
#pragma unroll
        for (int k = 1; k < kMaxBins; ++k)
            if ((int64_t)t >= tstart[k]) {
                b = k;
                tb = tstart[k];
            }
        const BinDesc* bd = &Ap->bins[b];
        const int tc = bd->task_cells, type = bd->type, variant = bd->variant;
        const bool mapped = bd->f0.map != nullptr;
        const int64_t local = ((int64_t)t - tb) * tc;
        const int64_t cnt = (int64_t)A.counts[b];
        const int n = (int)(cnt - local < tc ? cnt - local : tc);
        const int64_t first = (int64_t)A.offs[b] + local;
        if (variant == 2) batch_dispatch_v<PREC, 2>(Ap, bd, type, mapped, b, first, n, lane, wave_off);
        else if (variant == 0) batch_dispatch_v<PREC, 0>(Ap, bd, type, mapped, b, first, n, lane, wave_off);
        else batch_dispatch_v<PREC, 1>(Ap, bd, type, mapped, b, first, n, lane, wave_off);
    }
}

}  // namespace dev

// Workspace: header (counts, offs, ebase, queue), a copy of the kernel
// arguments, per-slice counts, then the binned output offsets and cell indices.
constexpr int64_t kWsHeader = 64 * 8;
constexpr int64_t kWsArgs = 2048;
constexpr int64_t kWsSlices = (int64_t)dev::kMaxSlices * dev::kMaxBins * 4;
static_assert(sizeof(dev::BatchArgs) <= kWsArgs, "batch arguments do not fit the workspace slot");

int64_t batch_workspace_bytes(int nseg, int64_t nentries) {
    (void)nseg;
    return kWsHeader + kWsArgs + kWsSlices + nentries * 12;
}

// Entries per task of the packed layout when the segment leaves it open
// (measured on the 3,000,000-entry batch: 256 beats 512 and 1024).
constexpr int kPackedTaskCells = 256;

static int batch_type(int form, int cell, int degree) {
    int shape = -1;
    if (cell == 2 && degree >= 1 && degree <= 4) shape = degree - 1;
    if (cell == 3 && degree >= 1 && degree <= 3) shape = 3 + degree;
    if (shape < 0) return -1;
    if (form == COFFEE_MASS) return shape;
    if (form == COFFEE_HELMHOLTZ) return 7 + shape;
    return -1;
}

// ---------------------------------------------------------------- allocation-free variant
//
// coffee_assemble_batch_packed_noalloc takes its workspace from `scratch`, a
// file-scope device array, and its reference tables from `table_pool`, a
// second one, instead of caller memory and hipMalloc. In host code these
// names are stand-ins, not device addresses: their addresses on the current
// device come from hipGetSymbolAddress (each device holds its own copies) and
// are the only form in which host code uses them.

constexpr int64_t kScratchMaxEntries = COFFEE_NOALLOC_MAX_ENTRIES;
constexpr int64_t kScratchBytes = kWsHeader + kWsArgs + kWsSlices + kScratchMaxEntries * 12;
constexpr int64_t kTablePoolBytes = 1 << 20;

__device__ __align__(256) unsigned char scratch[kScratchBytes];
__device__ __align__(256) unsigned char table_pool[kTablePoolBytes];

struct NoallocDev {
    unsigned char* scratch = nullptr;  // device address of `scratch`
    unsigned char* pool = nullptr;     // device address of `table_pool`
    int64_t used = 0;                  // bytes of the pool in use
    std::map<std::tuple<int, int, int, int, int, int>, const void*> tabs;  // (kind, form, cell, degree, q, prec)
};

static std::mutex g_noalloc_mu;
static std::map<int, NoallocDev> g_noalloc;

// Set-up once per device (with that device current): the arrays' addresses.
static coffee_status noalloc_device(int dev, NoallocDev** out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    NoallocDev& d = g_noalloc[dev];
    if (!d.scratch) {
        void* ps = nullptr;
        void* pt = nullptr;
        if (hipGetSymbolAddress(&ps, HIP_SYMBOL(scratch)) != hipSuccess || !ps) return COFFEE_E_HIP;
        if (hipGetSymbolAddress(&pt, HIP_SYMBOL(table_pool)) != hipSuccess || !pt) return COFFEE_E_HIP;
        d.scratch = static_cast<unsigned char*>(ps);
        d.pool = static_cast<unsigned char*>(pt);
    }
    *out = &d;
    return COFFEE_OK;
}

// A reference table in the pool, copied there on first use (a synchronous
// host-to-device copy into the pool; no allocation).
static coffee_status noalloc_table(NoallocDev& d, int kind, int form, int cell, int degree, int q, int prec,
                                   const void** out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    const auto key = std::make_tuple(kind, form, cell, degree, q, prec);
    auto it = d.tabs.find(key);
    if (it != d.tabs.end()) {
        *out = it->second;
        return COFFEE_OK;
    }
    std::vector<char> bytes;
    if (kind == 0) {
        if (!rtable_bytes(form, cell, degree, q, 1, prec, bytes)) return COFFEE_E_INVALID_ARG;
    } else {
        std::vector<double> h;
        if (!r64_table(form, cell, degree, q, 1, h)) return COFFEE_E_INVALID_ARG;
        bytes.resize(h.size() * sizeof(double));
        std::memcpy(bytes.data(), h.data(), bytes.size());
    }
    const int64_t n = ((int64_t)bytes.size() + 255) / 256 * 256;
    if (d.used + n > kTablePoolBytes) return COFFEE_E_NOMEM;
    unsigned char* dst = d.pool + d.used;
    if (hipMemcpy(dst, bytes.data(), bytes.size(), hipMemcpyHostToDevice) != hipSuccess) return COFFEE_E_HIP;
    d.used += n;
    d.tabs[key] = dst;
    *out = dst;
    return COFFEE_OK;
}

// packed = 0: tensors at the caller's out_offset (input); packed = 1: the
// library lays the bins out contiguously in segment order (entries of a bin in
// input order) and writes each entry's offset to out_offset_w. na != NULL:
// reference tables from the allocation-free pool.
static coffee_status assemble_batch(int precision, const coffee_segment* segs, int nseg, const int32_t* seg_of,
                                    const int64_t* cell_of, const int64_t* out_offset, int64_t* out_offset_w,
                                    int packed, int64_t nentries, void* out, void* workspace,
                                    int64_t workspace_bytes, void* hip_stream, NoallocDev* na = nullptr) {
    if (precision != COFFEE_FP64 && precision != COFFEE_FP32) return COFFEE_E_UNSUPPORTED;
    if (!segs || nseg < 1 || nseg > dev::kMaxBins || nentries < 0) return COFFEE_E_INVALID_ARG;
    if (nentries > INT32_MAX) return COFFEE_E_UNSUPPORTED;
    if (nentries > 0 && (!seg_of || !cell_of || !out || !workspace)) return COFFEE_E_INVALID_ARG;
    if (nentries > 0 && (packed ? !out_offset_w : !out_offset)) return COFFEE_E_INVALID_ARG;
    if (nentries > 0 && workspace_bytes < batch_workspace_bytes(nseg, nentries)) return COFFEE_E_BUFFER_TOO_SMALL;
    if (((uintptr_t)workspace & 7) != 0) return COFFEE_E_INVALID_ARG;
    if (packed && ((uintptr_t)out & 15) != 0) return COFFEE_E_INVALID_ARG;
    dev::BatchArgs a;
    std::memset(&a, 0, sizeof a);
    int devid = 0;
    if (hipGetDevice(&devid) != hipSuccess) return COFFEE_E_HIP;
    const int esz = precision == COFFEE_FP64 ? 8 : 4;
    int stage_elems = 8;  // staging area: 8 tensors of the largest bin that stages its stores
    for (int b = 0; b < nseg; ++b) {
        const coffee_segment& s = segs[b];
        const int type = batch_type(s.form, s.cell, s.degree);
        if (type < 0) return COFFEE_E_UNSUPPORTED;
        if (!s.coords || !s.cell_to_vertex || s.nvert < 0 || s.ncells_mesh < 0) return COFFEE_E_INVALID_ARG;
        if (s.ncells_mesh > INT32_MAX) return COFFEE_E_UNSUPPORTED;
        if (!s.coeff || !s.coeff->values || s.coeff->degree != 1 || s.coeff->ncomp != 1) return COFFEE_E_UNSUPPORTED;
        if (s.variant < 0 || s.variant > 1) return COFFEE_E_INVALID_ARG;
        if (s.task_cells != 0 && (s.task_cells % 64 != 0 || s.task_cells < 64 || s.task_cells > 1024))
            return COFFEE_E_INVALID_ARG;
        const int q = s.quad_degree >= 0 ? s.quad_degree : 2 * s.degree;
        if (rule_size(s.cell, q) <= 0) return COFFEE_E_INVALID_ARG;
        const void* rf = nullptr;
        coffee_status st = na ? noalloc_table(*na, 0, s.form, s.cell, s.degree, q, precision, &rf)
                              : get_rtable_public(devid, s.form, s.cell, s.degree, q, 1, precision, &rf);
        if (st != COFFEE_OK) return st;
        const int ns = n_scalar(s.cell, s.degree);
        dev::BinDesc& d = a.bins[b];
        d.coords = s.coords;
        d.c2v = s.cell_to_vertex;
        d.ncells = s.ncells_mesh;
        d.f0 = dev::FieldArg{s.coeff->values, s.coeff->cell_to_dof};
        d.rfrag = rf;
        d.r64 = nullptr;
        if (s.degree == 1) {
            if (na) {
                const void* r = nullptr;
                st = noalloc_table(*na, 1, s.form, s.cell, 1, q, COFFEE_FP64, &r);
                d.r64 = static_cast<const double*>(r);
            } else {
                st = reference_table_f64(devid, s.form, s.cell, 1, q, 1, &d.r64);
            }
            if (st != COFFEE_OK) return st;
        }
        d.type = type;
        d.nn = ns * ns;
        d.variant = s.variant;
        d.task_cells = s.task_cells ? s.task_cells : 256;
        int tv = 0, tt = 0;
        if (s.task_cells == 0 && tuned_batch(s.form, s.cell, s.degree, precision, &tv, &tt)) {
            d.variant = tv;
            d.task_cells = tt;
        }
        if (packed) {
            d.variant = 2;
            int pt = 0;
            if (s.task_cells == 0) d.task_cells = tuned_packed(s.form, s.cell, s.degree, precision, &pt) ? pt : kPackedTaskCells;
        }
        // the packed tiles stage 8 tensors when they fit 16 KiB (the
        // single-form engine's rule), the per-entry staged variant always
        const bool stages = packed ? 8 * d.nn * esz <= 16384 : d.variant == 0;
        if (stages) stage_elems = std::max(stage_elems, 8 * d.nn);
        if (s.degree == 1) stage_elems = std::max(stage_elems, 64 * (d.nn | 1));
    }
    if (nentries == 0) return COFFEE_OK;
    a.nbins = nseg;
    a.nentries = nentries;
    a.seg_of = seg_of;
    a.cell_of = cell_of;
    a.out_offset = out_offset;
    a.out_offset_w = out_offset_w;
    a.packed = packed;
    a.out = out;
    a.slice = std::max<int64_t>(256, (nentries + dev::kMaxSlices - 1) / dev::kMaxSlices);
    a.slice = (a.slice + 255) / 256 * 256;
    a.nslices = (int)((nentries + a.slice - 1) / a.slice);
    unsigned long long* ws = reinterpret_cast<unsigned long long*>(workspace);
    a.counts = ws;
    a.offs = ws + dev::kMaxBins;
    a.ebase = ws + 2 * dev::kMaxBins;
    a.queue = ws + 3 * dev::kMaxBins;
    a.self = reinterpret_cast<dev::BatchArgs*>(reinterpret_cast<char*>(workspace) + kWsHeader);
    a.scnt = reinterpret_cast<unsigned int*>(reinterpret_cast<char*>(workspace) + kWsHeader + kWsArgs);
    a.boff = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(workspace) + kWsHeader + kWsArgs + kWsSlices);
    a.bcell = reinterpret_cast<int32_t*>(a.boff + nentries);
    hipStream_t s = (hipStream_t)hip_stream;
    const int ncu = num_cu(devid);
    hipLaunchKernelGGL(dev::k_bin_count, dim3(a.nslices), dim3(256), 0, s, a);
    hipLaunchKernelGGL(dev::k_bin_scan, dim3(nseg), dim3(dev::kScanThreads), 0, s, a);
    hipLaunchKernelGGL(dev::k_bin_scatter, dim3(a.nslices), dim3(256), 0, s, a);
    stage_elems = (stage_elems + 3) / 4 * 4;  // 16-byte multiple for FP32
    const size_t gsz = esz;
    const size_t lds = 4 * ((size_t)16 * dev::kGtileRow * gsz + dev::kSoffs * 8 + (size_t)stage_elems * gsz);
    if (lds > 160 * 1024) return COFFEE_E_UNSUPPORTED;
    const void* kern = precision == COFFEE_FP64 ? (const void*)&dev::k_batch<dev::PREC_F64>
                                                : (const void*)&dev::k_batch<dev::PREC_F32>;
    if (lds > 64 * 1024 && hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return COFFEE_E_HIP;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 256, lds) != hipSuccess || nb <= 0) nb = 1;
    const int grid = ncu * nb * std::max(1, batch_grid_mult());
    if (precision == COFFEE_FP64)
        hipLaunchKernelGGL(dev::k_batch<dev::PREC_F64>, dim3(grid), dim3(256), lds, s,
                           (const dev::BatchArgs*)a.self, stage_elems);
    else
        hipLaunchKernelGGL(dev::k_batch<dev::PREC_F32>, dim3(grid), dim3(256), lds, s,
                           (const dev::BatchArgs*)a.self, stage_elems);
    return hipGetLastError() == hipSuccess ? COFFEE_OK : COFFEE_E_HIP;
}

}  // namespace coffee

extern "C" coffee_status coffee_assemble_batch(int precision, const coffee_segment* segs, int nseg,
                                               const int32_t* seg_of, const int64_t* cell_of,
                                               const int64_t* out_offset, int64_t nentries, void* out,
                                               void* workspace, int64_t workspace_bytes, void* hip_stream) {
    return coffee::assemble_batch(precision, segs, nseg, seg_of, cell_of, out_offset, nullptr, 0, nentries, out,
                                  workspace, workspace_bytes, hip_stream);
}

extern "C" coffee_status coffee_assemble_batch_packed(int precision, const coffee_segment* segs, int nseg,
                                                      const int32_t* seg_of, const int64_t* cell_of,
                                                      int64_t nentries, void* out, int64_t* out_offset,
                                                      void* workspace, int64_t workspace_bytes,
                                                      void* hip_stream) {
    return coffee::assemble_batch(precision, segs, nseg, seg_of, cell_of, nullptr, out_offset, 1, nentries, out,
                                  workspace, workspace_bytes, hip_stream);
}

extern "C" int64_t coffee_batch_workspace_size(int nseg, int64_t nentries) {
    return coffee::batch_workspace_bytes(nseg, nentries);
}

extern "C" coffee_status coffee_assemble_batch_packed_noalloc(int precision, const coffee_segment* segs, int nseg,
                                                              const int32_t* seg_of, const int64_t* cell_of,
                                                              int64_t nentries, void* out, int64_t* out_offset,
                                                              void* hip_stream) {
    using namespace coffee;
    if (nentries > kScratchMaxEntries) return COFFEE_E_BUFFER_TOO_SMALL;
    if (nentries < 0) return COFFEE_E_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return COFFEE_E_HIP;
    NoallocDev* na = nullptr;
    const coffee_status st = noalloc_device(dev, &na);
    if (st != COFFEE_OK) return st;
    return assemble_batch(precision, segs, nseg, seg_of, cell_of, nullptr, out_offset, 1, nentries, out, na->scratch,
                          kScratchBytes, hip_stream, na);
}
