// Mixed persistent batch: cells of different shape, degree and form in one
// launch (the paper's inter-kernel vectorization across cells, section 4,
// applied to a heterogeneous set of cells).
//
// 1. Binning on the device: per-workgroup histograms of the entries' segment
//    ids, a prefix sum, and a scatter of each entry's cell index and output
//    offset into its bin's contiguous range of the workspace (each workgroup
//    reserves one range per bin with one atomic).
// 2. One persistent kernel: every wave takes tasks (task_cells consecutive
//    binned entries of one bin) from a single atomic queue that lists the bins
//    in segment order, and runs the symmetric-form engine of that bin's
//    (form, shape, degree) on them 64 entries at a time, software-pipelined
//    three deep inside the task (while group g is contracted and stored, the
//    coordinates and coefficient dofs of group g+1, the vertex indices of
//    g+2 and the binned cell index and offset of g+3 are in flight). Element
//    tensors go to the entries' own offsets, either staged through LDS (8
//    tensors at a time) or stored straight from the accumulators.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "library.h"
#include "registry.h"
#include "tables.h"

namespace coffee {
namespace dev {

constexpr int kMaxBins = 16;

struct BinDesc {
    const double* coords;
    const int32_t* c2v;
    FieldArg f0;
    const void* rfrag;
    int type;        // 7 * form + shape, shape in tri P1..P4, tet P1..P3
    int variant;     // 0 staged stores, 1 direct stores
    int task_cells;  // multiple of 64
    int pad;
};

struct BatchArgs {
    BinDesc bins[kMaxBins];
    int nbins;
    int64_t nentries;
    const int32_t* seg_of;
    const int64_t* cell_of;
    const int64_t* out_offset;
    void* out;
    // workspace
    unsigned long long* counts;   // [kMaxBins]
    unsigned long long* offs;     // [kMaxBins]
    unsigned long long* cursor;   // [kMaxBins]
    unsigned long long* queue;    // [1]
    int64_t* boff;                // [nentries] output offsets in bin order
    int32_t* bcell;               // [nentries] cell indices in bin order
};

// ---------------------------------------------------------------- binning

__global__ __launch_bounds__(256) void k_bin_count(BatchArgs A) {
    __shared__ unsigned int h[kMaxBins];
    if (threadIdx.x < kMaxBins) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < A.nentries; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[A.seg_of[i]], 1u);
    __syncthreads();
    if (threadIdx.x < A.nbins && h[threadIdx.x]) atomicAdd(A.counts + threadIdx.x, (unsigned long long)h[threadIdx.x]);
}

__global__ void k_bin_scan(BatchArgs A) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned long long s = 0;
        for (int b = 0; b < A.nbins; ++b) {
            A.offs[b] = s;
            A.cursor[b] = s;
            s += A.counts[b];
        }
        A.queue[0] = 0;
    }
}

// Each workgroup takes a contiguous slice of entries, counts them per bin,
// reserves one range per bin and writes every entry's cell index and output
// offset into it (the order inside a workgroup's range is immaterial: each
// entry's result depends only on its own data).
__global__ __launch_bounds__(256) void k_bin_scatter(BatchArgs A, int64_t slice) {
    __shared__ unsigned int h[kMaxBins];
    __shared__ unsigned long long base[kMaxBins];
    const int64_t s0 = blockIdx.x * slice;
    const int64_t s1 = s0 + slice < A.nentries ? s0 + slice : A.nentries;
    if (threadIdx.x < kMaxBins) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) atomicAdd(&h[A.seg_of[i]], 1u);
    __syncthreads();
    if (threadIdx.x < A.nbins) {
        base[threadIdx.x] = h[threadIdx.x] ? atomicAdd(A.cursor + threadIdx.x, (unsigned long long)h[threadIdx.x]) : 0;
        h[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        const int sg = A.seg_of[i];
        const unsigned long long pos = base[sg] + atomicAdd(&h[sg], 1u);
        A.bcell[pos] = (int32_t)A.cell_of[i];
        A.boff[pos] = A.out_offset[i];
    }
}

// ---------------------------------------------------------------- tasks

constexpr int kGtileRow = 16;  // >= any G row of the compiled bin types (KR <= 10)

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
                    if (FULL || o >= 0) W.out[o + e] = W.stage[k];
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
                    W.out[roff[v] + a * NS + bb] = x;
                    W.out[roff[v] + bb * NS + a] = x;
                }
            }
        }
    }
    wave_sync();
}

// n binned entries first .. first + n - 1 of one bin, 64 per group.
template <int FORM, int D, int P, int FD, int PREC, int VARIANT>
__device__ void batch_task(const BatchArgs& A, const BinDesc& bd, int64_t first, int n, int lane,
                           typename PrecT<PREC>::gtype* gtile, typename PrecT<PREC>::otype* stage, int64_t* soffs) {
    using C = ScalarCfg<FORM, D, P, FD, PREC>;
    constexpr int KR = C::KR, NT = C::NT, KS = C::KS, NS = C::NS;
    ScalarWave<FORM, D, P, FD, PREC> W;
    W.lane = lane;
    W.col = lane & 15;
    W.gtile = gtile;
    W.stage = stage;
    W.rf = reinterpret_cast<const typename C::frag_t*>(bd.rfrag);
    W.out = reinterpret_cast<typename C::out_t*>(A.out);
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
            for (int s = 0; s < KS; ++s) W.rreg[t][s] = W.rf[(t * KS + s) * 64 + lane];
    }
    LinArgs L;
    L.coords = bd.coords;
    L.c2v = bd.c2v;
    L.f0 = bd.f0;
    L.f1 = FieldArg{nullptr, nullptr};
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
        const int c0 = A.bcell[p0];
        o0 = A.boff[p0];
        load_idx<FORM, D, FD>(L, c0, ix);
        load_raw<FORM, D, FD>(L, c0, ix, raw);
        G_from_raw<FORM, D, FD>(raw, L, true, Gv);
        const int64_t p1 = at(1);
        c1 = A.bcell[p1];
        o1 = A.boff[p1];
        load_idx<FORM, D, FD>(L, c1, ix);
        const int64_t p2 = at(2);
        c2 = A.bcell[p2];
        o2 = A.boff[p2];
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
    for (int g = 0; g < nfull; ++g) {
        load_raw<FORM, D, FD>(L, c1, ix, raw);  // group g + 1
        load_idx<FORM, D, FD>(L, c2, ix);       // group g + 2
        const int64_t p3 = at(g + 3);
        const int c3 = A.bcell[p3];
        const int64_t o3 = A.boff[p3];
        batch_tile<FORM, D, P, FD, PREC, VARIANT, true>(W, Gv, 0, o0, true, soffs);
        batch_tile<FORM, D, P, FD, PREC, VARIANT, true>(W, Gv, 1, o0, true, soffs);
        batch_tile<FORM, D, P, FD, PREC, VARIANT, true>(W, Gv, 2, o0, true, soffs);
        batch_tile<FORM, D, P, FD, PREC, VARIANT, true>(W, Gv, 3, o0, true, soffs);
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
            batch_tile<FORM, D, P, FD, PREC, VARIANT, false>(W, Gv, j, o0, valid, soffs);
        }
    }
}

template <int PREC, int VARIANT>
__device__ inline void batch_dispatch_v(const BatchArgs& A, const BinDesc& bd, int64_t first, int n, int lane,
                                        typename PrecT<PREC>::gtype* gtile, typename PrecT<PREC>::otype* stage,
                                        int64_t* soffs) {
    switch (bd.type) {
        case 0: batch_task<F_MASS, 2, 1, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 1: batch_task<F_MASS, 2, 2, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 2: batch_task<F_MASS, 2, 3, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 3: batch_task<F_MASS, 2, 4, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 4: batch_task<F_MASS, 3, 1, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 5: batch_task<F_MASS, 3, 2, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 6: batch_task<F_MASS, 3, 3, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 7: batch_task<F_HELM, 2, 1, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 8: batch_task<F_HELM, 2, 2, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 9: batch_task<F_HELM, 2, 3, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 10: batch_task<F_HELM, 2, 4, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 11: batch_task<F_HELM, 3, 1, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 12: batch_task<F_HELM, 3, 2, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 13: batch_task<F_HELM, 3, 3, 1, PREC, VARIANT>(A, bd, first, n, lane, gtile, stage, soffs); break;
        default: break;
    }
}

// Dynamic LDS per wave: G tile (16 x kGtileRow), output offsets (8), and the
// staging area of `stage_elems` elements (8 tensors of the largest staged bin).
template <int PREC>
__global__ __launch_bounds__(256) void k_batch(BatchArgs A, int stage_elems) {
    using g_t = typename PrecT<PREC>::gtype;
    using out_t = typename PrecT<PREC>::otype;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const size_t per_wave = (size_t)16 * kGtileRow * sizeof(g_t) + 8 * sizeof(int64_t) +
                            (size_t)stage_elems * sizeof(out_t);
    unsigned char* mine = lds + wave * per_wave;
    g_t* gtile = reinterpret_cast<g_t*>(mine);
    int64_t* soffs = reinterpret_cast<int64_t*>(mine + (size_t)16 * kGtileRow * sizeof(g_t));
    out_t* stage = reinterpret_cast<out_t*>(mine + (size_t)16 * kGtileRow * sizeof(g_t) + 8 * sizeof(int64_t));
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
        t = __shfl(t, 0);
        if ((int64_t)t >= total) break;
        int b = 0;
        int64_t tb = 0;
#pragma unroll
        for (int k = 1; k < kMaxBins; ++k)
            if ((int64_t)t >= tstart[k]) {
                b = k;
                tb = tstart[k];
            }
        const BinDesc& bd = A.bins[b];
        const int64_t local = ((int64_t)t - tb) * bd.task_cells;
        const int64_t cnt = (int64_t)A.counts[b];
        const int n = (int)(cnt - local < bd.task_cells ? cnt - local : bd.task_cells);
        const int64_t first = (int64_t)A.offs[b] + local;
        if (bd.variant == 0) batch_dispatch_v<PREC, 0>(A, bd, first, n, lane, gtile, stage, soffs);
        else batch_dispatch_v<PREC, 1>(A, bd, first, n, lane, gtile, stage, soffs);
    }
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace dev

int64_t batch_workspace_bytes(int nseg, int64_t nentries) {
    (void)nseg;
    return (int64_t)(4 * dev::kMaxBins) * 8 + 256 + nentries * 12;
}

static int batch_type(int form, int cell, int degree) {
    int shape = -1;
    if (cell == 2 && degree >= 1 && degree <= 4) shape = degree - 1;
    if (cell == 3 && degree >= 1 && degree <= 3) shape = 3 + degree;
    if (shape < 0) return -1;
    if (form == COFFEE_MASS) return shape;
    if (form == COFFEE_HELMHOLTZ) return 7 + shape;
    return -1;
}

coffee_status assemble_batch(int precision, const coffee_segment* segs, int nseg, const int32_t* seg_of,
                             const int64_t* cell_of, const int64_t* out_offset, int64_t nentries, void* out,
                             void* workspace, int64_t workspace_bytes, void* hip_stream) {
    if (precision != COFFEE_FP64 && precision != COFFEE_FP32) return COFFEE_E_UNSUPPORTED;
    if (!segs || nseg < 1 || nseg > dev::kMaxBins || nentries < 0) return COFFEE_E_INVALID_ARG;
    if (nentries > INT32_MAX) return COFFEE_E_UNSUPPORTED;
    if (nentries > 0 && (!seg_of || !cell_of || !out_offset || !out || !workspace)) return COFFEE_E_INVALID_ARG;
    if (nentries > 0 && workspace_bytes < batch_workspace_bytes(nseg, nentries)) return COFFEE_E_BUFFER_TOO_SMALL;
    if (((uintptr_t)workspace & 7) != 0) return COFFEE_E_INVALID_ARG;
    dev::BatchArgs a;
    std::memset(&a, 0, sizeof a);
    int devid = 0;
    if (hipGetDevice(&devid) != hipSuccess) return COFFEE_E_HIP;
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
        if (q > 10) return COFFEE_E_INVALID_ARG;
        const void* rf = nullptr;
        coffee_status st = get_rtable_public(devid, s.form, s.cell, s.degree, q, 1, precision, &rf);
        if (st != COFFEE_OK) return st;
        dev::BinDesc& d = a.bins[b];
        d.coords = s.coords;
        d.c2v = s.cell_to_vertex;
        d.f0 = dev::FieldArg{s.coeff->values, s.coeff->cell_to_dof};
        d.rfrag = rf;
        d.type = type;
        d.variant = s.variant;
        d.task_cells = s.task_cells ? s.task_cells : 256;
        int tv = 0, tt = 0;
        if (s.task_cells == 0 && tuned_batch(s.form, s.cell, s.degree, precision, &tv, &tt)) {
            d.variant = tv;
            d.task_cells = tt;
        }
    }
    if (nentries == 0) return COFFEE_OK;
    a.nbins = nseg;
    a.nentries = nentries;
    a.seg_of = seg_of;
    a.cell_of = cell_of;
    a.out_offset = out_offset;
    a.out = out;
    unsigned long long* ws = reinterpret_cast<unsigned long long*>(workspace);
    a.counts = ws;
    a.offs = ws + dev::kMaxBins;
    a.cursor = ws + 2 * dev::kMaxBins;
    a.queue = ws + 3 * dev::kMaxBins;
    a.boff = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(workspace) + 4 * dev::kMaxBins * 8 + 256);
    a.bcell = reinterpret_cast<int32_t*>(a.boff + nentries);
    hipStream_t s = (hipStream_t)hip_stream;
    const int ncu = num_cu(devid);
    hipLaunchKernelGGL(dev::k_fill_u64, dim3(1), dim3(64), 0, s, ws, (unsigned long long)0, (int64_t)(4 * dev::kMaxBins));
    const int gh = (int)std::min<int64_t>((nentries + 255) / 256, (int64_t)ncu * 4);
    hipLaunchKernelGGL(dev::k_bin_count, dim3(gh), dim3(256), 0, s, a);
    hipLaunchKernelGGL(dev::k_bin_scan, dim3(1), dim3(64), 0, s, a);
    const int64_t slice = std::max<int64_t>(256, (nentries + ncu * 4 - 1) / (ncu * 4));
    const int gs = (int)((nentries + slice - 1) / slice);
    hipLaunchKernelGGL(dev::k_bin_scatter, dim3(gs), dim3(256), 0, s, a, slice);
    // staging area: 8 tensors of the largest bin that stages its stores
    int stage_elems = 8;
    for (int b = 0; b < nseg; ++b)
        if (a.bins[b].variant == 0) {
            const int ns = n_scalar(segs[b].cell, segs[b].degree);
            stage_elems = std::max(stage_elems, 8 * ns * ns);
        }
    stage_elems = (stage_elems + 3) / 4 * 4;  // 16-byte multiple for FP32
    const size_t gsz = precision == COFFEE_FP64 ? 8 : 4;
    const size_t lds = 4 * ((size_t)16 * dev::kGtileRow * gsz + 8 * 8 + (size_t)stage_elems * gsz);
    if (lds > 160 * 1024) return COFFEE_E_UNSUPPORTED;
    const void* kern = precision == COFFEE_FP64 ? (const void*)&dev::k_batch<dev::PREC_F64>
                                                : (const void*)&dev::k_batch<dev::PREC_F32>;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, 256, lds) != hipSuccess || nb <= 0) nb = 1;
    const int grid = ncu * nb * std::max(1, batch_grid_mult());
    if (precision == COFFEE_FP64)
        hipLaunchKernelGGL(dev::k_batch<dev::PREC_F64>, dim3(grid), dim3(256), lds, s, a, stage_elems);
    else
        hipLaunchKernelGGL(dev::k_batch<dev::PREC_F32>, dim3(grid), dim3(256), lds, s, a, stage_elems);
    return hipGetLastError() == hipSuccess ? COFFEE_OK : COFFEE_E_HIP;
}

}  // namespace coffee

extern "C" coffee_status coffee_assemble_batch(int precision, const coffee_segment* segs, int nseg,
                                               const int32_t* seg_of, const int64_t* cell_of,
                                               const int64_t* out_offset, int64_t nentries, void* out,
                                               void* workspace, int64_t workspace_bytes, void* hip_stream) {
    return coffee::assemble_batch(precision, segs, nseg, seg_of, cell_of, out_offset, nentries, out, workspace,
                                  workspace_bytes, hip_stream);
}

extern "C" int64_t coffee_batch_workspace_size(int nseg, int64_t nentries) {
    return coffee::batch_workspace_bytes(nseg, nentries);
}
