// Mixed persistent batch: cells of different shape, degree and form in one
// launch (the paper's inter-kernel vectorization across cells, section 4,
// applied to a heterogeneous set of cells).
//
// 1. Binning on the device: per-workgroup histograms of the entries' segment
//    ids, a prefix sum, and a scatter of entry indices into per-bin lists
//    (each workgroup reserves one contiguous range per bin, so the relative
//    order of entries inside a workgroup's slice is kept).
// 2. One persistent kernel: every wave takes tasks (task_cells consecutive
//    entries of one bin) from a single atomic queue that lists the bins in
//    segment order, and runs the symmetric-form contraction of that bin's
//    (form, shape, degree) on them: FP64 geometry and G per lane, MFMA
//    contraction against the bin's reference tensors, element tensors written
//    to the entries' own output offsets, either staged through LDS (8 tensors
//    at a time) or stored straight from the accumulators.
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
    int32_t* list;                // [nentries]
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

// Each workgroup takes a contiguous slice of entries, counts per bin, reserves
// one range per bin and writes its entries in slice order.
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
    // in-order placement within the slice: one pass per 256 entries, ranks by prefix in LDS
    __shared__ int seg[256];
    for (int64_t c = s0; c < s1; c += blockDim.x) {
        const int64_t i = c + threadIdx.x;
        const int sg = i < s1 ? A.seg_of[i] : -1;
        seg[threadIdx.x] = sg;
        __syncthreads();
        if (sg >= 0) {
            int rank = 0;
            for (int t = 0; t < (int)threadIdx.x; ++t) rank += (seg[t] == sg);
            A.list[base[sg] + h[sg] + rank] = (int32_t)i;
        }
        __syncthreads();
        if (threadIdx.x < A.nbins) {
            int cnt = 0;
            for (int t = 0; t < (int)blockDim.x; ++t) cnt += (seg[t] == (int)threadIdx.x);
            h[threadIdx.x] += cnt;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- tasks

template <int D, int P, int PREC>
struct BatchCfg {
    static constexpr int NS = nsc(D, P);
    static constexpr int NN = NS * NS;
};

constexpr int kGtileRow = 16;  // >= any G row of the compiled bin types (KR <= 10)

template <int FORM, int D, int P, int FD, int PREC>
__device__ void batch_task(const BatchArgs& A, const BinDesc& bd, int64_t first, int n, int lane,
                           typename PrecT<PREC>::gtype* gtile, typename PrecT<PREC>::otype* stage, int64_t* soffs) {
    using frag_t = typename PrecT<PREC>::frag;
    using acc_t = typename PrecT<PREC>::acc;
    using out_t = typename PrecT<PREC>::otype;
    constexpr int NS = nsc(D, P), NN = NS * NS;
    constexpr int KR = kref(FORM, D, FD);
    constexpr int KS = ksteps(FORM, D, FD, PREC);
    constexpr int NT = ntiles_sym(D, P);
    constexpr int NU = nuniq(D, P);
    constexpr int ROW = GLayout<FORM, D, FD, PREC>::ROW;
    static_assert(ROW <= kGtileRow, "G row does not fit the batch tile");
    const int col = lane & 15;
    const frag_t* rf = reinterpret_cast<const frag_t*>(bd.rfrag);
    out_t* out = reinterpret_cast<out_t*>(A.out);
    LinArgs L;
    L.coords = bd.coords;
    L.c2v = bd.c2v;
    L.f0 = bd.f0;
    int ua[NT], ub[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        int u = t * 16 + col, a = 0;
        while (a < NS - 1 && u >= NS - a) { u -= NS - a; ++a; }
        ua[t] = a;
        ub[t] = a + u;
    }
#pragma unroll 1
    for (int g0 = 0; g0 < n; g0 += 64) {
        const bool valid = g0 + lane < n;
        const int64_t li = first + g0 + (valid ? lane : 0);
        const int64_t entry = A.list[li];
        const int64_t cell = A.cell_of[entry];
        const int64_t myoff = A.out_offset[entry];
        double Gv[KR];
        {
            CellIdx<FORM, D, FD> ix;
            CellRaw<FORM, D, FD> raw;
            load_idx<FORM, D, FD>(L, cell, ix);
            load_raw<FORM, D, FD>(L, cell, ix, raw);
            CellData<FORM, D, FD> cd;
            cell_from_raw<FORM, D, FD>(raw, cd);
            build_G<FORM, D, FD, 0, 0>(cd, L, Gv);
        }
#pragma unroll 1
        for (int j = 0; j < 4; ++j) {
            if (g0 + 16 * j >= n) break;  // wave-uniform
            if ((lane >> 4) == j) put_G_row<FORM, D, FD, PREC>(gtile + col * ROW, Gv);
            wave_sync();
            constexpr int NTC = NT;
            acc_t acc[NTC];
#pragma unroll
            for (int t = 0; t < NTC; ++t) acc[t] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const frag_t a = load_afrag<PREC>(gtile, ROW, lane, s);
#pragma unroll
                for (int t = 0; t < NTC; ++t) acc[t] = mfma<PREC>(a, rf[(t * KS + s) * 64 + lane], acc[t]);
            }
            if (bd.variant == 0) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    wave_sync();
                    // output offsets of the 8 cells of this half
                    if ((lane >> 3) == 2 * j + h) soffs[lane & 7] = valid ? myoff : -1;
#pragma unroll
                    for (int t = 0; t < NTC; ++t) {
                        if (t * 16 + col >= NU) continue;
                        const int oab = ua[t] * NS + ub[t], oba = ub[t] * NS + ua[t];
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = acc_row<PREC>(lane, v);
                            if ((row >> 3) != h) continue;
                            const out_t x = (out_t)acc[t][v];
                            stage[(row & 7) * NN + oab] = x;
                            stage[(row & 7) * NN + oba] = x;
                        }
                    }
                    wave_sync();
#pragma unroll 2
                    for (int k = lane; k < 8 * NN; k += 64) {
                        const int c = k / NN, e = k - (k / NN) * NN;
                        const int64_t o = soffs[c];
                        if (o >= 0) out[o + e] = stage[k];
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
                    rok[v] = g0 + src < n;
                }
#pragma unroll
                for (int t = 0; t < NTC; ++t) {
                    if (t * 16 + col >= NU) continue;
                    const int a = ua[t], bb = ub[t];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (rok[v]) {
                            const out_t x = (out_t)acc[t][v];
                            out[roff[v] + a * NS + bb] = x;
                            out[roff[v] + bb * NS + a] = x;
                        }
                    }
                }
            }
            wave_sync();
        }
    }
}

template <int PREC>
__device__ inline void batch_dispatch(const BatchArgs& A, const BinDesc& bd, int64_t first, int n, int lane,
                                      typename PrecT<PREC>::gtype* gtile, typename PrecT<PREC>::otype* stage,
                                      int64_t* soffs) {
    switch (bd.type) {
        case 0: batch_task<F_MASS, 2, 1, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 1: batch_task<F_MASS, 2, 2, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 2: batch_task<F_MASS, 2, 3, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 3: batch_task<F_MASS, 2, 4, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 4: batch_task<F_MASS, 3, 1, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 5: batch_task<F_MASS, 3, 2, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 6: batch_task<F_MASS, 3, 3, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 7: batch_task<F_HELM, 2, 1, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 8: batch_task<F_HELM, 2, 2, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 9: batch_task<F_HELM, 2, 3, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 10: batch_task<F_HELM, 2, 4, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 11: batch_task<F_HELM, 3, 1, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 12: batch_task<F_HELM, 3, 2, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
        case 13: batch_task<F_HELM, 3, 3, 1, PREC>(A, bd, first, n, lane, gtile, stage, soffs); break;
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
    int64_t ntask[kMaxBins], tstart[kMaxBins + 1];
    tstart[0] = 0;
#pragma unroll
    for (int b = 0; b < kMaxBins; ++b) {
        const int64_t c = b < A.nbins ? (int64_t)A.counts[b] : 0;
        const int tc = b < A.nbins ? A.bins[b].task_cells : 64;
        ntask[b] = (c + tc - 1) / tc;
        tstart[b + 1] = tstart[b] + ntask[b];
    }
    const int64_t total = tstart[kMaxBins];
    for (;;) {
        unsigned long long t = 0;
        if (lane == 0) t = atomicAdd(A.queue, 1ull);
        t = __shfl(t, 0);
        if ((int64_t)t >= total) break;
        int b = 0;
#pragma unroll
        for (int k = 1; k < kMaxBins; ++k)
            if ((int64_t)t >= tstart[k]) b = k;
        const BinDesc& bd = A.bins[b];
        const int64_t local = ((int64_t)t - tstart[b]) * bd.task_cells;
        const int64_t cnt = (int64_t)A.counts[b];
        const int n = (int)(cnt - local < bd.task_cells ? cnt - local : bd.task_cells);
        batch_dispatch<PREC>(A, bd, (int64_t)A.offs[b] + local, n, lane, gtile, stage, soffs);
    }
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace dev

int64_t batch_workspace_bytes(int nseg, int64_t nentries) {
    (void)nseg;
    return (int64_t)(4 * dev::kMaxBins) * 8 + 256 + nentries * 4;
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
        if (!s.coeff || !s.coeff->values || s.coeff->degree != 1 || s.coeff->ncomp != 1) return COFFEE_E_UNSUPPORTED;
        if (s.variant < 0 || s.variant > 1) return COFFEE_E_INVALID_ARG;
        if (s.task_cells != 0 && s.task_cells != 64 && s.task_cells != 128 && s.task_cells != 256)
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
        d.task_cells = s.task_cells ? s.task_cells : 64;
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
    a.list = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(workspace) + 4 * dev::kMaxBins * 8 + 256);
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
