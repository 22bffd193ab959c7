// Global assembly: the element tensors summed into the sparse matrix of the
// linear system (paper, section 2: the per-cell contributions are added to
// the global system; local assembly is the step before this one).
//
// Pattern (symbolic phase, once per mesh and space): every pair of dofs
// that share a cell is a nonzero. The pairs (dof_i, dof_j) of all cells,
// as 64-bit keys dof_i * ndofs + dof_j, are radix-sorted and deduplicated;
// the sorted unique keys are the scalar pattern in CSR order, the row
// pointers come from a histogram of their rows and a prefix sum. For a
// vector space with ncomp components (global index dof * ncomp + c) every
// scalar nonzero becomes an ncomp x ncomp block.
//
// Numeric phase: the cells are assembled in chunks into a workspace by the
// local-assembly engines (coffee_assemble), then every element-tensor entry
// is added to its matrix entry, found by binary search in the row's column
// indices, with an atomic add (FP64 or FP32 by precision).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "library.h"
#include "tables.h"

namespace coffee {
namespace dev {

__global__ __launch_bounds__(256) void k_pair_keys(const int32_t* __restrict__ c2d, int64_t ncells, int nloc,
                                                  uint64_t ndofs, uint64_t* __restrict__ keys) {
    const int64_t total = ncells * nloc * nloc;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / (nloc * nloc);
        const int ij = (int)(t - e * nloc * nloc), i = ij / nloc, j = ij - (ij / nloc) * nloc;
        keys[t] = (uint64_t)(uint32_t)c2d[e * nloc + i] * ndofs + (uint32_t)c2d[e * nloc + j];
    }
}

// flag[k] = 1 if sorted key k differs from key k-1 (first of its run)
__global__ __launch_bounds__(256) void k_run_heads(const uint64_t* __restrict__ sk, int64_t n,
                                                  int32_t* __restrict__ flag) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        flag[k] = (k == 0 || sk[k] != sk[k - 1]) ? 1 : 0;
}

// unique key u = pos[k] for run heads: scalar column and per-row count
__global__ __launch_bounds__(256) void k_compact(const uint64_t* __restrict__ sk, const int32_t* __restrict__ flag,
                                                const int64_t* __restrict__ pos, int64_t n, uint64_t ndofs,
                                                int32_t* __restrict__ scol, int64_t* __restrict__ rowcnt) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        if (!flag[k]) continue;
        const uint64_t key = sk[k];
        scol[pos[k]] = (int32_t)(key % ndofs);
        atomicAdd(reinterpret_cast<unsigned long long*>(&rowcnt[key / ndofs]), 1ull);
    }
}

// block expansion of the scalar pattern into the ncomp-component pattern
__global__ __launch_bounds__(256) void k_expand(const int64_t* __restrict__ srow, const int32_t* __restrict__ scol,
                                               int64_t ndofs, int nc, int64_t* __restrict__ row_ptr,
                                               int32_t* __restrict__ col_idx) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < ndofs; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = srow[r], len = srow[r + 1] - b;
        for (int c1 = 0; c1 < nc; ++c1) {
            const int64_t R = r * nc + c1, start = (int64_t)nc * nc * b + (int64_t)c1 * nc * len;
            row_ptr[R] = start;
            for (int64_t m = 0; m < len; ++m)
                for (int c2 = 0; c2 < nc; ++c2) col_idx[start + m * nc + c2] = scol[b + m] * nc + c2;
        }
        if (r == ndofs - 1) row_ptr[ndofs * nc] = (int64_t)nc * nc * srow[ndofs];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero(T* p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

// One thread per (cell, test row): the row's entries are added to the matrix.
// The element tensor is component-blocked ((c, a) -> c * n + a); the global
// index of local dof (c, a) is dof(a) * nc + c.
template <typename T>
__global__ __launch_bounds__(256) void k_scatter_csr(const T* __restrict__ A, const int32_t* __restrict__ c2d,
                                                    int64_t ncells, int n, int nc, const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col_idx, T* __restrict__ values) {
    const int N = n * nc;
    const int64_t total = ncells * N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / N;
        const int i = (int)(t - e * N), ci = i / n, ai = i - ci * n;
        const int64_t row = (int64_t)c2d[e * n + ai] * nc + ci;
        const int64_t b0 = row_ptr[row], b1 = row_ptr[row + 1];
        if (b1 <= b0) continue;  // a row outside the pattern: nothing to add to
        const T* Ae = A + (e * N + i) * N;
        for (int j = 0; j < N; ++j) {
            const int cj = j / n, aj = j - cj * n;
            const int32_t col = c2d[e * n + aj] * nc + cj;
            int64_t lo = b0, hi = b1 - 1;
            while (lo < hi) {  // first index with col_idx >= col
                const int64_t mid = (lo + hi) >> 1;
                if (col_idx[mid] < col) lo = mid + 1;
                else hi = mid;
            }
            atomicAdd(&values[lo], Ae[j]);
        }
    }
}

}  // namespace dev

namespace {

constexpr int64_t kAlign = 256;
int64_t al(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

unsigned pair_bits(int64_t ndofs) {
    const unsigned __int128 m = (unsigned __int128)ndofs * (unsigned __int128)ndofs;
    unsigned b = 1;
    while (b < 64 && ((unsigned __int128)1 << b) < m) ++b;
    return b;
}

bool pattern_temp(int64_t npairs, int64_t ndofs, size_t* sort_bytes, size_t* scan_bytes) {
    *sort_bytes = *scan_bytes = 0;
    if (npairs == 0) return true;
    if (rocprim::radix_sort_keys(nullptr, *sort_bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr, (size_t)npairs,
                                 0u, pair_bits(ndofs), (hipStream_t)0) != hipSuccess)
        return false;
    size_t a = 0, b = 0;
    if (rocprim::exclusive_scan(nullptr, a, (const int32_t*)nullptr, (int64_t*)nullptr, (int64_t)0, (size_t)npairs,
                                rocprim::plus<int64_t>(), (hipStream_t)0) != hipSuccess)
        return false;
    if (rocprim::exclusive_scan(nullptr, b, (const int64_t*)nullptr, (int64_t*)nullptr, (int64_t)0,
                                (size_t)(ndofs + 1), rocprim::plus<int64_t>(), (hipStream_t)0) != hipSuccess)
        return false;
    *scan_bytes = std::max(a, b);
    return true;
}

struct PatternWs {
    uint64_t *keys, *skeys;
    int32_t *flag, *scol;
    int64_t *pos, *rowcnt, *srow;
    void* temp;
    int64_t bytes;
};

bool pattern_layout(int64_t ncells, int nloc, int64_t ndofs, char* base, PatternWs* w) {
    const int64_t np = ncells * nloc * nloc;
    size_t sb = 0, scb = 0;
    if (!pattern_temp(np, ndofs, &sb, &scb)) return false;
    int64_t o = 0;
    auto take = [&](int64_t n) { char* p = base ? base + o : nullptr; o += al(n); return p; };
    w->keys = (uint64_t*)take(np * 8);
    w->skeys = (uint64_t*)take(np * 8);
    w->flag = (int32_t*)take(np * 4);
    w->pos = (int64_t*)take(np * 8);
    w->scol = (int32_t*)take(np * 4);
    w->rowcnt = (int64_t*)take((ndofs + 1) * 8);
    w->srow = (int64_t*)take((ndofs + 1) * 8);
    w->temp = take((int64_t)std::max(sb, scb));
    w->bytes = o;
    return true;
}

int grid_of(int64_t work) { return (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 16384)); }

}  // namespace

}  // namespace coffee

using namespace coffee;

extern "C" int64_t coffee_csr_pattern_workspace_size(int64_t ncells, int nloc, int64_t ndofs) {
    if (ncells < 0 || nloc < 1 || nloc > kMaxN || ndofs < 1 || ndofs > INT32_MAX) return -1;
    PatternWs w;
    if (!pattern_layout(ncells, nloc, ndofs, nullptr, &w)) return -1;
    return w.bytes;
}

extern "C" coffee_status coffee_csr_pattern(const int32_t* cell_to_dof, int64_t ncells, int nloc, int64_t ndofs,
                                            int ncomp, int64_t* row_ptr, int32_t* col_idx, int64_t col_capacity,
                                            int64_t* nnz, void* workspace, int64_t workspace_bytes,
                                            void* hip_stream) {
    if (!nnz || ncells < 0 || nloc < 1 || nloc > kMaxN || ndofs < 1 || ndofs > INT32_MAX || ncomp < 1 || ncomp > 3)
        return COFFEE_E_INVALID_ARG;
    if ((int64_t)ndofs * ncomp > INT32_MAX) return COFFEE_E_UNSUPPORTED;
    if (!row_ptr || (ncells > 0 && (!cell_to_dof || !workspace))) return COFFEE_E_INVALID_ARG;
    if (((uintptr_t)workspace & 255) != 0) return COFFEE_E_INVALID_ARG;
    PatternWs w;
    if (!pattern_layout(ncells, nloc, ndofs, (char*)workspace, &w)) return COFFEE_E_HIP;
    if (ncells > 0 && workspace_bytes < w.bytes) return COFFEE_E_BUFFER_TOO_SMALL;
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t np = ncells * nloc * nloc;
    int64_t nscal = 0;
    if (np > 0) {
        hipLaunchKernelGGL(dev::k_pair_keys, dim3(grid_of(np)), dim3(256), 0, s, cell_to_dof, ncells, nloc,
                           (uint64_t)ndofs, w.keys);
        size_t sb = 0, scb = 0;
        pattern_temp(np, ndofs, &sb, &scb);
        if (rocprim::radix_sort_keys(w.temp, sb, w.keys, w.skeys, (size_t)np, 0u, pair_bits(ndofs), s) != hipSuccess)
            return COFFEE_E_HIP;
        hipLaunchKernelGGL(dev::k_run_heads, dim3(grid_of(np)), dim3(256), 0, s, w.skeys, np, w.flag);
        if (rocprim::exclusive_scan(w.temp, scb, w.flag, w.pos, (int64_t)0, (size_t)np, rocprim::plus<int64_t>(), s) !=
            hipSuccess)
            return COFFEE_E_HIP;
        hipLaunchKernelGGL(dev::k_zero<int64_t>, dim3(grid_of(ndofs + 1)), dim3(256), 0, s, w.rowcnt, ndofs + 1);
        hipLaunchKernelGGL(dev::k_compact, dim3(grid_of(np)), dim3(256), 0, s, w.skeys, w.flag, w.pos, np,
                           (uint64_t)ndofs, w.scol, w.rowcnt);
        if (rocprim::exclusive_scan(w.temp, scb, w.rowcnt, w.srow, (int64_t)0, (size_t)(ndofs + 1),
                                    rocprim::plus<int64_t>(), s) != hipSuccess)
            return COFFEE_E_HIP;
        if (hipMemcpyAsync(&nscal, w.srow + ndofs, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return COFFEE_E_HIP;
    }
    const int64_t total = nscal * ncomp * ncomp;
    *nnz = total;
    if (!col_idx || col_capacity < total) return COFFEE_E_BUFFER_TOO_SMALL;
    if (np == 0) {
        hipLaunchKernelGGL(dev::k_zero<int64_t>, dim3(grid_of(ndofs * ncomp + 1)), dim3(256), 0, s, row_ptr,
                           ndofs * ncomp + 1);
    } else {
        hipLaunchKernelGGL(dev::k_expand, dim3(grid_of(ndofs)), dim3(256), 0, s, w.srow, w.scol, ndofs, ncomp, row_ptr,
                           col_idx);
    }
    return hipGetLastError() == hipSuccess ? COFFEE_OK : COFFEE_E_HIP;
}

namespace {

// chunk of cells assembled into the workspace at a time
constexpr int64_t kCsrChunk = 1 << 17;

}  // namespace

extern "C" int64_t coffee_assemble_csr_workspace_size(int form, int cell, int degree, int precision, int64_t ncells) {
    const int N = coffee_tensor_dim(form, cell, degree);
    if (N <= 0 || ncells < 0 || precision < COFFEE_FP64 || precision > COFFEE_BF16X3) return -1;
    const int64_t chunk = std::min<int64_t>(ncells, kCsrChunk);
    return al(chunk * N * N * (precision == COFFEE_FP64 ? 8 : 4));
}

extern "C" coffee_status coffee_assemble_csr(int form, int cell, int degree, int quad_degree, int precision,
                                             const double* coords, int64_t nvert, const int32_t* c2v,
                                             int64_t ncells, const coffee_field* coeffs, int ncoeff,
                                             const double* constants, int nconst, const int32_t* cell_to_dof,
                                             int64_t ndofs, const int64_t* row_ptr, const int32_t* col_idx,
                                             int64_t nnz, void* values, void* workspace, int64_t workspace_bytes,
                                             void* hip_stream) {
    if (form == COFFEE_SVK_ENERGY || form == COFFEE_SVK_RESIDUAL) return COFFEE_E_UNSUPPORTED;
    const int N = coffee_tensor_dim(form, cell, degree);
    if (N <= 0) return COFFEE_E_INVALID_ARG;
    const int n = cell_nscalar(cell, degree), nc = N / n;
    if (degree > 1 && !cell_to_dof) return COFFEE_E_INVALID_ARG;  // P1: the vertices are the dofs
    const int32_t* map = cell_to_dof ? cell_to_dof : c2v;
    if (ndofs < 1 || nnz < 0 || (nnz > 0 && (!row_ptr || !col_idx || !values))) return COFFEE_E_INVALID_ARG;
    const int64_t need = coffee_assemble_csr_workspace_size(form, cell, degree, precision, ncells);
    if (need < 0) return COFFEE_E_INVALID_ARG;
    if (ncells > 0 && (!workspace || workspace_bytes < need)) return workspace ? COFFEE_E_BUFFER_TOO_SMALL
                                                                               : COFFEE_E_INVALID_ARG;
    if (((uintptr_t)workspace & 15) != 0) return COFFEE_E_INVALID_ARG;
    if (ncoeff < 0 || ncoeff > 2 || (ncoeff > 0 && !coeffs)) return COFFEE_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    const bool f64 = precision == COFFEE_FP64;
    if (nnz > 0) {
        if (f64) hipLaunchKernelGGL(dev::k_zero<double>, dim3(grid_of(nnz)), dim3(256), 0, s, (double*)values, nnz);
        else hipLaunchKernelGGL(dev::k_zero<float>, dim3(grid_of(nnz)), dim3(256), 0, s, (float*)values, nnz);
    }
    coffee_field fl[2];
    for (int64_t e0 = 0; e0 < ncells; e0 += kCsrChunk) {
        const int64_t m = std::min<int64_t>(kCsrChunk, ncells - e0);
        for (int i = 0; i < ncoeff; ++i) {
            // the chunk's cells: offset the dof map, or the cell-major values
            fl[i] = coeffs[i];
            const int64_t nl = cell_nscalar(cell, coeffs[i].degree);
            if (coeffs[i].cell_to_dof) fl[i].cell_to_dof = coeffs[i].cell_to_dof + e0 * nl;
            else if (coeffs[i].values) fl[i].values = coeffs[i].values + e0 * nl * coeffs[i].ncomp;
        }
        coffee_status st = coffee_assemble(form, cell, degree, quad_degree, precision, coords, nvert,
                                           c2v + e0 * cell_nverts(cell), m, fl, ncoeff, constants, nconst, workspace,
                                           hip_stream);
        if (st != COFFEE_OK) return st;
        const int64_t work = m * N;
        if (f64)
            hipLaunchKernelGGL(dev::k_scatter_csr<double>, dim3(grid_of(work)), dim3(256), 0, s,
                               (const double*)workspace, map + e0 * n, m, n, nc, row_ptr, col_idx, (double*)values);
        else
            hipLaunchKernelGGL(dev::k_scatter_csr<float>, dim3(grid_of(work)), dim3(256), 0, s,
                               (const float*)workspace, map + e0 * n, m, n, nc, row_ptr, col_idx, (float*)values);
        if (hipGetLastError() != hipSuccess) return COFFEE_E_HIP;
    }
    return COFFEE_OK;
}
