// Deterministic scatter of per-cell gradients (the adjoint's reproducible
// mode).
//
// The atomic scatter adds the cells' contributions to a shared vertex or dof
// in whatever order the hardware completes them, so FP64 sums can differ in
// the last bits from run to run. In the deterministic mode every adjoint
// kernel writes its per-cell contributions to a workspace instead (entry j =
// cell * slots + local slot, `ncomp` values each), and this file sums them per
// target in a fixed order:
//   1. a stable radix sort of the entries by target index (the target of
//      entry j is keys[j], i.e. the cell-to-vertex or cell-to-dof map read as
//      one flat array), carrying j along: the entries of one target come out
//      in increasing j, i.e. in increasing cell order;
//   2. one thread per run of equal keys adds the run's values in that order
//      and then adds the sum to the target (grad[t] += sum).
// The result depends only on the mesh and the values, not on the launch or on
// timing. Targets given cell-major (no map) have one entry each: grad[j] +=
// local[j].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "library.h"

namespace coffee {
namespace dev {

template <int NC>
__global__ __launch_bounds__(256) void k_det_gather(const uint32_t* __restrict__ skeys,
                                                    const int32_t* __restrict__ sidx,
                                                    const double* __restrict__ local, double* __restrict__ grad,
                                                    int64_t n) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = skeys[p];
        if (p > 0 && skeys[p - 1] == k) continue;  // not the first entry of its run
        double acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = 0.0;
        for (int64_t q = p; q < n && skeys[q] == k; ++q) {
            const int64_t j = sidx[q];
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] += local[j * NC + c];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) grad[(int64_t)k * NC + c] += acc[c];
    }
}

__global__ __launch_bounds__(256) void k_det_add(const double* __restrict__ local, double* __restrict__ grad,
                                                 int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        grad[i] += local[i];
}

}  // namespace dev

namespace {

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

unsigned key_bits(int64_t ntargets) {
    unsigned b = 1;
    while (b < 31 && ((int64_t)1 << b) < ntargets) ++b;
    return b;
}

// rocPRIM's temporary storage for sorting n (key, index) pairs over `bits` key bits.
bool sort_temp_bytes(int64_t n, unsigned bits, size_t* bytes) {
    *bytes = 0;
    if (n == 0) return true;
    rocprim::counting_iterator<int32_t> iota(0);
    const hipError_t e = rocprim::radix_sort_pairs(nullptr, *bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr, iota,
                                                   (int32_t*)nullptr, (size_t)n, 0u, bits, (hipStream_t)0);
    return e == hipSuccess;
}

}  // namespace

int64_t det_workspace_bytes(const DetTarget* t, int nt) {
    int64_t bytes = 0, nmax = 0;
    size_t temp = 0;
    for (int i = 0; i < nt; ++i) {
        bytes += align_up(t[i].n * t[i].ncomp * (int64_t)sizeof(double));
        if (t[i].mapped) {
            nmax = std::max(nmax, t[i].n);
            size_t tb = 0;
            if (!sort_temp_bytes(t[i].n, key_bits(t[i].ntargets), &tb)) return -1;
            temp = std::max(temp, tb);
        }
    }
    bytes += 2 * align_up(nmax * 4) + align_up((int64_t)temp);
    return bytes;
}

coffee_status det_carve(void* ws, int64_t ws_bytes, DetTarget* t, int nt) {
    const int64_t need = det_workspace_bytes(t, nt);
    if (need < 0) return COFFEE_E_HIP;
    if (!ws || ws_bytes < need) return ws ? COFFEE_E_BUFFER_TOO_SMALL : COFFEE_E_INVALID_ARG;
    if (((uintptr_t)ws & 255) != 0) return COFFEE_E_INVALID_ARG;
    char* p = (char*)ws;
    for (int i = 0; i < nt; ++i) {
        t[i].local = (double*)p;
        p += align_up(t[i].n * t[i].ncomp * (int64_t)sizeof(double));
    }
    return COFFEE_OK;
}

coffee_status det_scatter(const DetTarget* t, int nt, void* ws, hipStream_t s) {
    int64_t nmax = 0, off = 0;
    size_t temp = 0;
    for (int i = 0; i < nt; ++i) {
        off += align_up(t[i].n * t[i].ncomp * (int64_t)sizeof(double));
        if (t[i].mapped) {
            nmax = std::max(nmax, t[i].n);
            size_t tb = 0;
            if (!sort_temp_bytes(t[i].n, key_bits(t[i].ntargets), &tb)) return COFFEE_E_HIP;
            temp = std::max(temp, tb);
        }
    }
    char* base = (char*)ws + off;
    uint32_t* skeys = (uint32_t*)base;
    int32_t* sidx = (int32_t*)(base + align_up(nmax * 4));
    void* tmp = base + 2 * align_up(nmax * 4);
    for (int i = 0; i < nt; ++i) {
        const DetTarget& x = t[i];
        if (!x.grad || x.n == 0) continue;
        const int64_t work = x.mapped ? x.n : x.n * x.ncomp;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 8192));
        if (!x.mapped) {
            hipLaunchKernelGGL(dev::k_det_add, dim3(grid), dim3(256), 0, s, x.local, x.grad, x.n * x.ncomp);
            if (hipGetLastError() != hipSuccess) return COFFEE_E_HIP;
            continue;
        }
        const unsigned bits = key_bits(x.ntargets);
        size_t tb = temp;
        rocprim::counting_iterator<int32_t> iota(0);
        // the map read as unsigned keys (valid indices are non-negative)
        const uint32_t* keys = reinterpret_cast<const uint32_t*>(x.keys);
        if (rocprim::radix_sort_pairs(tmp, tb, keys, skeys, iota, sidx, (size_t)x.n, 0u, bits, s) != hipSuccess)
            return COFFEE_E_HIP;
        switch (x.ncomp) {
            case 1: hipLaunchKernelGGL(dev::k_det_gather<1>, dim3(grid), dim3(256), 0, s, skeys, sidx, x.local, x.grad, x.n); break;
            case 2: hipLaunchKernelGGL(dev::k_det_gather<2>, dim3(grid), dim3(256), 0, s, skeys, sidx, x.local, x.grad, x.n); break;
            case 3: hipLaunchKernelGGL(dev::k_det_gather<3>, dim3(grid), dim3(256), 0, s, skeys, sidx, x.local, x.grad, x.n); break;
            default: return COFFEE_E_UNSUPPORTED;
        }
        if (hipGetLastError() != hipSuccess) return COFFEE_E_HIP;
    }
    return COFFEE_OK;
}

}  // namespace coffee
