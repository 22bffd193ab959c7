// libcoffee host library: argument validation, per-device table cache, kernel
// dispatch and the small utility kernels. The C ABI is declared in
// include/coffee.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "library.h"
#include "registry.h"
#include "tables.h"

namespace coffee {

// ---------------------------------------------------------------- registry

static std::vector<LinEntry>& lin_registry() {
    static std::vector<LinEntry> reg;
    static std::once_flag once;
    std::call_once(once, [] {
        register_mass_tri(reg);
        register_mass_tet(reg);
        register_helmholtz_tri(reg);
        register_helmholtz_tet(reg);
        register_elasticity(reg);
        register_burgers(reg);
        register_diffusion(reg);
        register_variants(reg);
    });
    return reg;
}

// The instance of a key with the given tile-shape variant, or variant 0.
const LinEntry* find_linear(int form, int dim, int p, int fd, int prec, int variant) {
    const LinEntry* base = nullptr;
    for (const LinEntry& e : lin_registry())
        if (e.form == form && e.dim == dim && e.p == p && e.fd == fd && e.prec == prec) {
            if (e.variant == variant) return &e;
            if (e.variant == 0) base = &e;
        }
    return base;
}

extern "C" int coffee_has_variant(int form, int cell, int degree, int field_degree, int precision, int variant) {
    const LinEntry* e = find_linear(form, cell, degree, field_degree, precision, variant);
    return e && e->variant == variant ? 1 : 0;
}

// ---------------------------------------------------------------- device table cache

struct DevTable {
    void* ptr = nullptr;
    size_t bytes = 0;
};

struct DeviceCtx {
    std::map<std::tuple<int, int, int, int, int, int>, DevTable> rtab;  // (form, dim, p, q, fd, prec)
    std::map<const void*, int> occupancy;                               // kernel -> blocks per CU
    int num_cu = 0;
};

static std::mutex g_mu;
static std::map<int, DeviceCtx> g_ctx;

static DeviceCtx& device_ctx(int dev) {
    DeviceCtx& c = g_ctx[dev];
    if (c.num_cu == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        c.num_cu = n;
    }
    return c;
}

static uint16_t bf16_bits_host(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static float bf16_float_host(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Pack reference tensors in MFMA B-fragment order: fragment (t, s) for lane l
// holds rows k of the K dimension and output column 16 t + l % 16. Columns are
// the entries a <= b of the upper triangle in row-major order (symmetric
// engine), or the entries ab = a n + b in row groups of `rows_per_group` rows,
// each group starting on a fresh 16-column tile (vector engine).
std::vector<char> pack_fragments(const RefTensor& R, int prec, bool sym, int rows_per_group) {
    const int NS = R.NS, NN = R.NS * R.NS, KR = R.KR;
    std::vector<int> colmap;  // packed column -> entry, -1 for padding
    if (sym) {
        for (int a = 0; a < NS; ++a)
            for (int b = a; b < NS; ++b) colmap.push_back(a * NS + b);
    } else {
        for (int a0 = 0; a0 < NS; a0 += rows_per_group) {
            const int a1 = std::min(NS, a0 + rows_per_group);
            const int ne = (a1 - a0) * NS, nt = (ne + 15) / 16;
            for (int c = 0; c < 16 * nt; ++c) colmap.push_back(c < ne ? a0 * NS + c : -1);
        }
    }
    const int NC = (int)colmap.size();
    const int NT = (NC + 15) / 16;
    std::vector<char> buf;
    if (prec == COFFEE_FP64 || prec == COFFEE_FP32) {
        const int KS = (KR + 3) / 4;
        const size_t elem = prec == COFFEE_FP64 ? 8 : 4;
        buf.assign((size_t)NT * KS * 64 * elem, 0);
        for (int t = 0; t < NT; ++t)
            for (int s = 0; s < KS; ++s)
                for (int l = 0; l < 64; ++l) {
                    const int k = 4 * s + l / 16, c = 16 * t + l % 16;
                    const long double v = (k < KR && c < NC && colmap[c] >= 0) ? R.R[(size_t)k * NN + colmap[c]] : 0.0L;
                    const size_t idx = ((size_t)(t * KS + s) * 64 + l);
                    if (prec == COFFEE_FP64) {
                        double d = (double)v;
                        std::memcpy(&buf[idx * 8], &d, 8);
                    } else {
                        float f = (float)v;
                        std::memcpy(&buf[idx * 4], &f, 4);
                    }
                }
    } else {
        // symmetric engine: k' = part KR + k, parts (R_hi, R_lo, R_hi) against
        // G's (hi, hi, lo); vector engine: k' = 4 k + slot, slots (R_hi, R_lo,
        // R_hi, 0) against (hi, hi, lo, 0)
        const int KE = (sym ? 3 : 4) * KR, KS = (KE + 31) / 32;
        buf.assign((size_t)NT * KS * 64 * 16, 0);
        for (int t = 0; t < NT; ++t)
            for (int s = 0; s < KS; ++s)
                for (int l = 0; l < 64; ++l)
                    for (int jj = 0; jj < 8; ++jj) {
                        const int kp = 32 * s + 8 * (l / 16) + jj, c = 16 * t + l % 16;
                        uint16_t h = 0;
                        const int k = sym ? kp % KR : kp / 4, part = sym ? kp / KR : kp % 4;
                        if (kp < KE && c < NC && colmap[c] >= 0 && part < 3) {
                            const float x = (float)R.R[(size_t)k * NN + colmap[c]];
                            const uint16_t hi = bf16_bits_host(x);
                            h = part == 1 ? bf16_bits_host(x - bf16_float_host(hi)) : hi;
                        }
                        const size_t idx = (((size_t)(t * KS + s) * 64 + l) * 8 + jj) * 2;
                        std::memcpy(&buf[idx], &h, 2);
                    }
    }
    return buf;
}

// Packed reference fragments of a key (host bytes, in the layout the engines read).
bool rtable_bytes(int form, int dim, int p, int q, int fd, int prec, std::vector<char>& buf) {
    RefTensor R;
    if (!build_reference(form, dim, p, q, fd, R)) return false;
    // the cell-row engine reads plain 16-entry column tiles: one row group
    const int rpg = uses_elast_engine(form, dim, p, fd, prec) ? R.NS
                                                              : dev::vec_rows_per_group(R.NS, dev::vec_group_tiles(form, prec));
    buf = pack_fragments(R, prec, uses_scalar_engine(form), rpg);
    return true;
}

// Reference fragments for a key, built and uploaded on first use.
static coffee_status get_rtable(int dev, int form, int dim, int p, int q, int fd, int prec, const void** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCtx& c = device_ctx(dev);
    auto key = std::make_tuple(form, dim, p, q, fd, prec);
    auto it = c.rtab.find(key);
    if (it != c.rtab.end()) {
        *out = it->second.ptr;
        return COFFEE_OK;
    }
    std::vector<char> buf;
    if (!rtable_bytes(form, dim, p, q, fd, prec, buf)) return COFFEE_E_INVALID_ARG;
    DevTable t;
    t.bytes = buf.size();
    if (hipMalloc(&t.ptr, t.bytes) != hipSuccess) return COFFEE_E_NOMEM;
    if (hipMemcpy(t.ptr, buf.data(), t.bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(t.ptr);
        return COFFEE_E_HIP;
    }
    c.rtab[key] = t;
    *out = t.ptr;
    return COFFEE_OK;
}

coffee_status get_rtable_public(int dev, int form, int dim, int p, int q, int fd, int prec, const void** out) {
    return get_rtable(dev, form, dim, p, q, fd, prec, out);
}

int blocks_per_cu(int dev, const void* kernel, int threads, int lds_bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCtx& c = device_ctx(dev);
    auto it = c.occupancy.find(kernel);
    if (it != c.occupancy.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds_bytes) != hipSuccess || nb <= 0)
        nb = 1;
    c.occupancy[kernel] = nb;
    return nb;
}

int num_cu(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    return device_ctx(dev).num_cu;
}

// Launch shape override used by the autotuner: grid = cu * blocks_per_cu * mult
// rounded to a multiple of 8 (XCD count); mult <= 0 selects the engine's
// default (1: both engines are persistent, one resident set of workgroups).
static int t_grid_mult = 0;
static int t_variant = -1;  // forced tile-shape variant (-1: tuned or 0)

int batch_grid_mult() { return t_grid_mult; }

int grid_for(int dev, const void* kernel, int threads, int lds_bytes, int64_t nchunks, int default_mult) {
    const int cus = num_cu(dev);
    const int nb = blocks_per_cu(dev, kernel, threads, lds_bytes);
    int64_t g = (int64_t)cus * nb * (t_grid_mult > 0 ? t_grid_mult : default_mult);
    g = std::max<int64_t>(8, (g + 7) / 8 * 8);
    if (g > nchunks) g = nchunks;
    return (int)std::max<int64_t>(1, g);
}

}  // namespace coffee

using namespace coffee;

extern "C" void coffee_set_launch_options(int grid_mult) { t_grid_mult = grid_mult; }

extern "C" void coffee_set_variant(int variant) { t_variant = variant; }

extern "C" const char* coffee_status_string(int s) {
    switch (s) {
        case COFFEE_OK: return "ok";
        case COFFEE_E_INVALID_ARG: return "invalid argument";
        case COFFEE_E_UNSUPPORTED: return "unsupported (outside the compiled set)";
        case COFFEE_E_BUFFER_TOO_SMALL: return "buffer too small";
        case COFFEE_E_DEGENERATE_CELL: return "degenerate cell";
        case COFFEE_E_HIP: return "HIP runtime error";
        case COFFEE_E_NOMEM: return "out of device memory";
        default: return "unknown status";
    }
}

int coffee::cell_nscalar(int cell, int p) { return cell == COFFEE_PRISM ? n_prism(p) : n_scalar(cell, p); }

extern "C" int coffee_tensor_dim(int form, int cell, int degree) {
    if (degree < 1 || degree > kMaxP) return -1;
    if (cell == COFFEE_PRISM)
        return (form == COFFEE_MASS || form == COFFEE_HELMHOLTZ || form == COFFEE_DIFFUSION) ? n_prism(degree) : -1;
    if (cell != COFFEE_TRIANGLE && cell != COFFEE_TETRAHEDRON) return -1;
    const int n = n_scalar(cell, degree);
    switch (form) {
        case COFFEE_MASS: case COFFEE_HELMHOLTZ: case COFFEE_DIFFUSION: return n;
        case COFFEE_ELASTICITY: case COFFEE_BURGERS: case COFFEE_SVK_RESIDUAL: case COFFEE_SVK_JACOBIAN:
            return cell * n;
        case COFFEE_SVK_ENERGY: return 0;
        default: return -1;
    }
}

// Validation shared by the forward and adjoint entry points.
coffee_status coffee::validate_common(int form, int cell, int degree, int quad_degree, const double* coords,
                                      int64_t nvert, const int32_t* c2v, int64_t ncells,
                                      const coffee_field* coeffs, int ncoeff, const double* constants,
                                      int nconst, int* q_out, int* fd_out) {
    if (form < COFFEE_MASS || form > COFFEE_DIFFUSION) return COFFEE_E_INVALID_ARG;
    if (cell != COFFEE_TRIANGLE && cell != COFFEE_TETRAHEDRON && cell != COFFEE_PRISM) return COFFEE_E_INVALID_ARG;
    if (degree < 1 || degree > kMaxP) return COFFEE_E_INVALID_ARG;
    const bool prism = cell == COFFEE_PRISM;
    // quad_degree: q or COFFEE_QUAD(q, rule); negative selects the default
    if (quad_degree >= 0 &&
        (prism ? prism_rule_size(quad_degree) : rule_size(cell == COFFEE_TRIANGLE ? 2 : 3, quad_degree)) <= 0)
        return COFFEE_E_INVALID_ARG;
    if (prism && form != COFFEE_MASS && form != COFFEE_HELMHOLTZ && form != COFFEE_DIFFUSION)
        return COFFEE_E_UNSUPPORTED;
    if (ncells < 0 || nvert < 0 || nvert > INT32_MAX) return COFFEE_E_INVALID_ARG;
    if (ncells > 0 && (!coords || !c2v)) return COFFEE_E_INVALID_ARG;
    if (ncoeff < 0 || ncoeff > 2 || (ncoeff > 0 && !coeffs)) return COFFEE_E_INVALID_ARG;
    if (nconst < 0 || (nconst > 0 && !constants)) return COFFEE_E_INVALID_ARG;
    const int d = prism ? 3 : cell;
    for (int i = 0; i < ncoeff; ++i) {
        if (!coeffs[i].values && ncells > 0) return COFFEE_E_INVALID_ARG;
        if (coeffs[i].degree < 1 || coeffs[i].degree > kMaxP) return COFFEE_E_INVALID_ARG;
    }
    int fd = 0;
    switch (form) {
        case COFFEE_MASS:
        case COFFEE_HELMHOLTZ:
            if (ncoeff > 1) return COFFEE_E_INVALID_ARG;
            if (ncoeff == 1) {
                if (coeffs[0].ncomp != 1) return COFFEE_E_INVALID_ARG;
                fd = coeffs[0].degree;
                if (prism && fd != 1) return COFFEE_E_UNSUPPORTED;
            }
            break;
        case COFFEE_DIFFUSION:
            if (ncoeff != 0) return COFFEE_E_INVALID_ARG;
            break;
        case COFFEE_ELASTICITY:
            if (ncoeff == 0) {
                if (nconst < 2) return COFFEE_E_INVALID_ARG;
            } else {
                if (ncoeff != 2 || coeffs[0].ncomp != 1 || coeffs[1].ncomp != 1) return COFFEE_E_INVALID_ARG;
                if (coeffs[0].degree != coeffs[1].degree) return COFFEE_E_UNSUPPORTED;
                fd = coeffs[0].degree;
            }
            break;
        default:  // Burgers and SVK: one vector field
            if (ncoeff != 1 || coeffs[0].ncomp != d) return COFFEE_E_INVALID_ARG;
            fd = coeffs[0].degree;
    }
    int q = quad_degree >= 0 ? quad_degree : (form == COFFEE_BURGERS ? 2 * degree + 1 : 2 * degree);
    if ((prism ? prism_rule_size(q) : rule_size(d, q)) <= 0) return COFFEE_E_UNSUPPORTED;
    *q_out = q;
    *fd_out = fd;
    return COFFEE_OK;
}

extern "C" coffee_status coffee_assemble(int form, int cell, int degree, int quad_degree, int precision,
                                         const double* coords, int64_t nvert, const int32_t* c2v,
                                         int64_t ncells, const coffee_field* coeffs, int ncoeff,
                                         const double* constants, int nconst, void* out, void* hip_stream) {
    int q = 0, fd = 0;
    coffee_status st = validate_common(form, cell, degree, quad_degree, coords, nvert, c2v, ncells, coeffs,
                                       ncoeff, constants, nconst, &q, &fd);
    if (st != COFFEE_OK) return st;
    if (precision < COFFEE_FP64 || precision > COFFEE_BF16X3) return COFFEE_E_INVALID_ARG;
    if (ncells > 0 && !out) return COFFEE_E_INVALID_ARG;
    if (((uintptr_t)out & 15) != 0) return COFFEE_E_INVALID_ARG;
    if (cell == COFFEE_PRISM)
        return assemble_prism(form, degree, q, precision, coords, c2v, ncells, coeffs, ncoeff, constants, nconst, out,
                              hip_stream);
    if (is_svk_form(form))
        return assemble_svk(form, cell, degree, q, precision, coords, nvert, c2v, ncells, coeffs, constants,
                            nconst, out, hip_stream);
    // degree 1 mass / Helmholtz / diffusion: thread-per-cell FMA kernel (p1.hip)
    if ((form == COFFEE_MASS || form == COFFEE_HELMHOLTZ || form == COFFEE_DIFFUSION) && degree == 1 && fd <= 1 &&
        precision != COFFEE_BF16X3)
        return assemble_p1(form, cell, fd, q, precision, coords, c2v, ncells, coeffs, ncoeff, constants, nconst, out,
                           hip_stream);
    int tuned_variant = 0;
    const int tuned = tuned_linear(form, cell, degree, fd, precision, &tuned_variant);
    const LinEntry* e = find_linear(form, cell, degree, fd, precision, t_variant >= 0 ? t_variant : tuned_variant);
    if (!e) return COFFEE_E_UNSUPPORTED;
    if (ncells == 0) return COFFEE_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return COFFEE_E_HIP;
    const void* rf = nullptr;
    st = get_rtable(dev, form, cell, degree, q, fd, precision, &rf);
    if (st != COFFEE_OK) return st;
    dev::LinArgs a;
    std::memset(&a, 0, sizeof a);
    a.coords = coords;
    a.c2v = c2v;
    a.ncells = ncells;
    if (ncoeff >= 1) a.f0 = dev::FieldArg{coeffs[0].values, coeffs[0].cell_to_dof};
    if (ncoeff >= 2) a.f1 = dev::FieldArg{coeffs[1].values, coeffs[1].cell_to_dof};
    if (form == COFFEE_BURGERS) {
        a.c0 = nconst > 0 ? constants[0] : 1.0;
        a.c1 = nconst > 1 ? constants[1] : 1.0;
    } else if (form == COFFEE_ELASTICITY && ncoeff == 0) {
        a.c0 = constants[0];
        a.c1 = constants[1];
    } else if (form == COFFEE_DIFFUSION) {
        a.c0 = (nconst > 0 ? constants[0] : 1.0) * (nconst > 1 ? constants[1] : 1.0);  // kappa dt
    }
    a.rfrag = rf;
    a.out = out;
    a.nchunks = (ncells + e->cells_per_chunk - 1) / e->cells_per_chunk;
    const int grid = grid_for(dev, e->kernel, e->threads, e->lds_bytes, a.nchunks, tuned > 0 ? tuned : 1);
    if (e->launch(a, (hipStream_t)hip_stream, grid) != hipSuccess) return COFFEE_E_HIP;
    return COFFEE_OK;
}

// ---------------------------------------------------------------- geometry check

template <int D>
__global__ void k_check_geometry(const double* coords, const int32_t* c2v, int64_t ncells, int64_t nvert,
                                 unsigned long long* first_bad) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ncells;
         e += (int64_t)gridDim.x * blockDim.x) {
        double x[D + 1][D];
        bool bad = false;
        for (int v = 0; v <= D; ++v) {
            const int64_t g = c2v[e * (D + 1) + v];
            if (g < 0 || g >= nvert) { bad = true; break; }
            for (int i = 0; i < D; ++i) {
                x[v][i] = coords[g * D + i];
                if (!isfinite(x[v][i])) bad = true;
            }
        }
        if (!bad) {
            double J[D][D];
            for (int i = 0; i < D; ++i)
                for (int j = 0; j < D; ++j) J[i][j] = x[j + 1][i] - x[0][i];
            double det;
            if constexpr (D == 2) det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            else
                det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                      J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            bad = !(det > 0.0) || !isfinite(det);
        }
        if (bad) atomicMin(first_bad, (unsigned long long)e);
    }
}

// Prisms: the map is not affine, so det J is checked at nine points: the six
// reference vertices and the mid-heights of the three vertical edges (det J
// is linear in (X, Y) on each horizontal slice and quadratic in Z).
__global__ void k_check_geometry_prism(const double* coords, const int32_t* c2v, int64_t ncells, int64_t nvert,
                                       unsigned long long* first_bad) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ncells;
         e += (int64_t)gridDim.x * blockDim.x) {
        double x[6][3];
        bool bad = false;
        for (int v = 0; v < 6; ++v) {
            const int64_t g = c2v[e * 6 + v];
            if (g < 0 || g >= nvert) { bad = true; break; }
            for (int i = 0; i < 3; ++i) {
                x[v][i] = coords[g * 3 + i];
                if (!isfinite(x[v][i])) bad = true;
            }
        }
        for (int pt = 0; pt < 9 && !bad; ++pt) {
            const int t = pt % 3;
            const double X = t == 1 ? 1.0 : 0.0, Y = t == 2 ? 1.0 : 0.0, Z = 0.5 * (pt / 3);
            const double zb = 1.0 - Z, l0 = 1.0 - X - Y;
            double J[3][3];
            for (int i = 0; i < 3; ++i) {
                J[i][0] = zb * (x[2][i] - x[0][i]) + Z * (x[3][i] - x[1][i]);
                J[i][1] = zb * (x[4][i] - x[0][i]) + Z * (x[5][i] - x[1][i]);
                J[i][2] = l0 * (x[1][i] - x[0][i]) + X * (x[3][i] - x[2][i]) + Y * (x[5][i] - x[4][i]);
            }
            const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            bad = !(det > 0.0) || !isfinite(det);
        }
        if (bad) atomicMin(first_bad, (unsigned long long)e);
    }
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

extern "C" coffee_status coffee_check_geometry(int cell, const double* coords, int64_t nvert,
                                               const int32_t* c2v, int64_t ncells, int64_t* first_bad,
                                               void* hip_stream) {
    if (cell != COFFEE_TRIANGLE && cell != COFFEE_TETRAHEDRON && cell != COFFEE_PRISM) return COFFEE_E_INVALID_ARG;
    if (!first_bad || ncells < 0 || nvert < 0 || (ncells > 0 && (!coords || !c2v))) return COFFEE_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    // the sentinel ~0 read as int64 is -1 ("no bad cell")
    unsigned long long* fb = reinterpret_cast<unsigned long long*>(first_bad);
    hipLaunchKernelGGL((k_fill<unsigned long long>), dim3(1), dim3(64), 0, s, fb, ~0ull, (int64_t)1);
    if (ncells > 0) {
        const int grid = (int)std::min<int64_t>((ncells + 255) / 256, 4096);
        if (cell == COFFEE_PRISM)
            hipLaunchKernelGGL(k_check_geometry_prism, dim3(grid), dim3(256), 0, s, coords, c2v, ncells, nvert, fb);
        else if (cell == 2)
            hipLaunchKernelGGL((k_check_geometry<2>), dim3(grid), dim3(256), 0, s, coords, c2v, ncells, nvert, fb);
        else
            hipLaunchKernelGGL((k_check_geometry<3>), dim3(grid), dim3(256), 0, s, coords, c2v, ncells, nvert, fb);
    }
    return hipGetLastError() == hipSuccess ? COFFEE_OK : COFFEE_E_HIP;
}

extern "C" void coffee_shutdown(void) {
    free_adjoint_tables();
    free_svk_tables();
    free_svkb_tables();
    free_prism_tables();
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_ctx) {
        (void)hipSetDevice(kv.first);
        for (auto& t : kv.second.rtab) (void)hipFree(t.second.ptr);
        kv.second.rtab.clear();
        kv.second.occupancy.clear();
    }
    g_ctx.clear();
    (void)hipSetDevice(cur);
}
