// Internal declarations shared by the host parts of libcoffee.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/coffee.h"

namespace coffee {

coffee_status validate_common(int form, int cell, int degree, int quad_degree, const double* coords,
                              int64_t nvert, const int32_t* c2v, int64_t ncells, const coffee_field* coeffs,
                              int ncoeff, const double* constants, int nconst, int* q_out, int* fd_out);

coffee_status assemble_svk(int form, int cell, int degree, int q, int precision, const double* coords,
                           int64_t nvert, const int32_t* c2v, int64_t ncells, const coffee_field* coeffs,
                           const double* constants, int nconst, void* out, void* hip_stream);

int grid_for(int dev, const void* kernel, int threads, int lds_bytes, int64_t nchunks, int default_mult);

struct DetTarget;
coffee_status adjoint_linear(int form, int cell, int degree, int q, int fd, const double* coords, int64_t nvert,
                             const int32_t* c2v, int64_t ncells, const coffee_field* coeffs, int ncoeff,
                             const double* constants, int nconst, const double* lam, const double* u,
                             double seed, double* grad_coords, double* const* grad_coeff_values,
                             double* cell_value, const DetTarget* det, void* hip_stream);
void free_adjoint_tables();
coffee_status reference_table_f64(int dev, int form, int dim, int p, int q, int fd, const double** out);
coffee_status assemble_p1(int form, int cell, int fd, int q, int precision, const double* coords, const int32_t* c2v,
                          int64_t ncells, const coffee_field* coeffs, int ncoeff, const double* constants, int nconst,
                          void* out, void* hip_stream);
coffee_status get_rtable_public(int dev, int form, int dim, int p, int q, int fd, int prec, const void** out);
// Host bytes of the packed reference fragments and of the FP64 reference tensors.
bool rtable_bytes(int form, int dim, int p, int q, int fd, int prec, std::vector<char>& buf);
bool r64_table(int form, int dim, int p, int q, int fd, std::vector<double>& h);
int batch_grid_mult();
int tuned_linear(int form, int cell, int degree, int fd, int prec, int* variant);
bool tuned_batch(int form, int cell, int degree, int prec, int* variant, int* task_cells);
bool tuned_packed(int form, int cell, int degree, int prec, int* task_cells);
void free_svk_tables();
coffee_status assemble_svk_bf16(int form, int cell, int degree, int q, const double* coords, const int32_t* c2v,
                                int64_t ncells, const coffee_field* coeffs, const double* constants, int nconst,
                                void* out, void* hip_stream);
void free_svkb_tables();
int num_cu(int dev);

struct RefTensor;
// Reference tensors packed in MFMA B-fragment order (library.hip).
std::vector<char> pack_fragments(const RefTensor& R, int prec, bool sym, int rows_per_group);

// Prism cells (prism.hip).
coffee_status assemble_prism(int form, int degree, int quad, int precision, const double* coords,
                             const int32_t* c2v, int64_t ncells, const coffee_field* coeffs, int ncoeff,
                             const double* constants, int nconst, void* out, void* hip_stream);
void free_prism_tables();

inline bool is_svk_form(int form) {
    return form == COFFEE_SVK_ENERGY || form == COFFEE_SVK_RESIDUAL || form == COFFEE_SVK_JACOBIAN;
}
// Vertices per cell and scalar Lagrange dofs of degree p for a cell code.
inline int cell_nverts(int cell) { return cell == COFFEE_PRISM ? 6 : cell + 1; }
int cell_nscalar(int cell, int p);

// Deterministic scatter of per-cell gradients (scatter.hip). One target array:
// `n` local entries of `ncomp` values (entry j = cell * slots + slot), added to
// grad[keys[j]] (or grad[j] if keys is NULL) in increasing j per target.
struct DetTarget {
    const int32_t* keys;  // [n] target index of each entry (used when mapped)
    int mapped;           // 0: entry j goes to target j (no sort)
    int64_t n;
    int ncomp;            // 1..3
    int64_t ntargets;
    double* local;        // [n][ncomp], placed in the workspace by det_carve
    double* grad;         // [ntargets][ncomp] accumulated; NULL skips the target
};
int64_t det_workspace_bytes(const DetTarget* t, int nt);  // -1 if the sort size query fails
coffee_status det_carve(void* ws, int64_t ws_bytes, DetTarget* t, int nt);
coffee_status det_scatter(const DetTarget* t, int nt, void* ws, hipStream_t s);
int blocks_per_cu(int dev, const void* kernel, int threads, int lds_bytes);

}  // namespace coffee
