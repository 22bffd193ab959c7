/*
 * coffee.h - C ABI of libcoffee, finite element local assembly on MI355X.
 *
 * Local assembly (paper, section 2 and Fig. 1) evaluates, for every cell of
 * a mesh, the element tensor of a variational form by mapping the cell to a
 * reference simplex, evaluating basis functions and coefficient fields at
 * quadrature points and summing integrand * |det J| * weight. The paper's
 * per-cell kernels (Fig. 1; Listings 1 and 2; Table 1 for the objects) take
 * a zeroed element matrix, the element's coordinates and its coefficient
 * fields. These entry points apply that contract to whole meshes on one GPU.
 *
 * Conventions shared by every entry point:
 *  - Reference cells: triangle (0,0),(1,0),(0,1); tetrahedron 0,e1,e2,e3;
 *    prism T x [0,1] with T the reference triangle (the paper's third cell
 *    shape, section 5.2).
 *  - Geometry: J has columns x_i - x_0, K = J^{-1} (row-major, so that
 *    d phi/d x_i = sum_a K[a][i] d phi/d X_a, as in Listing 1), integrals use
 *    |det J|. Geometry is always computed in FP64.
 *  - Quadrature of degree q: collapsed Gauss-Jacobi product rule with
 *    m = ceil((q+1)/2) points per direction (m^2 on triangles, m^3 on
 *    tetrahedra), first direction outermost. quad_degree < 0 selects 2p
 *    (Burgers: 2p+1).
 *  - Lagrange P_p dof order: vertices; edges (triangle (1,2),(0,2),(0,1);
 *    tetrahedron (2,3),(1,3),(1,2),(0,3),(0,2),(0,1)), points from the lower
 *    to the higher vertex; faces (face f opposite vertex f, lattice points
 *    (i,j) with j outermost); interior.
 *  - Vector spaces are component-blocked: local dof (c, a) has index
 *    c * n_scalar + a. Element matrices are row-major [row = test][col =
 *    trial], stored cell-major: out[e][i][j].
 *  - All device pointers are caller-owned; the library allocates nothing per
 *    call (it keeps one lazily built table cache per device, freed by
 *    coffee_shutdown). Calls are asynchronous on `hip_stream` (a hipStream_t,
 *    NULL for the default stream). Host-side validation happens before any
 *    HIP call and returns a status; faults inside a kernel surface at the
 *    caller's next synchronisation.
 *  - Degenerate cells (det J = 0, non-finite input) are not checked on the
 *    hot path: they yield non-finite output. coffee_check_geometry is the
 *    explicit check.
 */
#ifndef COFFEE_H
#define COFFEE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    COFFEE_OK = 0,
    COFFEE_E_INVALID_ARG = 1,      /* null pointer, bad enum, inconsistent sizes */
    COFFEE_E_UNSUPPORTED = 2,      /* valid request outside the compiled set */
    COFFEE_E_BUFFER_TOO_SMALL = 3,
    COFFEE_E_DEGENERATE_CELL = 4,  /* reported by coffee_check_geometry */
    COFFEE_E_HIP = 5,              /* a HIP runtime call or kernel launch failed */
    COFFEE_E_NOMEM = 6
} coffee_status;

/* Simplices are numbered by their dimension, the prism by its vertex count.
 * Prisms (section 5.2 of the paper): cell_to_vertex rows hold six vertices,
 * each vertex of the base triangle at the bottom, then at the top:
 * (t0,0), (t0,1), (t1,0), (t1,1), (t2,0), (t2,1). The cell map is spanned by
 * the six degree-1 prism basis functions, so J, det J and K = J^-1 depend on
 * the point (a prism need not be an affine image of the reference prism).
 * The degree-p prism element is the tensor product of the degree-p triangle
 * (dof order below) and the degree-p interval with nodes 0, 1, then the
 * interior ones ascending; local dof (a, b) has index a (p + 1) + b. The rule
 * of degree q is the triangle rule of degree q times Gauss-Legendre with
 * m = ceil((q+1)/2) points on [0,1], triangle point outermost. */
typedef enum { COFFEE_TRIANGLE = 2, COFFEE_TETRAHEDRON = 3, COFFEE_PRISM = 6 } coffee_cell;

typedef enum {
    COFFEE_MASS = 0,         /* int f u v                          fields: [f] or none (f = 1)     */
    COFFEE_HELMHOLTZ = 1,    /* int grad u . grad v + f u v        fields: [f] or none             */
    COFFEE_ELASTICITY = 2,   /* int 2 mu eps(u):eps(v) + lambda div u div v (vector)
                                fields: [mu, lambda] (same degree) or none with constants (mu, lambda) */
    COFFEE_BURGERS = 3,      /* Jacobian of backward-Euler viscous Burgers at state w (vector):
                                int (1/dt) du.v + ((w.grad)du).v + ((du.grad)w).v + nu grad du:grad v
                                fields: [w] (ncomp = d); constants (nu, 1/dt), default (1, 1)   */
    COFFEE_SVK_ENERGY = 4,   /* St Venant-Kirchhoff: int psi(F), F = I + grad u (one value per cell) */
    COFFEE_SVK_RESIDUAL = 5, /* int P(F) : grad v, P = F S (vector of N per cell)                  */
    COFFEE_SVK_JACOBIAN = 6, /* int dP[du] : grad v (N x N per cell)
                                SVK fields: [u] (ncomp = d); constants (mu, lambda), default (1, 1) */
    COFFEE_DIFFUSION = 7     /* int kappa dt grad u . grad v: the paper's diffusion kernel, the
                                Helmholtz operator without its basis-value (mass) term and with
                                extra constants (section 5.2). No fields; constants (kappa, dt),
                                default (1, 1)                                                  */
} coffee_form;

typedef enum {
    COFFEE_FP64 = 0,   /* FP64 everywhere, FP64 output                                          */
    COFFEE_FP32 = 1,   /* FP64 geometry (J, det J, K); FP32 contraction, FP32 output. The SVK
                          energy and residual compute their point arithmetic (F, E, S, P) in
                          FP32 from the FP64 geometry; the SVK Jacobian forms F, S and the
                          tangent in FP64 and accumulates the element matrix in FP32.           */
    COFFEE_BF16X3 = 2  /* FP64 geometry; each contraction operand x split as x_hi = bf16(x),
                          x_lo = bf16(x - x_hi); hi*hi + hi*lo + lo*hi on bf16 MFMA with FP32
                          accumulation; FP32 output                                             */
} coffee_precision;

/* Quadrature rule families. A quad_degree argument is q (collapsed
 * Gauss-Jacobi rule of degree q, 0 <= q <= 10) or COFFEE_QUAD(q, rule).
 * COFFEE_RULE_SYMMETRIC selects the fully symmetric rule of degree q,
 * 0 <= q <= 6, of the kind the paper's kernels use (a 3-point rule in
 * Listing 1, a 5-point rule in Listing 2): points in orbits of the simplex's
 * symmetry group, one weight per orbit, found from the moment equations.
 * Points per rule for q = 1..6: triangle 1, 3, 6, 6, 7, 12; tetrahedron 1, 4,
 * 5, 14, 14, 24 (the tetrahedral 5-point rule has a negative weight). */
typedef enum { COFFEE_RULE_GAUSS_JACOBI = 0, COFFEE_RULE_SYMMETRIC = 1 } coffee_rule;
#define COFFEE_QUAD(q, rule) ((q) + 16 * (rule))

/* A coefficient field on the cells (device pointers).
 * cell_to_dof != NULL: values is global [ndofs][ncomp], cell_to_dof is
 *   [ncells][nloc] int32 with nloc the Lagrange dof count of `degree`.
 * cell_to_dof == NULL: values is cell-major [ncells][nloc][ncomp].
 * degree 1..4 (P_p Lagrange). */
typedef struct {
    const double* values;
    const int32_t* cell_to_dof;
    int32_t degree;
    int32_t ncomp;
} coffee_field;

/* Reference quadrature and Lagrange basis tables (host, FP64; paper section 2:
 * the constant weight and basis tables W, X, Y that the kernels of Listings 1
 * and 2 declare, and Table 1). Buffers are caller-owned host memory; pass NULL
 * for all four to query *nq and *ndof. Layouts: points [nq][d], weights [nq],
 * basis [nq][ndof], dbasis [d][nq][ndof] (reference derivatives); d = 3 on
 * prisms. quad_degree: q or COFFEE_QUAD(q, rule) (on prisms the rule family
 * applies to the triangle factor).
 * Errors: COFFEE_E_INVALID_ARG (bad cell, degree outside 0..4, a quad_degree
 * naming no rule, null nq/ndof). */
coffee_status coffee_tabulate(int cell, int degree, int quad_degree, int* nq, int* ndof,
                              double* points, double* weights, double* basis, double* dbasis);

/* Rows N of the element tensor of (form, cell, degree): n_scalar for scalar
 * forms, d * n_scalar for vector forms, 0 for the energy, -1 if invalid. */
int coffee_tensor_dim(int form, int cell, int degree);

/* Element tensors of all cells (paper section 2: the per-cell kernel of Fig. 1
 * is run once for every cell of the mesh; here one call covers the mesh). Inputs (device): coords [nvert][d] FP64, cell_to_vertex [ncells][d+1]
 * int32, coefficient fields as described above, constants (host) per form.
 * Output (device, overwritten; equals "zero-initialise then +=" of Fig. 1):
 * [ncells][N][N] for bilinear forms, [ncells][N] for the residual, [ncells]
 * for the energy; FP64 if precision == COFFEE_FP64, else FP32. `out` must be
 * 16-byte aligned. cell_to_vertex and cell_to_dof entries must be valid
 * indices (coffee_check_geometry validates the vertex indices).
 * Prisms: cell_to_vertex is [ncells][6] (vertex order above) and coords
 * [nvert][3]; COFFEE_MASS and COFFEE_HELMHOLTZ (no field, or one degree-1
 * prism field: 6 dofs per cell through cell_to_dof or cell-major) and
 * COFFEE_DIFFUSION, at degree 1 (6 x 6), 2 (18 x 18) and 3 (40 x 40), with the
 * default rule (q = 2p: 8, 27 and 64 points), in every precision.
 * Errors: COFFEE_E_INVALID_ARG (null pointers, bad enums, negative sizes,
 * misaligned out,
 * field shape/count not matching the form), COFFEE_E_UNSUPPORTED (degree or
 * field degree outside the compiled set, precision not available for the
 * form, a form or rule not compiled for prisms), COFFEE_E_HIP (launch
 * failure), COFFEE_E_NOMEM (table upload). */
coffee_status coffee_assemble(int form, int cell, int degree, int quad_degree, int precision,
                              const double* coords, int64_t nvert, const int32_t* cell_to_vertex,
                              int64_t ncells, const coffee_field* coeffs, int ncoeff,
                              const double* constants, int nconst, void* out, void* hip_stream);

/* Reverse mode of the assembly (FP64), the derivative of the per-cell kernel
 * of section 2 (Fig. 1) with respect to its inputs; the paper itself has no
 * reverse pass (it serves PDE-constrained optimisation and shape derivatives).
 * S = sum_e lam_e^T A_e u_e for the bilinear forms (mass, Helmholtz,
 * elasticity, Burgers), sum_e lam_e^T b_e for COFFEE_SVK_RESIDUAL, sum_e Pi_e
 * for COFFEE_SVK_ENERGY. Accumulates (+=) seed * dS/dcoords into grad_coords
 * [nvert][d] and seed * dS/dvalues into grad_coeff_values[i] (shaped like
 * coeffs[i].values). A NULL grad_coords, a NULL grad_coeff_values array or a
 * NULL entry skips that gradient (all NULL: only the values). lam, u: device
 * [ncells][N] FP64, component-blocked like the element tensors (bilinear
 * forms need both; the residual needs lam; the energy neither). If
 * cell_value is not NULL it receives S_e per cell [ncells] FP64 (unscaled).
 * deterministic = 0: the per-cell gradients are combined per wave in LDS and
 *   scatter-added with FP64 atomics (sums are order-dependent in the last
 *   bits); workspace may be NULL.
 * deterministic = 1: the per-cell gradients are written to `workspace`, then
 *   each vertex's and dof's contributions are summed in increasing cell order
 *   (a stable sort of the cell-to-vertex / cell-to-dof entries by target):
 *   the result is bitwise reproducible. workspace: device buffer, 256-byte
 *   aligned, of at least coffee_adjoint_workspace_size(...) bytes.
 * COFFEE_SVK_JACOBIAN and prism cells have no reverse pass
 * (COFFEE_E_UNSUPPORTED); COFFEE_DIFFUSION has one at degree 1 and 2 on
 * triangles and tetrahedra (constants kappa, dt).
 * Errors as coffee_assemble, plus COFFEE_E_BUFFER_TOO_SMALL (workspace),
 * COFFEE_E_INVALID_ARG (deterministic not 0/1; NULL workspace with
 * deterministic = 1; NULL lam or u where the form needs them). */
coffee_status coffee_assemble_adjoint(int form, int cell, int degree, int quad_degree,
                                      const double* coords, int64_t nvert, const int32_t* cell_to_vertex,
                                      int64_t ncells, const coffee_field* coeffs, int ncoeff,
                                      const double* constants, int nconst,
                                      const double* lam, const double* u, double seed,
                                      double* grad_coords, double* const* grad_coeff_values,
                                      double* cell_value, int deterministic,
                                      void* workspace, int64_t workspace_bytes, void* hip_stream);

/* Workspace bytes of coffee_assemble_adjoint with deterministic = 1 for these
 * sizes and fields (coeffs are read for their degree, component count and
 * whether they have a dof map): per-cell gradients of the coordinates and of
 * every field, plus the sort buffers. -1 for invalid arguments, or if the
 * sort's size query fails (it needs a HIP device). */
int64_t coffee_adjoint_workspace_size(int form, int cell, int degree, int64_t nvert, int64_t ncells,
                                      const coffee_field* coeffs, int ncoeff);

/* One bin of a mixed batch: a form (mass or Helmholtz) on the cells of one mesh
 * with one degree. coords / cell_to_vertex describe the mesh the bin's cells
 * index into; coeff is NULL or one P1 coefficient field on that mesh (device
 * pointers). variant and task_cells are launch choices made by the autotuner:
 * variant 0 stages 8 element tensors through LDS before storing them, 1
 * stores them straight from the matrix-core registers; task_cells (a
 * multiple of 64, at most 1024) is how many of the bin's cells one wave takes
 * from the queue at a time. task_cells = 0 selects the autotuned pair for
 * this (form, shape, degree, precision) from the loaded tuning cache, else
 * (variant, 256). The bin's mesh must have at most 2^31 - 1 cells. */
typedef struct {
    int32_t form, cell, degree, quad_degree;
    const double* coords;
    int64_t nvert;
    const int32_t* cell_to_vertex;
    int64_t ncells_mesh;
    const coffee_field* coeff;
    int32_t variant, task_cells;
} coffee_segment;

/* Mixed persistent batch (the paper's vectorization across cells, section 4,
 * extended to cells of different shape, degree and form in one launch).
 * Entry i of the batch is cell cell_of[i] of segment seg_of[i]; its element
 * tensor is written at out + out_offset[i] (elements, FP64 or FP32 by
 * precision; FP32 and FP64 supported). An entry whose seg_of is outside
 * [0, nseg) or whose cell_of is outside its segment's mesh is skipped:
 * nothing is read or written for it. The entries are binned on the device
 * (histograms, prefix sums, stable scatter of each entry's cell index and
 * output offset into per-bin ranges of the workspace), then one persistent kernel drains a
 * queue of bin tasks in segment order (put the costliest bins first). Output
 * regions of different entries must not overlap; cell_of[i] must index a cell
 * of segment seg_of[i]'s mesh. Up to 16 segments. All arrays are device memory;
 * workspace must hold coffee_batch_workspace_size(nseg, nentries) bytes.
 * Errors: COFFEE_E_INVALID_ARG (null pointers, nseg outside 1..16, bad
 * segment), COFFEE_E_UNSUPPORTED (form/degree outside mass or Helmholtz on
 * P1-P4 triangles or P1-P3 tetrahedra with a P1 coefficient),
 * COFFEE_E_BUFFER_TOO_SMALL (workspace), COFFEE_E_HIP. */
coffee_status coffee_assemble_batch(int precision, const coffee_segment* segs, int nseg, const int32_t* seg_of,
                                    const int64_t* cell_of, const int64_t* out_offset, int64_t nentries,
                                    void* out, void* workspace, int64_t workspace_bytes, void* hip_stream);

/* The same mixed batch with the output layout chosen by the library: the
 * element tensors of segment 0 first, then segment 1, ..., each segment's
 * tensors contiguous and in increasing entry order, so that every tensor is
 * written as whole contiguous stores. out_offset (device, [nentries], int64)
 * is an output: out_offset[i] receives the element offset of entry i's tensor
 * (-1 for a skipped entry, see coffee_assemble_batch; skipped entries take no
 * space).
 * out must hold sum_i n_seg_of[i]^2 elements (16-byte aligned); the binning is
 * deterministic (the layout depends only on seg_of). Workspace, precision,
 * segments and errors as coffee_assemble_batch; the segments' variant is
 * ignored (every bin uses contiguous staged stores). */
coffee_status coffee_assemble_batch_packed(int precision, const coffee_segment* segs, int nseg,
                                           const int32_t* seg_of, const int64_t* cell_of, int64_t nentries,
                                           void* out, int64_t* out_offset, void* workspace,
                                           int64_t workspace_bytes, void* hip_stream);

/* Workspace bytes of coffee_assemble_batch and coffee_assemble_batch_packed. */
int64_t coffee_batch_workspace_size(int nseg, int64_t nentries);

/* Largest batch of coffee_assemble_batch_packed_noalloc. */
#define COFFEE_NOALLOC_MAX_ENTRIES 4194304

/* coffee_assemble_batch_packed for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, bit for bit, with no
 * workspace argument. Its scratch memory (binning counters, per-bin entry
 * lists, the task queue: 48.3 MiB) is a static device array of the library,
 * and its reference tables live in a second static device array of 1 MiB;
 * each GPU the library runs on holds its own copy of both until the process
 * ends. The call allocates nothing: the first call on a device looks up the
 * arrays' addresses, and the first call that uses a bin type copies that
 * type's tables into the table array with a synchronous hipMemcpy (make such
 * a call once before capturing a graph). Every call on one GPU shares its
 * scratch array, and the binning kernels rewrite all of it that a call reads
 * (no clearing needed), so calls that overlap in time on one GPU (different
 * streams, or host threads) race and must be serialised by the caller.
 * Errors: as coffee_assemble_batch_packed, plus COFFEE_E_BUFFER_TOO_SMALL for
 * nentries > COFFEE_NOALLOC_MAX_ENTRIES and COFFEE_E_NOMEM if the table array
 * is full (it holds every bin type's tables in both precisions). */
coffee_status coffee_assemble_batch_packed_noalloc(int precision, const coffee_segment* segs, int nseg,
                                                   const int32_t* seg_of, const int64_t* cell_of,
                                                   int64_t nentries, void* out, int64_t* out_offset,
                                                   void* hip_stream);

/* Global assembly (paper, section 2: the element tensors are the per-cell
 * contributions summed into the matrix of the linear system; local assembly
 * is the step before it).
 *
 * coffee_csr_pattern: the CSR sparsity pattern of that matrix for a space
 * whose cells map to dofs through cell_to_dof (device int32 [ncells][nloc],
 * values in [0, ndofs)); a vector space of ncomp components (1..3) numbers
 * its global dofs dof * ncomp + c and every scalar nonzero becomes an
 * ncomp x ncomp block. Every pair of dofs sharing a cell is a nonzero; rows
 * hold their columns in increasing order. row_ptr: device int64
 * [ndofs * ncomp + 1]; col_idx: device int32 of col_capacity entries. The
 * call synchronises on hip_stream to learn the count: *nnz (host) always
 * receives it, and if col_idx is NULL or col_capacity < *nnz the call
 * returns COFFEE_E_BUFFER_TOO_SMALL without writing col_idx (call again with
 * a large enough buffer). workspace: device, 256-byte aligned, at least
 * coffee_csr_pattern_workspace_size bytes (the 64-bit keys of every
 * (cell, i, j) pair, sorted). Deterministic.
 * Errors: COFFEE_E_INVALID_ARG, COFFEE_E_UNSUPPORTED (ndofs * ncomp beyond
 * int32), COFFEE_E_BUFFER_TOO_SMALL, COFFEE_E_HIP. */
int64_t coffee_csr_pattern_workspace_size(int64_t ncells, int nloc, int64_t ndofs);
coffee_status coffee_csr_pattern(const int32_t* cell_to_dof, int64_t ncells, int nloc, int64_t ndofs, int ncomp,
                                 int64_t* row_ptr, int32_t* col_idx, int64_t col_capacity, int64_t* nnz,
                                 void* workspace, int64_t workspace_bytes, void* hip_stream);

/* coffee_assemble_csr: the global matrix sum_e P_e^T A_e P_e of a bilinear
 * form (mass, Helmholtz, elasticity, Burgers, SVK Jacobian) in the CSR
 * pattern built by coffee_csr_pattern for the form's space (cell_to_dof: the
 * space's dof map, the one the pattern was built from; NULL at degree 1 means
 * cell_to_vertex). The other arguments are coffee_assemble's. values (device,
 * nnz entries, FP64 if precision is COFFEE_FP64, else FP32) is overwritten.
 * The cells are assembled in chunks of 131,072 into `workspace` (16-byte
 * aligned, coffee_assemble_csr_workspace_size bytes) and added to the matrix
 * with atomic adds: sums of shared entries are order-dependent in the last
 * bits. Errors: as coffee_assemble, plus COFFEE_E_BUFFER_TOO_SMALL. */
int64_t coffee_assemble_csr_workspace_size(int form, int cell, int degree, int precision, int64_t ncells);
coffee_status coffee_assemble_csr(int form, int cell, int degree, int quad_degree, int precision,
                                  const double* coords, int64_t nvert, const int32_t* cell_to_vertex,
                                  int64_t ncells, const coffee_field* coeffs, int ncoeff,
                                  const double* constants, int nconst, const int32_t* cell_to_dof, int64_t ndofs,
                                  const int64_t* row_ptr, const int32_t* col_idx, int64_t nnz, void* values,
                                  void* workspace, int64_t workspace_bytes, void* hip_stream);

/* Checks every cell for the geometry step of the per-cell kernel (section 2,
 * Fig. 1: the Jacobian of the affine map and its determinant, which the
 * kernels invert and use as |det J| without checking): writes to *first_bad
 * (device int64) the smallest cell index with a vertex index outside
 * [0, nvert), a non-finite coordinate or det J <= 0, or -1 if none. On
 * prisms (non-affine) det J is tested at the six reference vertices and at
 * the mid-heights of the three vertical edges.
 * Errors: COFFEE_E_INVALID_ARG. */
coffee_status coffee_check_geometry(int cell, const double* coords, int64_t nvert,
                                    const int32_t* cell_to_vertex, int64_t ncells,
                                    int64_t* first_bad, void* hip_stream);

/* Human-readable name of a status code (static string). */
const char* coffee_status_string(int status);

/* Launch-shape option for subsequent calls in this process (used by the
 * autotuner and the benchmark): grid_mult scales the grid (workgroups = CUs x
 * resident workgroups per CU x grid_mult, capped at one workgroup per 256
 * cells); 0 restores the defaults: 1 for mass and Helmholtz, whose kernel is
 * persistent, one workgroup per 256 cells for the other forms. Not
 * thread-safe with concurrent assembly calls. */
void coffee_set_launch_options(int grid_mult);

/* Tile-shape variant of the symmetric engine (mass, Helmholtz) used by
 * subsequent coffee_assemble calls in this process, for the autotuner: 0
 * keeps the reference fragments in registers, 1 stages them in LDS with the
 * register budget of two waves per SIMD, 2 reads them through the caches with
 * that budget; -1 (the default) takes the tuning cache's choice, else 0. A
 * key compiled without the requested variant runs variant 0
 * (coffee_has_variant tells which keys have them). Not thread-safe with
 * concurrent assembly calls. */
void coffee_set_variant(int variant);
int coffee_has_variant(int form, int cell, int degree, int field_degree, int precision, int variant);

/* Loads a tuning cache written by the autotuner (paper_1407_0904_amd/tuner.py):
 * per (form, cell, degree, field degree, precision) grid multipliers for
 * coffee_assemble, and per batch bin type the store variant and task size
 * (used when a segment's task_cells is 0). Without this call the file named by
 * the environment variable COFFEE_TUNE_CACHE is loaded on first use. NULL
 * clears the cache. Text format: lines "linear form cell degree fd prec
 * grid_mult [variant]", "batch form cell degree prec variant task_cells
 * ns_per_cell" and "packed form cell degree prec task_cells ns_per_cell".
 * Errors: COFFEE_E_INVALID_ARG (unreadable file or malformed line; the
 * previous cache is kept). */
coffee_status coffee_load_tuning(const char* path);

/* Frees every per-device table cache. Safe to call more than once. */
void coffee_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif
