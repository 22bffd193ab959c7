/*
 * oracle.h - plain FP64 CPU reference for finite element local assembly.
 *
 * TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
 * CPU-baseline leg call this library; the GPU library never includes, links
 * or calls it, and it shares no code, header or table with it.
 *
 * Every routine is written from the mathematics of local assembly as the
 * paper states it (section 2, Fig. 1 and Table 1): map each cell to the
 * reference simplex, evaluate basis functions and coefficient fields at the
 * points of a quadrature rule, and sum integrand * |det J| * weight. Nothing
 * is factorised, collapsed or reordered.
 *
 * Status codes (int): 0 ok, 1 invalid argument, 2 unsupported, 4 degenerate
 * cell (det J = 0 or a non-finite input), 6 out of memory.
 */
#ifndef COFFEE_ORACLE_H
#define COFFEE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_E_INVALID_ARG = 1, OR_E_UNSUPPORTED = 2, OR_E_DEGENERATE = 4, OR_E_NOMEM = 6 };

/* Forms (same numbering as the library's public enum). DIFFUSION is the
 * Helmholtz operator without its mass term, scaled by two constants:
 * kappa dt grad u . grad v (constants kappa, dt; both 1 if absent). */
enum { OR_MASS = 0, OR_HELMHOLTZ = 1, OR_ELASTICITY = 2, OR_BURGERS = 3,
       OR_SVK_ENERGY = 4, OR_SVK_RESIDUAL = 5, OR_SVK_JACOBIAN = 6, OR_DIFFUSION = 7 };

/* Cell argument `dim`: 2 triangle, 3 tetrahedron, OR_PRISM the prism
 * (triangle x interval, six vertices; prism.c). */
enum { OR_PRISM = 6 };

/* A coefficient field. values: global [ndofs][ncomp] if cell_to_dof is not
 * NULL (cell_to_dof is [ncells][nloc]); else cell-major [ncells][nloc][ncomp].
 * degree 0..4 (Lagrange; degree 0 is one value per cell). */
typedef struct {
    const double* values;
    const int32_t* cell_to_dof;
    int32_t degree;
    int32_t ncomp;
} oracle_field;

/* Reference quadrature and basis tables on the reference simplex
 * (triangle (0,0),(1,0),(0,1); tetrahedron 0,e1,e2,e3). The rule is the
 * collapsed Gauss-Jacobi product rule with m = ceil((q+1)/2) points per
 * direction. Outputs may be NULL to query nq and ndof.
 *   points [nq][d], weights [nq], basis [nq][ndof], dbasis [d][nq][ndof]. */
int oracle_tabulate(int dim, int degree, int quad_degree, int* nq, int* ndof,
                    double* points, double* weights, double* basis, double* dbasis);

/* Basis values [npts][ndof] and reference gradients [dim][npts][ndof] of the
 * degree-p Lagrange element at arbitrary reference points X[npts][dim]. */
int oracle_basis_at(int dim, int degree, int npts, const double* X, double* phi, double* dphi);

/* Fully symmetric rule of degree q (0..6) on the reference simplex, solved
 * from the moment equations (symrule.c): *nq points X[nq][dim], weights
 * W[nq]; X and W may be NULL. A quad_degree argument of the other routines
 * selects it as q + 16 (q alone: the collapsed Gauss-Jacobi rule). */
int oracle_symmetric_rule(int dim, int q, int* nq, double* X, double* W);

/* One-dimensional Gauss-Jacobi rule on [0,1] for weight (1-x)^alpha. */
int oracle_gauss_jacobi(int m, int alpha, double* x, double* w);

/* Number of rows of the element tensor (0 for an energy). */
int oracle_tensor_dim(int form, int dim, int degree);

/* Element tensors of the cells listed in `cells` (or of all cells if cells is
 * NULL; then nsel must equal ncells). out has nsel blocks of N*N (bilinear
 * forms), N (residual) or 1 (energy) doubles. quad_degree < 0 selects 2p
 * (Burgers: 2p+1). constants: Burgers (nu, 1/dt); SVK and constant-parameter
 * elasticity (mu, lambda). nthreads <= 0 uses the OpenMP default. */
int oracle_assemble(int form, int dim, int degree, int quad_degree,
                    const double* coords, int64_t nvert, const int32_t* cell_to_vertex,
                    int64_t ncells, const oracle_field* fields, int nfield,
                    const double* constants, int nconst,
                    const int64_t* cells, int64_t nsel, double* out, int nthreads);

/* Gradient of seed * S, S = sum_e lam_e^T A_e u_e (bilinear forms),
 * sum_e lam_e^T b_e (residual) or sum_e Pi_e (energy), with respect to the
 * vertex coordinates and to every coefficient value, by the complex-step
 * derivative of the per-cell functional. grad_coords [nvert][d] and each
 * grad_fields[i] (shaped like fields[i].values; NULL skips) are ACCUMULATED.
 * S (unscaled) is written to *value when value is not NULL. */
int oracle_adjoint(int form, int dim, int degree, int quad_degree,
                   const double* coords, int64_t nvert, const int32_t* cell_to_vertex,
                   int64_t ncells, const oracle_field* fields, int nfield,
                   const double* constants, int nconst,
                   const double* lam, const double* u, double seed,
                   double* grad_coords, double* const* grad_fields, double* value,
                   int nthreads);

/* Prism cells (prism.c), reached through the calls above with dim = OR_PRISM:
 * mass, Helmholtz and diffusion, degree 1..4, a degree-1 prism field. */
int prism_ndofs(int p);
int prism_tabulate(int degree, int quad_degree, int* nq, int* ndof, double* points, double* weights,
                   double* basis, double* dbasis);
int prism_basis_at(int degree, int npts, const double* X, double* phi, double* dphi);
int prism_assemble(int form, int degree, int quad_degree, const double* coords, int64_t nvert,
                   const int32_t* c2v, int64_t ncells, const oracle_field* fields, int nfield,
                   const double* constants, int nconst, const int64_t* cells, int64_t nsel, double* out,
                   int nthreads);

#ifdef __cplusplus
}
#endif
#endif
