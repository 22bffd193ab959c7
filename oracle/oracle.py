"""ctypes wrapper of the plain FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; the product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

FORMS = {"mass": 0, "helmholtz": 1, "elasticity": 2, "burgers": 3,
         "svk_energy": 4, "svk_residual": 5, "svk_jacobian": 6, "diffusion": 7}
PRISM = 6  # cell code of the prism (triangle x interval); simplices use their dimension


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc -O2 and OpenMP."""
    srcs = [os.path.join(_HERE, f) for f in ("oracle.c", "symrule.c", "prism.c")]
    deps = srcs + [os.path.join(_HERE, f) for f in ("element.inc", "oracle.h")]
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < max(os.path.getmtime(f) for f in deps):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
               "-o", _SO + ".tmp", *srcs, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Field(C.Structure):
    _fields_ = [("values", C.c_void_p), ("cell_to_dof", C.c_void_p),
                ("degree", C.c_int32), ("ncomp", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        L.oracle_tabulate.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_basis_at.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_gauss_jacobi.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p]
        L.oracle_symmetric_rule.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.c_void_p, C.c_void_p]
        L.oracle_tensor_dim.argtypes = [C.c_int, C.c_int, C.c_int]
        L.oracle_assemble.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int64,
                                      C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                      C.c_void_p, C.c_int64, C.c_void_p, C.c_int]
        L.oracle_adjoint.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int64,
                                     C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                     C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def _ptr(a):
    return None if a is None else a.ctypes.data


def gauss_jacobi(m: int, alpha: int):
    x = np.zeros(m)
    w = np.zeros(m)
    st = lib().oracle_gauss_jacobi(m, alpha, _ptr(x), _ptr(w))
    if st:
        raise OracleError(st)
    return x, w


RULE_SYMMETRIC = 1


def quad(q: int, rule: int = 0) -> int:
    """quad_degree argument selecting rule `rule` of degree q (q + 16 rule)."""
    return q + 16 * rule


def symmetric_rule(dim: int, q: int):
    """(points [nq, dim], weights [nq]) of the fully symmetric rule of degree q."""
    nq = C.c_int()
    X = np.zeros((64, dim))
    W = np.zeros(64)
    st = lib().oracle_symmetric_rule(dim, q, C.byref(nq), _ptr(X), _ptr(W))
    if st:
        raise OracleError(st)
    return X[:nq.value].copy(), W[:nq.value].copy()


def tabulate(dim: int, degree: int, quad_degree: int):
    """Rule and basis tables; dim 2, 3 or PRISM (points then have 3 coordinates)."""
    nq, nd = C.c_int(), C.c_int()
    st = lib().oracle_tabulate(dim, degree, quad_degree, C.byref(nq), C.byref(nd), None, None, None, None)
    if st:
        raise OracleError(st)
    q, n = nq.value, nd.value
    sd = 3 if dim == PRISM else dim
    X = np.zeros((q, sd)); W = np.zeros(q); B = np.zeros((q, n)); D = np.zeros((sd, q, n))
    st = lib().oracle_tabulate(dim, degree, quad_degree, C.byref(nq), C.byref(nd), _ptr(X), _ptr(W), _ptr(B), _ptr(D))
    if st:
        raise OracleError(st)
    return X, W, B, D


def basis_at(dim: int, degree: int, X: np.ndarray):
    """Basis values [npts, n] and reference gradients [dim, npts, n] at points X [npts, dim]."""
    sd = 3 if dim == PRISM else dim
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, sd)
    if dim == PRISM:
        n = (degree + 1) * (degree + 2) // 2 * (degree + 1)
    else:
        n = (degree + 1) * (degree + 2) // 2 if dim == 2 else (degree + 1) * (degree + 2) * (degree + 3) // 6
    phi = np.zeros((X.shape[0], n))
    dphi = np.zeros((sd, X.shape[0], n))
    st = lib().oracle_basis_at(dim, degree, X.shape[0], _ptr(X), _ptr(phi), _ptr(dphi))
    if st:
        raise OracleError(st)
    return phi, dphi


def tensor_dim(form: str, dim: int, degree: int) -> int:
    return lib().oracle_tensor_dim(FORMS[form], dim, degree)


def _fields(fields):
    keep = []
    arr = (_Field * max(1, len(fields)))()
    for i, f in enumerate(fields):
        v = np.ascontiguousarray(f.values, dtype=np.float64)
        c2d = None if f.cell_to_dof is None else np.ascontiguousarray(f.cell_to_dof, dtype=np.int32)
        keep += [v, c2d]
        arr[i] = _Field(v.ctypes.data, None if c2d is None else c2d.ctypes.data, f.degree, f.ncomp)
    return arr, keep


def assemble(form: str, mesh, degree: int, quad_degree: int = -1, fields=(), constants=(),
             cells=None, nthreads: int = 0) -> np.ndarray:
    """Element tensors [nsel, N, N] / [nsel, N] / [nsel] for the selected cells
    (simplex or prism meshes: the cell code comes from the connectivity)."""
    coords = np.ascontiguousarray(mesh.coords, dtype=np.float64)
    c2v = np.ascontiguousarray(mesh.cells, dtype=np.int32)
    E = c2v.shape[0]
    cell = PRISM if c2v.shape[1] == 6 else mesh.d
    sel = None if cells is None else np.ascontiguousarray(cells, dtype=np.int64)
    nsel = E if sel is None else sel.shape[0]
    N = tensor_dim(form, cell, degree)
    shape = (nsel,) if form == "svk_energy" else ((nsel, N) if form == "svk_residual" else (nsel, N, N))
    out = np.zeros(shape)
    farr, keep = _fields(list(fields))
    cst = np.ascontiguousarray(constants, dtype=np.float64)
    st = lib().oracle_assemble(FORMS[form], cell, degree, quad_degree, _ptr(coords), coords.shape[0],
                               _ptr(c2v), E, farr, len(fields), _ptr(cst) if cst.size else None, cst.size,
                               _ptr(sel), nsel, _ptr(out), nthreads)
    if st:
        raise OracleError(st)
    return out


def adjoint(form: str, mesh, degree: int, quad_degree: int = -1, fields=(), constants=(),
            lam=None, u=None, seed: float = 1.0, nthreads: int = 0):
    """(S, grad_coords [V, d], [grad of each field's values])."""
    coords = np.ascontiguousarray(mesh.coords, dtype=np.float64)
    c2v = np.ascontiguousarray(mesh.cells, dtype=np.int32)
    E = c2v.shape[0]
    farr, keep = _fields(list(fields))
    cst = np.ascontiguousarray(constants, dtype=np.float64)
    gc = np.zeros_like(coords)
    gfs = [np.zeros_like(np.asarray(f.values, dtype=np.float64)) for f in fields]
    gptr = (C.c_void_p * max(1, len(gfs)))(*[g.ctypes.data for g in gfs])
    lam_ = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
    u_ = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    val = C.c_double()
    st = lib().oracle_adjoint(FORMS[form], mesh.d, degree, quad_degree, _ptr(coords), coords.shape[0],
                              _ptr(c2v), E, farr, len(fields), _ptr(cst) if cst.size else None, cst.size,
                              _ptr(lam_), _ptr(u_), seed, _ptr(gc), gptr, C.byref(val), nthreads)
    if st:
        raise OracleError(st)
    return val.value, gc, gfs


def assemble_global(form: str, mesh, degree: int, space_map, ndofs: int, quad_degree: int = -1, fields=(),
                    constants=()):
    """The global matrix sum_e P_e^T A_e P_e as a scipy CSR matrix (FP64):
    element tensors from `assemble`, scattered entry by entry into a
    coordinate list with the global indices dof * ncomp + c of the local dofs
    (c, a) (component-blocked locally), duplicates summed by scipy.
    space_map [E, nloc] is the dof map of the form's space."""
    import scipy.sparse as sp
    A = assemble(form, mesh, degree, quad_degree, fields=fields, constants=constants)
    E, N, _ = A.shape
    nloc = space_map.shape[1]
    nc = N // nloc
    gidx = np.empty((E, N), dtype=np.int64)
    for c in range(nc):
        for a in range(nloc):
            gidx[:, c * nloc + a] = space_map[:, a].astype(np.int64) * nc + c
    rows = np.repeat(gidx, N, axis=1).reshape(-1)
    cols = np.tile(gidx, (1, N)).reshape(-1)
    M = sp.coo_matrix((A.reshape(-1), (rows, cols)), shape=(ndofs * nc, ndofs * nc)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return M
