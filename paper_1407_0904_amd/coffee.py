"""Thin Python binding of libcoffee (include/coffee.h): argument marshalling only.

Every function here forwards to the C ABI of the same name; all arithmetic
runs in the HIP kernels of libcoffee.so. PyTorch provides device memory and
the current stream. The library must be built (see build.py): importing this
module without it raises ImportError, there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_SO = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcoffee.so")

FORMS = {"mass": 0, "helmholtz": 1, "elasticity": 2, "burgers": 3,
         "svk_energy": 4, "svk_residual": 5, "svk_jacobian": 6, "diffusion": 7}
# cell codes: simplices by dimension, the prism (triangle x interval) by its vertex count
CELLS = {"triangle": 2, "tetrahedron": 3, "prism": 6, 2: 2, 3: 3, 6: 6}
PRISM = 6
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}


class CoffeeError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {status_string(code)} (status {code})")
        self.code = code


class _Field(C.Structure):
    _fields_ = [("values", C.c_void_p), ("cell_to_dof", C.c_void_p),
                ("degree", C.c_int32), ("ncomp", C.c_int32)]


class _Segment(C.Structure):
    _fields_ = [("form", C.c_int32), ("cell", C.c_int32), ("degree", C.c_int32), ("quad_degree", C.c_int32),
                ("coords", C.c_void_p), ("nvert", C.c_int64), ("cell_to_vertex", C.c_void_p),
                ("ncells_mesh", C.c_int64), ("coeff", C.c_void_p), ("variant", C.c_int32),
                ("task_cells", C.c_int32)]


def _load():
    if not os.path.exists(_SO):
        raise ImportError(f"{_SO} is not built: run paper_1407_0904_amd.build.build() first")
    L = C.CDLL(_SO)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    L.coffee_tabulate.argtypes = [i32, i32, i32, C.POINTER(C.c_int), C.POINTER(C.c_int), vp, vp, vp, vp]
    L.coffee_tabulate.restype = i32
    L.coffee_tensor_dim.argtypes = [i32, i32, i32]
    L.coffee_tensor_dim.restype = i32
    L.coffee_assemble.argtypes = [i32, i32, i32, i32, i32, vp, i64, vp, i64, vp, i32, vp, i32, vp, vp]
    L.coffee_assemble.restype = i32
    L.coffee_assemble_adjoint.argtypes = [i32, i32, i32, i32, vp, i64, vp, i64, vp, i32, vp, i32,
                                          vp, vp, dbl, vp, vp, vp, i32, vp, i64, vp]
    L.coffee_assemble_adjoint.restype = i32
    L.coffee_adjoint_workspace_size.argtypes = [i32, i32, i32, i64, i64, vp, i32]
    L.coffee_adjoint_workspace_size.restype = i64
    L.coffee_check_geometry.argtypes = [i32, vp, i64, vp, i64, vp, vp]
    L.coffee_check_geometry.restype = i32
    L.coffee_status_string.argtypes = [i32]
    L.coffee_status_string.restype = C.c_char_p
    L.coffee_shutdown.argtypes = []
    L.coffee_shutdown.restype = None
    L.coffee_assemble_batch.argtypes = [i32, vp, i32, vp, vp, vp, i64, vp, vp, i64, vp]
    L.coffee_assemble_batch.restype = i32
    L.coffee_assemble_batch_packed.argtypes = [i32, vp, i32, vp, vp, i64, vp, vp, vp, i64, vp]
    L.coffee_assemble_batch_packed.restype = i32
    L.coffee_assemble_batch_packed_noalloc.argtypes = [i32, vp, i32, vp, vp, i64, vp, vp, vp]
    L.coffee_assemble_batch_packed_noalloc.restype = i32
    L.coffee_batch_workspace_size.argtypes = [i32, i64]
    L.coffee_batch_workspace_size.restype = i64
    L.coffee_csr_pattern_workspace_size.argtypes = [i64, i32, i64]
    L.coffee_csr_pattern_workspace_size.restype = i64
    L.coffee_csr_pattern.argtypes = [vp, i64, i32, i64, i32, vp, vp, i64, C.POINTER(C.c_int64), vp, i64, vp]
    L.coffee_csr_pattern.restype = i32
    L.coffee_assemble_csr_workspace_size.argtypes = [i32, i32, i32, i32, i64]
    L.coffee_assemble_csr_workspace_size.restype = i64
    L.coffee_assemble_csr.argtypes = [i32, i32, i32, i32, i32, vp, i64, vp, i64, vp, i32, vp, i32, vp, i64, vp, vp,
                                      i64, vp, vp, i64, vp]
    L.coffee_assemble_csr.restype = i32
    L.coffee_load_tuning.argtypes = [C.c_char_p]
    L.coffee_load_tuning.restype = i32
    L.coffee_set_launch_options.argtypes = [i32]
    L.coffee_set_launch_options.restype = None
    L.coffee_set_variant.argtypes = [i32]
    L.coffee_set_variant.restype = None
    L.coffee_has_variant.argtypes = [i32, i32, i32, i32, i32, i32]
    L.coffee_has_variant.restype = i32
    return L


_lib = _load()
LIBRARY_PATH = _SO


def status_string(code: int) -> str:
    return _lib.coffee_status_string(int(code)).decode()


def _check(code: int, where: str):
    if code != 0:
        raise CoffeeError(code, where)


def _dptr(t, dtype, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


# Shape checks. They run before any device pointer is taken, so a wrong shape
# is a ValueError on the host instead of an out-of-bounds access on the GPU.
def _nloc(c: int, p: int) -> int:
    """Lagrange dofs of degree p on cell code c."""
    if c == PRISM:
        return (p + 1) * (p + 2) // 2 * (p + 1)
    return (p + 1) * (p + 2) // 2 if c == 2 else (p + 1) * (p + 2) * (p + 3) // 6


def _sdim(c: int) -> int:
    return 3 if c == PRISM else c


def _nverts(c: int) -> int:
    return 6 if c == PRISM else c + 1


def _need(t, name, dtype, shape=None, numel=None, allow_none=False):
    # `name` is a string or a callable giving it (formatted only for the error)
    if t is None:
        if allow_none:
            return
        raise ValueError(f"{_nm(name)} is required")
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{_nm(name)} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{_nm(name)} must be {dtype}, got {t.dtype}")
    if shape is not None and t.shape != shape:
        raise ValueError(f"{_nm(name)} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{_nm(name)} has {t.numel()} elements, expected {numel}")


def _nm(name):
    return name() if callable(name) else name


def _check_mesh(c, coords, cell_to_vertex, where=""):
    _need(coords, lambda: where + "coords", torch.float64)
    _need(cell_to_vertex, lambda: where + "cell_to_vertex", torch.int32)
    d, nv = _sdim(c), _nverts(c)
    if coords.ndim != 2 or coords.shape[1] != d:
        raise ValueError(f"{where}coords has shape {tuple(coords.shape)}, expected (nvert, {d})")
    if cell_to_vertex.ndim != 2 or cell_to_vertex.shape[1] != nv:
        raise ValueError(f"{where}cell_to_vertex has shape {tuple(cell_to_vertex.shape)}, expected (ncells, {nv})")


def _check_fields(coeffs, d, ncells, where="coeffs"):
    for i, f in enumerate(coeffs):
        name = lambda: f"{where}[{i}]"
        _need(f.values, lambda: name() + ".values", torch.float64)
        if not 1 <= f.degree <= 4 or f.ncomp < 1:
            continue  # the library reports the bad degree or component count
        nloc, nc = _nloc(d, f.degree), f.ncomp
        if f.cell_to_dof is not None:
            _need(f.cell_to_dof, lambda: name() + ".cell_to_dof", torch.int32, shape=(ncells, nloc))
            v = f.values
            if v.numel() % nc or (v.ndim >= 2 and v.shape[-1] != nc) or (v.ndim == 1 and nc != 1):
                raise ValueError(f"{name()}.values has shape {tuple(v.shape)}, expected (ndofs, {nc})")
        else:
            _need(f.values, lambda: name() + ".values", torch.float64, numel=ncells * nloc * nc)


@dataclass
class DeviceField:
    """A coefficient field on the device (see coffee_field in coffee.h)."""
    values: torch.Tensor              # float64, global [ndofs, ncomp] or cell-major [E, nloc, ncomp]
    cell_to_dof: torch.Tensor | None  # int32 [E, nloc] or None
    degree: int
    ncomp: int

    @staticmethod
    def from_host(f, device="cuda") -> "DeviceField":
        v = torch.as_tensor(np.ascontiguousarray(f.values, dtype=np.float64), device=device)
        m = None if f.cell_to_dof is None else torch.as_tensor(
            np.ascontiguousarray(f.cell_to_dof, dtype=np.int32), device=device)
        return DeviceField(v, m, int(f.degree), int(f.ncomp))


def _fields(coeffs):
    arr = (_Field * max(1, len(coeffs)))()
    for i, f in enumerate(coeffs):
        arr[i] = _Field(_dptr(f.values, torch.float64, f"coeffs[{i}].values"),
                        _dptr(f.cell_to_dof, torch.int32, f"coeffs[{i}].cell_to_dof", allow_none=True),
                        int(f.degree), int(f.ncomp))
    return arr


def coffee_tabulate(cell, degree: int, quad_degree: int):
    """Host FP64 tables: (points [nq, d], weights [nq], basis [nq, n], dbasis [d, nq, n]); d = 3 on prisms."""
    c = CELLS[cell]
    nq, nd = C.c_int(), C.c_int()
    _check(_lib.coffee_tabulate(c, degree, quad_degree, C.byref(nq), C.byref(nd), None, None, None, None),
           "coffee_tabulate")
    q, n, d = nq.value, nd.value, _sdim(c)
    X = np.zeros((q, d)); W = np.zeros(q); B = np.zeros((q, n)); D = np.zeros((d, q, n))
    _check(_lib.coffee_tabulate(c, degree, quad_degree, C.byref(nq), C.byref(nd), X.ctypes.data,
                                W.ctypes.data, B.ctypes.data, D.ctypes.data), "coffee_tabulate")
    return X, W, B, D


def coffee_tensor_dim(form, cell, degree: int) -> int:
    return _lib.coffee_tensor_dim(FORMS[form], CELLS[cell], degree)


def output_shape(form, ncells: int, cell, degree: int):
    N = _tensor_dim(FORMS[form], CELLS[cell], degree)
    if form == "svk_energy":
        return (ncells,)
    if form == "svk_residual":
        return (ncells, N)
    return (ncells, N, N)


_TDIM = {}


def _tensor_dim(form: int, cell: int, degree: int) -> int:
    key = (form, cell, degree)
    n = _TDIM.get(key)
    if n is None:
        n = _TDIM[key] = _lib.coffee_tensor_dim(form, cell, degree)
    return n


def _numel(shape) -> int:
    n = 1
    for s in shape:
        n *= s
    return n


def coffee_assemble(form, cell, degree: int, coords: torch.Tensor, cell_to_vertex: torch.Tensor,
                    coeffs=(), constants=(), quad_degree: int = -1, precision: str = "fp64",
                    out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Element tensors of every cell (coffee_assemble)."""
    c = CELLS[cell]
    _check_mesh(c, coords, cell_to_vertex)
    ncells = cell_to_vertex.shape[0]
    _check_fields(coeffs, c, ncells)
    odt = torch.float64 if precision == "fp64" else torch.float32
    shape = output_shape(form, ncells, c, degree)
    if min(shape) < 0:  # bad form or degree: the library reports it
        out = torch.empty(0, dtype=odt, device=coords.device) if out is None else out
    elif out is None:
        out = torch.empty(shape, dtype=odt, device=coords.device)
    else:
        _need(out, "out", odt, numel=_numel(shape))
    cst = np.ascontiguousarray(constants, dtype=np.float64)
    st = _lib.coffee_assemble(FORMS[form], c, degree, quad_degree, PRECISIONS[precision],
                              _dptr(coords, torch.float64, "coords"), coords.shape[0] if coords.ndim else 0,
                              _dptr(cell_to_vertex, torch.int32, "cell_to_vertex"), ncells,
                              _fields(list(coeffs)), len(coeffs),
                              cst.ctypes.data if cst.size else None, cst.size,
                              _dptr(out, odt, "out"), _stream(stream))
    _check(st, "coffee_assemble")
    return out


class PreparedAssemble:
    """One coffee_assemble call with its arguments checked and marshalled once,
    for callers that launch the same assembly repeatedly (time stepping, a
    serving loop, a benchmark): each call only re-enters the C ABI. The
    tensors are kept referenced; the stream is the one current at preparation
    unless given."""

    def __init__(self, form, cell, degree: int, coords, cell_to_vertex, coeffs=(), constants=(),
                 quad_degree: int = -1, precision: str = "fp64", out=None, stream=None):
        c = CELLS[cell]
        _check_mesh(c, coords, cell_to_vertex)
        ncells = cell_to_vertex.shape[0]
        _check_fields(coeffs, c, ncells)
        odt = torch.float64 if precision == "fp64" else torch.float32
        shape = output_shape(form, ncells, c, degree)
        if min(shape) < 0:
            raise CoffeeError(1, "PreparedAssemble")
        if out is None:
            out = torch.empty(shape, dtype=odt, device=coords.device)
        _need(out, "out", odt, numel=_numel(shape))
        self.out = out
        self._keep = (coords, cell_to_vertex, list(coeffs), np.ascontiguousarray(constants, dtype=np.float64))
        cst = self._keep[3]
        self._fields = _fields(list(coeffs))
        self._args = (FORMS[form], c, degree, quad_degree, PRECISIONS[precision],
                      _dptr(coords, torch.float64, "coords"), coords.shape[0],
                      _dptr(cell_to_vertex, torch.int32, "cell_to_vertex"), ncells,
                      self._fields, len(coeffs), cst.ctypes.data if cst.size else None, cst.size,
                      _dptr(out, odt, "out"), _stream(stream))

    def __call__(self) -> torch.Tensor:
        _check(_lib.coffee_assemble(*self._args), "coffee_assemble")
        return self.out


def coffee_adjoint_workspace_size(form, cell, degree: int, nvert: int, ncells: int, coeffs=()) -> int:
    """Workspace bytes of the deterministic adjoint (coffee_adjoint_workspace_size)."""
    fa = _fields(list(coeffs))
    n = int(_lib.coffee_adjoint_workspace_size(FORMS[form], CELLS[cell], degree, nvert, ncells, fa, len(coeffs)))
    if n < 0:
        raise CoffeeError(1, "coffee_adjoint_workspace_size")
    return n


def coffee_assemble_adjoint(form, cell, degree: int, coords, cell_to_vertex, coeffs=(), constants=(),
                            lam=None, u=None, seed: float = 1.0, grad_coords=None, grad_coeffs=None,
                            cell_value=None, deterministic: bool = False, quad_degree: int = -1,
                            workspace=None, grads: bool = True, stream=None):
    """Accumulates seed * dS/d(coords, coefficient values); returns (grad_coords, grad_coeffs).
    grads=False computes only the per-cell values (cell_value) and returns (None, [])."""
    c = CELLS[cell]
    _check_mesh(c, coords, cell_to_vertex)
    ncells = cell_to_vertex.shape[0]
    _check_fields(coeffs, c, ncells)
    N = _tensor_dim(FORMS[form], c, degree)
    if N > 0:
        _need(lam, "lam", torch.float64, shape=(ncells, N), allow_none=True)
        _need(u, "u", torch.float64, shape=(ncells, N), allow_none=True)
    _need(cell_value, "cell_value", torch.float64, numel=ncells, allow_none=True)
    if not grads:
        grad_coords, grad_coeffs = None, [None] * len(coeffs)
    elif grad_coords is None:
        grad_coords = torch.zeros_like(coords)
    _need(grad_coords, "grad_coords", torch.float64, shape=tuple(coords.shape), allow_none=not grads)
    if grad_coeffs is None:
        grad_coeffs = [torch.zeros_like(f.values) for f in coeffs]
    if len(grad_coeffs) != len(coeffs):
        raise ValueError(f"grad_coeffs has {len(grad_coeffs)} entries, expected {len(coeffs)}")
    for i, (g, f) in enumerate(zip(grad_coeffs, coeffs)):
        _need(g, f"grad_coeffs[{i}]", torch.float64, shape=tuple(f.values.shape), allow_none=True)
    gptr = (C.c_void_p * max(1, len(coeffs)))(
        *[_dptr(g, torch.float64, "grad_coeffs", allow_none=True) for g in grad_coeffs])
    fa = _fields(list(coeffs))
    if deterministic:
        nbytes = coffee_adjoint_workspace_size(form, c, degree, coords.shape[0], ncells, coeffs)
        if workspace is None:
            workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=coords.device)
        _need(workspace, "workspace", torch.uint8)
        if workspace.numel() < nbytes:
            raise ValueError(f"workspace has {workspace.numel()} bytes, expected at least {nbytes}")
    cst = np.ascontiguousarray(constants, dtype=np.float64)
    st = _lib.coffee_assemble_adjoint(
        FORMS[form], c, degree, quad_degree,
        _dptr(coords, torch.float64, "coords"), coords.shape[0],
        _dptr(cell_to_vertex, torch.int32, "cell_to_vertex"), ncells, fa, len(coeffs),
        cst.ctypes.data if cst.size else None, cst.size,
        _dptr(lam, torch.float64, "lam", allow_none=True), _dptr(u, torch.float64, "u", allow_none=True),
        float(seed), _dptr(grad_coords, torch.float64, "grad_coords", allow_none=not grads), gptr,
        _dptr(cell_value, torch.float64, "cell_value", allow_none=True), int(bool(deterministic)),
        None if workspace is None else workspace.data_ptr(), 0 if workspace is None else workspace.numel(),
        _stream(stream))
    _check(st, "coffee_assemble_adjoint")
    if not grads:
        return None, []
    return grad_coords, grad_coeffs


@dataclass
class Segment:
    """One bin of a mixed batch (see coffee_segment in coffee.h)."""
    form: str
    cell: int
    degree: int
    coords: torch.Tensor
    cell_to_vertex: torch.Tensor
    coeff: DeviceField
    quad_degree: int = -1
    variant: int = 0
    task_cells: int = 0


def coffee_batch_workspace_size(nseg: int, nentries: int) -> int:
    return int(_lib.coffee_batch_workspace_size(int(nseg), int(nentries)))


def _check_batch(segments, seg_of, cell_of, out_offset, out, odt, total_elems, workspace):
    for i, sg in enumerate(segments):
        d = CELLS[sg.cell]
        _check_mesh(d, sg.coords, sg.cell_to_vertex, where=f"segments[{i}].")
        _check_fields([sg.coeff], d, sg.cell_to_vertex.shape[0], where=f"segments[{i}].coeff")
    _need(seg_of, "seg_of", torch.int32)
    if seg_of.ndim != 1:
        raise ValueError(f"seg_of has shape {tuple(seg_of.shape)}, expected (nentries,)")
    n = seg_of.shape[0]
    _need(cell_of, "cell_of", torch.int64, shape=(n,))
    _need(out_offset, "out_offset", torch.int64, shape=(n,))
    _need(out, "out", odt)
    if out.numel() < total_elems:
        raise ValueError(f"out has {out.numel()} elements, fewer than total_elems = {total_elems}")
    need = coffee_batch_workspace_size(len(segments), n)
    _need(workspace, "workspace", torch.uint8)
    if workspace.numel() < need:
        raise ValueError(f"workspace has {workspace.numel()} bytes, expected at least {need}")


def _segments(segments):
    segs = (_Segment * len(segments))()
    fields = (_Field * len(segments))()
    for i, sg in enumerate(segments):
        f = sg.coeff
        fields[i] = _Field(_dptr(f.values, torch.float64, "coeff.values"),
                           _dptr(f.cell_to_dof, torch.int32, "coeff.cell_to_dof", allow_none=True),
                           int(f.degree), int(f.ncomp))
        segs[i] = _Segment(FORMS[sg.form], CELLS[sg.cell], int(sg.degree), int(sg.quad_degree),
                           _dptr(sg.coords, torch.float64, "coords"), sg.coords.shape[0],
                           _dptr(sg.cell_to_vertex, torch.int32, "cell_to_vertex"), sg.cell_to_vertex.shape[0],
                           C.addressof(fields[i]), int(sg.variant), int(sg.task_cells))
    return segs, fields  # fields must outlive the call


def coffee_assemble_batch(segments, seg_of: torch.Tensor, cell_of: torch.Tensor, out_offset: torch.Tensor,
                          total_elems: int, precision: str = "fp32", out: torch.Tensor | None = None,
                          workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Packed element tensors of a mixed batch at the caller's offsets (coffee_assemble_batch)."""
    odt = torch.float64 if precision == "fp64" else torch.float32
    dev = seg_of.device
    n = seg_of.shape[0]
    if out is None:
        out = torch.empty(total_elems, dtype=odt, device=dev)
    if workspace is None:
        workspace = torch.empty(coffee_batch_workspace_size(len(segments), n), dtype=torch.uint8, device=dev)
    _check_batch(segments, seg_of, cell_of, out_offset, out, odt, total_elems, workspace)
    segs, _keep = _segments(segments)
    st = _lib.coffee_assemble_batch(PRECISIONS[precision], segs, len(segments),
                                    _dptr(seg_of, torch.int32, "seg_of"), _dptr(cell_of, torch.int64, "cell_of"),
                                    _dptr(out_offset, torch.int64, "out_offset"), n, _dptr(out, odt, "out"),
                                    workspace.data_ptr(), workspace.numel(), _stream(stream))
    _check(st, "coffee_assemble_batch")
    return out


def coffee_assemble_batch_packed(segments, seg_of: torch.Tensor, cell_of: torch.Tensor, total_elems: int,
                                 precision: str = "fp32", out: torch.Tensor | None = None,
                                 out_offset: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                                 stream=None):
    """Element tensors of a mixed batch in the library's segment-major layout
    (coffee_assemble_batch_packed); returns (out, out_offset)."""
    odt = torch.float64 if precision == "fp64" else torch.float32
    dev = seg_of.device
    n = seg_of.shape[0]
    if out is None:
        out = torch.empty(total_elems, dtype=odt, device=dev)
    if out_offset is None:
        out_offset = torch.empty(n, dtype=torch.int64, device=dev)
    if workspace is None:
        workspace = torch.empty(coffee_batch_workspace_size(len(segments), n), dtype=torch.uint8, device=dev)
    _check_batch(segments, seg_of, cell_of, out_offset, out, odt, total_elems, workspace)
    segs, _keep = _segments(segments)
    st = _lib.coffee_assemble_batch_packed(PRECISIONS[precision], segs, len(segments),
                                           _dptr(seg_of, torch.int32, "seg_of"),
                                           _dptr(cell_of, torch.int64, "cell_of"), n, _dptr(out, odt, "out"),
                                           _dptr(out_offset, torch.int64, "out_offset"),
                                           workspace.data_ptr(), workspace.numel(), _stream(stream))
    _check(st, "coffee_assemble_batch_packed")
    return out, out_offset


def coffee_csr_pattern(cell_to_dof: torch.Tensor, ndofs: int, ncomp: int = 1, stream=None):
    """CSR pattern (row_ptr int64 [ndofs * ncomp + 1], col_idx int32 [nnz]) of
    the global matrix of the space with this cell-to-dof map."""
    _need(cell_to_dof, "cell_to_dof", torch.int32)
    if cell_to_dof.ndim != 2:
        raise ValueError(f"cell_to_dof has shape {tuple(cell_to_dof.shape)}, expected (ncells, nloc)")
    ncells, nloc = cell_to_dof.shape
    dev = cell_to_dof.device
    wsb = int(_lib.coffee_csr_pattern_workspace_size(ncells, nloc, ndofs))
    if wsb < 0:
        raise CoffeeError(1, "coffee_csr_pattern_workspace_size")
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    row_ptr = torch.empty(ndofs * ncomp + 1, dtype=torch.int64, device=dev)
    nnz = C.c_int64()
    args = [_dptr(cell_to_dof, torch.int32, "cell_to_dof"), ncells, nloc, ndofs, ncomp,
            _dptr(row_ptr, torch.int64, "row_ptr")]
    st = _lib.coffee_csr_pattern(*args, None, 0, C.byref(nnz), ws.data_ptr(), ws.numel(), _stream(stream))
    if st not in (0, 3):
        _check(st, "coffee_csr_pattern")
    col_idx = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
    st = _lib.coffee_csr_pattern(*args, col_idx.data_ptr(), col_idx.numel(), C.byref(nnz), ws.data_ptr(),
                                 ws.numel(), _stream(stream))
    _check(st, "coffee_csr_pattern")
    return row_ptr, col_idx[:nnz.value]


def coffee_assemble_csr(form, cell, degree: int, coords, cell_to_vertex, row_ptr, col_idx, ndofs: int,
                        cell_to_dof=None, coeffs=(), constants=(), quad_degree: int = -1, precision: str = "fp64",
                        values=None, workspace=None, stream=None) -> torch.Tensor:
    """Values of the global matrix in the CSR pattern (coffee_assemble_csr)."""
    c = CELLS[cell]
    _check_mesh(c, coords, cell_to_vertex)
    ncells = cell_to_vertex.shape[0]
    _check_fields(coeffs, c, ncells)
    nloc = _nloc(c, degree)
    N = _tensor_dim(FORMS[form], c, degree)
    if N <= 0:
        raise ValueError(f"{form} has no element matrix")
    ncomp = N // nloc
    if cell_to_dof is not None:
        _need(cell_to_dof, "cell_to_dof", torch.int32, shape=(ncells, nloc))
    elif degree != 1:
        raise ValueError("cell_to_dof is required above degree 1")
    _need(row_ptr, "row_ptr", torch.int64, shape=(ndofs * ncomp + 1,))
    _need(col_idx, "col_idx", torch.int32)
    nnz = col_idx.numel()
    odt = torch.float64 if precision == "fp64" else torch.float32
    if values is None:
        values = torch.empty(nnz, dtype=odt, device=coords.device)
    _need(values, "values", odt, numel=nnz)
    wsb = int(_lib.coffee_assemble_csr_workspace_size(FORMS[form], c, degree, PRECISIONS[precision], ncells))
    if workspace is None:
        workspace = torch.empty(max(wsb, 16), dtype=torch.uint8, device=coords.device)
    if workspace.numel() < wsb:
        raise ValueError(f"workspace has {workspace.numel()} bytes, expected at least {wsb}")
    cst = np.ascontiguousarray(constants, dtype=np.float64)
    st = _lib.coffee_assemble_csr(FORMS[form], c, degree, quad_degree, PRECISIONS[precision],
                                  _dptr(coords, torch.float64, "coords"), coords.shape[0],
                                  _dptr(cell_to_vertex, torch.int32, "cell_to_vertex"), ncells,
                                  _fields(list(coeffs)), len(coeffs), cst.ctypes.data if cst.size else None, cst.size,
                                  _dptr(cell_to_dof, torch.int32, "cell_to_dof", allow_none=True), ndofs,
                                  _dptr(row_ptr, torch.int64, "row_ptr"), _dptr(col_idx, torch.int32, "col_idx"), nnz,
                                  _dptr(values, odt, "values"), workspace.data_ptr(), workspace.numel(),
                                  _stream(stream))
    _check(st, "coffee_assemble_csr")
    return values


NOALLOC_MAX_ENTRIES = 4194304  # COFFEE_NOALLOC_MAX_ENTRIES


def coffee_assemble_batch_packed_noalloc(segments, seg_of: torch.Tensor, cell_of: torch.Tensor, out: torch.Tensor,
                                         out_offset: torch.Tensor, precision: str = "fp32", stream=None):
    """coffee_assemble_batch_packed without a workspace: the library's static
    device scratch array (at most NOALLOC_MAX_ENTRIES entries). The caller
    passes the outputs; nothing is allocated."""
    odt = torch.float64 if precision == "fp64" else torch.float32
    n = seg_of.shape[0]
    for i, sg in enumerate(segments):
        d = CELLS[sg.cell]
        _check_mesh(d, sg.coords, sg.cell_to_vertex, where=f"segments[{i}].")
        _check_fields([sg.coeff], d, sg.cell_to_vertex.shape[0], where=f"segments[{i}].coeff")
    _need(seg_of, "seg_of", torch.int32, shape=(n,))
    _need(cell_of, "cell_of", torch.int64, shape=(n,))
    _need(out_offset, "out_offset", torch.int64, shape=(n,))
    _need(out, "out", odt)
    segs, _keep = _segments(segments)
    st = _lib.coffee_assemble_batch_packed_noalloc(PRECISIONS[precision], segs, len(segments),
                                                   _dptr(seg_of, torch.int32, "seg_of"),
                                                   _dptr(cell_of, torch.int64, "cell_of"), n,
                                                   _dptr(out, odt, "out"),
                                                   _dptr(out_offset, torch.int64, "out_offset"), _stream(stream))
    _check(st, "coffee_assemble_batch_packed_noalloc")
    return out, out_offset


def coffee_check_geometry(cell, coords, cell_to_vertex, stream=None) -> int:
    """Smallest bad cell index (det J <= 0 or non-finite), or -1."""
    _check_mesh(CELLS[cell], coords, cell_to_vertex)
    fb = torch.empty(1, dtype=torch.int64, device=coords.device)
    st = _lib.coffee_check_geometry(CELLS[cell], _dptr(coords, torch.float64, "coords"), coords.shape[0],
                                    _dptr(cell_to_vertex, torch.int32, "cell_to_vertex"),
                                    cell_to_vertex.shape[0], fb.data_ptr(), _stream(stream))
    _check(st, "coffee_check_geometry")
    return int(fb.item())


def coffee_set_launch_options(grid_mult: int = 0):
    _lib.coffee_set_launch_options(int(grid_mult))


def coffee_set_variant(variant: int = -1):
    _lib.coffee_set_variant(int(variant))


def coffee_has_variant(form, cell, degree: int, field_degree: int, precision: str, variant: int) -> bool:
    return bool(_lib.coffee_has_variant(FORMS[form], CELLS[cell], degree, field_degree, PRECISIONS[precision],
                                        variant))


def coffee_load_tuning(path: str | None):
    _check(_lib.coffee_load_tuning(None if path is None else path.encode()), "coffee_load_tuning")


def coffee_shutdown():
    _lib.coffee_shutdown()
