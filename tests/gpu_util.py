"""Helpers for the GPU parity tests: move seeded workloads to the device, run
the HIP path through the binding, compare with the oracle per cell."""
from __future__ import annotations

import numpy as np
import torch

# Parity bars (per-cell normwise relative error, max over cells):
#   FP64    1e-12 (both sides compute the same quadrature sum in FP64)
#   FP32    1e-5
#   BF16X3  TOL_BF16: three bf16 products with FP32 accumulation lose about
#           3 * 2^-16 of sum_k |G_k R_k| per entry; cancellation between the
#           terms of an entry raises the error relative to the entry norm.
TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 2e-4}


def dev():
    return torch.device("cuda:0")


def to_dev(mesh, fields):
    from paper_1407_0904_amd.coffee import DeviceField
    coords = torch.as_tensor(mesh.coords, device=dev())
    c2v = torch.as_tensor(mesh.cells, device=dev())
    dfs = [DeviceField.from_host(f, dev()) for f in fields]
    return coords, c2v, dfs


def cell_rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max over cells of max_ij |got - ref| / max_ij |ref|."""
    E = ref.shape[0]
    g = got.reshape(E, -1).astype(np.float64)
    r = ref.reshape(E, -1)
    num = np.max(np.abs(g - r), axis=1)
    den = np.maximum(np.max(np.abs(r), axis=1), 1e-300)
    return float(np.max(num / den)) if E else 0.0


def assemble_gpu(form, mesh, degree, fields, constants=(), quad_degree=-1, precision="fp64"):
    from paper_1407_0904_amd import coffee
    coords, c2v, dfs = to_dev(mesh, fields)
    out = coffee.coffee_assemble(form, mesh.cell, degree, coords, c2v, coeffs=dfs, constants=constants,
                                 quad_degree=quad_degree, precision=precision)
    torch.cuda.synchronize()
    return out
