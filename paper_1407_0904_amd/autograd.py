"""torch.autograd Functions over the C ABI.

BilinearAction:  S = sum_e lam_e^T A_e(coords, coefficients) u_e, differentiable
                 with respect to the vertex coordinates and the coefficient
                 values (coffee_assemble_adjoint). lam and u are data: their
                 gradients are not provided.
Assemble:        the element tensors (forward only).
"""
from __future__ import annotations

import torch

from . import coffee


class BilinearAction(torch.autograd.Function):
    """S = sum_e lam_e^T A_e u_e for a bilinear form."""

    @staticmethod
    def forward(ctx, coords, *args):
        (form, cell, degree, quad_degree, constants, maps, degrees, ncomps, lam, u, c2v, deterministic) = args[-12:]
        values = args[:-12]
        fields = [coffee.DeviceField(v.detach().contiguous(), m, d, nc)
                  for v, m, d, nc in zip(values, maps, degrees, ncomps)]
        cell_value = torch.empty(c2v.shape[0], dtype=torch.float64, device=coords.device)
        # one reverse pass gives S_e and the gradients; keep the gradients for backward
        gc, gf = coffee.coffee_assemble_adjoint(form, cell, degree, coords.detach().contiguous(), c2v,
                                                coeffs=fields, constants=constants, lam=lam, u=u, seed=1.0,
                                                cell_value=cell_value, deterministic=deterministic,
                                                quad_degree=quad_degree)
        ctx.save_for_backward(gc, *gf)
        return cell_value.sum()

    @staticmethod
    def backward(ctx, grad_out):
        gc, *gf = ctx.saved_tensors
        grads = [gc * grad_out] + [g * grad_out for g in gf]
        return tuple(grads) + (None,) * 12


def bilinear_action(form: str, cell, degree: int, coords: torch.Tensor, cell_to_vertex: torch.Tensor,
                    fields=(), constants=(), lam=None, u=None, quad_degree: int = -1,
                    deterministic: bool = False) -> torch.Tensor:
    """Differentiable S = sum_e lam_e^T A_e u_e; `fields` are DeviceFields whose
    `values` may require grad."""
    if lam is None or u is None:
        raise ValueError("lam and u are required")
    vals = [f.values for f in fields]
    return BilinearAction.apply(coords, *vals, form, cell, degree, quad_degree, tuple(constants),
                                [f.cell_to_dof for f in fields], [f.degree for f in fields],
                                [f.ncomp for f in fields], lam.contiguous(), u.contiguous(), cell_to_vertex,
                                deterministic)


class Assemble(torch.autograd.Function):
    """Element tensors (forward only; use BilinearAction for derivatives)."""

    @staticmethod
    def forward(ctx, coords, form, cell, degree, cell_to_vertex, fields, constants, quad_degree, precision):
        return coffee.coffee_assemble(form, cell, degree, coords, cell_to_vertex, coeffs=fields,
                                      constants=constants, quad_degree=quad_degree, precision=precision)

    @staticmethod
    def backward(ctx, grad_out):
        raise RuntimeError("Assemble is forward-only: differentiate a functional with bilinear_action")
