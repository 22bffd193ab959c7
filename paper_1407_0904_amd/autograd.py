"""torch.autograd Functions over the C ABI.

Each functional is a sum of per-cell values whose gradient with respect to
the vertex coordinates and the coefficient values comes from one reverse
pass of the assembly (coffee_assemble_adjoint):

BilinearActionFn:  S = sum_e lam_e^T A_e(coords, coefficients) u_e for a
                   bilinear form (mass, Helmholtz, elasticity, Burgers);
EnergyFn:          Pi = sum_e Pi_e(coords, u), the St Venant-Kirchhoff
                   energy, differentiable in the coordinates and in the
                   displacement (dPi/du is the assembled residual);
ResidualActionFn:  S = sum_e lam_e^T b_e(coords, u) for the SVK residual
                   (dS/du = sum_e A_e lam_e with A_e the SVK Jacobian).
Assemble:          the element tensors (forward only).

lam and u of the bilinear action, and lam of the residual action, are data:
their gradients are not provided. The forward pass runs the reverse pass
only when some input needs a gradient (it then keeps the gradients for
backward); otherwise it computes the per-cell values alone.
"""
from __future__ import annotations

import torch

from . import coffee


class _AdjointFunctional(torch.autograd.Function):
    """sum_e S_e for the functional described by `spec`, differentiable in
    coords and in the values of the coefficient fields."""

    @staticmethod
    def forward(ctx, spec, coords, *values):
        fields = [coffee.DeviceField(v.detach().contiguous(), m, d, nc)
                  for v, m, d, nc in zip(values, spec["maps"], spec["degrees"], spec["ncomps"])]
        c2v = spec["cell_to_vertex"]
        cell_value = torch.empty(c2v.shape[0], dtype=torch.float64, device=coords.device)
        need = any(ctx.needs_input_grad[1:])
        gc, gf = coffee.coffee_assemble_adjoint(
            spec["form"], spec["cell"], spec["degree"], coords.detach().contiguous(), c2v, coeffs=fields,
            constants=spec["constants"], lam=spec["lam"], u=spec["u"], seed=1.0, cell_value=cell_value,
            deterministic=spec["deterministic"], quad_degree=spec["quad_degree"], grads=need)
        if need:
            ctx.save_for_backward(gc, *gf)
        return cell_value.sum()

    @staticmethod
    def backward(ctx, grad_out):
        gc, *gf = ctx.saved_tensors
        return (None, gc * grad_out, *[g * grad_out for g in gf])


class BilinearActionFn(_AdjointFunctional):
    """S = sum_e lam_e^T A_e u_e of a bilinear form (mass, Helmholtz, elasticity, Burgers)."""


class EnergyFn(_AdjointFunctional):
    """Pi = sum_e Pi_e(coords, u), the St Venant-Kirchhoff energy."""


class ResidualActionFn(_AdjointFunctional):
    """S = sum_e lam_e^T b_e(coords, u), b the St Venant-Kirchhoff residual."""


_FN = {"svk_energy": EnergyFn, "svk_residual": ResidualActionFn}


def _apply(form, cell, degree, coords, cell_to_vertex, fields, constants, lam, u, quad_degree, deterministic):
    spec = {"form": form, "cell": cell, "degree": degree, "quad_degree": quad_degree,
            "constants": tuple(constants), "maps": [f.cell_to_dof for f in fields],
            "degrees": [f.degree for f in fields], "ncomps": [f.ncomp for f in fields],
            "lam": None if lam is None else lam.detach().contiguous(),
            "u": None if u is None else u.detach().contiguous(),
            "cell_to_vertex": cell_to_vertex, "deterministic": bool(deterministic)}
    return _FN.get(form, BilinearActionFn).apply(spec, coords, *[f.values for f in fields])


def bilinear_action(form: str, cell, degree: int, coords: torch.Tensor, cell_to_vertex: torch.Tensor,
                    fields=(), constants=(), lam=None, u=None, quad_degree: int = -1,
                    deterministic: bool = False) -> torch.Tensor:
    """Differentiable S = sum_e lam_e^T A_e u_e; `fields` are DeviceFields whose
    `values` may require grad."""
    if lam is None or u is None:
        raise ValueError("lam and u are required")
    return _apply(form, cell, degree, coords, cell_to_vertex, fields, constants, lam, u, quad_degree, deterministic)


def svk_energy(cell, degree: int, coords: torch.Tensor, cell_to_vertex: torch.Tensor, u, constants=(),
               quad_degree: int = -1, deterministic: bool = False) -> torch.Tensor:
    """Differentiable St Venant-Kirchhoff energy Pi(coords, u); `u` is a
    DeviceField (ncomp = d) whose values may require grad."""
    return _apply("svk_energy", cell, degree, coords, cell_to_vertex, [u], constants, None, None, quad_degree,
                  deterministic)


def svk_residual_action(cell, degree: int, coords: torch.Tensor, cell_to_vertex: torch.Tensor, u, lam,
                        constants=(), quad_degree: int = -1, deterministic: bool = False) -> torch.Tensor:
    """Differentiable S = sum_e lam_e^T b_e(coords, u) for the SVK residual b."""
    if lam is None:
        raise ValueError("lam is required")
    return _apply("svk_residual", cell, degree, coords, cell_to_vertex, [u], constants, lam, None, quad_degree,
                  deterministic)


BilinearAction = BilinearActionFn


class Assemble(torch.autograd.Function):
    """Element tensors (forward only; differentiate a functional instead)."""

    @staticmethod
    def forward(ctx, coords, form, cell, degree, cell_to_vertex, fields, constants, quad_degree, precision):
        return coffee.coffee_assemble(form, cell, degree, coords, cell_to_vertex, coeffs=fields,
                                      constants=constants, quad_degree=quad_degree, precision=precision)

    @staticmethod
    def backward(ctx, grad_out):
        raise RuntimeError("Assemble is forward-only: differentiate a functional (bilinear_action, svk_energy)")
