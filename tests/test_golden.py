"""Closed-form fixtures (tests/golden/closed_forms.txt) against the oracle and
against the library's host tabulation."""
import ast
import math
import os

import numpy as np
import pytest

from paper_1407_0904_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")


def _eval(expr: str) -> float:
    """Exact-expression evaluator: numbers, + - * /, unary minus, sqrt()."""
    def ev(n):
        if isinstance(n, ast.Expression):
            return ev(n.body)
        if isinstance(n, ast.Constant) and isinstance(n.value, (int, float)):
            return float(n.value)
        if isinstance(n, ast.UnaryOp) and isinstance(n.op, ast.USub):
            return -ev(n.operand)
        if isinstance(n, ast.BinOp) and isinstance(n.op, (ast.Add, ast.Sub, ast.Mult, ast.Div)):
            a, b = ev(n.left), ev(n.right)
            return {ast.Add: a + b, ast.Sub: a - b, ast.Mult: a * b, ast.Div: a / b}[type(n.op)]
        if isinstance(n, ast.Call) and isinstance(n.func, ast.Name) and n.func.id == "sqrt" and len(n.args) == 1:
            return math.sqrt(ev(n.args[0]))
        raise ValueError(f"unsupported expression {expr!r}")
    return ev(ast.parse(expr.strip(), mode="eval"))


def golden():
    out = {}
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        name, _src, vals = (s.strip() for s in line.split(" | "))
        out[name] = np.array([_eval(v) for v in vals.split(",")])
    return out


G = golden()


def test_fixture_parses():
    assert len(G) == 18
    assert abs(G["gj_a1_m2_w"].sum() - 0.5) < 1e-15


@pytest.mark.parametrize("alpha,m", [(0, 1), (0, 2), (1, 1), (1, 2), (2, 1)])
def test_gauss_jacobi_closed_forms(oracle, alpha, m):
    x, w = oracle.gauss_jacobi(m, alpha)
    order = np.argsort(x)
    np.testing.assert_allclose(x[order], G[f"gj_a{alpha}_m{m}_x"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w[order], G[f"gj_a{alpha}_m{m}_w"], rtol=0, atol=1e-15)


@pytest.mark.parametrize("d,name", [(2, "tri"), (3, "tet")])
def test_one_point_rules(oracle, d, name):
    X, W, _, _ = oracle.tabulate(d, 1, 1)
    np.testing.assert_allclose(X.reshape(-1), G[f"{name}_q1_x"], atol=1e-15)
    np.testing.assert_allclose(W, G[f"{name}_q1_w"], atol=1e-15)


@pytest.mark.parametrize("d,name", [(2, "tri"), (3, "tet")])
def test_library_tabulate_one_point_rules(d, name):
    from paper_1407_0904_amd import coffee
    X, W, _, _ = coffee.coffee_tabulate(d, 1, 1)
    np.testing.assert_allclose(X.reshape(-1), G[f"{name}_q1_x"], atol=1e-15)
    np.testing.assert_allclose(W, G[f"{name}_q1_w"], atol=1e-15)


@pytest.mark.parametrize("d,name", [(2, "tri"), (3, "tet")])
def test_reference_p1_matrices(oracle, d, name):
    verts = np.vstack([np.zeros(d), np.eye(d)])
    mesh = I.single_cell_mesh(d, verts)
    n = d + 1
    mass = oracle.assemble("mass", mesh, 1)[0]
    np.testing.assert_allclose(mass.reshape(-1), G[f"{name}_p1_mass"], rtol=1e-14, atol=1e-16)
    zero = I.Field(values=np.zeros((n, 1)), cell_to_dof=np.arange(n, dtype=np.int32)[None], degree=1, ncomp=1)
    stiff = oracle.assemble("helmholtz", mesh, 1, fields=[zero])[0]
    np.testing.assert_allclose(stiff.reshape(-1), G[f"{name}_p1_stiff"], rtol=1e-14, atol=1e-15)
