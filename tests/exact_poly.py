"""Exact integration of polynomial integrands on one simplex (test helper).

An independent route to element tensors, used to pin the oracle: every basis
function, coefficient and integrand is a polynomial in the reference
coordinates, held as a dense coefficient array, multiplied by convolution and
integrated with the exact simplex moments
    int_{ref} X^i Y^j (Z^k) = i! j! (k!) / (i + j (+ k) + d)!.
The Lagrange basis comes from inverting the monomial Vandermonde matrix at
the nodes, a different construction from the oracle's product formula.
Results are exact up to float64 rounding of the coefficients.
"""
from __future__ import annotations

from itertools import product
from math import factorial

import numpy as np
from scipy.signal import convolve

TRI_EDGES = ((1, 2), (0, 2), (0, 1))
TET_EDGES = ((2, 3), (1, 3), (1, 2), (0, 3), (0, 2), (0, 1))


def ref_vertices(d):
    v = np.zeros((d + 1, d))
    v[1:] = np.eye(d)
    return v


def lagrange_nodes(d: int, p: int) -> np.ndarray:
    """Reference coordinates of the degree-p nodes: vertices, edges (lower to
    higher vertex), faces (face f opposite vertex f, (i, j) with j outer),
    interior (k outer, then j, then i)."""
    V = ref_vertices(d)
    if p == 0:
        return V.mean(axis=0, keepdims=True)
    pts = [V[i] for i in range(d + 1)]
    for (a, b) in (TRI_EDGES if d == 2 else TET_EDGES):
        for k in range(1, p):
            pts.append(V[a] + k / p * (V[b] - V[a]))
    faces = [(0, 1, 2)] if d == 2 else [tuple(v for v in range(4) if v != f) for f in range(4)]
    for (a, b, c) in faces:
        for j in range(1, p):
            for i in range(1, p - j):
                pts.append(V[a] + i / p * (V[b] - V[a]) + j / p * (V[c] - V[a]))
    if d == 3:
        for k in range(1, p):
            for j in range(1, p - k):
                for i in range(1, p - j - k):
                    pts.append(V[0] + i / p * (V[1] - V[0]) + j / p * (V[2] - V[0]) + k / p * (V[3] - V[0]))
    return np.array(pts)


def monomials(d: int, p: int):
    return [e for e in product(range(p + 1), repeat=d) if sum(e) <= p]


class Poly:
    """Dense polynomial in d reference variables."""

    def __init__(self, c: np.ndarray):
        self.c = np.asarray(c, dtype=np.float64)

    @property
    def d(self):
        return self.c.ndim

    @staticmethod
    def const(d, v):
        return Poly(np.full((1,) * d, float(v)))

    def __add__(self, o):
        if not isinstance(o, Poly):
            o = Poly.const(self.d, o)
        shape = tuple(max(a, b) for a, b in zip(self.c.shape, o.c.shape))
        r = np.zeros(shape)
        r[tuple(slice(0, s) for s in self.c.shape)] += self.c
        r[tuple(slice(0, s) for s in o.c.shape)] += o.c
        return Poly(r)

    __radd__ = __add__

    def __neg__(self):
        return Poly(-self.c)

    def __sub__(self, o):
        return self + (-o if isinstance(o, Poly) else -o)

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        if isinstance(o, Poly):
            return Poly(convolve(self.c, o.c, method="direct"))
        return Poly(self.c * float(o))

    __rmul__ = __mul__

    def deriv(self, j):
        c = self.c
        n = c.shape[j]
        if n == 1:
            return Poly(np.zeros((1,) * self.d))
        idx = [slice(None)] * self.d
        idx[j] = slice(1, n)
        r = c[tuple(idx)].copy()
        shape = [1] * self.d
        shape[j] = n - 1
        r *= np.arange(1, n).reshape(shape)
        return Poly(r)

    def integrate(self) -> float:
        """Integral over the reference simplex."""
        d = self.d
        tot = 0.0
        for e in zip(*np.nonzero(self.c)):
            num = 1
            for k in e:
                num *= factorial(int(k))
            tot += self.c[e] * num / factorial(int(sum(e)) + d)
        return float(tot)

    def __call__(self, X):
        X = np.atleast_2d(X)
        out = np.zeros(X.shape[0])
        for e in zip(*np.nonzero(self.c)):
            out += self.c[e] * np.prod(X ** np.array(e), axis=1)
        return out


def _exact_inverse_vandermonde(d: int, p: int) -> np.ndarray:
    """Inverse of the monomial Vandermonde matrix at the (rational) nodes,
    computed in exact rational arithmetic and rounded once."""
    from fractions import Fraction
    V0 = ref_vertices(d)
    nodes = lagrange_nodes(d, p)
    # nodes are multiples of 1/p: recover them exactly
    nodes_q = [[Fraction(int(round(c * p)), p) for c in x] for x in nodes]
    assert np.allclose(np.array(nodes_q, dtype=float), nodes)
    mons = monomials(d, p)
    n = len(mons)
    A = [[_fpow(x, m) for m in mons] + [Fraction(int(i == r)) for i in range(n)] for r, x in enumerate(nodes_q)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [a / pv for a in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    return np.array([[float(A[r][n + c]) for c in range(n)] for r in range(n)])


def _fpow(x, m):
    from fractions import Fraction
    out = Fraction(1)
    for xi, k in zip(x, m):
        out *= xi ** k
    return out


def lagrange_basis(d: int, p: int) -> list[Poly]:
    """Nodal basis by inverting the monomial Vandermonde matrix."""
    Cm = _exact_inverse_vandermonde(d, p)  # column a: coefficients of phi_a
    mons = monomials(d, p)
    nodes = lagrange_nodes(d, p)
    basis = []
    for a in range(len(nodes)):
        c = np.zeros((p + 1,) * d)
        for k, m in enumerate(mons):
            c[m] = Cm[k, a]
        basis.append(Poly(c))
    return basis


class Cell:
    """Affine cell: reference polynomials, physical gradients, exact integrals."""

    def __init__(self, verts):
        verts = np.asarray(verts, dtype=np.float64)
        self.d = d = verts.shape[1]
        J = (verts[1:] - verts[0]).T  # column j = x_{j+1} - x_0
        self.J = J
        self.K = np.linalg.inv(J)
        self.adet = abs(np.linalg.det(J))

    def grad(self, f: Poly) -> list[Poly]:
        """Physical gradient: d/dx_i = sum_alpha K[alpha, i] d/dX_alpha."""
        ref = [f.deriv(a) for a in range(self.d)]
        return [sum((ref[a] * self.K[a, i] for a in range(self.d)), Poly.const(self.d, 0.0))
                for i in range(self.d)]

    def integral(self, f: Poly) -> float:
        return self.adet * f.integrate()


def field_poly(d: int, degree: int, values: np.ndarray) -> list[Poly]:
    """Polynomial components of a field with local dof values [nloc, ncomp]."""
    values = np.asarray(values, dtype=np.float64).reshape(-1, values.shape[-1] if np.ndim(values) > 1 else 1)
    basis = lagrange_basis(d, degree) if degree > 0 else [Poly.const(d, 1.0)]
    out = []
    for c in range(values.shape[1]):
        acc = Poly.const(d, 0.0)
        for r, b in enumerate(basis):
            acc = acc + b * values[r, c]
        out.append(acc)
    return out


def mass(cell: Cell, p: int, f: Poly | None = None, stiff: bool = False) -> np.ndarray:
    d = cell.d
    B = lagrange_basis(d, p)
    G = [cell.grad(b) for b in B] if stiff else None
    n = len(B)
    A = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            integrand = B[a] * B[b]
            if f is not None:
                integrand = integrand * f
            if stiff:
                for i in range(d):
                    integrand = integrand + G[a][i] * G[b][i]
            A[a, b] = cell.integral(integrand)
    return A


def elasticity(cell: Cell, p: int, mu: Poly, lm: Poly) -> np.ndarray:
    """Index form: mu (delta_cc' grad a . grad b + d_c' phi_a d_c phi_b) + lambda d_c phi_a d_c' phi_b."""
    d = cell.d
    B = lagrange_basis(d, p)
    G = [cell.grad(b) for b in B]
    n = len(B)
    A = np.zeros((d * n, d * n))
    for c1 in range(d):
        for a in range(n):
            for c2 in range(d):
                for b in range(n):
                    t = mu * (G[a][c2] * G[b][c1]) + lm * (G[a][c1] * G[b][c2])
                    if c1 == c2:
                        for i in range(d):
                            t = t + mu * (G[a][i] * G[b][i])
                    A[c1 * n + a, c2 * n + b] = cell.integral(t)
    return A


def burgers(cell: Cell, p: int, w: list[Poly], nu: float, inv_dt: float) -> np.ndarray:
    d = cell.d
    B = lagrange_basis(d, p)
    G = [cell.grad(b) for b in B]
    gw = [cell.grad(wc) for wc in w]  # gw[c][i] = d_i w_c
    n = len(B)
    A = np.zeros((d * n, d * n))
    for c1 in range(d):
        for a in range(n):
            for c2 in range(d):
                for b in range(n):
                    # ((du . grad) w) . v with du = phi_b e_c2, v = phi_a e_c1
                    t = B[b] * gw[c1][c2] * B[a]
                    if c1 == c2:
                        adv = sum((w[j] * G[b][j] for j in range(d)), Poly.const(d, 0.0))
                        t = t + adv * B[a] + B[a] * B[b] * inv_dt
                        for i in range(d):
                            t = t + G[a][i] * G[b][i] * nu
                    A[c1 * n + a, c2 * n + b] = cell.integral(t)
    return A


def svk(cell: Cell, p: int, u: list[Poly], mu: float, lm: float):
    """(energy, residual [d n], jacobian [d n, d n]) of St Venant-Kirchhoff."""
    d = cell.d
    B = lagrange_basis(d, p)
    G = [cell.grad(b) for b in B]
    n = len(B)
    gu = [cell.grad(uc) for uc in u]  # gu[i][j] = d_j u_i
    F = [[gu[i][j] + (1.0 if i == j else 0.0) for j in range(d)] for i in range(d)]
    E = [[(sum((F[k][i] * F[k][j] for k in range(d)), Poly.const(d, 0.0)) - (1.0 if i == j else 0.0)) * 0.5
          for j in range(d)] for i in range(d)]
    trE = sum((E[i][i] for i in range(d)), Poly.const(d, 0.0))
    S = [[E[i][j] * (2 * mu) + (trE * lm if i == j else 0.0) for j in range(d)] for i in range(d)]
    P = [[sum((F[i][k] * S[k][j] for k in range(d)), Poly.const(d, 0.0)) for j in range(d)] for i in range(d)]
    EE = sum((E[i][j] * E[i][j] for i in range(d) for j in range(d)), Poly.const(d, 0.0))
    energy = cell.integral(trE * trE * (0.5 * lm) + EE * mu)
    res = np.zeros(d * n)
    for c in range(d):
        for a in range(n):
            res[c * n + a] = cell.integral(sum((P[c][j] * G[a][j] for j in range(d)), Poly.const(d, 0.0)))
    jac = np.zeros((d * n, d * n))
    for c2 in range(d):
        for b in range(n):
            H = [[G[b][j] if i == c2 else Poly.const(d, 0.0) for j in range(d)] for i in range(d)]
            dE = [[sum((H[k][i] * F[k][j] + F[k][i] * H[k][j] for k in range(d)), Poly.const(d, 0.0)) * 0.5
                   for j in range(d)] for i in range(d)]
            trdE = sum((dE[i][i] for i in range(d)), Poly.const(d, 0.0))
            dS = [[dE[i][j] * (2 * mu) + (trdE * lm if i == j else 0.0) for j in range(d)] for i in range(d)]
            dP = [[sum((H[i][k] * S[k][j] + F[i][k] * dS[k][j] for k in range(d)), Poly.const(d, 0.0))
                   for j in range(d)] for i in range(d)]
            for c1 in range(d):
                for a in range(n):
                    jac[c1 * n + a, c2 * n + b] = cell.integral(
                        sum((dP[c1][j] * G[a][j] for j in range(d)), Poly.const(d, 0.0)))
    return energy, res, jac
