"""Pins of the oracle's diffusion form and prism cells.

The paper's benchmarks include a diffusion operator (Helmholtz without the
basis-value array, with a few extra constants) and prism cells (section 5.2).
Each test below fixes a result by something other than the oracle's own code:
exact polynomial integrals (exact_poly, a Vandermonde basis), Kronecker
closed forms of tensor-product elements on right prisms, a tensor
Gauss-Legendre rule from scipy on the Duffy-collapsed triangle, and
invariants that hold on warped (non-affine) prisms.
"""
from math import factorial

import numpy as np
import pytest
from scipy.special import roots_legendre

import exact_poly as X
from paper_1407_0904_amd import inputs as I

PRISM = 6


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def rational_cell(d, rng):
    while True:
        v = rng.integers(-8, 9, size=(d + 1, d)) / 8.0
        det = np.linalg.det((v[1:] - v[0]).T)
        if abs(det) > 0.05:
            if det < 0:
                v[[-2, -1]] = v[[-1, -2]]
            return v


# ---------------------------------------------------------------- diffusion on simplices

@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_diffusion_exact(oracle, d, p):
    """kappa dt times the exact stiffness integral (exact_poly), at degree 2p."""
    rng = np.random.default_rng(40 + 10 * d + p)
    v = rational_cell(d, rng)
    cell = X.Cell(v)
    stiff = X.mass(cell, p, stiff=True) - X.mass(cell, p)
    got = oracle.assemble("diffusion", I.single_cell_mesh(d, v), p, constants=[0.7, 1.9])[0]
    assert rel(got, 0.7 * 1.9 * stiff) < 1e-12


def test_diffusion_p1_closed_form_and_patch(oracle):
    """P1 triangle: |T| G G^T (G from a linear solve); coordinate functions:
    x_i^T A x_j = delta_ij |T| on any cell."""
    v = np.array([[0.2, 0.1], [1.3, 0.4], [0.5, 1.2]])
    Mx = np.hstack([np.ones((3, 1)), v])
    G = np.linalg.solve(Mx, np.eye(3))[1:, :].T
    area = 0.5 * abs(np.linalg.det((v[1:] - v[0]).T))
    A = oracle.assemble("diffusion", I.single_cell_mesh(2, v), 1)[0]
    np.testing.assert_allclose(A, area * G @ G.T, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(v.T @ A @ v, area * np.eye(2), rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- prism rule and basis

def interval_nodes(p):
    return np.array([0.0, 1.0] + [k / p for k in range(1, p)])


def prism_nodes(p):
    """Reference nodes (a, b) -> a (p+1) + b: triangle nodes (exact_poly's
    order) times interval nodes 0, 1, interior."""
    tri = X.lagrange_nodes(2, p)
    z = interval_nodes(p)
    return np.array([[t[0], t[1], zz] for t in tri for zz in z])


@pytest.mark.parametrize("q", range(0, 9))
def test_prism_rule_exact_on_monomials(oracle, q):
    """int X^a Y^b Z^c = a! b! / (a+b+2)! / (c+1) for a + b <= q, c <= q."""
    Xq, W, _, _ = oracle.tabulate(PRISM, 1, q)
    m = (q + 2) // 2
    assert W.shape[0] == m ** 3 and np.all(W > 0)
    assert abs(W.sum() - 0.5) < 1e-15
    assert np.all(Xq[:, 0] + Xq[:, 1] <= 1 + 1e-15) and np.all((Xq[:, 2] > 0) & (Xq[:, 2] < 1))
    for a in range(q + 1):
        for b in range(q + 1 - a):
            for c in range(q + 1):
                exact = factorial(a) * factorial(b) / factorial(a + b + 2) / (c + 1)
                got = np.sum(W * Xq[:, 0] ** a * Xq[:, 1] ** b * Xq[:, 2] ** c)
                assert abs(got - exact) < 1e-14 * max(1.0, exact), (a, b, c)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_prism_basis_nodal(oracle, p):
    """phi_i(node_j) = delta_ij at the tensor-product nodes; partition of unity;
    reference gradients sum to zero."""
    nodes = prism_nodes(p)
    phi, dphi = oracle.basis_at(PRISM, p, nodes)
    np.testing.assert_allclose(phi, np.eye(nodes.shape[0]), atol=1e-12)
    rng = np.random.default_rng(p)
    pts = np.column_stack([rng.uniform(0, 0.5, 20), rng.uniform(0, 0.5, 20), rng.uniform(0, 1, 20)])
    phi, dphi = oracle.basis_at(PRISM, p, pts)
    np.testing.assert_allclose(phi.sum(axis=1), 1.0, atol=1e-13)
    np.testing.assert_allclose(dphi.sum(axis=2), 0.0, atol=1e-11)


# ---------------------------------------------------------------- independent prism integration

def interval_basis(p, z):
    """Degree-p Lagrange basis on [0,1] at z (Vandermonde solve) and its derivative."""
    nodes = interval_nodes(p)
    V = np.vander(nodes, p + 1, increasing=True)
    C = np.linalg.inv(V)                     # column b: monomial coefficients of l_b
    pw = np.vander(np.atleast_1d(z), p + 1, increasing=True)
    dpw = np.zeros_like(pw)
    dpw[:, 1:] = pw[:, :-1] * np.arange(1, p + 1)
    return pw @ C, dpw @ C


def prism_basis_indep(p, pts):
    """Tensor-product basis from exact_poly's triangle basis and interval_basis."""
    tri = X.lagrange_basis(2, p)
    l, dl = interval_basis(p, pts[:, 2])
    nt = len(tri)
    phi = np.zeros((pts.shape[0], nt * (p + 1)))
    dphi = np.zeros((3, pts.shape[0], nt * (p + 1)))
    for a, t in enumerate(tri):
        tv, tx, ty = t(pts[:, :2]), t.deriv(0)(pts[:, :2]), t.deriv(1)(pts[:, :2])
        for b in range(p + 1):
            i = a * (p + 1) + b
            phi[:, i] = tv * l[:, b]
            dphi[0, :, i] = tx * l[:, b]
            dphi[1, :, i] = ty * l[:, b]
            dphi[2, :, i] = tv * dl[:, b]
    return phi, dphi


def geometry_basis(pts):
    """Degree-1 prism basis written out: lambda_t(X, Y) l_z(Z)."""
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    lam = [1 - x - y, x, y]
    dlam = [(-1.0, -1.0), (1.0, 0.0), (0.0, 1.0)]
    l = [1 - z, z]
    dl = [-1.0, 1.0]
    psi = np.zeros((pts.shape[0], 6))
    dpsi = np.zeros((3, pts.shape[0], 6))
    for t in range(3):
        for s in range(2):
            i = 2 * t + s
            psi[:, i] = lam[t] * l[s]
            dpsi[0, :, i] = dlam[t][0] * l[s]
            dpsi[1, :, i] = dlam[t][1] * l[s]
            dpsi[2, :, i] = lam[t] * dl[s]
    return psi, dpsi


def gl_prism_rule(m):
    """Tensor Gauss-Legendre on [0,1]^3 through X = u, Y = (1-u) v (Duffy
    factor 1 - u in the weight), Z = w: exact for polynomials of degree
    <= 2m - 2 in (X, Y) and <= 2m - 1 in Z."""
    x, w = roots_legendre(m)
    x = (x + 1) / 2
    w = w / 2
    U, V, Z = np.meshgrid(x, x, x, indexing="ij")
    WU, WV, WZ = np.meshgrid(w, w, w, indexing="ij")
    pts = np.column_stack([U.ravel(), ((1 - U) * V).ravel(), Z.ravel()])
    wts = (WU * WV * WZ * (1 - U)).ravel()
    return pts, wts


def indep_mass(xv, p, f=None, m=8):
    """int f phi_a phi_b |det J| on the prism with vertices xv [6, 3]."""
    pts, wts = gl_prism_rule(m)
    phi, _ = prism_basis_indep(p, pts)
    psi, dpsi = geometry_basis(pts)
    J = np.einsum("vi,aqv->qia", xv, dpsi)
    det = np.abs(np.linalg.det(J))
    fq = np.ones(pts.shape[0]) if f is None else psi @ f
    return np.einsum("q,qa,qb->ab", wts * det * fq, phi, phi)


def right_prism(rng):
    tri = np.array([[0.1, 0.2], [1.2, 0.3], [0.4, 1.1]]) + rng.uniform(-0.1, 0.1, (3, 2))
    z0, h = 0.3, 0.7
    xv = np.array([[tri[t, 0], tri[t, 1], z0 + s * h] for t in range(3) for s in range(2)])
    return tri, z0, h, xv


def warped_prism(rng):
    _, _, _, xv = right_prism(rng)
    return xv + rng.uniform(-0.08, 0.08, xv.shape)


def one_prism_mesh(xv):
    return I.Mesh(d=3, n=1, coords=np.ascontiguousarray(xv), cells=np.arange(6, dtype=np.int32)[None])


def test_p1_right_prism_kronecker(oracle):
    """Right prism T x [z0, z0+h]: M = M_T (x) M_I and K = K_T (x) M_I + M_T (x) K_I with
    M_T = |T|/12 (1 + delta), K_T = |T| G G^T, M_I = h/6 [[2,1],[1,2]], K_I = 1/h [[1,-1],[-1,1]]."""
    tri, z0, h, xv = right_prism(np.random.default_rng(3))
    area = 0.5 * abs(np.linalg.det((tri[1:] - tri[0]).T))
    G = np.linalg.solve(np.hstack([np.ones((3, 1)), tri]), np.eye(3))[1:, :].T
    MT, KT = area / 12 * (np.ones((3, 3)) + np.eye(3)), area * G @ G.T
    MI, KI = h / 6 * np.array([[2.0, 1.0], [1.0, 2.0]]), np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    M, K = np.kron(MT, MI), np.kron(KT, MI) + np.kron(MT, KI)
    mesh = one_prism_mesh(xv)
    np.testing.assert_allclose(oracle.assemble("mass", mesh, 1)[0], M, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(oracle.assemble("diffusion", mesh, 1, constants=[2.0, 0.25])[0], 0.5 * K,
                               rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(oracle.assemble("helmholtz", mesh, 1)[0], K + M, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("p", [2, 3])
def test_right_prism_kronecker_exact(oracle, p):
    """Degree p on a right prism: the exact triangle matrices (exact_poly) times
    the exact interval matrices (numpy polynomial integration)."""
    tri, z0, h, xv = right_prism(np.random.default_rng(10 + p))
    cell = X.Cell(tri)
    MT = X.mass(cell, p)
    KT = X.mass(cell, p, stiff=True) - MT
    nodes = interval_nodes(p)
    C = np.linalg.inv(np.vander(nodes, p + 1, increasing=True))
    polys = [np.polynomial.Polynomial(C[:, b]) for b in range(p + 1)]
    MI = np.array([[(a * b).integ()(1.0) * h for b in polys] for a in polys])
    KI = np.array([[(a.deriv() * b.deriv()).integ()(1.0) / h for b in polys] for a in polys])
    mesh = one_prism_mesh(xv)
    assert rel(oracle.assemble("mass", mesh, p)[0], np.kron(MT, MI)) < 1e-12
    assert rel(oracle.assemble("diffusion", mesh, p)[0], np.kron(KT, MI) + np.kron(MT, KI)) < 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_warped_prism_mass_exact(oracle, p):
    """On a warped prism the mass integrand f phi_a phi_b |det J| is a
    polynomial of degree <= 2p+2 in (X, Y) and 2p+3 in Z: at a rule of degree
    2p+3 the oracle is exact and equals an 8^3-point Gauss-Legendre integral
    with the basis and geometry built independently."""
    rng = np.random.default_rng(20 + p)
    xv = warped_prism(rng)
    f = rng.uniform(0.5, 1.5, 6)
    mesh = one_prism_mesh(xv)
    fld = I.Field(values=f.reshape(6, 1), cell_to_dof=np.arange(6, dtype=np.int32)[None], degree=1, ncomp=1)
    got = oracle.assemble("mass", mesh, p, quad_degree=2 * p + 3, fields=[fld])[0]
    assert rel(got, indep_mass(xv, p, f)) < 1e-12
    got1 = oracle.assemble("mass", mesh, p, quad_degree=2 * p + 2)[0]
    assert rel(got1, indep_mass(xv, p)) < 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_warped_prism_patch_test(oracle, p):
    """Coordinate functions lie in the prism space, so on a warped prism
    x_i^T A x_j = kappa dt delta_ij |cell| and A 1 = 0 exactly at any rule,
    with |cell| = sum of the mass matrix = an independent volume integral."""
    rng = np.random.default_rng(30 + p)
    xv = warped_prism(rng)
    mesh = one_prism_mesh(xv)
    A = oracle.assemble("diffusion", mesh, p, constants=[1.5, 2.0])[0]
    M = oracle.assemble("mass", mesh, p)[0]
    vol = indep_mass(xv, 1).sum()
    assert abs(M.sum() - vol) < 1e-13
    psi, _ = geometry_basis(prism_nodes(p))
    xn = psi @ xv                                  # coordinates of the degree-p nodes
    np.testing.assert_allclose(xn.T @ A @ xn, 3.0 * vol * np.eye(3), rtol=0, atol=1e-12)
    np.testing.assert_allclose(A.sum(axis=1), 0.0, atol=1e-12)
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-14)


def test_warped_prism_rigid_motion(oracle):
    """Rotating and translating a warped prism leaves every form unchanged."""
    rng = np.random.default_rng(5)
    xv = warped_prism(rng)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    moved = xv @ Q.T + np.array([0.3, -1.0, 2.0])
    for form in ("mass", "helmholtz", "diffusion"):
        a = oracle.assemble(form, one_prism_mesh(xv), 2)[0]
        b = oracle.assemble(form, one_prism_mesh(moved), 2)[0]
        assert rel(b, a) < 1e-12, form


@pytest.mark.parametrize("p", [1, 2])
def test_prism_mesh_volume(oracle, p):
    """The jittered extruded cube keeps its boundary: total mass = 1."""
    mesh = I.make_prism_mesh(4, 0.15, np.random.default_rng(0))
    M = oracle.assemble("mass", mesh, p)
    assert abs(M.sum() - 1.0) < 1e-12


def test_prism_global_p2_dofmap_consistent(oracle):
    """The P2 prism dof map puts every node at one place: assembling the
    coordinate functions from the map gives x_i^T A x_j = delta_ij on the unit cube."""
    import scipy.sparse as sp
    n = 3
    mesh = I.make_prism_mesh(n, 0.15, np.random.default_rng(1))
    c2d, nd = I.prism_p2_dofmap(n)
    A = oracle.assemble_global("diffusion", mesh, 2, c2d, nd)
    psi, _ = geometry_basis(prism_nodes(2))
    xn = np.zeros((nd, 3))
    for e in range(mesh.ncells):
        xn[c2d[e]] = psi @ mesh.coords[mesh.cells[e]]
    np.testing.assert_allclose(xn.T @ (A @ xn), np.eye(3), rtol=0, atol=1e-11)
    assert sp.issparse(A) and A.shape == (nd, nd)
