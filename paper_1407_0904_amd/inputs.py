"""Seeded synthetic inputs for local assembly: jittered simplex meshes, P2 dof
maps and coefficient draws.

This module is shared by the tests, the benchmark and the oracle checks. It
holds no finite-element arithmetic (no basis, quadrature, geometry or
integrand): only lattice indexing, connectivity and random numbers.

Mesh recipes (the paper measured on unstructured meshes that are not
available; these stand in for them):

* Triangles: the unit square cut into n x n squares, each split along its
  (0,0)-(1,1) diagonal into T0 = (a, b, d) and T1 = (a, d, c) with
  a = v(i,j), b = v(i+1,j), c = v(i,j+1), d = v(i+1,j+1). Both are
  counter-clockwise. Square s = i + n*j owns cells 2s and 2s+1.
* Tetrahedra: the unit cube cut into n^3 cubes, each split into 6 Kuhn
  tetrahedra, one per permutation pi of the axes (lexicographic order): the
  path v000 -> +e_pi0 -> +e_pi1 -> v111. For odd pi the last two vertices
  are swapped so that every tetrahedron is positively oriented.
* Prisms: the triangle mesh of the unit square extruded through n layers of
  height h. The prism over base triangle (a, b, c) in layer k has vertices
  (a,k), (a,k+1), (b,k), (b,k+1), (c,k), (c,k+1) (each base vertex at the
  bottom, then at the top), and cells run layer-fastest within the column of
  each base triangle (cell t n + k). Jitter moves interior vertices in all
  three directions, so the prisms are not affine images of the reference
  prism (their top and bottom triangles differ and their sides are warped).
* Vertex index v = i + (n+1) j (+ (n+1)^2 k) on triangles and tetrahedra; on
  prisms the vertices are numbered column by column as extruded meshes are,
  v = b (n+1) + k for base vertex b = i + (n+1) j and level k (the jitter is
  drawn in lattice order, then the vertices are renumbered).
* Jitter: every coordinate of every interior vertex moves by an independent
  draw from U[-r h, r h] (h = 1/n); boundary vertices do not move, so the
  domain measure stays exactly 1.
* Draw order from one numpy PCG64 generator: jitter for all V x d
  coordinates (boundary entries then zeroed), then coefficient values, then
  the adjoint weights lam_e, then u_e.

Local dof order used by the P2 dof map (the same order the library and the
oracle use): vertices, then edge midpoints with triangle edges
(1,2), (0,2), (0,1) and tetrahedron edges (2,3), (1,3), (1,2), (0,3), (0,2),
(0,1). Global P2 dofs are the points of the twice-refined lattice: vertex p
maps to R(2p) and edge pq to R(p+q), R(I,J,K) = I + (2n+1) J + (2n+1)^2 K.
On prisms the local dof (a, b) of a triangle dof a and an interval dof b is
a (p+1) + b, interval dofs ordered bottom, top, then interior (middle);
the global P2 prism dof of base dof R2 at refined level l is R2 + (2n+1)^2 l.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import permutations

import numpy as np

TRI_EDGES = ((1, 2), (0, 2), (0, 1))
TET_EDGES = ((2, 3), (1, 3), (1, 2), (0, 3), (0, 2), (0, 1))


def _lattice_index(ijk: np.ndarray, m: int) -> np.ndarray:
    """Index of integer lattice points (rows of ijk) on an m-per-side lattice."""
    idx = np.zeros(ijk.shape[0], dtype=np.int64)
    stride = 1
    for a in range(ijk.shape[1]):
        idx += ijk[:, a].astype(np.int64) * stride
        stride *= m
    return idx


def _lattice_points(n: int, d: int) -> np.ndarray:
    """Integer lattice coordinates of the (n+1)^d vertices in index order."""
    g = np.arange(n + 1)
    grids = np.meshgrid(*([g] * d), indexing="ij")
    # index v = i + (n+1) j + ...: the first axis varies fastest
    pts = np.stack([gr.transpose(tuple(reversed(range(d)))).reshape(-1) for gr in grids], axis=1)
    return pts


def square_cells(n: int) -> np.ndarray:
    """Connectivity [2 n^2, 3] int32 of the split unit square."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    i = i.reshape(-1)
    j = j.reshape(-1)  # square s = i + n j
    m = n + 1
    a = i + m * j
    b = a + 1
    c = a + m
    dd = a + m + 1
    cells = np.empty((2 * n * n, 3), dtype=np.int64)
    cells[0::2] = np.stack([a, b, dd], axis=1)
    cells[1::2] = np.stack([a, dd, c], axis=1)
    return cells.astype(np.int32)


def cube_cells(n: int) -> np.ndarray:
    """Connectivity [6 n^3, 4] int32 of the Kuhn-split unit cube."""
    m = n + 1
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = (i + m * j + m * m * k).reshape(-1).astype(np.int64)  # cube-major, i fastest
    step = np.array([1, m, m * m], dtype=np.int64)
    cells = np.empty((base.shape[0], 6, 4), dtype=np.int64)
    for t, perm in enumerate(permutations(range(3))):
        p1 = step[perm[0]]
        p2 = p1 + step[perm[1]]
        p3 = step.sum()
        inversions = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        verts = [0, p1, p2, p3]
        if inversions % 2 == 1:
            verts = [0, p1, p3, p2]
        for q in range(4):
            cells[:, t, q] = base + verts[q]
    return cells.reshape(-1, 4).astype(np.int32)


def lattice_coords(n: int, d: int) -> np.ndarray:
    return _lattice_points(n, d).astype(np.float64) / n


def jitter(coords: np.ndarray, n: int, r: float, rng: np.random.Generator) -> np.ndarray:
    """Move interior vertices by U[-r h, r h] per coordinate (h = 1/n)."""
    h = 1.0 / n
    V, d = coords.shape
    shift = rng.uniform(-r * h, r * h, size=(V, d))
    lat = np.rint(coords * n).astype(np.int64)
    boundary = np.any((lat == 0) | (lat == n), axis=1)
    shift[boundary] = 0.0
    return coords + shift


def p2_dofmap(cells: np.ndarray, n: int, d: int) -> tuple[np.ndarray, int]:
    """P2 cell->dof map [E, (d+1)(d+2)/2] int32 via the refined lattice."""
    m = n + 1
    mr = 2 * n + 1
    lat = _lattice_points(n, d)  # [V, d] integer coordinates
    edges = TRI_EDGES if d == 2 else TET_EDGES
    cv = cells.astype(np.int64)
    cols = [_lattice_index(2 * lat[cv[:, a]], mr) for a in range(d + 1)]
    for (a, b) in edges:
        cols.append(_lattice_index(lat[cv[:, a]] + lat[cv[:, b]], mr))
    c2d = np.stack(cols, axis=1)
    ndofs = mr ** d
    assert m ** d == lat.shape[0]
    return c2d.astype(np.int32), ndofs


@dataclass
class Mesh:
    """A jittered simplex mesh of the unit square (d=2) or cube (d=3)."""
    d: int
    n: int
    coords: np.ndarray  # [V, d] float64
    cells: np.ndarray   # [E, d+1] int32

    @property
    def nvert(self) -> int:
        return self.coords.shape[0]

    @property
    def ncells(self) -> int:
        return self.cells.shape[0]

    @property
    def cell(self) -> int:
        """Cell code of the library and the oracle: d for simplices, 6 for prisms."""
        return 6 if self.cells.shape[1] == 6 else self.d


def make_mesh(d: int, n: int, jitter_frac: float, rng: np.random.Generator) -> Mesh:
    coords = lattice_coords(n, d)
    coords = jitter(coords, n, jitter_frac, rng)
    cells = square_cells(n) if d == 2 else cube_cells(n)
    return Mesh(d=d, n=n, coords=np.ascontiguousarray(coords), cells=np.ascontiguousarray(cells))


def prism_cells(n: int) -> np.ndarray:
    """Connectivity [2 n^2 n, 6] int32 of the extruded split unit square,
    numbered column by column as extruded meshes are: cell (t, k) = t n + k
    for base triangle t and layer k, vertex (b, k) = b (n+1) + k for base
    vertex b and level k."""
    m = n + 1
    base = square_cells(n).astype(np.int64)              # [T, 3] base-lattice vertices
    k = np.arange(n, dtype=np.int64)
    bot = base[:, None, :] * m + k[None, :, None]        # [T, n, 3]
    top = bot + 1
    cells = np.stack([bot[..., 0], top[..., 0], bot[..., 1], top[..., 1], bot[..., 2], top[..., 2]], axis=-1)
    return cells.reshape(-1, 6).astype(np.int32)


def make_prism_mesh(n: int, jitter_frac: float, rng: np.random.Generator) -> Mesh:
    # jitter drawn in lattice order (i + m j + m^2 k), then the vertices are
    # renumbered column by column: new index b m + k holds lattice point b + m^2 k
    m = n + 1
    lat = jitter(lattice_coords(n, 3), n, jitter_frac, rng)
    b = np.arange(m * m, dtype=np.int64)
    k = np.arange(m, dtype=np.int64)
    coords = lat[(b[:, None] + (m * m) * k[None, :]).reshape(-1)]
    return Mesh(d=3, n=n, coords=np.ascontiguousarray(coords), cells=np.ascontiguousarray(prism_cells(n)))


def prism_p2_dofmap(n: int) -> tuple[np.ndarray, int]:
    """P2 prism cell->dof map [2 n^2 n, 18] int32 (local order a * 3 + b)."""
    mr = 2 * n + 1
    tri, _ = p2_dofmap(square_cells(n), n, 2)            # [T, 6] refined 2-D lattice indices
    tri = tri.astype(np.int64)
    k = np.arange(n, dtype=np.int64)
    levels = np.stack([2 * k, 2 * k + 2, 2 * k + 1], axis=1)   # [n, 3]: bottom, top, middle
    c2d = tri[:, None, :, None] + (mr * mr) * levels[None, :, None, :]  # [T, n, 6, 3]
    return c2d.reshape(-1, 18).astype(np.int32), mr ** 3


def n_prism_dofs(p: int) -> int:
    return (p + 1) * (p + 2) // 2 * (p + 1)


@dataclass
class Field:
    """A coefficient field: global values [ndofs, ncomp] plus a cell->dof map
    [E, nloc] (or cell-major local values [E, nloc, ncomp] with no map)."""
    values: np.ndarray
    cell_to_dof: np.ndarray | None
    degree: int
    ncomp: int


@dataclass
class Workload:
    name: str
    form: str          # mass | helmholtz | diffusion | elasticity | burgers | svk_energy | svk_residual | svk_jacobian
    mesh: Mesh
    degree: int
    quad_degree: int
    fields: list = field(default_factory=list)
    constants: list = field(default_factory=list)
    lam: np.ndarray | None = None
    u: np.ndarray | None = None


def n_scalar_dofs(d: int, p: int) -> int:
    if d == 2:
        return (p + 1) * (p + 2) // 2
    return (p + 1) * (p + 2) * (p + 3) // 6


def _p1_field(mesh: Mesh, values: np.ndarray, ncomp: int) -> Field:
    return Field(values=np.ascontiguousarray(values.reshape(mesh.nvert, ncomp)),
                 cell_to_dof=mesh.cells, degree=1, ncomp=ncomp)


def _p2_field(mesh: Mesh, draw, rng, ncomp: int) -> Field:
    c2d, ndofs = p2_dofmap(mesh.cells, mesh.n, mesh.d)
    vals = draw(rng, (ndofs, ncomp))
    return Field(values=np.ascontiguousarray(vals), cell_to_dof=c2d, degree=2, ncomp=ncomp)


def workload(name: str, n: int | None = None, seed: int | None = None) -> Workload:
    """Build one of the named synthetic workloads.

    helmholtz_p1_tri   Helmholtz P1 triangles, f P1 ~ U[0.5,1.5], jitter 20%, q=2 (n=64: 8192 cells)
    helmholtz_p2_tet   Helmholtz P2 tetrahedra, f P2 ~ U[0.5,1.5], jitter 10%, q=4 (n=64: 1,572,864 cells)
    elasticity_p2_tet  vector P2 elasticity, mu, lambda P1 ~ U[1,10], q=4, adjoint weights ~ N(0,1) (n=48)
    svk_p1_tet / svk_p2_tet  St Venant-Kirchhoff, u ~ N(0, 0.01) per component, mu = lambda = 1 (n=32)
    burgers_p1_tet / burgers_p2_tet  Burgers Jacobian, w ~ U[-1,1], nu = 1/dt = 1, q = 2p+1 (n=48)
    helmholtz_p1_prism  Helmholtz P1 on warped prisms, f P1 ~ U[0.5,1.5], jitter 10%, q=2 (n=64: 524,288 cells)
    diffusion_p2_prism  diffusion P2 on warped prisms, kappa = 1, dt = 1, jitter 10%, q=4 (n=64)
    diffusion_p3_prism  diffusion P3 on warped prisms, kappa = 1, dt = 1, jitter 10%, q=6 (n=32: 65,536 cells)
    mass_pK_tri / helmholtz_pK_tet etc. are built by mixed_batch().
    """
    defaults = {
        "helmholtz_p1_tri": 64, "helmholtz_p2_tet": 64, "elasticity_p2_tet": 48,
        "elasticity_p1_tet": 48, "svk_p1_tet": 32, "svk_p2_tet": 32,
        "burgers_p1_tet": 48, "burgers_p2_tet": 48, "helmholtz_p1_prism": 64, "diffusion_p2_prism": 64,
        "diffusion_p3_prism": 32,
    }
    if name not in defaults:
        raise KeyError(name)
    n = defaults[name] if n is None else n
    rng = np.random.default_rng(0 if seed is None else seed)
    unif = lambda lo, hi: (lambda g, shape: g.uniform(lo, hi, size=shape))
    if name == "helmholtz_p1_tri":
        mesh = make_mesh(2, n, 0.20, rng)
        f = _p1_field(mesh, rng.uniform(0.5, 1.5, size=mesh.nvert), 1)
        return Workload(name, "helmholtz", mesh, 1, 2, [f])
    if name == "helmholtz_p2_tet":
        mesh = make_mesh(3, n, 0.10, rng)
        f = _p2_field(mesh, unif(0.5, 1.5), rng, 1)
        return Workload(name, "helmholtz", mesh, 2, 4, [f])
    if name in ("elasticity_p2_tet", "elasticity_p1_tet"):
        p = 2 if name.endswith("p2_tet") else 1
        mesh = make_mesh(3, n, 0.10, rng)
        mu = _p1_field(mesh, rng.uniform(1.0, 10.0, size=mesh.nvert), 1)
        lm = _p1_field(mesh, rng.uniform(1.0, 10.0, size=mesh.nvert), 1)
        N = 3 * n_scalar_dofs(3, p)
        lam = rng.standard_normal((mesh.ncells, N))
        u = rng.standard_normal((mesh.ncells, N))
        return Workload(name, "elasticity", mesh, p, 2 * p, [mu, lm], [], lam, u)
    if name in ("svk_p1_tet", "svk_p2_tet"):
        p = 1 if name == "svk_p1_tet" else 2
        mesh = make_mesh(3, n, 0.10, rng)
        normal = lambda g, shape: g.normal(0.0, 0.01, size=shape)
        if p == 1:
            u = _p1_field(mesh, rng.normal(0.0, 0.01, size=(mesh.nvert, 3)), 3)
        else:
            u = _p2_field(mesh, normal, rng, 3)
        return Workload(name, "svk_jacobian", mesh, p, 2 * p, [u], [1.0, 1.0])
    if name == "helmholtz_p1_prism":
        mesh = make_prism_mesh(n, 0.10, rng)
        f = _p1_field(mesh, rng.uniform(0.5, 1.5, size=mesh.nvert), 1)
        return Workload(name, "helmholtz", mesh, 1, 2, [f])
    if name in ("diffusion_p2_prism", "diffusion_p3_prism"):
        p = 2 if name == "diffusion_p2_prism" else 3
        mesh = make_prism_mesh(n, 0.10, rng)
        return Workload(name, "diffusion", mesh, p, 2 * p, [], [1.0, 1.0])
    if name in ("burgers_p1_tet", "burgers_p2_tet"):
        p = 1 if name == "burgers_p1_tet" else 2
        mesh = make_mesh(3, n, 0.10, rng)
        if p == 1:
            w = _p1_field(mesh, rng.uniform(-1.0, 1.0, size=(mesh.nvert, 3)), 3)
        else:
            w = _p2_field(mesh, unif(-1.0, 1.0), rng, 3)
        return Workload(name, "burgers", mesh, p, 2 * p + 1, [w], [1.0, 1.0])
    raise KeyError(name)


def single_cell_mesh(d: int, verts: np.ndarray) -> Mesh:
    """A one-cell mesh with the given vertex coordinates [d+1, d]."""
    verts = np.ascontiguousarray(np.asarray(verts, dtype=np.float64).reshape(d + 1, d))
    cells = np.arange(d + 1, dtype=np.int32).reshape(1, d + 1)
    return Mesh(d=d, n=1, coords=verts, cells=cells)


def random_cells(d: int, ncells: int, rng: np.random.Generator, scale: float = 1.0) -> Mesh:
    """Disconnected mesh of independent, positively oriented random simplices.

    Each cell is x0 + Q L (reference vertices) with Q a product of plane
    rotations and L lower triangular with a positive diagonal, so every cell
    is non-degenerate and positively oriented by construction.
    """
    ref = np.zeros((d + 1, d))
    ref[1:, :] = np.eye(d)
    verts = np.empty((ncells, d + 1, d))
    for e in range(ncells):
        L = np.tril(rng.uniform(-0.5, 0.5, size=(d, d)), -1) + np.diag(rng.uniform(0.3, 1.5, size=d))
        Q = np.eye(d)
        for (i, j) in ([(0, 1)] if d == 2 else [(0, 1), (0, 2), (1, 2)]):
            t = rng.uniform(0.0, 2.0 * np.pi)
            G = np.eye(d)
            G[i, i] = G[j, j] = np.cos(t)
            G[i, j] = -np.sin(t)
            G[j, i] = np.sin(t)
            Q = G @ Q
        x0 = rng.uniform(-1.0, 1.0, size=d)
        verts[e] = (x0 + (ref @ (Q @ L).T)) * scale
    coords = verts.reshape(-1, d)
    cells = np.arange(ncells * (d + 1), dtype=np.int32).reshape(ncells, d + 1)
    return Mesh(d=d, n=0, coords=np.ascontiguousarray(coords), cells=cells)


@dataclass
class MixedBatch:
    """Cells of mixed shape, degree and form in one random order.

    segments: list of (form, d, degree) bin types; seg_of[i], cell_of[i]: the
    bin and the cell (in that shape's mesh) of batch entry i; out_offset[i]:
    element offset of entry i's tensor in the packed output (batch order).
    """
    tri: Mesh
    tet: Mesh
    f_tri: Field
    f_tet: Field
    segments: list
    seg_of: np.ndarray
    cell_of: np.ndarray
    out_offset: np.ndarray
    total_elems: int


def mixed_batch(n_tri: int = 1000, n_tet: int = 56, tri_counts=(800_000, 600_000, 400_000, 200_000),
                tet_counts=(500_000, 300_000, 200_000), seed: int = 1) -> MixedBatch:
    """Triangles P1-P4 drawn from an n_tri^2 x 2 mesh (every cell used once when
    the counts sum to the mesh size) and tetrahedra P1-P3 drawn without
    replacement from an n_tet^3 x 6 mesh; Mass and Helmholtz 50/50; f a P1
    field ~ U[0.5, 1.5] on each mesh; quadrature degree 2p; all entries
    interleaved in one random order. One PCG64 generator (seed) draws, in
    order: triangle jitter (20%), tetrahedron jitter (10%), f on triangles,
    f on tetrahedra, triangle degree assignment, tetrahedron subset and
    degrees, forms, the interleaving permutation."""
    rng = np.random.default_rng(seed)
    tri = make_mesh(2, n_tri, 0.20, rng)
    tet = make_mesh(3, n_tet, 0.10, rng)
    f_tri = Field(rng.uniform(0.5, 1.5, size=(tri.nvert, 1)), tri.cells, 1, 1)
    f_tet = Field(rng.uniform(0.5, 1.5, size=(tet.nvert, 1)), tet.cells, 1, 1)
    ntri = int(sum(tri_counts))
    ntet = int(sum(tet_counts))
    if ntri > tri.ncells or ntet > tet.ncells:
        raise ValueError("more cells requested than the meshes hold")
    tri_cells = rng.permutation(tri.ncells)[:ntri]
    tet_cells = rng.permutation(tet.ncells)[:ntet]
    segments = []
    seg_parts, cell_parts = [], []
    forms = ("mass", "helmholtz")
    start = 0
    for p, cnt in enumerate(tri_counts, start=1):
        cells = tri_cells[start:start + cnt]
        start += cnt
        fsel = rng.integers(0, 2, size=cnt)
        for fi, fname in enumerate(forms):
            segments.append((fname, 2, p))
            seg_parts.append(np.full(int((fsel == fi).sum()), len(segments) - 1, dtype=np.int32))
            cell_parts.append(np.sort(cells[fsel == fi]))
    start = 0
    for p, cnt in enumerate(tet_counts, start=1):
        cells = tet_cells[start:start + cnt]
        start += cnt
        fsel = rng.integers(0, 2, size=cnt)
        for fi, fname in enumerate(forms):
            segments.append((fname, 3, p))
            seg_parts.append(np.full(int((fsel == fi).sum()), len(segments) - 1, dtype=np.int32))
            cell_parts.append(np.sort(cells[fsel == fi]))
    seg_of = np.concatenate(seg_parts)
    cell_of = np.concatenate(cell_parts).astype(np.int64)
    perm = rng.permutation(seg_of.shape[0])
    seg_of = np.ascontiguousarray(seg_of[perm])
    cell_of = np.ascontiguousarray(cell_of[perm])
    sizes = np.array([n_scalar_dofs(d, p) ** 2 for (_, d, p) in segments], dtype=np.int64)[seg_of]
    out_offset = np.zeros(seg_of.shape[0], dtype=np.int64)
    np.cumsum(sizes[:-1], out=out_offset[1:])
    return MixedBatch(tri, tet, f_tri, f_tet, segments, seg_of, cell_of, out_offset, int(sizes.sum()))
