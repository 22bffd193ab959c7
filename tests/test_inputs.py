"""Seeded synthetic meshes: measure, orientation, topology and dof counts."""
import numpy as np
import pytest

from paper_1407_0904_amd import inputs as I


def _dets(mesh):
    c = mesh.coords[mesh.cells]
    return np.linalg.det(np.transpose(c[:, 1:] - c[:, :1], (0, 2, 1)))


@pytest.mark.parametrize("d,n,r", [(2, 8, 0.2), (3, 4, 0.1), (2, 1, 0.0), (3, 1, 0.0)])
def test_mesh_measure_and_orientation(d, n, r):
    m = I.make_mesh(d, n, r, np.random.default_rng(0))
    det = _dets(m)
    assert np.all(det > 0)
    fact = 2 if d == 2 else 6
    assert abs(det.sum() / fact - 1.0) < 1e-13
    assert m.ncells == (2 * n * n if d == 2 else 6 * n ** 3)
    assert m.nvert == (n + 1) ** d


def test_triangle_euler_characteristic():
    n = 5
    m = I.make_mesh(2, n, 0.2, np.random.default_rng(0))
    edges = set()
    for c in m.cells:
        for a, b in ((0, 1), (1, 2), (0, 2)):
            edges.add(tuple(sorted((c[a], c[b]))))
    assert m.nvert - len(edges) + m.ncells == 1


def test_tet_euler_characteristic():
    n = 3
    m = I.make_mesh(3, n, 0.1, np.random.default_rng(0))
    edges, faces = set(), set()
    for c in m.cells:
        for a in range(4):
            for b in range(a + 1, 4):
                edges.add(tuple(sorted((c[a], c[b]))))
        for f in range(4):
            faces.add(tuple(sorted(np.delete(c, f))))
    assert m.nvert - len(edges) + len(faces) - m.ncells == 1


@pytest.mark.parametrize("d,n", [(2, 4), (3, 3)])
def test_p2_dofmap(d, n):
    m = I.make_mesh(d, n, 0.0, np.random.default_rng(0))
    c2d, nd = I.p2_dofmap(m.cells, n, d)
    assert nd == (2 * n + 1) ** d
    assert c2d.min() >= 0 and c2d.max() < nd
    # every refined-lattice point that is a vertex or an edge midpoint is used;
    # on the Kuhn / diagonal split every refined point is one of those
    assert np.unique(c2d).size == nd
    # geometric check: the dof's refined-lattice position equals the node position
    mr = 2 * n + 1
    pos = np.stack([(c2d // mr ** a) % mr for a in range(d)], axis=-1) / (2 * n)
    x = m.coords[m.cells]
    edges = I.TRI_EDGES if d == 2 else I.TET_EDGES
    want = np.concatenate([x] + [0.5 * (x[:, a:a + 1] + x[:, b:b + 1]) for a, b in edges], axis=1)
    np.testing.assert_allclose(pos, want, atol=1e-14)


def test_workloads_are_seeded():
    a = I.workload("helmholtz_p1_tri", n=4)
    b = I.workload("helmholtz_p1_tri", n=4)
    np.testing.assert_array_equal(a.mesh.coords, b.mesh.coords)
    np.testing.assert_array_equal(a.fields[0].values, b.fields[0].values)
    w = I.workload("elasticity_p2_tet", n=2)
    assert w.lam.shape == (48, 30) and w.u.shape == (48, 30)
    assert w.fields[0].values.min() >= 1.0 and w.fields[0].values.max() <= 10.0
