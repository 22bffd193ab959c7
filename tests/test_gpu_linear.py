"""GPU parity of the linear-form engine (mass, Helmholtz, elasticity, Burgers)
against the FP64 oracle, through the C ABI."""
import os

import numpy as np
import pytest

from paper_1407_0904_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cf():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a device"
    from paper_1407_0904_amd import coffee
    return coffee


def _field_of_degree(mesh, deg, rng, lo=0.5, hi=1.5, ncomp=1):
    if deg == 1:
        return I.Field(rng.uniform(lo, hi, size=(mesh.nvert, ncomp)), mesh.cells, 1, ncomp)
    if deg == 2:
        c2d, nd = I.p2_dofmap(mesh.cells, mesh.n, mesh.d)
        return I.Field(rng.uniform(lo, hi, size=(nd, ncomp)), c2d, 2, ncomp)
    nl = I.n_scalar_dofs(mesh.d, deg)
    return I.Field(rng.uniform(lo, hi, size=(mesh.ncells, nl, ncomp)), None, deg, ncomp)


PRECS = ["fp64", "fp32", "bf16x3"]


@pytest.mark.parametrize("prec", PRECS)
def test_helmholtz_p1_tri_full_config(cf, oracle, prec):
    """8192-cell Helmholtz P1 triangle workload, every cell."""
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    w = I.workload("helmholtz_p1_tri")
    ref = oracle.assemble(w.form, w.mesh, w.degree, w.quad_degree, fields=w.fields)
    got = assemble_gpu(w.form, w.mesh, w.degree, w.fields, quad_degree=w.quad_degree, precision=prec).cpu().numpy()
    err = cell_rel_err(got, ref)
    print(f"helmholtz_p1_tri {prec} max cell rel err {err:.3e}")
    assert err < TOL[prec]


CASES = [
    # form, d, p, field degree (0 = none)
    ("mass", 2, 1, 0), ("mass", 2, 2, 1), ("mass", 2, 3, 2), ("mass", 2, 4, 1),
    ("mass", 3, 1, 1), ("mass", 3, 2, 2), ("mass", 3, 3, 1), ("mass", 3, 4, 0),
    ("helmholtz", 2, 1, 1), ("helmholtz", 2, 2, 2), ("helmholtz", 2, 3, 1), ("helmholtz", 2, 4, 2),
    ("helmholtz", 3, 1, 0), ("helmholtz", 3, 2, 2), ("helmholtz", 3, 3, 1), ("helmholtz", 3, 4, 1),
]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("form,d,p,fd", CASES)
def test_scalar_forms(cf, oracle, form, d, p, fd, prec):
    """Small meshes spanning several 256-cell chunks with a ragged tail."""
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    rng = np.random.default_rng(100 + 10 * d + p)
    mesh = I.make_mesh(d, 13 if d == 2 else 5, 0.2 if d == 2 else 0.1, rng)  # 338 / 750 cells
    fields = [] if fd == 0 else [_field_of_degree(mesh, fd, rng)]
    ref = oracle.assemble(form, mesh, p, fields=fields)
    got = assemble_gpu(form, mesh, p, fields, precision=prec).cpu().numpy()
    err = cell_rel_err(got, ref)
    print(f"{form} d{d} p{p} fd{fd} {prec}: {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("d,p,fields", [(3, 2, True), (3, 1, True), (3, 2, False), (2, 2, True), (3, 3, True),
                                        (2, 3, False), (2, 1, True), (2, 1, False), (3, 1, False), (2, 3, True)])
def test_elasticity(cf, oracle, d, p, fields, prec):
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    rng = np.random.default_rng(7 + p)
    mesh = I.make_mesh(d, 10 if d == 2 else 4, 0.1, rng)
    if fields:
        flds = [_field_of_degree(mesh, 1, rng, 1, 10), _field_of_degree(mesh, 1, rng, 1, 10)]
        cst = []
    else:
        flds, cst = [], [2.5, 7.0]
    ref = oracle.assemble("elasticity", mesh, p, fields=flds, constants=cst)
    got = assemble_gpu("elasticity", mesh, p, flds, constants=cst, precision=prec).cpu().numpy()
    err = cell_rel_err(got, ref)
    print(f"elasticity d{d} p{p} {prec}: {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("d,p", [(3, 1), (3, 2), (2, 1), (2, 2), (2, 3)])
def test_burgers(cf, oracle, d, p, prec):
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    rng = np.random.default_rng(70 + p)
    mesh = I.make_mesh(d, 10 if d == 2 else 4, 0.1, rng)
    w = _field_of_degree(mesh, p, rng, -1, 1, ncomp=d)
    cst = [0.7, 1.3]
    ref = oracle.assemble("burgers", mesh, p, fields=[w], constants=cst)
    got = assemble_gpu("burgers", mesh, p, [w], constants=cst, precision=prec).cpu().numpy()
    err = cell_rel_err(got, ref)
    print(f"burgers d{d} p{p} {prec}: {err:.3e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("form,p", [("elasticity", 2), ("burgers", 2), ("burgers", 1)])
def test_vector_ragged_counts(cf, oracle, form, p, prec):
    """Cell counts around the 16-cell tile and the 128-cell chunk of the
    vector engine (one cell, a partial first tile, full tiles plus a partial
    one, several chunks plus a tail), on tetrahedra with P1 Lame fields or a
    vector Burgers state of the trial degree."""
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    rng = np.random.default_rng(90 + p)
    mesh = I.make_mesh(3, 6, 0.1, rng)  # 1296 cells
    if form == "elasticity":
        mu = rng.uniform(1, 10, size=(mesh.nvert, 1))
        lm = rng.uniform(1, 10, size=(mesh.nvert, 1))
        cst = []
    else:
        w = rng.uniform(-1, 1, size=(mesh.nvert if p == 1 else I.p2_dofmap(mesh.cells, mesh.n, 3)[1], 3))
        cst = [0.7, 1.3]
    for n in (1, 15, 17, 48, 133, 1291):
        sub = I.Mesh(3, mesh.n, mesh.coords, mesh.cells[:n])
        if form == "elasticity":
            flds = [I.Field(mu, sub.cells, 1, 1), I.Field(lm, sub.cells, 1, 1)]
        elif p == 1:
            flds = [I.Field(w, sub.cells, 1, 3)]
        else:
            flds = [I.Field(w, I.p2_dofmap(mesh.cells, mesh.n, 3)[0][:n], 2, 3)]
        ref = oracle.assemble(form, sub, p, fields=flds, constants=cst)
        got = assemble_gpu(form, sub, p, flds, constants=cst, precision=prec).cpu().numpy()
        err = cell_rel_err(got, ref)
        print(f"{form} p{p} {n} cells {prec}: {err:.3e}")
        assert err < TOL[prec]


TUNING = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1407_0904_amd",
                      "tuning_mi355x.txt")


@pytest.fixture(params=["default", "tuned"])
def launch_config(request, cf):
    """The library's default launch shape, and the shipped tuning cache that
    the benchmark loads before it times anything (grid multipliers per kernel
    instance); the defaults are restored afterwards."""
    if request.param == "tuned":
        assert os.path.exists(TUNING), TUNING
        cf.coffee_load_tuning(TUNING)
    yield request.param
    cf.coffee_load_tuning(None)
    cf.coffee_set_launch_options(0)


def test_full_size_elasticity_p2_tet_sampled(cf, oracle, launch_config):
    """The 663,552-cell elasticity P2 tetrahedron workload (P1 Lame fields) in
    the library's default launch shape and in the tuned one the benchmark
    times: sampled cells against the oracle in every precision, and rigid
    translations in the kernel of all cells."""
    import torch
    from gpu_util import TOL, cell_rel_err, to_dev
    w = I.workload("elasticity_p2_tet")
    coords, c2v, dfs = to_dev(w.mesh, w.fields)
    rng = np.random.default_rng(12)
    E = w.mesh.ncells
    sample = np.unique(np.concatenate([[0, 1, 15, 16, 127, 128, E - 1], rng.integers(0, E, 1500)]))
    ref = oracle.assemble(w.form, w.mesh, 2, w.quad_degree, fields=w.fields, cells=sample)
    idx = torch.as_tensor(sample, device=coords.device)
    for prec in PRECS:
        out = cf.coffee_assemble(w.form, 3, 2, coords, c2v, coeffs=dfs, quad_degree=w.quad_degree, precision=prec)
        torch.cuda.synchronize()
        got = out[idx].cpu().numpy()
        err = cell_rel_err(got, ref)
        print(f"elasticity_p2_tet full {prec}: {err:.3e}")
        assert err < TOL[prec]
        if prec == "fp64":
            # rigid translations (component block c all ones) are in the kernel of
            # every A_e: the row sums over each block of 10 columns vanish (a sum,
            # not a batched matrix-vector product, so that no BLAS path is involved)
            scale = out.abs().amax(dim=(1, 2))
            for c in range(3):
                r = out[:, :, 10 * c:10 * c + 10].sum(dim=2).abs().amax(dim=1) / scale
                assert float(r.max()) < 1e-12, (c, float(r.max()))
        del out


def test_edge_cases(cf, oracle):
    """Empty input, a single cell, exactly one chunk, one chunk + 1, cell-major fields."""
    import torch
    from gpu_util import assemble_gpu, cell_rel_err, to_dev
    rng = np.random.default_rng(5)
    mesh = I.random_cells(3, 257, rng)
    f = I.Field(rng.uniform(0.5, 1.5, size=(257, 10, 1)), None, 2, 1)  # cell-major (no map)
    for ncell in (1, 64, 256, 257):
        sub = I.Mesh(3, 0, mesh.coords, mesh.cells[:ncell])
        fs = I.Field(f.values[:ncell], None, 2, 1)
        ref = oracle.assemble("helmholtz", sub, 3, fields=[fs])
        got = assemble_gpu("helmholtz", sub, 3, [fs]).cpu().numpy()
        assert cell_rel_err(got, ref) < 1e-12
    coords, c2v, _ = to_dev(mesh, [])
    empty = torch.empty((0, 4), dtype=torch.int32, device=coords.device)
    out = cf.coffee_assemble("mass", 3, 2, coords, empty)
    assert out.shape == (0, 10, 10)
    # a field degree outside the compiled set is reported, not silently run
    f3 = I.Field(rng.uniform(0.5, 1.5, size=(4, 20, 1)), None, 3, 1)
    sub = I.Mesh(3, 0, mesh.coords, mesh.cells[:4])
    with pytest.raises(cf.CoffeeError) as ei:
        assemble_gpu("helmholtz", sub, 3, [f3])
    assert ei.value.code == 2


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("form,d,fd", [("helmholtz", 2, 1), ("helmholtz", 3, 1), ("mass", 2, 0), ("mass", 3, 1),
                                       ("helmholtz", 3, 0)])
def test_p1_ragged_counts(cf, oracle, form, d, fd, prec):
    """Degree-1 forms (the thread-per-cell kernel in FP64/FP32, the MFMA engine
    in BF16X3) at counts around a 64-cell wave and a 256-cell workgroup."""
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    rng = np.random.default_rng(40 + d)
    mesh = I.make_mesh(d, 20 if d == 2 else 5, 0.15, rng)  # 800 / 750 cells
    f = rng.uniform(0.5, 1.5, size=(mesh.nvert, 1))
    for n in (1, 63, 64, 65, 255, 257, mesh.ncells):
        sub = I.Mesh(d, mesh.n, mesh.coords, mesh.cells[:n])
        flds = [I.Field(f, sub.cells, 1, 1)] if fd else []
        ref = oracle.assemble(form, sub, 1, fields=flds)
        got = assemble_gpu(form, sub, 1, flds, precision=prec).cpu().numpy()
        err = cell_rel_err(got, ref)
        assert err < TOL[prec], (n, err)


def test_full_size_helmholtz_p2_tet_sampled(cf, oracle, launch_config):
    """The 1,572,864-cell Helmholtz P2 tetrahedron workload, in the library's
    default launch shape and in the tuned one the benchmark times; sampled
    cells against the oracle, plus the total mass identity on all cells."""
    import torch
    from gpu_util import TOL, cell_rel_err, to_dev
    w = I.workload("helmholtz_p2_tet")
    coords, c2v, dfs = to_dev(w.mesh, w.fields)
    rng = np.random.default_rng(11)
    E = w.mesh.ncells
    sample = np.unique(np.concatenate([[0, 1, 255, 256, E - 1], rng.integers(0, E, 3000)]))
    ref = oracle.assemble(w.form, w.mesh, 2, 4, fields=w.fields, cells=sample)
    idx = torch.as_tensor(sample, device=coords.device)
    for prec in PRECS:
        out = cf.coffee_assemble(w.form, 3, 2, coords, c2v, coeffs=dfs, quad_degree=4, precision=prec)
        torch.cuda.synchronize()
        got = out[idx].cpu().numpy()
        err = cell_rel_err(got, ref)
        print(f"helmholtz_p2_tet full {prec} ({launch_config} launch): {err:.3e}")
        assert err < TOL[prec]
        del out
    # f = 1 mass over the whole mesh sums to the cube's volume
    m = cf.coffee_assemble("mass", 3, 2, coords, c2v)
    assert abs(float(m.sum()) - 1.0) < 1e-10


def test_check_geometry(cf):
    import torch
    from gpu_util import to_dev
    mesh = I.make_mesh(3, 4, 0.1, np.random.default_rng(0))
    coords, c2v, _ = to_dev(mesh, [])
    assert cf.coffee_check_geometry(3, coords, c2v) == -1
    bad = c2v.clone()
    bad[37] = bad[37][[0, 2, 1, 3]]  # inverted orientation
    bad[200, 1] = bad[200, 0]        # collapsed
    assert cf.coffee_check_geometry(3, coords, bad) == 37


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("form,d,p,fd,q", [("helmholtz", 3, 2, 2, 4), ("mass", 2, 3, 1, 6), ("helmholtz", 3, 3, 1, 6),
                                           ("burgers", 3, 1, 1, 3), ("elasticity", 3, 2, 1, 4)])
def test_symmetric_rule_forms(cf, oracle, form, d, p, fd, q, prec):
    """Forms integrated with the fully symmetric rule (COFFEE_QUAD(q, 1)),
    against the oracle with its own symmetric rule. The coefficient mass terms
    are under-integrated at these degrees, so they match only if both sides
    use the same rule; the Burgers case is the paper's 5-point tetrahedral
    rule (negative centroid weight)."""
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    rng = np.random.default_rng(300 + 10 * p + q)
    mesh = I.make_mesh(d, 8 if d == 2 else 4, 0.15, rng)
    qs = oracle.quad(q, oracle.RULE_SYMMETRIC)
    cst = []
    if form == "burgers":
        flds = [_field_of_degree(mesh, p, rng, -1, 1, ncomp=d)]
        cst = [0.7, 1.3]
    elif form == "elasticity":
        flds = [_field_of_degree(mesh, 1, rng, 1, 10), _field_of_degree(mesh, 1, rng, 1, 10)]
    else:
        flds = [_field_of_degree(mesh, fd, rng)]
    ref = oracle.assemble(form, mesh, p, quad_degree=qs, fields=flds, constants=cst)
    got = assemble_gpu(form, mesh, p, flds, constants=cst, quad_degree=qs, precision=prec).cpu().numpy()
    err = cell_rel_err(got, ref)
    print(f"{form} d{d} p{p} symmetric q{q} {prec}: {err:.3e}")
    assert err < TOL[prec]
    if form in ("helmholtz", "mass") and fd > 0:
        # the Gauss-Jacobi rule of the same degree gives a different tensor
        gj = oracle.assemble(form, mesh, p, quad_degree=q, fields=flds)
        assert cell_rel_err(gj, ref) > 1e-10


def test_prepared_assemble_equals_assemble(cf):
    """PreparedAssemble (arguments checked and marshalled once) launches the
    same kernel: bitwise equal to coffee_assemble, on repeated calls."""
    import torch
    from gpu_util import to_dev
    w = I.workload("helmholtz_p2_tet", n=6)
    coords, c2v, dfs = to_dev(w.mesh, w.fields)
    ref = cf.coffee_assemble(w.form, 3, 2, coords, c2v, coeffs=dfs, quad_degree=w.quad_degree)
    call = cf.PreparedAssemble(w.form, 3, 2, coords, c2v, coeffs=dfs, quad_degree=w.quad_degree)
    for _ in range(3):
        out = call()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


VARIANT_KEYS = [("helmholtz", 3, 2, 2), ("helmholtz", 3, 2, 1), ("mass", 3, 2, 2), ("mass", 3, 2, 1),
                ("helmholtz", 2, 3, 1), ("helmholtz", 2, 4, 1)]


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("form,d,p,fd", VARIANT_KEYS)
def test_tile_shape_variants(cf, oracle, form, d, p, fd, prec, variant):
    """Every tile-shape variant the autotuner can choose (reference fragments
    in registers, in LDS, or through the caches) against the oracle, on a mesh
    of several 256-cell chunks with a ragged tail."""
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    assert variant == 0 or cf.coffee_has_variant(form, d, p, fd, prec, variant)
    rng = np.random.default_rng(500 + 10 * p + fd)
    mesh = I.make_mesh(d, 14 if d == 2 else 5, 0.15, rng)  # 392 / 750 cells
    fields = [_field_of_degree(mesh, fd, rng)]
    ref = oracle.assemble(form, mesh, p, fields=fields)
    cf.coffee_set_variant(variant)
    try:
        got = assemble_gpu(form, mesh, p, fields, precision=prec).cpu().numpy()
    finally:
        cf.coffee_set_variant(-1)
    err = cell_rel_err(got, ref)
    assert err < TOL[prec], err
