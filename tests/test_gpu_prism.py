"""GPU diffusion form (simplices and prisms) and prism cells against the oracle.

Prisms are not affine images of the reference prism, so the library forms
J, det J and K at every quadrature point; the oracle does the same by a
separate route (prism.c). Cases span several 16-cell tiles with a ragged
tail, every precision, fields through a dof map and cell-major, and the
full-size workloads of the benchmark (sampled cells).
"""
import numpy as np
import pytest

from paper_1407_0904_amd import inputs as I

pytestmark = pytest.mark.gpu

PRISM = 6


@pytest.fixture(scope="module")
def cf():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a device"
    from paper_1407_0904_amd import coffee
    return coffee


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_diffusion_simplex_vs_oracle(cf, oracle, d, p, prec):
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    rng = np.random.default_rng(60 + 10 * d + p)
    mesh = I.make_mesh(d, 7 if d == 2 else 3, 0.15, rng)  # 98 / 162 cells: ragged against the chunks
    cst = [0.7, 1.9]
    ref = oracle.assemble("diffusion", mesh, p, constants=cst)
    got = assemble_gpu("diffusion", mesh, p, [], constants=cst, precision=prec).cpu().numpy()
    err = cell_rel_err(got, ref)
    print(f"diffusion d{d} p{p} {prec}: {err:.2e}")
    assert err < TOL[prec]


def _prism_fields(kind, mesh, rng):
    if kind == "none":
        return []
    vals = rng.uniform(0.5, 1.5, (mesh.nvert, 1))
    if kind == "mapped":
        return [I.Field(vals, mesh.cells, 1, 1)]
    return [I.Field(vals[mesh.cells.reshape(-1)].reshape(mesh.ncells, 6, 1), None, 1, 1)]  # cell-major


PRISM_CASES = [("mass", "none"), ("mass", "mapped"), ("helmholtz", "none"), ("helmholtz", "mapped"),
               ("helmholtz", "cellmajor"), ("diffusion", "none")]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("form,kind", PRISM_CASES)
def test_prism_vs_oracle(cf, oracle, form, kind, p, prec):
    from gpu_util import TOL, assemble_gpu, cell_rel_err
    rng = np.random.default_rng(70 + p)
    mesh = I.make_prism_mesh(4, 0.15, rng)  # 128 cells; warped prisms
    assert mesh.cell == PRISM
    fields = _prism_fields(kind, mesh, rng)
    cst = [1.3, 0.8] if form == "diffusion" else []
    ref = oracle.assemble(form, mesh, p, fields=fields, constants=cst)
    got = assemble_gpu(form, mesh, p, fields, constants=cst, precision=prec).cpu().numpy()
    err = cell_rel_err(got, ref)
    print(f"prism {form} ({kind}) p{p} {prec}: {err:.2e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("ncells", [1, 15, 16, 17, 31, 32, 33, 64, 250])
def test_prism_ragged_counts(cf, oracle, ncells):
    """Cell counts around the 16-cell tile: the first ncells cells of a mesh."""
    from gpu_util import assemble_gpu, cell_rel_err
    rng = np.random.default_rng(ncells)
    full = I.make_prism_mesh(5, 0.15, rng)
    mesh = I.Mesh(d=3, n=5, coords=full.coords, cells=np.ascontiguousarray(full.cells[:ncells]))
    for p in (1, 2, 3):
        ref = oracle.assemble("helmholtz", mesh, p)
        got = assemble_gpu("helmholtz", mesh, p, []).cpu().numpy()
        assert got.shape == ref.shape
        assert cell_rel_err(got, ref) < 1e-12


@pytest.mark.parametrize("name,p,form", [("p1", 1, "helmholtz"), ("p2", 2, "diffusion"), ("p3", 3, "diffusion")])
def test_prism_full_size_sampled(cf, oracle, name, p, form):
    """The benchmark's prism workloads at full size, in its launch
    configuration (the shipped tuning cache): 2,000 sampled cells against the
    oracle, every precision; the FP64 mass of the whole mesh sums to the
    cube's volume."""
    import os
    import torch
    from gpu_util import TOL, cell_rel_err, to_dev
    tuning = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1407_0904_amd",
                          "tuning_mi355x.txt")
    cf.coffee_load_tuning(tuning)
    try:
        _prism_full_size(cf, oracle, name, p, form)
    finally:
        cf.coffee_load_tuning(None)


def _prism_full_size(cf, oracle, name, p, form):
    import torch
    from gpu_util import TOL, cell_rel_err, to_dev
    w = I.workload(f"{'helmholtz' if p == 1 else 'diffusion'}_{name}_prism")
    assert w.form == form and w.degree == p
    coords, c2v, dfs = to_dev(w.mesh, w.fields)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(w.mesh.ncells, 2000, replace=False))
    sample[-1] = w.mesh.ncells - 1
    ref = oracle.assemble(w.form, w.mesh, p, fields=w.fields, constants=w.constants, cells=sample)
    for prec in ("fp64", "fp32", "bf16x3"):
        out = cf.coffee_assemble(w.form, PRISM, p, coords, c2v, coeffs=dfs, constants=w.constants, precision=prec)
        torch.cuda.synchronize()
        got = out[torch.as_tensor(sample, device=out.device)].cpu().numpy()
        err = cell_rel_err(got, ref)
        print(f"{w.name} {prec}: {err:.2e} on {len(sample)} sampled cells of {w.mesh.ncells}")
        assert err < TOL[prec]
        del out
    m = cf.coffee_assemble("mass", PRISM, p, coords, c2v)
    assert abs(float(m.sum()) - 1.0) < 1e-10


def test_prism_errors_and_geometry_check(cf):
    """Refusals are reported (prism adjoint, non-default rule, degree 4,
    vector forms), an empty mesh is accepted, and the geometry check finds an
    inverted prism."""
    import torch
    from gpu_util import to_dev
    mesh = I.make_prism_mesh(3, 0.1, np.random.default_rng(2))
    coords, c2v, _ = to_dev(mesh, [])
    U = 2  # COFFEE_E_UNSUPPORTED
    for kwargs in (dict(quad_degree=3), dict(quad_degree=COFFEE_QUAD(2, 1))):
        with pytest.raises(cf.CoffeeError) as e:
            cf.coffee_assemble("helmholtz", PRISM, 1, coords, c2v, **kwargs)
        assert e.value.code == U
    with pytest.raises(cf.CoffeeError) as e:
        cf.coffee_assemble("helmholtz", PRISM, 4, coords, c2v)
    assert e.value.code == U
    with pytest.raises(cf.CoffeeError) as e:
        cf.coffee_assemble("svk_energy", PRISM, 1, coords, c2v,
                           coeffs=[cf.DeviceField(torch.zeros(mesh.nvert, 3, dtype=torch.float64,
                                                              device=coords.device), c2v, 1, 3)])
    assert e.value.code == U
    lam = torch.zeros(mesh.ncells, 6, dtype=torch.float64, device=coords.device)
    with pytest.raises(cf.CoffeeError) as e:
        cf.coffee_assemble_adjoint("helmholtz", PRISM, 1, coords, c2v, lam=lam, u=lam)
    assert e.value.code == U
    empty = cf.coffee_assemble("helmholtz", PRISM, 2, coords, c2v[:0])
    torch.cuda.synchronize()
    assert tuple(empty.shape) == (0, 18, 18)
    assert cf.coffee_check_geometry("prism", coords, c2v) == -1
    bad = c2v.clone()
    bad[7] = bad[7][[1, 0, 3, 2, 5, 4]]  # bottom and top swapped: det J < 0
    assert cf.coffee_check_geometry("prism", coords, bad) == 7


def COFFEE_QUAD(q, rule):
    return q + 16 * rule


def test_prism_global_csr(cf, oracle):
    """Global P2 prism diffusion matrix (NEXT to local assembly: the scatter
    into CSR) against the oracle's global assembler."""
    import torch
    from gpu_util import to_dev
    n = 3
    mesh = I.make_prism_mesh(n, 0.12, np.random.default_rng(8))
    c2d, nd = I.prism_p2_dofmap(n)
    ref = oracle.assemble_global("diffusion", mesh, 2, c2d, nd)
    coords, c2v, _ = to_dev(mesh, [])
    map_d = torch.as_tensor(c2d, device=coords.device)
    row_ptr, col_idx = cf.coffee_csr_pattern(map_d, nd)
    np.testing.assert_array_equal(row_ptr.cpu().numpy(), ref.indptr)
    np.testing.assert_array_equal(col_idx.cpu().numpy(), ref.indices)
    vals = cf.coffee_assemble_csr("diffusion", PRISM, 2, coords, c2v, row_ptr, col_idx, nd, cell_to_dof=map_d)
    torch.cuda.synchronize()
    assert rel(vals.cpu().numpy(), ref.data) < 1e-12


@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (3, 1), (3, 2)])
@pytest.mark.parametrize("deterministic", [0, 1])
def test_diffusion_adjoint_vs_oracle(cf, oracle, d, p, deterministic):
    """Reverse pass of the diffusion form against the oracle's complex-step gradient."""
    import torch
    from gpu_util import to_dev
    rng = np.random.default_rng(90 + 10 * d + p)
    mesh = I.make_mesh(d, 6 if d == 2 else 3, 0.15, rng)
    cst = [0.6, 1.7]
    N = oracle.tensor_dim("diffusion", d, p)
    lam = rng.standard_normal((mesh.ncells, N))
    u = rng.standard_normal((mesh.ncells, N))
    S_ref, gc_ref, _ = oracle.adjoint("diffusion", mesh, p, constants=cst, lam=lam, u=u)
    coords, c2v, _ = to_dev(mesh, [])
    cv = torch.empty(mesh.ncells, dtype=torch.float64, device=coords.device)
    gc, _ = cf.coffee_assemble_adjoint("diffusion", d, p, coords, c2v, constants=cst,
                                       lam=torch.as_tensor(lam, device=coords.device),
                                       u=torch.as_tensor(u, device=coords.device), cell_value=cv,
                                       deterministic=bool(deterministic))
    torch.cuda.synchronize()
    S = float(cv.sum())
    assert abs(S - S_ref) <= 1e-11 * abs(S_ref)
    assert rel(gc.cpu().numpy(), gc_ref) < 1e-10
