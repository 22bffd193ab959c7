"""GPU adjoint (coffee_assemble_adjoint) against the oracle's complex-step
gradients, central differences and invariants."""
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


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _gpu_adjoint(cf, form, mesh, p, fields, constants, lam, u, q=-1):
    import torch
    from gpu_util import to_dev
    coords, c2v, dfs = to_dev(mesh, fields)
    lam_d = torch.as_tensor(lam, device=coords.device)
    u_d = torch.as_tensor(u, device=coords.device)
    cv = torch.empty(mesh.ncells, dtype=torch.float64, device=coords.device)
    gc, gf = cf.coffee_assemble_adjoint(form, mesh.d, p, coords, c2v, coeffs=dfs, constants=constants,
                                        lam=lam_d, u=u_d, cell_value=cv, quad_degree=q)
    torch.cuda.synchronize()
    return float(cv.sum()), gc.cpu().numpy(), [g.cpu().numpy() for g in gf], cv.cpu().numpy()


CASES = [("elasticity", 3, 2), ("elasticity", 3, 1), ("elasticity", 2, 2), ("helmholtz", 3, 2), ("helmholtz", 2, 1),
         ("mass", 3, 2), ("burgers", 3, 2), ("burgers", 3, 1), ("burgers", 2, 1)]


@pytest.mark.parametrize("form,d,p", CASES)
def test_adjoint_vs_oracle_complex_step(cf, oracle, form, d, p):
    rng = np.random.default_rng(3 + p)
    mesh = I.make_mesh(d, 6 if d == 2 else 3, 0.15, rng)
    if form == "elasticity":
        fields = [I.Field(rng.uniform(1, 10, (mesh.nvert, 1)), mesh.cells, 1, 1),
                  I.Field(rng.uniform(1, 10, (mesh.nvert, 1)), mesh.cells, 1, 1)]
        cst = []
    elif form == "burgers":
        if p == 1:
            fields = [I.Field(rng.uniform(-1, 1, (mesh.nvert, d)), mesh.cells, 1, d)]
        else:
            c2d, nd = I.p2_dofmap(mesh.cells, mesh.n, d)
            fields = [I.Field(rng.uniform(-1, 1, (nd, d)), c2d, 2, d)]
        cst = [0.6, 1.4]
    else:
        if p == 1:
            fields = [I.Field(rng.uniform(0.5, 1.5, (mesh.nvert, 1)), mesh.cells, 1, 1)]
        else:
            c2d, nd = I.p2_dofmap(mesh.cells, mesh.n, d)
            fields = [I.Field(rng.uniform(0.5, 1.5, (nd, 1)), c2d, 2, 1)]
        cst = []
    N = oracle.tensor_dim(form, d, p)
    lam = rng.standard_normal((mesh.ncells, N))
    u = rng.standard_normal((mesh.ncells, N))
    S_ref, gc_ref, gf_ref = oracle.adjoint(form, mesh, p, fields=fields, constants=cst, lam=lam, u=u)
    S, gc, gf, _ = _gpu_adjoint(cf, form, mesh, p, fields, cst, lam, u)
    print(f"{form} d{d} p{p}: S rel {abs(S - S_ref) / abs(S_ref):.2e} coords {rel(gc, gc_ref):.2e} "
          + " ".join(f"f{i} {rel(a, b):.2e}" for i, (a, b) in enumerate(zip(gf, gf_ref))))
    assert abs(S - S_ref) <= 1e-11 * abs(S_ref)
    assert rel(gc, gc_ref) < 1e-10
    for a, b in zip(gf, gf_ref):
        assert rel(a, b) < 1e-10


def test_adjoint_central_differences(cf):
    """GPU gradient vs central differences (h = 1e-6) of the GPU forward on one coordinate and one Lame dof."""
    import torch
    from gpu_util import to_dev
    w = I.workload("elasticity_p2_tet", n=3)
    mesh = w.mesh
    S, gc, gf, _ = _gpu_adjoint(cf, "elasticity", mesh, 2, w.fields, [], w.lam, w.u)

    def S_of(coords_np, mu_np):
        f0 = I.Field(mu_np, mesh.cells, 1, 1)
        m = I.Mesh(3, mesh.n, coords_np, mesh.cells)
        coords, c2v, dfs = to_dev(m, [f0, w.fields[1]])
        A = cf.coffee_assemble("elasticity", 3, 2, coords, c2v, coeffs=dfs).cpu().numpy()
        return float(np.einsum("ei,eij,ej->", w.lam, A, w.u))

    h = 1e-6
    for (v, i) in ((21, 0), (30, 2)):  # interior vertices
        cp = mesh.coords.copy(); cp[v, i] += h
        cm = mesh.coords.copy(); cm[v, i] -= h
        fd = (S_of(cp, w.fields[0].values) - S_of(cm, w.fields[0].values)) / (2 * h)
        assert abs(fd - gc[v, i]) <= 1e-6 * max(abs(fd), np.max(np.abs(gc)) * 1e-3)
    mp = w.fields[0].values.copy(); mp[17, 0] += h
    mm = w.fields[0].values.copy(); mm[17, 0] -= h
    fd = (S_of(mesh.coords, mp) - S_of(mesh.coords, mm)) / (2 * h)
    assert abs(fd - gf[0][17, 0]) <= 1e-6 * abs(fd)


def test_adjoint_full_size_elasticity(cf, oracle):
    """663,552-cell elasticity P2: invariants on the whole gradient, per-cell values
    on sampled cells and the gradient at sampled vertices from their cell patches."""
    w = I.workload("elasticity_p2_tet")
    mesh = w.mesh
    S, gc, gf, cv = _gpu_adjoint(cf, "elasticity", mesh, 2, w.fields, [], w.lam, w.u)
    scale = np.max(np.abs(gc))
    # translation invariance and Euler homogeneity (3-D stiffness: degree d - 2 = 1)
    assert np.max(np.abs(gc.sum(axis=0))) < 1e-9 * scale * np.sqrt(mesh.nvert)
    assert abs(np.sum(mesh.coords * gc) - S) < 1e-9 * abs(S) + 1e-9 * scale
    # linearity in the Lame fields
    lin = np.sum(w.fields[0].values * gf[0]) + np.sum(w.fields[1].values * gf[1])
    assert abs(lin - S) < 1e-10 * np.sum(np.abs(cv))
    # per-cell values on sampled cells
    rng = np.random.default_rng(2)
    sample = rng.integers(0, mesh.ncells, 500)
    A = oracle.assemble("elasticity", mesh, 2, fields=w.fields, cells=sample)
    ref = np.einsum("ei,eij,ej->e", w.lam[sample], A, w.u[sample])
    np.testing.assert_allclose(cv[sample], ref, rtol=1e-10, atol=1e-12 * np.max(np.abs(ref)))
    # gradient at sampled vertices = oracle adjoint over the cells touching them
    for v in rng.integers(0, mesh.nvert, 4):
        cells = np.nonzero(np.any(mesh.cells == v, axis=1))[0]
        sub = I.Mesh(3, mesh.n, mesh.coords, mesh.cells[cells])
        flds = [I.Field(f.values, f.cell_to_dof[cells], 1, 1) for f in w.fields]
        _, gref, fref = oracle.adjoint("elasticity", sub, 2, fields=flds, lam=w.lam[cells], u=w.u[cells])
        np.testing.assert_allclose(gc[v], gref[v], rtol=1e-9, atol=1e-10 * np.max(np.abs(gref[v])))
        np.testing.assert_allclose(gf[0][v], fref[0][v], rtol=1e-9, atol=1e-12)


def test_autograd_bilinear_action(cf):
    """torch.autograd through BilinearAction: gradient of 2 S equals twice the adjoint."""
    import torch
    from paper_1407_0904_amd.autograd import bilinear_action
    from gpu_util import to_dev
    w = I.workload("elasticity_p2_tet", n=2)
    coords, c2v, dfs = to_dev(w.mesh, w.fields)
    coords.requires_grad_(True)
    dfs[0].values.requires_grad_(True)
    lam = torch.as_tensor(w.lam, device=coords.device)
    u = torch.as_tensor(w.u, device=coords.device)
    S = bilinear_action("elasticity", 3, 2, coords, c2v, fields=dfs, lam=lam, u=u)
    (2.0 * S).backward()
    S0, gc, gf, _ = _gpu_adjoint(cf, "elasticity", w.mesh, 2, w.fields, [], w.lam, w.u)
    assert abs(float(S.detach()) - S0) < 1e-12 * abs(S0)
    np.testing.assert_allclose(coords.grad.cpu().numpy(), 2 * gc, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(dfs[0].values.grad.cpu().numpy(), 2 * gf[0], rtol=1e-12, atol=1e-14)


def _det_case(form, d, p, rng, cellmajor=False):
    """A small mesh with the form's coefficient fields (mapped, or cell-major)."""
    mesh = I.make_mesh(d, 6 if d == 2 else 3, 0.15, rng)
    if form == "elasticity":
        fields = [I.Field(rng.uniform(1, 10, (mesh.nvert, 1)), mesh.cells, 1, 1),
                  I.Field(rng.uniform(1, 10, (mesh.nvert, 1)), mesh.cells, 1, 1)]
    elif form == "burgers":
        c2d, nd = (mesh.cells, mesh.nvert) if p == 1 else I.p2_dofmap(mesh.cells, mesh.n, d)
        fields = [I.Field(rng.uniform(-1, 1, (nd, d)), c2d, p, d)]
    else:
        c2d, nd = (mesh.cells, mesh.nvert) if p == 1 else I.p2_dofmap(mesh.cells, mesh.n, d)
        fields = [I.Field(rng.uniform(0.5, 1.5, (nd, 1)), c2d, p, 1)]
    if cellmajor:
        fields = [I.Field(np.ascontiguousarray(f.values[f.cell_to_dof]), None, f.degree, f.ncomp) for f in fields]
    return mesh, fields


@pytest.mark.parametrize("form,d,p,cellmajor", [("elasticity", 3, 2, False), ("helmholtz", 3, 2, False),
                                                ("mass", 3, 2, True), ("burgers", 3, 2, False),
                                                ("burgers", 2, 1, True)])
def test_deterministic_adjoint(cf, oracle, form, d, p, cellmajor):
    """deterministic=1: two runs give the same bits; the result matches the
    atomic scatter to rounding and the oracle's complex-step gradient."""
    import torch
    from gpu_util import to_dev
    rng = np.random.default_rng(31 + p)
    mesh, fields = _det_case(form, d, p, rng, cellmajor)
    cst = [0.6, 1.4] if form == "burgers" else []
    N = oracle.tensor_dim(form, d, p)
    lam = rng.standard_normal((mesh.ncells, N))
    u = rng.standard_normal((mesh.ncells, N))
    S_ref, gc_ref, gf_ref = oracle.adjoint(form, mesh, p, fields=fields, constants=cst, lam=lam, u=u)
    coords, c2v, dfs = to_dev(mesh, fields)
    lam_d = torch.as_tensor(lam, device=coords.device)
    u_d = torch.as_tensor(u, device=coords.device)
    nbytes = cf.coffee_adjoint_workspace_size(form, d, p, mesh.nvert, mesh.ncells, dfs)
    assert nbytes > 0
    runs = []
    for det in (True, True, False):
        gc, gf = cf.coffee_assemble_adjoint(form, d, p, coords, c2v, coeffs=dfs, constants=cst, lam=lam_d, u=u_d,
                                            deterministic=det)
        torch.cuda.synchronize()
        runs.append((gc.cpu().numpy(), [g.cpu().numpy() for g in gf]))
    (a, af), (b, bf), (c, cfl) = runs
    assert np.array_equal(a, b) and all(np.array_equal(x, y) for x, y in zip(af, bf))
    assert rel(a, c) < 1e-13 and all(rel(x, y) < 1e-13 for x, y in zip(af, cfl))
    assert rel(a, gc_ref) < 1e-10 and all(rel(x, y) < 1e-10 for x, y in zip(af, gf_ref))


def test_deterministic_adjoint_full_size_elasticity(cf):
    """The 663,552-cell elasticity adjoint in deterministic mode: bitwise
    repeatable, and equal to the atomic scatter to rounding."""
    import torch
    from gpu_util import to_dev
    w = I.workload("elasticity_p2_tet")
    coords, c2v, dfs = to_dev(w.mesh, w.fields)
    lam = torch.as_tensor(w.lam, device=coords.device)
    u = torch.as_tensor(w.u, device=coords.device)
    ws = torch.empty(cf.coffee_adjoint_workspace_size("elasticity", 3, 2, w.mesh.nvert, w.mesh.ncells, dfs),
                     dtype=torch.uint8, device=coords.device)
    out = []
    for det in (True, True, False):
        gc, gf = cf.coffee_assemble_adjoint("elasticity", 3, 2, coords, c2v, coeffs=dfs, lam=lam, u=u,
                                            deterministic=det, workspace=ws if det else None)
        torch.cuda.synchronize()
        out.append([gc] + gf)
    for x, y in zip(out[0], out[1]):
        assert torch.equal(x, y)
    for x, z in zip(out[0], out[2]):
        assert float((x - z).abs().max()) <= 1e-12 * float(z.abs().max())


def test_adjoint_workspace_checks(cf):
    import torch
    from gpu_util import to_dev
    rng = np.random.default_rng(2)
    mesh, fields = _det_case("helmholtz", 3, 2, rng)
    coords, c2v, dfs = to_dev(mesh, fields)
    N = 10
    lam = torch.zeros((mesh.ncells, N), dtype=torch.float64, device=coords.device)
    nbytes = cf.coffee_adjoint_workspace_size("helmholtz", 3, 2, mesh.nvert, mesh.ncells, dfs)
    with pytest.raises(ValueError, match="workspace has"):
        cf.coffee_assemble_adjoint("helmholtz", 3, 2, coords, c2v, coeffs=dfs, lam=lam, u=lam, deterministic=True,
                                   workspace=torch.empty(nbytes - 1, dtype=torch.uint8, device=coords.device))
    # the SVK Jacobian has no reverse pass
    ud = cf.DeviceField(torch.zeros((mesh.nvert, 3), dtype=torch.float64, device=coords.device), c2v, 1, 3)
    with pytest.raises(cf.CoffeeError) as ei:
        cf.coffee_assemble_adjoint("svk_jacobian", 3, 1, coords, c2v, coeffs=[ud], lam=torch.zeros(
            (mesh.ncells, 12), dtype=torch.float64, device=coords.device), u=torch.zeros(
            (mesh.ncells, 12), dtype=torch.float64, device=coords.device))
    assert ei.value.code == 2


def test_value_only_reverse_pass(cf):
    """grads=False computes the per-cell values alone, equal to those of the
    full reverse pass."""
    import torch
    from gpu_util import to_dev
    w = I.workload("elasticity_p2_tet", n=3)
    coords, c2v, dfs = to_dev(w.mesh, w.fields)
    lam = torch.as_tensor(w.lam, device=coords.device)
    u = torch.as_tensor(w.u, device=coords.device)
    cv0 = torch.empty(w.mesh.ncells, dtype=torch.float64, device=coords.device)
    cv1 = torch.empty_like(cv0)
    cf.coffee_assemble_adjoint("elasticity", 3, 2, coords, c2v, coeffs=dfs, lam=lam, u=u, cell_value=cv0)
    gc, gf = cf.coffee_assemble_adjoint("elasticity", 3, 2, coords, c2v, coeffs=dfs, lam=lam, u=u, cell_value=cv1,
                                        grads=False)
    torch.cuda.synchronize()
    assert gc is None and gf == []
    assert torch.equal(cv0, cv1)
