"""C ABI of libcoffee without a GPU: exported symbols, host validation and the
host tabulation (checked against the oracle's independent tables)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SO = os.path.join(ROOT, "paper_1407_0904_amd", "libcoffee.so")
HDR = os.path.join(ROOT, "include", "coffee.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(SO):
        from paper_1407_0904_amd import build
        build.build()
    return C.CDLL(SO)


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(coffee_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "coffee_assemble" in names and "coffee_tabulate" in names and "coffee_assemble_adjoint" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    lib.coffee_status_string.restype = C.c_char_p
    assert lib.coffee_status_string(0) == b"ok"
    assert b"invalid" in lib.coffee_status_string(1)
    assert lib.coffee_status_string(99) == b"unknown status"


def _assemble(lib, form=1, cell=2, degree=1, q=-1, prec=0, coords=None, nvert=3, c2v=None, ncells=1,
              coeffs=None, ncoeff=0, consts=None, nconst=0, out=None):
    f = lib.coffee_assemble
    f.argtypes = [C.c_int] * 5 + [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_int,
                                  C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
    return f(form, cell, degree, q, prec, coords, nvert, c2v, ncells, coeffs, ncoeff, consts, nconst, out, None)


def test_validation_before_any_hip_call(lib):
    """Invalid arguments are rejected on the host (status 1/2), never reaching HIP."""
    dummy = C.c_void_p(16)  # never dereferenced: validation fails first
    assert _assemble(lib, coords=None, c2v=dummy, out=dummy) == 1
    assert _assemble(lib, coords=dummy, c2v=None, out=dummy) == 1
    assert _assemble(lib, coords=dummy, c2v=dummy, out=None) == 1
    assert _assemble(lib, form=9, coords=dummy, c2v=dummy, out=dummy) == 1
    assert _assemble(lib, cell=4, coords=dummy, c2v=dummy, out=dummy) == 1
    assert _assemble(lib, degree=0, coords=dummy, c2v=dummy, out=dummy) == 1
    assert _assemble(lib, degree=5, coords=dummy, c2v=dummy, out=dummy) == 1
    assert _assemble(lib, prec=3, coords=dummy, c2v=dummy, out=dummy) == 1
    assert _assemble(lib, ncells=-1, coords=dummy, c2v=dummy, out=dummy) == 1
    assert _assemble(lib, q=11, coords=dummy, c2v=dummy, out=dummy) == 1
    # elasticity without fields needs (mu, lambda)
    assert _assemble(lib, form=2, coords=dummy, c2v=dummy, out=dummy) == 1
    # Burgers needs one vector field
    assert _assemble(lib, form=3, coords=dummy, c2v=dummy, out=dummy) == 1
    # prisms (cell 6): vector forms, degree 4 and a non-default rule are outside the compiled set;
    # diffusion (form 7) takes no field
    assert _assemble(lib, form=2, cell=6, coords=dummy, c2v=dummy, out=dummy) == 2
    assert _assemble(lib, form=1, cell=6, degree=4, coords=dummy, c2v=dummy, out=dummy) == 2
    assert _assemble(lib, form=7, cell=6, q=3, coords=dummy, c2v=dummy, out=dummy) == 2
    assert _assemble(lib, form=8, coords=dummy, c2v=dummy, out=dummy) == 1


def test_tensor_dims(lib):
    f = lib.coffee_tensor_dim
    assert f(1, 2, 1) == 3 and f(1, 3, 2) == 10 and f(2, 3, 2) == 30 and f(3, 3, 1) == 12
    assert f(0, 3, 4) == 35 and f(4, 3, 2) == 0 and f(6, 3, 2) == 30 and f(9, 3, 2) == -1
    # diffusion (7) is scalar; prisms (6): 6, 18, 40, 75 dofs, scalar forms only
    assert f(7, 2, 3) == 10 and f(7, 3, 2) == 10
    assert [f(1, 6, p) for p in (1, 2, 3, 4)] == [6, 18, 40, 75] and f(7, 6, 2) == 18 and f(2, 6, 1) == -1


def test_diffusion_instances_registered(lib):
    """Every diffusion key (triangles and tetrahedra, P1-P4, no field) has a
    kernel in every precision (a registry lookup, no HIP call)."""
    f = lib.coffee_has_variant
    for d in (2, 3):
        for p in (1, 2, 3, 4):
            for prec in (0, 1, 2):
                assert f(7, d, p, 0, prec, 0) == 1, (d, p, prec)
    assert f(7, 3, 2, 1, 0, 0) == 0  # no field-carrying diffusion


@pytest.mark.parametrize("p,q", [(1, 2), (2, 4), (3, 6), (4, 8), (2, 2 + 16), (0, 3)])
def test_prism_tabulate_matches_oracle(lib, oracle, p, q):
    """Library prism tables (Golub-Welsch rules, Vandermonde bases) equal the oracle's."""
    nq, nd = C.c_int(), C.c_int()
    tab = lib.coffee_tabulate
    tab.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)] + [C.c_void_p] * 4
    assert tab(6, p, q, C.byref(nq), C.byref(nd), None, None, None, None) == 0
    X = np.zeros((nq.value, 3)); W = np.zeros(nq.value); B = np.zeros((nq.value, nd.value))
    D = np.zeros((3, nq.value, nd.value))
    assert tab(6, p, q, C.byref(nq), C.byref(nd), X.ctypes.data, W.ctypes.data, B.ctypes.data, D.ctypes.data) == 0
    Xo, Wo, Bo, Do = oracle.tabulate(6, p, q)
    np.testing.assert_allclose(X, Xo, atol=1e-15)
    np.testing.assert_allclose(W, Wo, rtol=1e-14)
    np.testing.assert_allclose(B, Bo, atol=2e-14)
    np.testing.assert_allclose(D, Do, atol=1e-13)


@pytest.mark.parametrize("d,p,q", [(2, 1, 2), (2, 4, 8), (3, 2, 4), (3, 3, 6), (3, 4, 8), (2, 2, 5), (3, 0, 3)])
def test_tabulate_matches_oracle(lib, oracle, d, p, q):
    """Golub-Welsch + Vandermonde tables equal the oracle's Newton + Silvester tables."""
    nq, nd = C.c_int(), C.c_int()
    tab = lib.coffee_tabulate
    tab.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)] + [C.c_void_p] * 4
    assert tab(d, p, q, C.byref(nq), C.byref(nd), None, None, None, None) == 0
    X = np.zeros((nq.value, d)); W = np.zeros(nq.value); B = np.zeros((nq.value, nd.value))
    D = np.zeros((d, nq.value, nd.value))
    assert tab(d, p, q, C.byref(nq), C.byref(nd), X.ctypes.data, W.ctypes.data, B.ctypes.data, D.ctypes.data) == 0
    Xo, Wo, Bo, Do = oracle.tabulate(d, p, q)
    np.testing.assert_allclose(X, Xo, atol=1e-15)
    np.testing.assert_allclose(W, Wo, rtol=1e-14)
    np.testing.assert_allclose(B, Bo, atol=2e-14)
    np.testing.assert_allclose(D, Do, atol=1e-13)
    assert tab(5, p, q, C.byref(nq), C.byref(nd), None, None, None, None) == 1


def test_tuning_cache_parsing(lib, tmp_path):
    """The tuning cache loader accepts the tuner's format and rejects malformed lines."""
    f = lib.coffee_load_tuning
    f.argtypes = [C.c_char_p]
    good = tmp_path / "good.txt"
    good.write_text("# comment\nlinear 1 3 2 2 0 2\nlinear 1 3 2 2 1 4 1\nbatch 0 2 1 1 1 128 0.25\n"
                    "packed 0 2 1 1 512 0.2\n\n")
    assert f(str(good).encode()) == 0
    bad = tmp_path / "bad.txt"
    bad.write_text("batch 0 2 1 1 1 100 0.25\n")
    assert f(str(bad).encode()) == 1
    bad.write_text("linear 1 3 2 2 0 4 4\n")  # no tile-shape variant 4
    assert f(str(bad).encode()) == 1
    bad.write_text("packed 0 2 1 1 96 0.25\n")
    assert f(str(bad).encode()) == 1
    assert f(str(tmp_path / "missing.txt").encode()) == 1
    assert f(None) == 0
    from paper_1407_0904_amd import tuner
    out = tmp_path / "w.txt"
    tuner.write_cache(str(out), [("linear", 1, 3, 2, 2, 0, 4, 1), ("batch", 1, 3, 3, 1, 0, 256, 1.5),
                                 ("packed", 1, 3, 3, 1, 512, 1.25)])
    assert f(str(out).encode()) == 0
    assert tuner.read_batch_costs(str(out)) == {("helmholtz", 3, 3, "fp32"): 1.5}
    assert tuner.read_batch_costs(str(out), "packed") == {("helmholtz", 3, 3, "fp32"): 1.25}
    # the cache shipped with the package (the benchmark's launch configuration) loads
    shipped = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1407_0904_amd",
                           "tuning_mi355x.txt")
    assert f(shipped.encode()) == 0
    assert f(None) == 0


def test_batch_workspace_size_checked_on_host(lib):
    """A workspace smaller than coffee_batch_workspace_size is reported
    (status 3) before anything is read from the segment array or the device."""
    lib.coffee_batch_workspace_size.restype = C.c_int64
    lib.coffee_batch_workspace_size.argtypes = [C.c_int, C.c_int64]
    need = lib.coffee_batch_workspace_size(1, 1000)
    assert need >= 1000 * 12
    for name in ("coffee_assemble_batch",):
        f = getattr(lib, name)
        f.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                      C.c_void_p, C.c_int64, C.c_void_p]
        f.restype = C.c_int
        dummy = C.c_void_p(16)  # never dereferenced
        assert f(1, dummy, 1, dummy, dummy, dummy, 1000, dummy, dummy, need - 1, None) == 3
        assert f(1, dummy, 17, dummy, dummy, dummy, 1000, dummy, dummy, need, None) == 1


def test_noalloc_batch_limit_checked_on_host(lib):
    """The allocation-free batch rejects more entries than its static scratch
    array holds (status 3) before any HIP call."""
    f = lib.coffee_assemble_batch_packed_noalloc
    f.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                  C.c_void_p]
    f.restype = C.c_int
    dummy = C.c_void_p(16)  # never dereferenced
    assert f(1, dummy, 1, dummy, dummy, 4194304 + 1, dummy, dummy, None) == 3
    assert f(1, dummy, 1, dummy, dummy, -1, dummy, dummy, None) == 1


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("q", range(1, 7))
def test_symmetric_rules_match_oracle(lib, oracle, d, q):
    """The library's symmetric rules (Gauss-Newton on Cartesian moments) and
    the oracle's (Gauss-Newton on barycentric moments, separate code) are the
    same point sets with the same weights."""
    from paper_1407_0904_amd import coffee as cf
    Xo, Wo = oracle.symmetric_rule(d, q)
    Xl, Wl, _, _ = cf.coffee_tabulate(d, 1, q + 16)
    assert Wl.shape == Wo.shape
    a = np.lexsort(np.c_[Xo, Wo].T[::-1])
    b = np.lexsort(np.c_[Xl, Wl].T[::-1])
    np.testing.assert_allclose(Xl[b], Xo[a], atol=1e-14)
    np.testing.assert_allclose(Wl[b], Wo[a], rtol=1e-13, atol=1e-16)
