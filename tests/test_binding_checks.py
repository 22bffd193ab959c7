"""Host-side argument checks of the Python binding (no GPU needed).

Every shape the C ABI takes on trust (coordinates, maps, field values,
outputs, adjoint vectors and gradients, batch arrays, workspaces) is checked
in the binding before a device pointer is taken, so a mismatch is a
ValueError on the host and never an out-of-bounds access on the device. The
tensors here live on the CPU: the shape check must fire before the
device-tensor check would."""
import numpy as np
import pytest
import torch

from paper_1407_0904_amd import coffee as cf


def f64(*shape):
    return torch.zeros(shape, dtype=torch.float64)


def i32(*shape):
    return torch.zeros(shape, dtype=torch.int32)


def i64(*shape):
    return torch.zeros(shape, dtype=torch.int64)


def test_assemble_mesh_shapes():
    with pytest.raises(ValueError, match="coords has shape"):
        cf.coffee_assemble("mass", 3, 2, f64(10, 2), i32(5, 4))
    with pytest.raises(ValueError, match="cell_to_vertex has shape"):
        cf.coffee_assemble("mass", 3, 2, f64(10, 3), i32(5, 3))
    with pytest.raises(ValueError, match="cell_to_vertex must be"):
        cf.coffee_assemble("mass", 3, 2, f64(10, 3), i64(5, 4))


def test_assemble_field_shapes():
    coords, c2v = f64(10, 3), i32(5, 4)
    # P2 dof map of the wrong width
    bad_map = cf.DeviceField(f64(20, 1), i32(5, 4), 2, 1)
    with pytest.raises(ValueError, match="cell_to_dof has shape"):
        cf.coffee_assemble("helmholtz", 3, 2, coords, c2v, coeffs=[bad_map])
    # dof map for fewer cells than the mesh has
    short = cf.DeviceField(f64(20, 1), i32(4, 10), 2, 1)
    with pytest.raises(ValueError, match="cell_to_dof has shape"):
        cf.coffee_assemble("helmholtz", 3, 2, coords, c2v, coeffs=[short])
    # values with the wrong component count
    vec = cf.DeviceField(f64(20, 2), i32(5, 10), 2, 3)
    with pytest.raises(ValueError, match="values has shape"):
        cf.coffee_assemble("burgers", 3, 2, coords, c2v, coeffs=[vec])
    # cell-major values of the wrong size
    cm = cf.DeviceField(f64(5, 9, 1), None, 2, 1)
    with pytest.raises(ValueError, match="values has 45 elements"):
        cf.coffee_assemble("helmholtz", 3, 2, coords, c2v, coeffs=[cm])


def test_assemble_output_shape():
    coords, c2v = f64(10, 3), i32(5, 4)
    with pytest.raises(ValueError, match="out has 499 elements"):
        cf.coffee_assemble("mass", 3, 2, coords, c2v, out=f64(499))
    with pytest.raises(ValueError, match="out must be"):
        cf.coffee_assemble("mass", 3, 2, coords, c2v, out=torch.zeros(500, dtype=torch.float32))
    with pytest.raises(ValueError, match="out has"):
        cf.coffee_assemble("svk_residual", 3, 1, coords, c2v, out=torch.zeros(5 * 13, dtype=torch.float32),
                           coeffs=[cf.DeviceField(f64(10, 3), c2v, 1, 3)], precision="fp32")


def test_adjoint_shapes():
    coords, c2v = f64(10, 3), i32(5, 4)
    mu = cf.DeviceField(f64(10, 1), c2v, 1, 1)
    lm = cf.DeviceField(f64(10, 1), c2v, 1, 1)
    N = 30
    good = dict(coeffs=[mu, lm], lam=f64(5, N), u=f64(5, N))
    with pytest.raises(ValueError, match="lam has shape"):
        cf.coffee_assemble_adjoint("elasticity", 3, 2, coords, c2v, coeffs=[mu, lm], lam=f64(5, N - 1), u=f64(5, N))
    with pytest.raises(ValueError, match="u has shape"):
        cf.coffee_assemble_adjoint("elasticity", 3, 2, coords, c2v, coeffs=[mu, lm], lam=f64(5, N), u=f64(4, N))
    with pytest.raises(ValueError, match="grad_coords has shape"):
        cf.coffee_assemble_adjoint("elasticity", 3, 2, coords, c2v, grad_coords=f64(9, 3), **good)
    with pytest.raises(ValueError, match=r"grad_coeffs\[1\] has shape"):
        cf.coffee_assemble_adjoint("elasticity", 3, 2, coords, c2v, grad_coeffs=[f64(10, 1), f64(11, 1)], **good)
    with pytest.raises(ValueError, match="grad_coeffs has 1 entries"):
        cf.coffee_assemble_adjoint("elasticity", 3, 2, coords, c2v, grad_coeffs=[f64(10, 1)], **good)
    with pytest.raises(ValueError, match="cell_value has"):
        cf.coffee_assemble_adjoint("elasticity", 3, 2, coords, c2v, cell_value=f64(4), **good)


def _segments(n_cells=6):
    coords, c2v = f64(10, 2), i32(n_cells, 3)
    f = cf.DeviceField(f64(10, 1), c2v, 1, 1)
    return [cf.Segment("mass", 2, 1, coords, c2v, f), cf.Segment("helmholtz", 2, 2, coords, c2v, f)]


def test_batch_shapes():
    segs = _segments()
    n = 4
    seg_of, cell_of, offs = i32(n), i64(n), i64(n)
    total = 4 * 36
    ws = torch.zeros(cf.coffee_batch_workspace_size(2, n), dtype=torch.uint8)
    out = torch.zeros(total, dtype=torch.float32)
    kw = dict(out=out, workspace=ws)
    with pytest.raises(ValueError, match="cell_of has shape"):
        cf.coffee_assemble_batch(segs, seg_of, i64(n + 1), offs, total, **kw)
    with pytest.raises(ValueError, match="out_offset has shape"):
        cf.coffee_assemble_batch(segs, seg_of, cell_of, i64(n - 1), total, **kw)
    with pytest.raises(ValueError, match="seg_of must be"):
        cf.coffee_assemble_batch(segs, i64(n), cell_of, offs, total, **kw)
    with pytest.raises(ValueError, match="fewer than total_elems"):
        cf.coffee_assemble_batch(segs, seg_of, cell_of, offs, total + 1, **kw)
    with pytest.raises(ValueError, match="workspace has"):
        cf.coffee_assemble_batch(segs, seg_of, cell_of, offs, total, out=out, workspace=ws[:-1])
    bad = list(segs)
    bad[1] = cf.Segment("mass", 2, 2, f64(10, 3), segs[1].cell_to_vertex, segs[1].coeff)
    with pytest.raises(ValueError, match=r"segments\[1\]\.coords has shape"):
        cf.coffee_assemble_batch(bad, seg_of, cell_of, offs, total, **kw)
    with pytest.raises(ValueError, match="out_offset has shape"):
        cf.coffee_assemble_batch_packed(segs, seg_of, cell_of, total, out=out, out_offset=i64(n + 2), workspace=ws)


def test_check_geometry_shapes():
    with pytest.raises(ValueError, match="cell_to_vertex has shape"):
        cf.coffee_check_geometry(2, f64(10, 2), i32(5, 4))
