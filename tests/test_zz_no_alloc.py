"""The allocation-free packed batch (coffee_assemble_batch_packed_noalloc)
against the workspace entry point (coffee_assemble_batch_packed): the same
kernels, so the same offsets and the same bits, on two calls in a row, the
second with a smaller batch (the static scratch keeps the first call's
contents)."""
import numpy as np
import pytest

from paper_1407_0904_amd import inputs as I

pytestmark = pytest.mark.gpu


def _device_batch(cf, mb):
    import torch
    dev = torch.device("cuda:0")
    tri_c = torch.as_tensor(mb.tri.coords, device=dev)
    tri_v = torch.as_tensor(mb.tri.cells, device=dev)
    tet_c = torch.as_tensor(mb.tet.coords, device=dev)
    tet_v = torch.as_tensor(mb.tet.cells, device=dev)
    f_tri = cf.DeviceField.from_host(mb.f_tri, dev)
    f_tet = cf.DeviceField.from_host(mb.f_tet, dev)
    segs = []
    for (form, d, p) in mb.segments:
        c, v, f = (tri_c, tri_v, f_tri) if d == 2 else (tet_c, tet_v, f_tet)
        segs.append(cf.Segment(form, d, p, c, v, f, task_cells=128))
    return segs, torch.as_tensor(mb.seg_of, device=dev), torch.as_tensor(mb.cell_of, device=dev)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_batch_equals_workspace_batch(precision):
    import torch
    assert torch.cuda.is_available()
    from paper_1407_0904_amd import coffee as cf
    odt = torch.float64 if precision == "fp64" else torch.float32
    big = I.mixed_batch(n_tri=24, n_tet=6, tri_counts=(400, 300, 200, 100), tet_counts=(500, 300, 200), seed=7)
    small = I.mixed_batch(n_tri=10, n_tet=3, tri_counts=(30, 20, 10, 5), tet_counts=(40, 9, 17), seed=8)
    for mb in (big, small):
        segs, seg_of, cell_of = _device_batch(cf, mb)
        n = seg_of.shape[0]
        ref, roff = cf.coffee_assemble_batch_packed(segs, seg_of, cell_of, mb.total_elems, precision=precision)
        out = torch.full((mb.total_elems,), -3.0, dtype=odt, device=seg_of.device)
        off = torch.full((n,), -7, dtype=torch.int64, device=seg_of.device)
        print(f"noalloc batch {precision}: {n} entries", flush=True)
        cf.coffee_assemble_batch_packed_noalloc(segs, seg_of, cell_of, out, off, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(off, roff)
        assert torch.equal(out, ref)
