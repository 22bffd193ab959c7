"""Offline autotuner of libcoffee's launch choices.

For every key it times each candidate on the GPU (median of repeated launches,
with events on the current stream) and keeps the fastest, the way the paper
reports the best over every feasible unroll factor for its register tiling
(section 5.6); the search runs offline, so its cost never reaches the assembly
call. Keys and candidates:

* coffee_assemble (form, cell, degree, field degree, precision): the
  tile-shape variant of the symmetric engine (reference fragments in
  registers at one wave per SIMD, in LDS at two waves per SIMD, read through
  the caches at two waves per SIMD, or through the caches at three waves per
  SIMD with no prefetch across chunks; coffee_set_variant) x the grid
  multiplier (persistent grid of CUs x resident workgroups x m, or one
  workgroup per 256 cells);
* mixed-batch bins (form, cell, degree, precision): store variant (LDS-staged
  or direct) x cells per queue task for the caller's layout, and cells per
  queue task for the packed layout; the measured ns per cell is kept so that
  callers can order bins by cost.

The result is a text cache read by coffee_load_tuning / COFFEE_TUNE_CACHE.

    python -m paper_1407_0904_amd.tuner --out tuning.txt [--quick]
"""
from __future__ import annotations

import argparse
import os
import statistics
import sys

import numpy as np

FORM_IDS = {"mass": 0, "helmholtz": 1, "elasticity": 2, "burgers": 3, "diffusion": 7}
PREC_IDS = {"fp64": 0, "fp32": 1, "bf16x3": 2}


def _time(fn, reps: int = 7, warm: int = 2) -> float:
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def tune_linear(workload_name: str, precisions=("fp64",), candidates=(1, 2, 3, 4, 8, 64), variants=(0, 1, 2, 3),
                log=print):
    """Best (tile-shape variant, grid multiplier) per precision for one named workload."""
    import torch
    from . import coffee, inputs
    dev = torch.device("cuda:0")
    w = inputs.workload(workload_name)
    coords = torch.as_tensor(w.mesh.coords, device=dev)
    c2v = torch.as_tensor(w.mesh.cells, device=dev)
    fields = [coffee.DeviceField.from_host(f, dev) for f in w.fields]
    fd = w.fields[0].degree if w.fields else 0
    entries = []
    for prec in precisions:
        out = torch.empty(coffee.output_shape(w.form, w.mesh.ncells, w.mesh.cell, w.degree),
                          dtype=torch.float64 if prec == "fp64" else torch.float32, device=dev)
        best = None
        for var in variants:
            if var and not coffee.coffee_has_variant(w.form, w.mesh.cell, w.degree, fd, prec, var):
                continue
            coffee.coffee_set_variant(var)
            for m in candidates:
                coffee.coffee_set_launch_options(m)
                call = coffee.PreparedAssemble(w.form, w.mesh.cell, w.degree, coords, c2v, coeffs=fields,
                                               constants=w.constants, quad_degree=w.quad_degree, precision=prec,
                                               out=out)
                ms = _time(call)
                log(f"  {workload_name} {prec} variant {var} grid_mult {m}: {ms * 1e3:.1f} us")
                if best is None or ms < best[2]:
                    best = (var, m, ms)
        coffee.coffee_set_launch_options(0)
        coffee.coffee_set_variant(-1)
        entries.append(("linear", FORM_IDS[w.form], w.mesh.cell, w.degree, fd, PREC_IDS[prec], best[1], best[0]))
        del out
    return entries


def tune_batch(mb, precision: str = "fp32", variants=(0, 1), task_cells=(64, 128, 256, 512, 1024), log=print):
    """Best (variant, task_cells) per bin of a mixed batch, timed one bin at a time."""
    import torch
    from . import coffee
    dev = torch.device("cuda:0")
    tri_c = torch.as_tensor(mb.tri.coords, device=dev)
    tri_v = torch.as_tensor(mb.tri.cells, device=dev)
    tet_c = torch.as_tensor(mb.tet.coords, device=dev)
    tet_v = torch.as_tensor(mb.tet.cells, device=dev)
    f_tri = coffee.DeviceField.from_host(mb.f_tri, dev)
    f_tet = coffee.DeviceField.from_host(mb.f_tet, dev)
    entries = []
    for b, (form, d, p) in enumerate(mb.segments):
        idx = np.nonzero(mb.seg_of == b)[0]
        n = idx.size
        if n == 0:
            continue
        c, v, f = (tri_c, tri_v, f_tri) if d == 2 else (tet_c, tet_v, f_tet)
        seg_of = torch.zeros(n, dtype=torch.int32, device=dev)
        cell_of = torch.as_tensor(mb.cell_of[idx], device=dev)
        size = (p + 1) * (p + 2) // 2 if d == 2 else (p + 1) * (p + 2) * (p + 3) // 6
        offs = torch.arange(n, dtype=torch.int64, device=dev) * (size * size)
        out = torch.empty(n * size * size, dtype=torch.float64 if precision == "fp64" else torch.float32, device=dev)
        ws = torch.empty(coffee.coffee_batch_workspace_size(1, n), dtype=torch.uint8, device=dev)
        best = None
        for var in variants:
            for tc in task_cells:
                seg = coffee.Segment(form, d, p, c, v, f, variant=var, task_cells=tc)
                ms = _time(lambda: coffee.coffee_assemble_batch([seg], seg_of, cell_of, offs, out.numel(),
                                                                precision=precision, out=out, workspace=ws))
                log(f"  bin {form} d{d} p{p} {precision} variant {var} task {tc}: {ms * 1e3:.1f} us ({n} cells)")
                if best is None or ms < best[2]:
                    best = (var, tc, ms)
        entries.append(("batch", FORM_IDS[form], d, p, PREC_IDS[precision], best[0], best[1],
                        best[2] * 1e6 / n))
        del out, ws
    return entries


def tune_batch_packed(mb, precision: str = "fp32", task_cells=(64, 128, 256, 512, 1024), log=print):
    """Best cells per task per bin of a mixed batch in the packed layout, timed one bin at a time."""
    import torch
    from . import coffee
    dev = torch.device("cuda:0")
    tri_c = torch.as_tensor(mb.tri.coords, device=dev)
    tri_v = torch.as_tensor(mb.tri.cells, device=dev)
    tet_c = torch.as_tensor(mb.tet.coords, device=dev)
    tet_v = torch.as_tensor(mb.tet.cells, device=dev)
    f_tri = coffee.DeviceField.from_host(mb.f_tri, dev)
    f_tet = coffee.DeviceField.from_host(mb.f_tet, dev)
    entries = []
    for b, (form, d, p) in enumerate(mb.segments):
        idx = np.nonzero(mb.seg_of == b)[0]
        n = idx.size
        if n == 0:
            continue
        c, v, f = (tri_c, tri_v, f_tri) if d == 2 else (tet_c, tet_v, f_tet)
        seg_of = torch.zeros(n, dtype=torch.int32, device=dev)
        cell_of = torch.as_tensor(mb.cell_of[idx], device=dev)
        size = (p + 1) * (p + 2) // 2 if d == 2 else (p + 1) * (p + 2) * (p + 3) // 6
        out = torch.empty(n * size * size, dtype=torch.float64 if precision == "fp64" else torch.float32, device=dev)
        offs = torch.empty(n, dtype=torch.int64, device=dev)
        ws = torch.empty(coffee.coffee_batch_workspace_size(1, n), dtype=torch.uint8, device=dev)
        best = None
        for tc in task_cells:
            seg = coffee.Segment(form, d, p, c, v, f, task_cells=tc)
            ms = _time(lambda: coffee.coffee_assemble_batch_packed([seg], seg_of, cell_of, out.numel(),
                                                                   precision=precision, out=out, out_offset=offs,
                                                                   workspace=ws))
            log(f"  packed bin {form} d{d} p{p} {precision} task {tc}: {ms * 1e3:.1f} us ({n} cells)")
            if best is None or ms < best[1]:
                best = (tc, ms)
        entries.append(("packed", FORM_IDS[form], d, p, PREC_IDS[precision], best[0], best[1] * 1e6 / n))
        del out, offs, ws
    return entries


def write_cache(path: str, entries, header: str = ""):
    with open(path, "w") as f:
        f.write("# coffee tuning cache (written by paper_1407_0904_amd.tuner)\n")
        if header:
            f.write(f"# {header}\n")
        for e in entries:
            if e[0] == "linear":
                f.write("linear %d %d %d %d %d %d %d\n" % e[1:])
            elif e[0] == "packed":
                f.write("packed %d %d %d %d %d %.6f\n" % e[1:])
            else:
                f.write("batch %d %d %d %d %d %d %.6f\n" % e[1:])


def read_batch_costs(path: str, kind: str = "batch"):
    """{(form, cell, degree, precision): ns_per_cell} of a cache file's "batch"
    (caller's layout) or "packed" lines."""
    costs = {}
    if not path or not os.path.exists(path):
        return costs
    inv_f = {v: k for k, v in FORM_IDS.items()}
    inv_p = {v: k for k, v in PREC_IDS.items()}
    for line in open(path):
        line = line.split("#", 1)[0].split()
        if line and line[0] == kind:
            form, cell, deg, prec = (int(x) for x in line[1:5])
            costs[(inv_f[form], cell, deg, inv_p[prec])] = float(line[-1])
    return costs


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--quick", action="store_true", help="small mixed batch (for tests)")
    args = ap.parse_args(argv)
    import torch
    from . import coffee, inputs
    name = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "unknown"
    entries = []
    if not args.quick:
        entries += tune_linear("helmholtz_p2_tet", ("fp64", "fp32", "bf16x3"))
        entries += tune_linear("helmholtz_p1_tri", ("fp64",))
        entries += tune_linear("elasticity_p2_tet", ("fp64", "fp32", "bf16x3"), candidates=(1, 2, 4, 8))
        entries += tune_linear("burgers_p2_tet", ("fp64", "fp32", "bf16x3"), candidates=(1, 2, 4, 8))
        entries += tune_linear("helmholtz_p1_prism", ("fp64", "fp32", "bf16x3"), candidates=(1, 2, 4), variants=(0,))
        entries += tune_linear("diffusion_p2_prism", ("fp64", "fp32", "bf16x3"), candidates=(1, 2, 3, 4, 8),
                               variants=(0,))
        entries += tune_linear("diffusion_p3_prism", ("fp64", "fp32", "bf16x3"), candidates=(1, 2, 3, 4, 8),
                               variants=(0,))
        mb = inputs.mixed_batch()
    else:
        mb = inputs.mixed_batch(n_tri=64, n_tet=12, tri_counts=(3000, 2000, 1500, 1000),
                                tet_counts=(3000, 2000, 1000))
    entries += tune_batch(mb, "fp32")
    entries += tune_batch_packed(mb, "fp32")
    write_cache(args.out, entries, header=f"device {name}")
    coffee.coffee_load_tuning(args.out)
    print(f"wrote {len(entries)} entries to {args.out}")


if __name__ == "__main__":
    sys.exit(main())
