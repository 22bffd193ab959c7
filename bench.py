#!/usr/bin/env python3
"""Benchmark of the local-assembly hot path on one MI355X.

A step is one coffee_assemble call over the whole workload (geometry, coefficient
gather, G construction, contraction and element-tensor store for every cell),
with inputs resident in HBM. Default workload: Helmholtz P2 on 64^3 x 6 =
1,572,864 jittered tetrahedra, f in P2, quadrature degree 4, FP64. The same
line reports the FP32 and BF16X3 variants of that workload with their error
against the FP64 oracle, the roofline of the assembly kernel, and the oracle
itself timed on the host cores over a bounded sample of cells.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision P]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cells/s + GB/s (frac of roofline) per form; FP32/BF16 vs FP64 at stated err"

WORKLOADS = {
    # name: description used in the JSON config
    "helmholtz_p2_tet": "Helmholtz P2 tetrahedra, 64^3 x 6 cells, f P2 ~ U[0.5,1.5], jitter 10%, q = 4",
    "helmholtz_p1_tri": "Helmholtz P1 triangles, 64^2 x 2 cells, f P1 ~ U[0.5,1.5], jitter 20%, q = 2",
    "elasticity_p2_tet": "elasticity vector P2 tetrahedra, 48^3 x 6 cells, mu, lambda P1 ~ U[1,10], q = 4",
    "burgers_p2_tet": "Burgers Jacobian vector P2 tetrahedra, 48^3 x 6 cells, w P2 ~ U[-1,1], q = 5",
    "burgers_p1_tet": "Burgers Jacobian vector P1 tetrahedra, 48^3 x 6 cells, w P1 ~ U[-1,1], q = 3",
}


def algorithmic_bytes(w, out_elem: int) -> int:
    """Each input array read once, element tensors written once (int32 maps)."""
    from paper_1407_0904_amd.coffee import output_shape
    E = w.mesh.ncells
    b = w.mesh.coords.nbytes + w.mesh.cells.nbytes
    for f in w.fields:
        b += f.values.nbytes
        if f.cell_to_dof is not None and f.cell_to_dof is not w.mesh.cells:
            b += f.cell_to_dof.nbytes
    b += int(np.prod(output_shape(w.form, E, w.mesh.d, w.degree))) * out_elem
    return int(b)


def cell_rel_err(got, ref):
    E = ref.shape[0]
    g = got.reshape(E, -1).astype(np.float64)
    r = ref.reshape(E, -1)
    return float(np.max(np.max(np.abs(g - r), 1) / np.maximum(np.max(np.abs(r), 1), 1e-300)))


def time_gpu(fn, steps: int, warmup: int):
    """(ms per step over the bracketed region, mean per-launch ms from events)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(s)
    for k in range(steps):
        starts[k].record(s)
        fn()
        ends[k].record(s)
    t1.record(s)
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    return t0.elapsed_time(t1) / steps, float(np.mean(per)), per


def cpu_baseline(w, target_s: float = 12.0):
    """The oracle on the host cores over the first cells of the same workload."""
    from oracle import oracle as O
    cores = len(os.sched_getaffinity(0))
    E = w.mesh.ncells
    n0 = min(E, 2048)
    t = time.perf_counter()
    O.assemble(w.form, w.mesh, w.degree, w.quad_degree, fields=w.fields, constants=w.constants,
               cells=np.arange(n0), nthreads=cores)
    dt = time.perf_counter() - t
    n = int(min(E, max(n0, n0 * target_s / max(dt, 1e-6))))
    t = time.perf_counter()
    O.assemble(w.form, w.mesh, w.degree, w.quad_degree, fields=w.fields, constants=w.constants,
               cells=np.arange(n), nthreads=cores)
    dt = time.perf_counter() - t
    return {"value": n / dt, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of {E} cells of the same workload, FP64, OpenMP static over cells, "
                      f"{dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="helmholtz_p2_tet", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of the output's byte size (counter calibration)")
    ap.add_argument("--grid-mult", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: local assembly needs no communication on the forward path, "
              "and this build runs on a single MI355X (see the sharding note in the design notes). "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1407_0904_amd import coffee, inputs
    from oracle import oracle as O

    dev = torch.device("cuda:0")
    w = inputs.workload(args.workload)
    coords = torch.as_tensor(w.mesh.coords, device=dev)
    c2v = torch.as_tensor(w.mesh.cells, device=dev)
    fields = [coffee.DeviceField.from_host(f, dev) for f in w.fields]
    coffee.coffee_set_launch_options(args.grid_mult)

    def run(prec, out):
        return lambda: coffee.coffee_assemble(w.form, w.mesh.d, w.degree, coords, c2v, coeffs=fields,
                                              constants=w.constants, quad_degree=w.quad_degree,
                                              precision=prec, out=out)

    E = w.mesh.ncells
    shape = coffee.output_shape(w.form, E, w.mesh.d, w.degree)
    sample = np.unique(np.concatenate([[0, E - 1], np.random.default_rng(3).integers(0, E, 1500)]))
    ref = O.assemble(w.form, w.mesh, w.degree, w.quad_degree, fields=w.fields, constants=w.constants,
                     cells=sample)
    idx = torch.as_tensor(sample, device=dev)

    results = {}
    precs = [args.precision] + ([] if args.no_variants else [p for p in ("fp64", "fp32", "bf16x3")
                                                             if p != args.precision])
    for prec in precs:
        out = torch.empty(shape, dtype=torch.float64 if prec == "fp64" else torch.float32, device=dev)
        ms, kms, per = time_gpu(run(prec, out), args.steps, args.warmup)
        err = cell_rel_err(out[idx].cpu().numpy(), ref)
        nbytes = algorithmic_bytes(w, 8 if prec == "fp64" else 4)
        results[prec] = {"ms": ms, "kernel_ms": kms, "cells_per_s": E / (ms * 1e-3),
                         "gbs": nbytes / (kms * 1e-3) / 1e9, "bytes": nbytes, "err": err}
        del out
        torch.cuda.synchronize()

    if args.calibrate_copy:
        # a plain copy kernel of known size, for scaling the HBM byte counters
        nb = int(np.prod(shape)) * 8
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"calibration copy: {nb} bytes read and {nb} bytes written per launch", file=sys.stderr)
        del src, dst

    main_r = results[args.precision]
    line = {
        "metric": METRIC,
        "value": main_r["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 (f64 geometry)", "bf16x3": "bf16x3->f32 (f64 geometry)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "cells": E,
                   "element_tensor": list(shape[1:]), "precision": args.precision,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": main_r["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": main_r["gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": main_r["bytes"],
                     "kernel_ms": main_r["kernel_ms"]},
        "max_cell_rel_err_vs_oracle": main_r["err"],
        "variants": {p: {"cells_per_s": r["cells_per_s"], "ms": r["ms"], "gbs": r["gbs"],
                         "frac_hbm": r["gbs"] / HBM_PEAK_GBS, "max_cell_rel_err": r["err"],
                         "speedup_vs_fp64": (results["fp64"]["ms"] / r["ms"]) if "fp64" in results else None}
                     for p, r in results.items()},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
