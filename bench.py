#!/usr/bin/env python3
"""Benchmark of the local-assembly hot path on one MI355X.

A step is one coffee_assemble call over the whole workload: gather of vertex
coordinates and coefficient dofs, FP64 geometry, geometry tensor, contraction
and element-tensor store for every cell, with inputs resident in HBM. The
headline workload is Helmholtz P2 on 64^3 x 6 = 1,572,864 jittered
tetrahedra, f in P2, quadrature degree 4, FP64. The JSON line also carries:
  - variants: the FP32 and BF16X3 runs of that workload, with their error
    against the FP64 oracle and their speedup over the FP64 GPU path;
  - roofline: achieved algorithmic GB/s of the assembly kernel (mean launch
    time from events on the launching stream) against the 8 TB/s HBM peak;
  - cpu_baseline: the FP64 oracle timed on the host cores (and on one core);
  - forms: the other workloads (P1 triangles at 8,192 and 2,097,152 cells,
    vector P2 elasticity forward and adjoint, St Venant-Kirchhoff P1/P2
    energy, residual, Jacobian and energy adjoint, Burgers P1/P2, and the
    3,000,000-entry mixed batch against per-bin launches), each with cells/s,
    GB/s, the binding roofline (max of bytes/HBM and flops/peak) and the
    error against the oracle on sampled cells.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision P] [--no-forms]
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
FLOP_PEAK_TF = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}
METRIC = "cells/s + GB/s (frac of roofline) per form; FP32/BF16 vs FP64 at stated err"
TUNING = os.path.join(ROOT, "paper_1407_0904_amd", "tuning_mi355x.txt")
# HBM bytes per launch of the headline kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE, scaled by a plain copy of known size (profiles/
# k_scalar_helmholtz_p2_tet_fp64.md); valid only for the kernel they were taken on.
TRAFFIC = {("helmholtz_p2_tet", "fp64"): 1374.4e6}

WORKLOADS = {
    "helmholtz_p2_tet": "Helmholtz P2 tetrahedra, 64^3 x 6 cells, f P2 ~ U[0.5,1.5], jitter 10%, q = 4",
    "helmholtz_p1_tri": "Helmholtz P1 triangles, 64^2 x 2 cells, f P1 ~ U[0.5,1.5], jitter 20%, q = 2",
    "elasticity_p2_tet": "elasticity vector P2 tetrahedra, 48^3 x 6 cells, mu, lambda P1 ~ U[1,10], q = 4",
    "burgers_p2_tet": "Burgers Jacobian vector P2 tetrahedra, 48^3 x 6 cells, w P2 ~ U[-1,1], q = 5",
    "burgers_p1_tet": "Burgers Jacobian vector P1 tetrahedra, 48^3 x 6 cells, w P1 ~ U[-1,1], q = 3",
    "svk_p2_tet": "St Venant-Kirchhoff Jacobian vector P2 tetrahedra, 32^3 x 6 cells, u P2 ~ N(0, 0.01^2), q = 4",
    "helmholtz_p1_prism": "Helmholtz P1 warped prisms, 64^2 x 2 x 64 cells, f P1 ~ U[0.5,1.5], jitter 10%, q = 2",
    "diffusion_p2_prism": "diffusion P2 warped prisms, 64^2 x 2 x 64 cells, kappa = dt = 1, jitter 10%, q = 4",
    "diffusion_p3_prism": "diffusion P3 warped prisms, 32^2 x 2 x 32 cells, kappa = dt = 1, jitter 10%, q = 6",
}

log = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)


def n_scalar(d, p):
    return (p + 1) * (p + 2) // 2 if d == 2 else (p + 1) * (p + 2) * (p + 3) // 6


def algorithmic_bytes(w, out_elems: int, out_elem: int) -> int:
    """Each input array read once, the outputs written once (int32 maps)."""
    b = w.mesh.coords.nbytes + w.mesh.cells.nbytes
    for f in w.fields:
        b += f.values.nbytes
        if f.cell_to_dof is not None and f.cell_to_dof is not w.mesh.cells:
            b += f.cell_to_dof.nbytes
    return int(b + out_elems * out_elem)


# Peaks (MI355X published figures): HBM 8 TB/s; FP64 vector and matrix 78.6
# TFLOP/s; FP32 vector and matrix 157.3 TFLOP/s; dense BF16 matrix 2.5 PFLOP/s,
# of which BF16X3 spends three products per useful multiply-add.
PEAK_TF = {"mfma_f64": 78.6, "mfma_f32": 157.3, "mfma_bf16x3": 2500.0 / 3.0, "valu_f64": 78.6, "valu_f32": 157.3}


def svk_work(d: int, p: int, form: str, prec: str) -> dict:
    """Flops per cell (2 per multiply-add) that each SVK kernel executes, by
    the unit that executes them. Points: 1 at P1 (the integrand is constant),
    the symmetric rule at P2 (6 triangle / 14 tetrahedron points)."""
    ns, D, nb = n_scalar(d, p), d, d * (d + 1) // 2
    nq = 1 if p == 1 else {2: 6, 3: 14}[d]
    U = 2 * D * D * ns                                   # reference displacement gradient
    pt = 2 * D ** 3 + D * D * (2 * D + 2) + 3 * D * D + 2 * D * D   # H = U K, E, S, psi
    P = 2 * D ** 3                                       # P = F S
    if prec in ("fp64", "fp32"):
        unit = "valu_f64" if prec == "fp64" else "valu_f32"
        if form == "svk_energy":
            return {unit: nq * (U + pt + P)}
        if form == "svk_residual":
            return {unit: nq * (U + pt + P + 2 * D ** 3 + 2 * D * D * ns)}
        # Jacobian: F, S and S^ = K S K^T once per (cell, point); per block
        # k1, k2, F.F, H, the row products dphi^T H and the rank updates of the
        # block's n x n entries
        per_pt = U + 2 * D ** 3 + D * D * (2 * D + 2) + 3 * D * D + 2 * D ** 3 + nb * 2 * D * D
        per_blk = 4 * D * D + 2 * D + 8 * D * D + 2 * D * D * ns + 2 * D * ns * ns
        if prec == "fp64":
            return {"valu_f64": nq * (per_pt + nb * per_blk)}
        # FP32 mode: point data in FP64, the block accumulation in FP32
        return {"valu_f64": nq * (per_pt + nb * (4 * D * D + 2 * D + 8 * D * D)),
                "valu_f32": nq * nb * (2 * D * D * ns + 2 * D * ns * ns)}
    # BF16X3: useful multiply-adds of the contractions on the matrix cores,
    # point arithmetic in FP32 on the vector units
    interp = 2 * ns * (nq * D) * D
    if form == "svk_energy":
        return {"mfma_bf16x3": interp, "valu_f32": nq * pt}
    if form == "svk_residual":
        return {"mfma_bf16x3": interp + 2 * (nq * D) * ns * D, "valu_f32": nq * (pt + P + 2 * D ** 3)}
    kj = nq * D * D
    return {"mfma_bf16x3": interp + nb * 2 * kj * ns * ns,
            "valu_f32": nq * (pt + P + 4 * D ** 3 + 2 * D * D) + nb * kj * 10}


def prism_work(w, prec: str) -> dict:
    """Prisms (non-affine): per point, J, det J, K = J^-1, K K^T and the
    mass factor on the FP64 vector units (about 150 flops), then the
    contraction over K = nq x (terms per point) for the n(n+1)/2 unique
    entries on the matrix cores of the precision."""
    p, form = w.degree, w.form
    ns = (p + 1) * (p + 2) // 2 * (p + 1)
    m = (w.quad_degree + 2) // 2
    nq = m * m * m
    jq = {"mass": 1, "helmholtz": 7, "diffusion": 6}[form]
    mm = {"fp64": "mfma_f64", "fp32": "mfma_f32", "bf16x3": "mfma_bf16x3"}[prec]
    return {mm: 2.0 * nq * jq * ns * (ns + 1) / 2, "valu_f64": 150.0 * nq}


def work_model(w, prec: str) -> dict:
    """Flops per cell of the formulation each kernel implements, by unit.

    Linear forms: the q-collapsed contraction, 2 * K * (entries computed), K =
    number of geometry-tensor terms per block (mass and Helmholtz compute the
    upper triangle only; elasticity the upper blocks, Burgers every block), on the matrix
    cores of the precision (degree-1 mass and Helmholtz in FP64/FP32 on the
    vector units). St Venant-Kirchhoff: svk_work."""
    d, p, form = w.mesh.d, w.degree, w.form
    if form.startswith("svk"):
        return svk_work(d, p, form, prec)
    if w.mesh.cell == 6:
        return prism_work(w, prec)
    ns = n_scalar(d, p)
    nd = d * (d + 1) // 2
    fd = w.fields[0].degree if w.fields else 0
    nf = n_scalar(d, fd) if fd else 0
    if form == "mass":
        f = 2.0 * max(nf, 1) * ns * (ns + 1) / 2
    elif form == "helmholtz":
        f = 2.0 * (nf + nd) * ns * (ns + 1) / 2
    elif form == "elasticity":
        # the d(d+1)/2 upper blocks; the lower ones are their transposes
        # (tet P3, on the panel engine, contracts all d^2 blocks)
        nblk = d * d if (d == 3 and p == 3) else nd
        f = 2.0 * (max(nf, 1) * d * d) * nblk * ns * ns
    else:
        f = 2.0 * (1 + nd + 2 * nf * d) * (d * ns) ** 2
    if p == 1 and form in ("mass", "helmholtz") and prec != "bf16x3":
        return {"valu_f64" if prec == "fp64" else "valu_f32": f}
    return {{"fp64": "mfma_f64", "fp32": "mfma_f32", "bf16x3": "mfma_bf16x3"}[prec]: f}


def cell_rel_err(got, ref):
    E = ref.shape[0]
    g = got.reshape(E, -1).astype(np.float64)
    r = ref.reshape(E, -1)
    return float(np.max(np.max(np.abs(g - r), 1) / np.maximum(np.max(np.abs(r), 1), 1e-300)))


def time_gpu(fn, steps: int, warmup: int):
    """Bracketed ms per step, and per-launch ms from events on the launching stream."""
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
    per = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    return t0.elapsed_time(t1) / steps, per


def pct(per):
    return {"mean": float(per.mean()), "p10": float(np.percentile(per, 10)),
            "p50": float(np.median(per)), "p90": float(np.percentile(per, 90))}


def cpu_baseline(w, target_s: float = 12.0):
    """The oracle on all host cores over the first cells of the same workload,
    then on one core over a smaller prefix."""
    from oracle import oracle as O
    cores = len(os.sched_getaffinity(0))
    E = w.mesh.ncells

    def run(n, threads):
        t = time.perf_counter()
        O.assemble(w.form, w.mesh, w.degree, w.quad_degree, fields=w.fields, constants=w.constants,
                   cells=np.arange(n), nthreads=threads)
        return time.perf_counter() - t

    n0 = min(E, 4096)
    dt = run(n0, cores)
    n = int(min(E, max(n0, n0 * target_s / max(dt, 1e-6))))
    times = [run(n, cores) for _ in range(1 if n * dt / n0 > 5 else 3)]
    dt = float(np.median(times))
    n1 = min(E, 4096)
    dt1 = run(n1, 1)
    return {"value": n / dt, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of {E} cells of the same workload, FP64, OpenMP static over cells, "
                      f"median of {len(times)} x {dt:.2f} s wall",
            "single_core_cells_per_s": n1 / dt1, "single_core_sample": f"first {n1} cells, {dt1:.2f} s"}


class Ctx:
    def __init__(self, steps, warmup):
        import torch
        from paper_1407_0904_amd import coffee
        self.torch = torch
        self.cf = coffee
        self.dev = torch.device("cuda:0")
        self.steps = steps
        self.warmup = warmup

    def upload(self, w):
        coords = self.torch.as_tensor(w.mesh.coords, device=self.dev)
        c2v = self.torch.as_tensor(w.mesh.cells, device=self.dev)
        fields = [self.cf.DeviceField.from_host(f, self.dev) for f in w.fields]
        return coords, c2v, fields


def roof(nbytes, work, kms):
    """Binding roofline: t_bound = max(bytes / HBM peak, flops_u / peak_u over
    the units u doing the work); frac = t_bound / measured."""
    t = {"hbm": nbytes / (HBM_PEAK_GBS * 1e9) * 1e3}
    for unit, flops in work.items():
        t[unit] = flops / (PEAK_TF[unit] * 1e12) * 1e3
    bound = max(t, key=t.get)
    return {"bound": bound, "frac": t[bound] / kms, "gbs": nbytes / (kms * 1e-3) / 1e9,
            "gflops": sum(work.values()) / (kms * 1e-3) / 1e9, "t_bound_ms": t[bound]}


def measure_forward(ctx, w, prec, sample_n=300, seed=3, tag=None):
    """One form: time, throughput, binding roofline, error on sampled cells."""
    from oracle import oracle as O
    torch, cf = ctx.torch, ctx.cf
    coords, c2v, fields = ctx.upload(w)
    E = w.mesh.ncells
    shape = cf.output_shape(w.form, E, w.mesh.cell, w.degree)
    out = torch.empty(shape, dtype=torch.float64 if prec == "fp64" else torch.float32, device=ctx.dev)
    fn = cf.PreparedAssemble(w.form, w.mesh.cell, w.degree, coords, c2v, coeffs=fields, constants=w.constants,
                             quad_degree=w.quad_degree, precision=prec, out=out)
    ms, per = time_gpu(fn, ctx.steps, ctx.warmup)
    sample = np.unique(np.concatenate([[0, E - 1], np.random.default_rng(seed).integers(0, E, sample_n)]))
    ref = O.assemble(w.form, w.mesh, w.degree, w.quad_degree, fields=w.fields, constants=w.constants, cells=sample)
    err = cell_rel_err(out[torch.as_tensor(sample, device=ctx.dev)].cpu().numpy(), ref)
    nbytes = algorithmic_bytes(w, int(np.prod(shape)), 8 if prec == "fp64" else 4)
    work = {k: v * E for k, v in work_model(w, prec).items()}
    flops = sum(work.values())
    del out, coords, c2v, fields
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    r = roof(nbytes, work, float(per.mean()))
    log(f"{tag or w.name} {w.form} {prec}: {per.mean() * 1e3:.1f} us, {r['gbs']:.0f} GB/s, frac {r['frac']:.2f}, "
        f"err {err:.2e}")
    return {"workload": tag or w.name, "form": w.form, "cells": E, "precision": prec,
            "ms_per_step": ms, "kernel_ms": pct(per), "cells_per_s": E / (ms * 1e-3),
            "algorithmic_bytes": nbytes, "algorithmic_flops": flops, "flops_by_unit": work, "gbs": r["gbs"],
            "gflops": r["gflops"], "bound": r["bound"], "frac": r["frac"], "max_cell_rel_err": err}


def adjoint_flops_per_cell(w):
    """Multiply-adds x 2 of the contraction the elasticity adjoint implements:
    V_k = R_k u_c2, then lam_c1 . V_k, for every entry k and block (c1, c2)."""
    if w.form != "elasticity":
        return None
    d, ns = w.mesh.d, n_scalar(w.mesh.d, w.degree)
    nf = n_scalar(d, 1) if w.fields else 1
    return 2.0 * nf * d * d * d * (ns * ns + d * ns)


def measure_adjoint(ctx, w, tag):
    torch, cf = ctx.torch, ctx.cf
    coords, c2v, fields = ctx.upload(w)
    E = w.mesh.ncells
    gc = torch.zeros_like(coords)
    gfs = [torch.zeros_like(f.values) for f in fields]
    cv = torch.empty(E, dtype=torch.float64, device=ctx.dev)
    lam = None if w.lam is None else torch.as_tensor(w.lam, device=ctx.dev)
    u = None if w.u is None else torch.as_tensor(w.u, device=ctx.dev)
    fn = lambda: cf.coffee_assemble_adjoint(w.form, w.mesh.d, w.degree, coords, c2v, coeffs=fields,
                                            constants=w.constants, lam=lam, u=u, grad_coords=gc, grad_coeffs=gfs,
                                            cell_value=cv, quad_degree=w.quad_degree)
    ms, per = time_gpu(fn, ctx.steps, ctx.warmup)
    # reads: inputs (+ lam, u); writes: per-cell values; gradients read-modify-written once each
    nbytes = algorithmic_bytes(w, E, 8) + 2 * w.mesh.coords.nbytes + sum(2 * f.values.nbytes for f in w.fields)
    if w.lam is not None:
        nbytes += w.lam.nbytes + w.u.nbytes
    del coords, c2v, fields, gc, gfs, cv, lam, u
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    gbs = nbytes / (per.mean() * 1e-3) / 1e9
    fpc = adjoint_flops_per_cell(w)
    extra = {}
    if fpc is not None:
        t_b = max(nbytes / (HBM_PEAK_GBS * 1e9), E * fpc / (FLOP_PEAK_TF["fp64"] * 1e12))
        extra = {"algorithmic_flops": E * fpc, "gflops": E * fpc / (per.mean() * 1e-3) / 1e9,
                 "bound": "fp64" if E * fpc / (FLOP_PEAK_TF["fp64"] * 1e12) > nbytes / (HBM_PEAK_GBS * 1e9)
                 else "hbm", "frac": t_b / (per.mean() * 1e-3)}
    log(f"{tag} adjoint: {per.mean() * 1e3:.1f} us, {gbs:.0f} GB/s"
        + (f", frac {extra['frac']:.2f} ({extra['bound']})" if extra else ""))
    return {"workload": tag, "form": f"{w.form} adjoint (vertex coords and coefficients)", "cells": E,
            "precision": "fp64", "ms_per_step": ms, "kernel_ms": pct(per), "cells_per_s": E / (ms * 1e-3),
            "algorithmic_bytes": nbytes, "gbs": gbs, "frac_hbm": gbs / HBM_PEAK_GBS, **extra,
            "parity": "tests/test_gpu_adjoint.py, tests/test_gpu_svk.py (oracle complex-step gradient, "
                      "central differences)"}


def mixed_batch_section(ctx):
    import torch
    from oracle import oracle as O
    from paper_1407_0904_amd import inputs as I
    from paper_1407_0904_amd import tuner
    cf = ctx.cf
    dev = ctx.dev
    mb = I.mixed_batch()
    tri_c = torch.as_tensor(mb.tri.coords, device=dev)
    tri_v = torch.as_tensor(mb.tri.cells, device=dev)
    tet_c = torch.as_tensor(mb.tet.coords, device=dev)
    tet_v = torch.as_tensor(mb.tet.cells, device=dev)
    f_tri = cf.DeviceField.from_host(mb.f_tri, dev)
    f_tet = cf.DeviceField.from_host(mb.f_tet, dev)
    costs = tuner.read_batch_costs(TUNING, "packed") or tuner.read_batch_costs(TUNING)
    # queue order: costliest bins first (tuned ns per cell, else the tensor size)
    key = lambda b: -costs.get((mb.segments[b][0], mb.segments[b][1], mb.segments[b][2], "fp32"),
                               n_scalar(mb.segments[b][1], mb.segments[b][2]) ** 2 * 1e-3)
    order = sorted(range(len(mb.segments)), key=key)
    remap = np.empty(len(order), dtype=np.int32)
    remap[np.array(order)] = np.arange(len(order), dtype=np.int32)
    segs = []
    for b in order:
        form, d, p = mb.segments[b]
        c, v, f = (tri_c, tri_v, f_tri) if d == 2 else (tet_c, tet_v, f_tet)
        segs.append(cf.Segment(form, d, p, c, v, f))  # task_cells 0: the tuned choice when cached
    seg_of = torch.as_tensor(remap[mb.seg_of], device=dev)
    cell_of = torch.as_tensor(mb.cell_of, device=dev)
    offs = torch.as_tensor(mb.out_offset, device=dev)
    out = torch.empty(mb.total_elems, dtype=torch.float32, device=dev)
    ws = torch.empty(cf.coffee_batch_workspace_size(len(segs), len(mb.seg_of)), dtype=torch.uint8, device=dev)
    # the library's packed layout (segment-major, offsets returned)
    poff = torch.empty(len(mb.seg_of), dtype=torch.int64, device=dev)
    fn_packed = lambda: cf.coffee_assemble_batch_packed(segs, seg_of, cell_of, mb.total_elems, precision="fp32",
                                                        out=out, out_offset=poff, workspace=ws)
    ms_p, per_p = time_gpu(fn_packed, ctx.steps, ctx.warmup)
    rng = np.random.default_rng(4)
    worst_p = 0.0
    poff_h = poff.cpu().numpy()
    for b, (form, d, p) in enumerate(mb.segments):
        idx = np.nonzero(mb.seg_of == b)[0]
        pick = rng.choice(idx, size=min(40, idx.size), replace=False)
        mesh, f = (mb.tri, mb.f_tri) if d == 2 else (mb.tet, mb.f_tet)
        ref = O.assemble(form, mesh, p, fields=[f], cells=mb.cell_of[pick])
        nn = ref.shape[1] * ref.shape[2]
        gidx = torch.as_tensor((poff_h[pick][:, None] + np.arange(nn)[None, :]).reshape(-1), device=dev)
        g = out[gidx].reshape(len(pick), nn).cpu().numpy()
        worst_p = max(worst_p, cell_rel_err(g, ref))
    # the caller's layout (entry order, the offsets of the input)
    fn = lambda: cf.coffee_assemble_batch(segs, seg_of, cell_of, offs, mb.total_elems, precision="fp32",
                                          out=out, workspace=ws)
    ms, per = time_gpu(fn, ctx.steps, ctx.warmup)
    rng = np.random.default_rng(4)
    worst = 0.0
    for b, (form, d, p) in enumerate(mb.segments):
        idx = np.nonzero(mb.seg_of == b)[0]
        pick = rng.choice(idx, size=min(40, idx.size), replace=False)
        mesh, f = (mb.tri, mb.f_tri) if d == 2 else (mb.tet, mb.f_tet)
        ref = O.assemble(form, mesh, p, fields=[f], cells=mb.cell_of[pick])
        nn = ref.shape[1] * ref.shape[2]
        gidx = torch.as_tensor((mb.out_offset[pick][:, None] + np.arange(nn)[None, :]).reshape(-1), device=dev)
        g = out[gidx].reshape(len(pick), nn).cpu().numpy()
        worst = max(worst, cell_rel_err(g, ref))
    del out, ws, poff
    # the same bins as 14 separate launches on pre-gathered per-bin inputs
    sub = []
    for b, (form, d, p) in enumerate(mb.segments):
        idx = np.nonzero(mb.seg_of == b)[0]
        c, v, f = (tri_c, tri_v, f_tri) if d == 2 else (tet_c, tet_v, f_tet)
        cells = torch.as_tensor(mb.cell_of[idx], device=dev)
        sf = cf.DeviceField(f.values, f.cell_to_dof[cells].contiguous(), 1, 1)
        ns = n_scalar(d, p)
        sub.append((form, d, p, c, v[cells].contiguous(), sf,
                    torch.empty((idx.size, ns, ns), dtype=torch.float32, device=dev)))

    calls = [cf.PreparedAssemble(form, d, p, c, v, coeffs=[sf], precision="fp32", out=o)
             for (form, d, p, c, v, sf, o) in sub]

    def per_bin():
        for call in calls:
            call()

    ms_sep, per_sep = time_gpu(per_bin, ctx.steps, ctx.warmup)
    del sub
    torch.cuda.empty_cache()
    reads = (mb.tri.coords.nbytes + mb.tri.cells.nbytes + mb.f_tri.values.nbytes + mb.tet.coords.nbytes
             + mb.tet.cells.nbytes + mb.f_tet.values.nbytes + mb.seg_of.nbytes + mb.cell_of.nbytes)
    n = len(mb.seg_of)
    # packed: offsets are written (8 B per entry); caller's layout: offsets are read
    nbytes_p = reads + mb.total_elems * 4 + 8 * n
    nbytes = reads + mb.total_elems * 4 + mb.out_offset.nbytes
    gbs_p = nbytes_p / (per_p.mean() * 1e-3) / 1e9
    gbs = nbytes / (per.mean() * 1e-3) / 1e9
    log(f"mixed batch packed: {per_p.mean() * 1e3:.1f} us ({gbs_p:.0f} GB/s), caller layout {per.mean() * 1e3:.1f} us "
        f"({gbs:.0f} GB/s), per-bin {per_sep.mean() * 1e3:.1f} us; err {worst_p:.2e} / {worst:.2e}")
    return {"workload": "mixed_batch", "form": "mass + Helmholtz, tri P1-P4 + tet P1-P3, random order",
            "cells": n, "precision": "fp32 (fp64 geometry)", "layout": "packed (segment-major, offsets returned)",
            "ms_per_step": ms_p, "kernel_ms": pct(per_p),
            "cells_per_s": n / (ms_p * 1e-3), "algorithmic_bytes": nbytes_p, "gbs": gbs_p, "bound": "hbm",
            "frac": gbs_p / HBM_PEAK_GBS, "max_cell_rel_err": worst_p,
            "caller_layout": {"ms_per_step": ms, "kernel_ms": pct(per), "cells_per_s": n / (ms * 1e-3),
                              "algorithmic_bytes": nbytes, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
                              "max_cell_rel_err": worst},
            "per_bin_launches_ms": ms_sep, "per_bin_cells_per_s": n / (ms_sep * 1e-3),
            "batch_speedup_vs_per_bin": ms_sep / ms_p, "tuning_cache": os.path.exists(TUNING),
            "note": "one coffee_assemble_batch_packed call (stable device binning + one persistent kernel) against "
                    "14 coffee_assemble launches on pre-gathered per-bin inputs (their gathers not timed); the "
                    "caller-layout call writes each tensor at the input offset (entry order)"}


def forms_section(ctx):
    from paper_1407_0904_amd import inputs as I
    res = []
    w = I.workload("helmholtz_p1_tri")
    r = measure_forward(ctx, w, "fp64")
    r["note"] = "8,192 cells: launch latency binds; the 2,097,152-cell run carries the roofline"
    res.append(r)
    res.append(measure_forward(ctx, I.workload("helmholtz_p1_tri", n=1024), "fp64", tag="helmholtz_p1_tri_2M"))
    w = I.workload("elasticity_p2_tet")
    for prec in ("fp64", "fp32", "bf16x3"):
        res.append(measure_forward(ctx, w, prec, sample_n=150))
    res.append(measure_adjoint(ctx, w, "elasticity_p2_tet"))
    for name in ("svk_p1_tet", "svk_p2_tet"):
        w = I.workload(name)
        for form in ("svk_energy", "svk_residual", "svk_jacobian"):
            w.form = form
            for prec in ("fp64", "fp32", "bf16x3"):
                res.append(measure_forward(ctx, w, prec, sample_n=150))
        w.form = "svk_energy"
        res.append(measure_adjoint(ctx, w, name))
    for name in ("burgers_p1_tet", "burgers_p2_tet", "helmholtz_p1_prism", "diffusion_p2_prism", "diffusion_p3_prism"):
        w = I.workload(name)
        for prec in ("fp64", "fp32", "bf16x3"):
            res.append(measure_forward(ctx, w, prec, sample_n=150))
    res.append(mixed_batch_section(ctx))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="helmholtz_p2_tet", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of the output's byte size (counter calibration)")
    ap.add_argument("--grid-mult", type=int, default=0)
    ap.add_argument("--only-batch", action="store_true",
                    help="run only the mixed-batch section and print its JSON (for profiling that kernel)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; runs on more than one GPU are not part of this implementation "
              "(local assembly shards by cell ranges with no exchange on the forward path). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1407_0904_amd import coffee, inputs
    from oracle import oracle as O

    if os.path.exists(TUNING):
        coffee.coffee_load_tuning(TUNING)
    ctx = Ctx(args.steps, args.warmup)
    if args.only_batch:
        print(json.dumps(mixed_batch_section(ctx), default=str), flush=True)
        return
    dev = ctx.dev
    w = inputs.workload(args.workload)
    coords, c2v, fields = ctx.upload(w)
    coffee.coffee_set_launch_options(args.grid_mult)
    E = w.mesh.ncells
    shape = coffee.output_shape(w.form, E, w.mesh.cell, w.degree)
    sample = np.unique(np.concatenate([[0, E - 1], np.random.default_rng(3).integers(0, E, 1500)]))
    ref = O.assemble(w.form, w.mesh, w.degree, w.quad_degree, fields=w.fields, constants=w.constants, cells=sample)
    idx = torch.as_tensor(sample, device=dev)

    results = {}
    precs = [args.precision] + ([] if args.no_variants else [p for p in ("fp64", "fp32", "bf16x3")
                                                             if p != args.precision])
    for prec in precs:
        out = torch.empty(shape, dtype=torch.float64 if prec == "fp64" else torch.float32, device=dev)
        fn = coffee.PreparedAssemble(w.form, w.mesh.cell, w.degree, coords, c2v, coeffs=fields,
                                     constants=w.constants, quad_degree=w.quad_degree, precision=prec, out=out)
        ms, per = time_gpu(fn, args.steps, args.warmup)
        err = cell_rel_err(out[idx].cpu().numpy(), ref)
        nbytes = algorithmic_bytes(w, int(np.prod(shape)), 8 if prec == "fp64" else 4)
        kms = float(per.mean())
        results[prec] = {"ms": ms, "kernel_ms": pct(per), "cells_per_s": E / (ms * 1e-3),
                         "gbs": nbytes / (kms * 1e-3) / 1e9, "bytes": nbytes, "err": err}
        log(f"{args.workload} {prec}: {kms * 1e3:.1f} us, {results[prec]['gbs']:.0f} GB/s, err {err:.2e}")
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
        log(f"calibration copy: {nb} bytes read and {nb} bytes written per launch")
        del src, dst
    del coords, c2v, fields
    torch.cuda.empty_cache()

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
                     "frac": main_r["gbs"] / HBM_PEAK_GBS,
                     "traffic": TRAFFIC.get((args.workload, args.precision)),
                     "algorithmic_bytes_per_launch": main_r["bytes"], "kernel_ms": main_r["kernel_ms"]},
        "max_cell_rel_err_vs_oracle": main_r["err"],
        "variants": {p: {"cells_per_s": r["cells_per_s"], "ms": r["ms"], "gbs": r["gbs"],
                         "frac_hbm": r["gbs"] / HBM_PEAK_GBS, "max_cell_rel_err": r["err"],
                         "speedup_vs_fp64": (results["fp64"]["ms"] / r["ms"]) if "fp64" in results else None}
                     for p, r in results.items()},
    }
    if not args.no_forms:
        line["forms"] = forms_section(ctx)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
