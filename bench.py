#!/usr/bin/env python3
"""Benchmark of the mesh-operator hot path on one MI355X.

Workload (the closed-surface solve of the plain method): icosphere at
subdivision level 7 (163,842 vertices, 327,680 triangles), radial noise
sigma = 1e-3 (seed 0), 8 right-hand sides f ~ N(0, 1) (seed 1). One step is
one outer iteration of a position-dependent solve, as in the MCF application
(Sec. 7.1): assemble K and M from the positions, form b = M f, and solve
(M + 1e-3 K) u = b with Jacobi PCG to relative tolerance 1e-8 on every column.
Inputs are resident in HBM before the timed region; the topology is built once
before it (it is static) and timed separately.

Output: one JSON line. `value` is triangles per second through the whole step
(nF * steps / wall time). `roofline` describes the kernel with the largest
share of step time. Per-kernel durations come from a second pass over the same
steps with every library kernel timed (dgo_trace_*): the reported kernels by
the start and stop events their launches carry (hipExtLaunchKernel, the
timestamps a profiler's kernel trace reads), the others bracketed by events. `cpu_baseline` times the FP64 oracle (single thread) on the
same step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0

PAPER_NOTE = "paper publishes no figure for this metric/workload"

ROOT = os.path.dirname(os.path.abspath(__file__))
# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE on this
# workload, scaled by the same counters on a plain copy of known size
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_icosphere_L{level}_{dtype}.json")
# the sources whose change makes a stored traffic figure stale
KERNEL_SOURCES = ["paper_2602_12105_amd/csrc/internal.hpp",
                  "paper_2602_12105_amd/csrc/kernels.hpp",
                  "paper_2602_12105_amd/csrc/assemble.hip",
                  "paper_2602_12105_amd/csrc/solve.hip"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--level", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--kernel-reps", type=int, default=30)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-suite", action="store_true",
                    help="skip the other workloads (tets, grid, VJP batch, size sweep)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--no-extra-steps", action="store_true",
                    help="skip the past-cache (L9) and other-precision PCG steps")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-pool", type=int, default=256,
                    help="distinct generated payloads the arrivals are drawn from")
    ap.add_argument("--cpu-baseline-suite", action="store_true",
                    help="only time the FP64 oracle on every workload (single thread per "
                         "workload, and a process pool for the batched serving and "
                         "differentiation workloads), print one JSON line and exit")
    ap.add_argument("--sweeps-only", action="store_true",
                    help="only the kernel sweeps on icosphere L9 and the Kuhn cube 160^3 "
                         "(--kernel-reps launches each, warm and cold), one JSON line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a plain elementwise copy of 256 MiB (read) into 256 MiB "
                         "(write), the reference for scaling the HBM byte counters")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def alg_bytes(kind, s, nV, nF, nnz, k):
    """Algorithmic bytes of one launch: the method's inputs and outputs, each
    moved once (index arrays at 4 bytes, values at s bytes)."""
    if kind == "assemble_tri":
        return 3 * s * nV + 12 * nF + s * nnz + s * nV
    if kind == "assemble_tet":
        return 3 * s * nV + 16 * nF + s * nnz + s * nV
    if kind == "assemble_vjp_tri":
        # X, gK, gM read, gX written, triangles
        return 3 * s * nV + 12 * nF + s * nnz + s * nV + 3 * s * nV
    if kind in ("spmm", "cg_sdot"):
        # CSR values + columns, row pointers, a diagonal (mass, or D^-1), x
        # read, y written
        return nnz * (s + 4) + 4 * (nV + 1) + s * nV + 2 * k * s * nV
    if kind == "cg_start":
        # A x0 as in the SpMM (x0 read), then beff and D^-1 read, r, p, s and
        # the row-order copy of x0 written
        return nnz * (s + 4) + 4 * (nV + 1) + s * nV + k * s * nV + k * s * nV + s * nV + 4 * k * s * nV
    if kind == "cg_vupdate":
        # read r w p s, write p s r, read D^-1; x (read and written) only in
        # every second iteration (two steps at once): 8 vectors on average
        return 8 * k * s * nV + s * nV
    if kind == "assemble_intrinsic":
        # edge lengths and the face -> edge map read, K and M written
        return s * (nnz - nV) // 2 + 12 * nF + s * nnz + s * nV
    if kind == "face_gradient":
        # positions, triangles and k vertex fields read, k face vectors written
        return 3 * s * nV + 12 * nF + k * s * nV + 3 * k * s * nF
    if kind == "face_divergence":
        # positions, triangles and k face vectors read, k vertex fields written
        return 3 * s * nV + 12 * nF + 3 * k * s * nF + k * s * nV
    if kind == "cg_values":
        # K, columns, row pointers, M, D^-1 read; scaled values written
        return nnz * (2 * s + 4) + 4 * (nV + 1) + 2 * s * nV
    return None


def kernel_sources_sha256():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update(rel.encode())
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, dtype, level):
    """Counter-measured HBM bytes per launch of `kernel`, or None when no
    measurement exists for this workload or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE.format(level=level, dtype=dtype)) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if (d.get("sources_sha256") != kernel_sources_sha256() or d.get("dtype") != dtype
            or d.get("level") != level):
        return None
    e = d.get("kernels", {}).get(kernel)
    return None if e is None else e.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; runs on several GPUs are not "
                                   "supported (the path is not sharded)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.cpu_baseline_suite:
        print(json.dumps(cpu_baseline_suite(args)), flush=True)
        return
    if args.sweeps_only:
        print(json.dumps(sweeps_only(args)), flush=True)
        return

    import numpy as np
    import torch

    import meshgen
    import paper_2602_12105_amd as dgo

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    td = torch.float64 if args.dtype == "f64" else torch.float32
    s = 8 if args.dtype == "f64" else 4
    k = 8
    head = pcg_step(args, dgo, torch, meshgen, args.level, args.dtype, args.steps, args.warmup)
    mesh, Xd, fd, K, M = head.pop("_objects")
    X, F, f = head.pop("_host")
    nV, nF, nnz = mesh.nV, mesh.n_elem, mesh.nnz
    value, ms_per_step, roofline = head["value"], head["ms_per_step"], head["roofline"]
    roofline["regime"] = ("effective: measured in the solve loop, whose working set "
                          f"({head['working_set_mb']:.0f} MB) stays in the 256 MB last-level "
                          "cache; the HBM fractions past the cache are under past_cache")

    # the same step past the last-level cache (icosphere L9, 2.6 M vertices,
    # 8 columns; working set about 1.1 GB in FP64): the dominant kernel's
    # fraction there is an HBM figure
    past = {}
    for dt in (() if args.no_extra_steps else ("f64", "f32")):
        log(args, f"PCG step past the cache: icosphere L9 {dt}")
        r = pcg_step(args, dgo, torch, meshgen, 9, dt, max(3, args.steps // 4), 1)
        r.pop("_objects")
        r.pop("_host")
        past[f"icosphere_L9_{dt}"] = r
        torch.cuda.empty_cache()
    if past:
        roofline["past_cache"] = {"workload": "the same step on icosphere L9 (2,621,442 V, "
                                              "5,242,880 F), 8 RHS, rtol 1e-8",
                                  "f64": past["icosphere_L9_f64"]["roofline"],
                                  "f32": past["icosphere_L9_f32"]["roofline"]}
        # the headline workload in the other precision
        other = "f32" if args.dtype == "f64" else "f64"
        log(args, f"PCG step icosphere L{args.level} {other}")
        r = pcg_step(args, dgo, torch, meshgen, args.level, other, args.steps, args.warmup)
        r.pop("_objects")
        r.pop("_host")
        past[f"icosphere_L{args.level}_{other}"] = r

    # kernel-level rooflines outside the solve: assembly and SpMM (k = 8 and 1),
    # warm (back to back) and cold (1 GiB written between launches)
    log(args, "kernel sweeps")
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)

    def timed(fn, name, cold):
        dgo.trace_reset()
        dgo.trace_enable(True, name)
        for _ in range(args.kernel_reps):
            if cold:
                flush.zero_()
            fn()
        torch.cuda.synchronize()
        dgo.trace_enable(False)
        e = dgo.trace_read().get(name)
        return None if e is None else e["total_ms"] / e["count"] * 1e3

    x1 = fd[:, 0].contiguous()
    y8 = torch.empty_like(fd)
    y1 = torch.empty_like(x1)
    sweeps = {}
    for label, fn, name, kk in [
        ("assemble", lambda: dgo.assemble(mesh, Xd, out=(K, M)), "assemble_tri", k),
        ("spmv_k8", lambda: dgo.spmv(mesh, 1.0, M, 1e-3, K, fd, out=y8), "spmm", 8),
        ("spmv_k1", lambda: dgo.spmv(mesh, 1.0, M, 1e-3, K, x1, out=y1), "spmm", 1),
    ]:
        ent = {}
        for cold in (False, True):
            us = timed(fn, name, cold)
            ab = alg_bytes(name, s, nV, nF, nnz, kk)
            gbs = ab / (us * 1e-6) / 1e9
            ent["cold" if cold else "warm"] = {"us": us, "gbps": gbs, "frac": gbs / HBM_PEAK_GBS}
        ent["alg_bytes"] = ab
        if label == "assemble":
            ent["elements_per_s_cold"] = nF / (ent["cold"]["us"] * 1e-6)
            ent["elements_per_s_warm"] = nF / (ent["warm"]["us"] * 1e-6)
        sweeps[label] = ent
    del flush

    # reference: a plain device-to-device copy of 512 MiB (read 512 MiB, write
    # 512 MiB), beyond the last-level cache, timed with events on torch's stream
    src = torch.ones(1 << 26, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 10 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst
    roofline["frac_of_stream_copy"] = roofline["achieved"] / copy_gbs

    out = {
        "metric": "elements assembled/s + SpMV HBM GB/s (frac of peak); req/s, p50/p99 latency",
        "value": value,
        "unit": "triangles/s (assembly + M f + PCG to 1e-8, 8 RHS, per step)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded icosphere + N(0,1) right-hand sides)",
        "config": {"workload": f"icosphere L{args.level} ({nV} V, {nF} F), radial noise 1e-3; "
                               "assemble K,M; b = M f; Jacobi PCG (M + 1e-3 K) u = b, "
                               "8 RHS, rtol 1e-8",
                   "nV": nV, "nF": nF, "nnz": nnz, "k": k, "parallelism": "single GPU"},
        "roofline": roofline,
        "pcg": {"iters": head["iters"], "max_true_relres": head["max_true_relres"]},
        "topology_ms": head["topology_ms"],
        "kernels": head["kernels"],
        "pcg_steps": past,
        "kernel_sweeps": sweeps,
        "stream_copy_gbps": copy_gbs,
        "device": device_info(torch, dev),
        "baseline_note": PAPER_NOTE,
    }

    if not args.no_suite:
        out["suite"] = suite(args, dgo, torch, meshgen)
    if not args.no_serving:
        out["serving"] = serving(args, meshgen)
    if not args.no_cpu_baseline:
        log(args, "cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(X, F, f, args.cpu_seconds)
    if args.calibrate_copy:
        a = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        b_ = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 1.0, out=b_)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


def device_info(torch, dev):
    """The GPU the numbers were taken on, as the runtime reports it (the peak
    figures used above are the chip's published ones)."""
    p = torch.cuda.get_device_properties(dev)
    info = {"name": p.name, "compute_units": p.multi_processor_count,
            "memory_gib": round(p.total_memory / 2 ** 30, 1)}
    arch = getattr(p, "gcnArchName", None)
    if arch:
        info["arch"] = arch
    return info


def pcg_step(args, dgo, torch, meshgen, level, dtype, steps, warmup):
    """One step of the headline workload on the icosphere of `level`: assemble
    K and M, b = M f, Jacobi PCG on (M + 1e-3 K) u = b to rtol 1e-8 on 8
    columns. Times `steps` steps (after `warmup`), then the same steps again
    with every library kernel timed; returns the step rate, the per-kernel
    table and the dominant kernel's roofline."""
    dev = torch.device("cuda:0")
    td = torch.float64 if dtype == "f64" else torch.float32
    s = 8 if dtype == "f64" else 4
    k = 8
    log(args, f"generating icosphere level {level}")
    X, F = meshgen.icosphere(level, 1e-3, 0)
    f = meshgen.normal(1, X.shape[0] * k).reshape(-1, k)
    nV, nF = X.shape[0], F.shape[0]
    Fd = torch.from_numpy(F).to(dev)
    Xd = torch.from_numpy(X).to(dev, td)
    fd = torch.from_numpy(f).to(dev, td)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh = dgo.Mesh(Fd, nV)
    torch.cuda.synchronize()
    topo_ms = (time.perf_counter() - t0) * 1e3
    nnz = mesh.nnz
    K = torch.empty(nnz, dtype=td, device=dev)
    M = torch.empty(nV, dtype=td, device=dev)
    b = torch.empty_like(fd)
    u0 = torch.zeros_like(fd)
    stall = 20 if dtype == "f32" else 0
    reports = []

    def step():
        dgo.assemble(mesh, Xd, out=(K, M))
        dgo.spmv(mesh, 1.0, M, 0.0, K, fd, out=b)  # b = M f
        u, rep = dgo.pcg(mesh, 1.0, M, 1e-3, K, b, u0=u0, rtol=1e-8, max_iter=1000,
                         check_every=8, stall_iters=stall)
        reports.append(rep)
        return u

    log(args, f"L{level} {dtype}: topology {topo_ms:.1f} ms; warmup {warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    reports.clear()
    log(args, f"L{level} {dtype}: timed {steps} steps")
    # nothing is timed per kernel inside the timed steps: even the events a
    # launch carries itself slowed the step by about 14% (measured)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iters = reports[-1]["iters"]
    true_rr = max(reports[-1]["true_relres"])

    # second pass: the same steps with every library kernel timed (the
    # reported ones by their dispatch events, the others bracketed by events)
    dgo.trace_reset()
    dgo.trace_enable(True)
    torch.cuda.synchronize()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dgo.trace_enable(False)
    tr = dgo.trace_read()
    # The solver queues the next chunk of iterations before it has seen the
    # previous one finish (it never waits on the host), so each solve ends
    # with launches that find every column stopped and exit at once. Their
    # time is charged to the iterations that did work: the per-launch figures
    # of the iteration kernels divide by the iterations run, not the launches.
    maxit = max(iters)
    effective = {"cg_vupdate": maxit, "cg_sdot": maxit + 1}
    kernels = {}
    for n, e in tr.items():
        ab = alg_bytes(n, s, nV, nF, nnz, k)
        per_step = e["count"] / steps
        n_eff = effective.get(n, per_step)
        ent = {"launches_per_step": per_step, "effective_launches_per_step": n_eff,
               "avg_us": e["total_ms"] / steps / n_eff * 1e3,
               "ms_per_step": e["total_ms"] / steps}
        if ab is not None and ent["avg_us"] > 0:
            gbs = ab / (ent["avg_us"] * 1e-6) / 1e9
            ent.update({"alg_bytes": ab, "gbps": gbs, "frac": gbs / HBM_PEAK_GBS})
        kernels[n] = ent
    dom = max((n for n in kernels if "gbps" in kernels[n]), key=lambda n: kernels[n]["ms_per_step"])
    dk = kernels[dom]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["gbps"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dk["frac"],
                "traffic": measured_traffic(dom, dtype, level),
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_us": dk["avg_us"]}
    # the PCG loop's resident data: K values and pattern (padded rows), D^-1,
    # and the vectors r p s w x b (nV x k each)
    ws_mb = (nV * 8 * (s + 4) + 2 * s * nV + 6 * k * s * nV) / 1e6
    return {"level": level, "dtype": dtype, "nV": nV, "nF": nF, "nnz": nnz, "k": k,
            "steps": steps, "value_triangles_per_s": nF * steps / wall, "value": nF * steps / wall,
            "ms_per_step": wall / steps * 1e3, "iters": iters, "max_true_relres": true_rr,
            "topology_ms": topo_ms, "working_set_mb": ws_mb, "kernels": kernels,
            "roofline": roofline, "_objects": (mesh, Xd, fd, K, M), "_host": (X, F, f)}


def kernel_time(dgo, torch, fn, name, reps, flush=None):
    """Median over reps calls of fn of the duration (us) of the library kernel
    `name`, each call's from the library's hipEvents around its launches (read
    after every call); with flush, 1 GiB is written before each call."""
    dgo.trace_reset()
    dgo.trace_enable(True, name)
    ds = []
    for _ in range(reps):
        if flush is not None:
            flush.zero_()
        dgo.trace_reset()  # the totals below are this call's alone
        fn()
        e = dgo.trace_read().get(name)  # synchronises this call's events
        if e is not None and e["count"] > 0:
            ds.append(e["total_ms"] / e["count"] * 1e3)
    torch.cuda.synchronize()
    dgo.trace_enable(False)
    dgo.trace_reset()
    if not ds:
        return None
    ds.sort()
    n = len(ds)
    return ds[n // 2] if n % 2 else 0.5 * (ds[n // 2 - 1] + ds[n // 2])


def roof(ab, us):
    gbs = ab / (us * 1e-6) / 1e9
    return {"us": us, "alg_bytes": ab, "gbps": gbs, "frac": gbs / HBM_PEAK_GBS}


def _cube_sweep(args, dgo, torch, meshgen, dev, td, s, reps, flush, nc, out):
    """Tet assembly and SpMV (k = 1) on the Kuhn cube nc^3, warm and cold."""
    log(args, f"suite: Kuhn cube {nc}^3")
    X, T = meshgen.cube_tets(nc, 0.15, 0)
    m = dgo.Mesh(torch.from_numpy(T).to(dev), X.shape[0])
    Xd = torch.from_numpy(X).to(dev, td)
    K, M = dgo.assemble(m, Xd)
    ent = {"nV": m.nV, "nT": m.n_elem, "nnz": m.nnz}
    ab = alg_bytes("assemble_tet", s, m.nV, m.n_elem, m.nnz, 1)
    abs1 = alg_bytes("spmm", s, m.nV, m.n_elem, m.nnz, 1)
    x1 = torch.rand(m.nV, dtype=td, device=dev)
    y1 = torch.empty_like(x1)
    for cold in (False, True):
        tag = "cold" if cold else "warm"
        us = kernel_time(dgo, torch, lambda: dgo.assemble(m, Xd, out=(K, M)), "assemble_tet", reps,
                         flush if cold else None)
        ent["assemble_" + tag] = roof(ab, us)
        us = kernel_time(dgo, torch, lambda: dgo.spmv(m, 0.0, M, 1.0, K, x1, out=y1), "spmm", reps,
                         flush if cold else None)
        ent["spmv_k1_" + tag] = roof(abs1, us)
    ent["tets_per_s_cold"] = m.n_elem / (ent["assemble_cold"]["us"] * 1e-6)
    out[f"cube{nc}_tet"] = ent
    del m, K, M, Xd, x1, y1
    torch.cuda.empty_cache()


def suite(args, dgo, torch, meshgen):
    """The other workloads, each timed per kernel (warm and cache-flushed)."""
    dev = torch.device("cuda:0")
    reps = max(5, args.kernel_reps // 3)
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    out = {}
    td, s = (torch.float64, 8) if args.dtype == "f64" else (torch.float32, 4)

    # tetrahedral volume: Kuhn cube 64^3, jitter 0.15 h, Dirichlet Poisson to 1e-8,
    # in both precisions
    import numpy as np
    X, T = meshgen.cube_tets(64, 0.15, 0)
    m = dgo.Mesh(torch.from_numpy(T).to(dev), X.shape[0])
    mask = m.boundary()
    us_ = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    for dt in (args.dtype, "f32" if args.dtype == "f64" else "f64"):
        log(args, f"suite: Kuhn cube 64^3 {dt}")
        tdd, ss = (torch.float64, 8) if dt == "f64" else (torch.float32, 4)
        Xd = torch.from_numpy(X).to(dev, tdd)
        K, M = dgo.assemble(m, Xd)
        ent = {"dtype": dt, "nV": m.nV, "nT": m.n_elem, "nnz": m.nnz}
        ab = alg_bytes("assemble_tet", ss, m.nV, m.n_elem, m.nnz, 1)
        for cold in (False, True):
            us = kernel_time(dgo, torch, lambda: dgo.assemble(m, Xd, out=(K, M)), "assemble_tet",
                             reps, flush if cold else None)
            ent["assemble_" + ("cold" if cold else "warm")] = roof(ab, us)
        ent["tets_per_s_cold"] = m.n_elem / (ent["assemble_cold"]["us"] * 1e-6)
        x1 = torch.rand(m.nV, dtype=tdd, device=dev)
        y1 = torch.empty_like(x1)
        ab = alg_bytes("spmm", ss, m.nV, m.n_elem, m.nnz, 1)
        for cold in (False, True):
            us = kernel_time(dgo, torch, lambda: dgo.spmv(m, 0.0, M, 1.0, K, x1, out=y1), "spmm",
                             reps, flush if cold else None)
            ent["spmv_k1_" + ("cold" if cold else "warm")] = roof(ab, us)
        g = torch.from_numpy(us_).to(dev, tdd)
        b = (M * torch.from_numpy(3 * np.pi ** 2 * us_).to(dev, tdd)).contiguous()
        times = []
        for r in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, rep = dgo.pcg(m, 0.0, M, 1.0, K, b, mask=mask, g=g, rtol=1e-8, max_iter=5000,
                             check_every=16, stall_iters=50 if dt == "f32" else 0)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        ent["dirichlet_pcg"] = {"ms": float(np.median(times)), "iters": rep["iters"][0],
                                "true_relres": rep["true_relres"][0],
                                "nodal_err_vs_exact": float((u.double() - g.double()).abs().max())}
        out["cube64_tet" if dt == args.dtype else f"cube64_tet_{dt}"] = ent
        del K, M, Xd
    del m

    # the same generator past the last-level cache: Kuhn cubes 128^3 (2.1 M
    # vertices, 12.3 M tets) and 160^3 (4.1 M vertices, 24.1 M tets): tet
    # assembly and SpMV, warm and cold
    for nc in (128, 160):
        _cube_sweep(args, dgo, torch, meshgen, dev, td, s, reps, flush, nc, out)

    # plain method on the 64 x 64 grid: 100 SpMVs with K on a uniform[-1, 1] vector
    log(args, "suite: grid 64x64")
    X, F = meshgen.grid2d(64, 0.2, 0)
    m = dgo.Mesh(torch.from_numpy(F).to(dev), X.shape[0])
    Xd = torch.from_numpy(X).to(dev, td)
    K, M = dgo.assemble(m, Xd)
    x = torch.from_numpy(meshgen.uniform(1, m.nV) * 2 - 1).to(dev, td)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(100):
        dgo.spmv(m, 0.0, M, 1.0, K, x, out=y)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e6 / 100
    # GPU time of the 100 back-to-back SpMVs (events on torch's stream, which
    # the library launches on) and of 20 assemblies: per-launch events are not
    # meaningful at this size, where a launch's start overlaps the previous one
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(100):
        dgo.spmv(m, 0.0, M, 1.0, K, x, out=y)
    ev1.record()
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / 100
    ev0.record()
    for _ in range(20):
        dgo.assemble(m, Xd, out=(K, M))
    ev1.record()
    torch.cuda.synchronize()
    ua = ev0.elapsed_time(ev1) * 1e3 / 20
    # the same 100 SpMVs captured once as a graph and replayed (five replays,
    # the median per SpMV), every replay checked bitwise against the eager y
    y_ref = y.clone()
    graph = {"spmv_us_per_call": None}
    try:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(100):
                dgo.spmv(m, 0.0, M, 1.0, K, x, out=y)
        times, same = [], True
        for _ in range(5):
            y.zero_()
            torch.cuda.synchronize()
            ev0.record()
            g.replay()
            ev1.record()
            torch.cuda.synchronize()
            times.append(ev0.elapsed_time(ev1) * 1e3 / 100)
            same = same and torch.equal(y, y_ref)
        graph = {"spmv_us_per_call": sorted(times)[2], "replays": 5, "replays_equal_eager": same}
        del g
    except Exception as e:  # a launch the capture refuses: reported, not fatal
        graph["error"] = str(e)[:200]
    out["grid64"] = {"spmv_us_gpu_per_call": us, "spmv_us_wall_per_call": wall, "assemble_us": ua,
                     "spmv_graph_x100": graph,
                     "note": "latency-bound size (0.4 MB per SpMV): reported in microseconds"}
    del m

    # differentiation batch: 256 icosphere L5 meshes, assembly and its VJP, in
    # both precisions
    B = 256
    X0, F = meshgen.icosphere(5)
    m = dgo.Mesh(torch.from_numpy(F).to(dev), X0.shape[0])
    Xs = np.stack([meshgen.icosphere(5, 1e-2, sd)[0] for sd in range(B)])
    for dt in (args.dtype, "f32" if args.dtype == "f64" else "f64"):
        log(args, f"suite: 256 x icosphere L5 VJP {dt}")
        tdd, ss = (torch.float64, 8) if dt == "f64" else (torch.float32, 4)
        Xb = torch.from_numpy(Xs).to(dev, tdd)
        Kb, Mb = dgo.assemble(m, Xb)
        gK = torch.randn_like(Kb)
        gM = torch.randn_like(Mb)
        ent = {"dtype": dt, "batch": B, "nV": m.nV, "nF": m.n_elem}
        ab = B * alg_bytes("assemble_tri", ss, m.nV, m.n_elem, m.nnz, 1)
        abv = B * alg_bytes("assemble_vjp_tri", ss, m.nV, m.n_elem, m.nnz, 1)
        for cold in (False, True):
            tag = "cold" if cold else "warm"
            us = kernel_time(dgo, torch, lambda: dgo.assemble(m, Xb, out=(Kb, Mb)), "assemble_tri",
                             reps, flush if cold else None)
            ent["assemble_" + tag] = roof(ab, us)
            us = kernel_time(dgo, torch, lambda: dgo.assemble_vjp(m, Xb, gK, gM),
                             "assemble_vjp_tri", reps, flush if cold else None)
            ent["vjp_" + tag] = roof(abv, us)
        ent["triangles_per_s_cold"] = B * m.n_elem / (ent["assemble_cold"]["us"] * 1e-6)
        out["diff_batch_ico5" if dt == args.dtype else f"diff_batch_ico5_{dt}"] = ent
        del Xb, Kb, Mb, gK, gM
    del m

    # one differentiable implicit MCF step (Sec. 7.1) on the icosphere L7:
    # forward (assemble, b = M X, PCG on (M + tau K) u = b, 3 columns) and
    # backward (adjoint PCG, solve VJP, assembly VJP, M lambda)
    log(args, "suite: MCF step L7")
    X, F = meshgen.icosphere(args.level, 1e-3, 0)
    m = dgo.Mesh(torch.from_numpy(F).to(dev), X.shape[0])
    W = torch.from_numpy(meshgen.normal(3, X.size).reshape(X.shape)).to(dev, td)
    Xd = torch.from_numpy(X).to(dev, td)
    tau, rtol = 1e-3, 1e-10
    fw, bw = [], []
    for r in range(reps + 2):
        Xg = Xd.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = dgo.mcf_step(m, Xg, tau, rtol=rtol)
        loss = (u * W).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if r >= 2:
            fw.append((t1 - t0) * 1e3)
            bw.append((t2 - t1) * 1e3)
    out["mcf_step_L7"] = {"nV": m.nV, "nF": m.n_elem, "tau": tau, "rtol": rtol, "columns": 3,
                          "forward_ms": float(np.median(fw)), "backward_ms": float(np.median(bw))}
    del m, W, Xd, Xg, u, loss

    # spectral layer forward (Sec. 5.2): the 9 smallest eigenpairs of the
    # icosphere L7 Laplacian (0, the l = 1 and l = 2 clusters) to 1e-8
    log(args, "suite: eigenpairs L7")
    X, F = meshgen.icosphere(args.level, 1e-3, 0)
    m = dgo.Mesh(torch.from_numpy(F).to(dev), X.shape[0])
    K, M = dgo.assemble(m, torch.from_numpy(X).to(dev, td))
    times = []
    for r in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, U, rep = dgo.eigs_smallest(m, M, K, 9)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    out["eigs_L7"] = {"nV": m.nV, "k": 9, "block": rep["block"], "sigma": rep["sigma"],
                      "outer_iters": rep["iters"], "inner_pcg_iters": rep["inner_iters"],
                      "converged": rep["converged"], "max_resid": max(rep["resid"]),
                      "ms": float(np.median(times)), "lambda": [float(v) for v in lam]}
    del m, K, M, U

    # size sweep past the 256 MB last-level cache: icosphere L8 and L9
    _ico_sweep(args, dgo, torch, meshgen, dev, td, s, reps, flush, (8, 9), out)
    del flush
    torch.cuda.empty_cache()
    return out


def _ico_sweep(args, dgo, torch, meshgen, dev, td, s, reps, flush, levels, out):
    """Triangle assembly, SpMM (k = 8), intrinsic assembly, face gradient and
    divergence (k = 1, 3) on icospheres of the given levels, warm and cold."""
    for L in levels:
        log(args, f"suite: icosphere L{L}")
        X, F = meshgen.icosphere(L, 1e-3, 0)
        m = dgo.Mesh(torch.from_numpy(F).to(dev), X.shape[0])
        Xd = torch.from_numpy(X).to(dev, td)
        K, M = dgo.assemble(m, Xd)
        xk = torch.randn(m.nV, 8, dtype=td, device=dev)
        yk = torch.empty_like(xk)
        ent = {"nV": m.nV, "nF": m.n_elem, "nnz": m.nnz}
        ab = alg_bytes("assemble_tri", s, m.nV, m.n_elem, m.nnz, 8)
        abs_ = alg_bytes("spmm", s, m.nV, m.n_elem, m.nnz, 8)
        for cold in (False, True):
            tag = "cold" if cold else "warm"
            us = kernel_time(dgo, torch, lambda: dgo.assemble(m, Xd, out=(K, M)), "assemble_tri",
                             reps, flush if cold else None)
            ent["assemble_" + tag] = roof(ab, us)
            us = kernel_time(dgo, torch, lambda: dgo.spmv(m, 1.0, M, 1e-3, K, xk, out=yk), "spmm",
                             reps, flush if cold else None)
            ent["spmv_k8_" + tag] = roof(abs_, us)
        ent["triangles_per_s_cold"] = m.n_elem / (ent["assemble_cold"]["us"] * 1e-6)
        # intrinsic assembly from edge lengths, per-face gradient and divergence
        EVd = m.edges()[0].long()
        Ld = (Xd[EVd[:, 0]] - Xd[EVd[:, 1]]).norm(dim=1).contiguous()
        Ki, Mi = dgo.assemble_intrinsic(m, Ld)
        ab = alg_bytes("assemble_intrinsic", s, m.nV, m.n_elem, m.nnz, 1)
        for cold in (False, True):
            us = kernel_time(dgo, torch, lambda: dgo.assemble_intrinsic(m, Ld, out=(Ki, Mi)),
                             "assemble_intrinsic", reps, flush if cold else None)
            ent["assemble_intrinsic_" + ("cold" if cold else "warm")] = roof(ab, us)
        for k in (1, 3):
            u = torch.randn(m.nV, k, dtype=td, device=dev)
            g = dgo.face_gradient(m, Xd, u)
            y = torch.randn(k, 3, m.n_elem, dtype=td, device=dev)
            d = dgo.face_divergence(m, Xd, y)
            abg = alg_bytes("face_gradient", s, m.nV, m.n_elem, m.nnz, k)
            abd = alg_bytes("face_divergence", s, m.nV, m.n_elem, m.nnz, k)
            for cold in (False, True):
                tag = f"k{k}_" + ("cold" if cold else "warm")
                us = kernel_time(dgo, torch, lambda: dgo.face_gradient(m, Xd, u, out=g),
                                 "face_gradient", reps, flush if cold else None)
                ent["face_gradient_" + tag] = roof(abg, us)
                us = kernel_time(dgo, torch, lambda: dgo.face_divergence(m, Xd, y, out=d),
                                 "face_divergence", reps, flush if cold else None)
                ent["face_divergence_" + tag] = roof(abd, us)
        out[f"icosphere_L{L}"] = ent
        del m, K, M, Xd, xk, yk, Ki, Mi, Ld, u, g, y, d
        torch.cuda.empty_cache()


def sweeps_only(args):
    """Only the kernel sweeps past the last-level cache (icosphere L9, Kuhn
    cube 160^3), for counter collection: one JSON line."""
    import torch
    import meshgen
    import paper_2602_12105_amd as dgo
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    td, s = (torch.float64, 8) if args.dtype == "f64" else (torch.float32, 4)
    reps = max(1, args.kernel_reps)
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    out = {}
    _ico_sweep(args, dgo, torch, meshgen, dev, td, s, reps, flush, (9,), out)
    _cube_sweep(args, dgo, torch, meshgen, dev, td, s, reps, flush, 160, out)
    return {"dtype": args.dtype, "kernel_reps": reps, "sweeps": out}


def _serve_payloads(meshgen, n_pool, seed=0):
    """Synthetic requests: vertex count ~ logU[1e3, 2e5], grid or icosphere
    (p = 1/2), k ~ U{1..16}, f ~ N(0, 1), FP32."""
    import numpy as np
    specs = meshgen.serving_requests(n_pool, seed)
    base = {}
    pool = []
    for sp in specs:
        key = (sp["kind"], sp["size"])
        if key not in base:
            base[key] = (meshgen.grid2d(sp["size"]) if sp["kind"] == "grid"
                         else meshgen.icosphere(sp["size"]))
        X0, F = base[key]
        if sp["kind"] == "grid":
            n = sp["size"]
            X, _ = meshgen.grid2d(n, 0.2, sp["mesh_seed"])
        else:
            xi = meshgen.normal(sp["mesh_seed"], X0.shape[0])
            X = X0 * (1.0 + 1e-3 * xi)[:, None]
        f = meshgen.normal(sp["rhs_seed"], X.shape[0] * sp["k"]).reshape(-1, sp["k"])
        pool.append((F, X.astype(np.float32), f.astype(np.float32), sp))
    return pool


def _run_server(dgo_serve, pool, n_req, rate, batched, seed):
    """Submit n_req requests drawn cyclically from the pool, as a Poisson
    stream of the given rate (req/s; None = all at once); returns
    throughput and latency percentiles on the server's clock."""
    import threading

    import numpy as np
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_req) if rate else np.zeros(n_req)
    srv = dgo_serve.Server(hbm_budget_bytes=32 << 30, max_slots=128 if batched else 1,
                           cg_iters=50, cg_chunk=10, batched=batched, prep_threads=4)
    tickets = [None] * n_req
    submitted = threading.Event()
    lat, starts, ends = [], [], []

    def producer():
        t_next = time.perf_counter()
        for r in range(n_req):
            t_next += gaps[r]
            d = t_next - time.perf_counter()
            if d > 0:
                time.sleep(d)
            F, X, f, _ = pool[r % len(pool)]
            tickets[r] = srv.submit(F, X, f, user=r)
            if r == 0:
                submitted.set()

    th = threading.Thread(target=producer)
    t0 = time.perf_counter()
    th.start()
    submitted.wait()
    for r in range(n_req):
        while tickets[r] is None:
            time.sleep(0.0005)
        _, st = srv.wait(tickets[r], timeout=600.0)
        lat.append(st["t_done"] - st["t_submit"])
        starts.append(st["t_submit"])
        ends.append(st["t_done"])
    th.join()
    wall = time.perf_counter() - t0
    c = srv.stats()
    srv.close()
    lat = np.array(lat) * 1e3
    span = max(ends) - min(starts)
    return {"requests": n_req, "offered_rate": rate, "req_per_s": n_req / span,
            "wall_s": wall, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_batch": c["max_batch"], "ticks": c["ticks"], "hbm_peak": c["hbm_peak"],
            "gpu_busy_frac": c["busy_s"] / span}


def serving(args, meshgen):
    """Continuous batching vs one request at a time (each with its own
    per-mesh launches): closed-loop capacity of the batched server, then a
    Poisson stream at 0.8 x that capacity offered to both."""
    import numpy as np
    from paper_2602_12105_amd import serve as dgo_serve
    log(args, f"serving: generating {args.serve_pool} payloads")
    pool = _serve_payloads(meshgen, args.serve_pool)
    nv = np.array([p[1].shape[0] for p in pool])
    ks = np.array([p[2].shape[1] for p in pool])
    n = args.serve_requests
    log(args, "serving: closed loop (batched)")
    cap = _run_server(dgo_serve, pool, n, None, True, 1)
    sweep = {}
    for frac in (0.5, 0.8, 1.0):
        r = frac * cap["req_per_s"]
        log(args, f"serving: Poisson {r:.0f} req/s = {frac} x capacity (batched)")
        sweep[f"{frac:.1f}x"] = _run_server(dgo_serve, pool, n, r, True, 2 + int(10 * frac))
    rate = 0.8 * cap["req_per_s"]
    b = sweep["0.8x"]
    log(args, "serving: closed loop (one request at a time)")
    cap1 = _run_server(dgo_serve, pool, max(64, n // 8), None, False, 3)
    log(args, f"serving: Poisson {rate:.0f} req/s (one request at a time)")
    one = _run_server(dgo_serve, pool, max(64, n // 8), rate, False, 4)
    return {"workload": f"{n} requests, nV ~ logU[1e3, 2e5] (mean {nv.mean():.0f}), "
                        f"k ~ U{{1..16}} (mean {ks.mean():.1f}), FP32, assembly + 50 PCG "
                        "iterations on (M + 1e-3 K) u = M f",
            "payload_pool": len(pool),
            "batched_closed_loop": cap, "batched_poisson": b,
            "batched_rate_sweep": sweep,
            "one_at_a_time_closed_loop": cap1, "one_at_a_time_poisson": one,
            "speedup_req_per_s": b["req_per_s"] / one["req_per_s"],
            "note": "one-at-a-time runs use n/8 requests of the same stream (its queue "
                    "grows without bound at the offered rate)"}


def cpu_baseline(X, F, f, budget_s):
    """The FP64 oracle on the same step (single thread): assemble, b = M f,
    PCG to 1e-8 on the 8 columns. Repeats whole steps until budget_s."""
    import numpy as np

    import oracle
    nF = F.shape[0]
    t0 = time.perf_counter()
    EV, _, _ = oracle.edges(X.shape[0], F)
    rp, col = oracle.csr(X.shape[0], EV)
    topo = time.perf_counter() - t0
    n = 0
    t0 = time.perf_counter()
    while True:
        K, M, _, _ = oracle.assemble(X, F, rp, col)
        b = oracle.spmv(rp, col, 1.0, M, 0.0, K, f)
        u, its, rr = oracle.pcg(rp, col, 1.0, M, 1e-3, K, b, rtol=1e-8, max_iter=1000)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": nF * n / el, "unit": "triangles/s (assembly + M f + PCG to 1e-8, 8 RHS, per step)",
            "cores": 1, "kind": "oracle",
            "sample": f"{n} full step(s) of the same workload in {el:.1f} s, FP64, one thread "
                      f"(topology once, {topo:.2f} s, not counted); host has {os.cpu_count()} CPUs",
            "iters": [int(i) for i in its]}


# ------------------------------------------------------ oracle on every workload

_POOL_DATA = {}


def _pool_serving(i):
    """One serving request through the FP64 oracle: assemble, b = M f, 50 PCG
    iterations on (M + 1e-3 K) u = b."""
    import oracle
    F, X, f, _ = _POOL_DATA["serving"][i]
    X = X.astype("float64")
    K, M, rp, col = oracle.assemble(X, F)
    b = M[:, None] * f.astype("float64")
    oracle.pcg(rp, col, 1.0, M, 1e-3, K, b, rtol=0.0, max_iter=50)
    return i


def _pool_diff(i):
    """One mesh of the differentiation batch through the FP64 oracle: the
    assembly, then its VJP for the loss u^T K u + sum(M)."""
    import numpy as np
    import oracle
    X, F, rp, col, u = _POOL_DATA["diff"][i]
    K, M, _, _ = oracle.assemble(X, F, rp, col)
    rows = np.repeat(np.arange(X.shape[0]), np.diff(rp))
    gK = u[rows] * u[col]
    oracle.assemble_vjp_tri(X, F, rp, col, gK, np.ones(X.shape[0]))
    return i


def _timed_pool(fn, n, workers):
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(fn, range(min(n, workers)))  # start the workers
        t0 = time.perf_counter()
        pool.map(fn, range(n), chunksize=1)
        return time.perf_counter() - t0


def cpu_baseline_suite(args):
    """The FP64 oracle (single-threaded C) on every workload, on this host.
    Batched workloads also run in a process pool of one process per core of
    this process's CPU share (at most 16): measured, not extrapolated."""
    import numpy as np

    import meshgen
    import oracle
    oracle.lib()
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, min(16, cores))
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out = {"kind": "oracle", "dtype": "f64", "host": {"cpus_available": cores, "pool_workers": workers,
                                                      "cpu_model": model}}

    def clock(fn, reps=1):
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        return (time.perf_counter() - t0) / reps, r

    # grid 64 x 64: assembly and 100 SpMVs with K
    log(args, "cpu suite: grid 64")
    X, F = meshgen.grid2d(64, 0.2, 0)
    EV, _, _ = oracle.edges(X.shape[0], F)
    rp, col = oracle.csr(X.shape[0], EV)
    ta, (K, M, _, _) = clock(lambda: oracle.assemble(X, F, rp, col), 10)
    x = meshgen.uniform(1, X.shape[0]) * 2 - 1
    ts, _ = clock(lambda: [oracle.spmv(rp, col, 0.0, M, 1.0, K, x) for _ in range(100)])
    out["grid64"] = {"assemble_ms": ta * 1e3, "spmv_x100_ms": ts * 1e3, "threads": 1}

    # icosphere L7 step: assembly, b = M f, PCG to 1e-8 on 8 columns
    log(args, "cpu suite: icosphere L7 step")
    X, F = meshgen.icosphere(7, 1e-3, 0)
    f = meshgen.normal(1, X.shape[0] * 8).reshape(-1, 8)
    EV, _, _ = oracle.edges(X.shape[0], F)
    rp, col = oracle.csr(X.shape[0], EV)

    def step():
        K, M, _, _ = oracle.assemble(X, F, rp, col)
        b = oracle.spmv(rp, col, 1.0, M, 0.0, K, f)
        return oracle.pcg(rp, col, 1.0, M, 1e-3, K, b, rtol=1e-8, max_iter=1000)
    ta, _ = clock(lambda: oracle.assemble(X, F, rp, col), 3)
    tstep, (_, its, _) = clock(step)
    out["icosphere_L7"] = {"assemble_ms": ta * 1e3, "step_ms": tstep * 1e3,
                           "triangles_per_s": F.shape[0] / tstep, "pcg_iters": [int(i) for i in its],
                           "threads": 1}

    # Kuhn cube 64^3: tet assembly and the Dirichlet Poisson solve to 1e-8
    log(args, "cpu suite: Kuhn cube 64^3")
    X, T = meshgen.cube_tets(64, 0.15, 0)
    EV, _, _ = oracle.edges(X.shape[0], T)
    rp, col = oracle.csr(X.shape[0], EV)
    ta, (K, M, _, _) = clock(lambda: oracle.assemble(X, T, rp, col))
    mask, _ = oracle.boundary(X.shape[0], T)
    us = np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2])
    b = M * (3 * np.pi ** 2 * us)
    tp, (_, its, _) = clock(lambda: oracle.pcg(rp, col, 0.0, M, 1.0, K, b, mask=mask, g=us,
                                                rtol=1e-8, max_iter=5000))
    out["cube64_tet"] = {"assemble_ms": ta * 1e3, "dirichlet_pcg_ms": tp * 1e3,
                         "pcg_iters": int(its[0]), "tets_per_s": T.shape[0] / ta, "threads": 1}

    # serving requests: the first 4 * workers of the same request stream
    log(args, "cpu suite: serving requests")
    _POOL_DATA["serving"] = _serve_payloads(meshgen, 4 * workers, seed=0)
    n1 = min(8, len(_POOL_DATA["serving"]))
    t1, _ = clock(lambda: [_pool_serving(i) for i in range(n1)])
    tp = _timed_pool(_pool_serving, len(_POOL_DATA["serving"]), workers)
    out["serving"] = {"req_per_s_one_thread": n1 / t1, "requests_one_thread": n1,
                      "req_per_s_pool": len(_POOL_DATA["serving"]) / tp,
                      "requests_pool": len(_POOL_DATA["serving"]), "pool_workers": workers,
                      "work": "FP64 assembly + b = M f + 50 PCG iterations per request"}

    # differentiation batch: 256 icosphere L5 meshes, assembly + VJP each
    log(args, "cpu suite: 256 x icosphere L5 VJP")
    X0, F = meshgen.icosphere(5)
    EV, _, _ = oracle.edges(X0.shape[0], F)
    rp, col = oracle.csr(X0.shape[0], EV)
    u = meshgen.normal(1000, X0.shape[0])
    _POOL_DATA["diff"] = [(meshgen.icosphere(5, 1e-2, sd)[0], F, rp, col, u) for sd in range(256)]
    t1, _ = clock(lambda: [_pool_diff(i) for i in range(16)])
    tp = _timed_pool(_pool_diff, 256, workers)
    out["diff_batch_ico5"] = {"meshes_per_s_one_thread": 16 / t1, "meshes_one_thread": 16,
                              "meshes_per_s_pool": 256 / tp, "meshes_pool": 256,
                              "pool_workers": workers,
                              "work": "FP64 assembly + assembly VJP per mesh"}
    return out


if __name__ == "__main__":
    main()
