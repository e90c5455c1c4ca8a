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
(nF * steps / wall time). Per-kernel durations come from hipEvents recorded by
the library around its own launches (dgo_trace_*), in a second pass over the
same steps; `roofline` describes the kernel with the largest share of step
time. `cpu_baseline` times the FP64 oracle (single thread) on the same step.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0

PAPER_NOTE = "paper publishes no figure for this metric/workload"


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
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def alg_bytes(kind, s, nV, nF, nnz, k):
    """Algorithmic bytes of one launch: the method's inputs and outputs, each
    moved once (index arrays at 4 bytes, values at s bytes)."""
    if kind == "assemble_tri":
        return 3 * s * nV + 12 * nF + s * nnz + s * nV
    if kind in ("spmm", "cg_spmm_dot"):
        # CSR values + columns, row pointers, mass diagonal, x read, y written
        return nnz * (s + 4) + 4 * (nV + 1) + s * nV + 2 * k * s * nV
    if kind == "cg_update":
        # read x p r q, write x r z, read D^-1
        return 7 * k * s * nV + s * nV
    if kind == "cg_pupdate":
        return 3 * k * s * nV
    return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not "
                                   "supported (the sharding design is described in DESIGN.md)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import meshgen
    import paper_2602_12105_amd as dgo

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    td = torch.float64 if args.dtype == "f64" else torch.float32
    s = 8 if args.dtype == "f64" else 4
    k = 8
    log(args, "generating icosphere level", args.level)
    X, F = meshgen.icosphere(args.level, 1e-3, 0)
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
    rtol = 1e-8
    stall = 20 if args.dtype == "f32" else 0
    reports = []

    def step():
        dgo.assemble(mesh, Xd, out=(K, M))
        dgo.spmv(mesh, 1.0, M, 0.0, K, fd, out=b)  # b = M f
        u, rep = dgo.pcg(mesh, 1.0, M, 1e-3, K, b, u0=u0, rtol=rtol, max_iter=1000,
                         check_every=8, stall_iters=stall)
        reports.append(rep)
        return u

    log(args, f"topology {topo_ms:.1f} ms; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    reports.clear()
    log(args, f"timed {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        u = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    value = nF * args.steps / wall
    iters = reports[-1]["iters"]
    true_rr = max(reports[-1]["true_relres"])

    # second pass: the same steps with every library kernel bracketed by events
    log(args, "traced pass")
    dgo.trace_reset()
    dgo.trace_enable(True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dgo.trace_enable(False)
    tr = dgo.trace_read()
    step_ms_by_kernel = {n: e["total_ms"] / args.steps for n, e in tr.items()}
    kernels = {}
    for n, e in tr.items():
        ab = alg_bytes(n, s, nV, nF, nnz, k)
        ent = {"launches_per_step": e["count"] / args.steps, "avg_us": e["avg_ms"] * 1e3,
               "ms_per_step": e["total_ms"] / args.steps}
        if ab is not None and e["avg_ms"] > 0:
            gbs = ab / (e["avg_ms"] * 1e-3) / 1e9
            ent.update({"alg_bytes": ab, "gbps": gbs, "frac": gbs / HBM_PEAK_GBS})
        kernels[n] = ent
    dom = max((n for n in kernels if "gbps" in kernels[n]), key=lambda n: kernels[n]["ms_per_step"])
    dk = kernels[dom]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["gbps"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dk["frac"], "traffic": None,
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_us": dk["avg_us"]}

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
        "pcg": {"iters": iters, "max_true_relres": true_rr},
        "topology_ms": topo_ms,
        "kernels": kernels,
        "kernel_sweeps": sweeps,
        "baseline_note": PAPER_NOTE,
    }

    if not args.no_cpu_baseline:
        log(args, "cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(X, F, f, args.cpu_seconds)
    print(json.dumps(out), flush=True)


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


if __name__ == "__main__":
    main()
