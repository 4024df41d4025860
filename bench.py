#!/usr/bin/env python3
"""Benchmark of one full IB-LB step on one MI355X.

Workload (default): the 64^3 shear case -- walls moving at -+0.01, a rigidly
coated capsule alpha = abar(1,1,1) at Ca = 0.05 meshed as a level-4 icosphere
(2562 vertices, 5120 faces, R = 10), FP32 deviation populations with FP64
positions and volume reductions.  Synthetic seeded inputs, no datasets.

Timed region: K steps replayed from a captured hipGraph, inputs resident in
HBM, bracketed by torch.cuda.synchronize().  value = fluid nodes x steps /
seconds / 1e6 (MLUPS) for the whole step (forces, spreading, LB, interpolation
and move).  A second, instrumented pass times every kernel with hipEvents on
the library's stream; the LB kernel's average duration gives the achieved
algorithmic HBM bandwidth (38 population accesses of 4 bytes per fluid node).
The FP64 CPU oracle is timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline per IB-LB step; adjoint/forward time ratio at stated accuracy"
HBM_PEAK_GBS = 8000.0


def workload(name: str):
    from paper_2305_18919_amd import inputs as I
    if name == "shear64":
        return I.c2_shear(0.05), 1
    if name == "droplet32":
        return I.c1_droplet(), 0
    if name == "wetting128":
        return I.c3_wetting(1.0), 1
    if name == "probe256":
        w = I.c3_wetting(1.0)
        w.domain = I.Domain(256, 256, 256)
        w.mesh.vertices = w.mesh.vertices + [64.0, 64.0, 0.0]
        w.mesh.ref_vertices = w.mesh.ref_vertices + [64.0, 64.0, 0.0]
        w.name = "probe256_f32"
        return w, 1
    raise SystemExit(f"unknown workload {name}")


def lb_bytes_per_node(precision: int) -> int:
    return 38 * (8 if precision == 0 else 4)


def cpu_baseline(w, budget_s: float):
    """The FP64 oracle on this host, on a bounded number of steps of the same workload."""
    from oracle import oracle as O
    sim = O.OracleSim(w.domain, w.mesh)
    sim.step(2)  # warm-up
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        sim.step(5)
        steps += 5
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return {"value": round(w.domain.n_fluid * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{w.name}: {steps} FP64 oracle steps after 2 warm-up steps ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="shear64")
    ap.add_argument("--timed-steps", type=int, default=500, help="steps of the hipEvent-instrumented pass")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not part of "
                                   "this build (see the sharding notes in the design document)"}))
        raise SystemExit(2)

    import torch
    from paper_2305_18919_amd import iblb

    w, prec = workload(args.workload)
    dom, mesh = w.domain, w.mesh
    sim = iblb.Simulation(dom, mesh, precision=prec, graph=True)
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    mlups = dom.n_fluid * args.steps / dt / 1e6

    # instrumented pass: per-kernel hipEvent durations on the library stream
    sim.set_timing(True)
    sim.reset_timing()
    sim.step(args.timed_steps)
    sim.sync()
    kernels = {}
    for name in ("forces", "spread", "lb", "move"):
        ms, n = sim.kernel_time(name)
        if n:
            kernels[name] = {"avg_us": round(ms * 1e3 / n, 3), "launches": n}
    sim.set_timing(False)
    lb_us = kernels["lb"]["avg_us"]
    lb_alg = dom.n_fluid * lb_bytes_per_node(prec)
    achieved = lb_alg / (lb_us * 1e-6) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_lb", "alg_bytes_per_launch": lb_alg, "avg_us": lb_us}
    sim.close()

    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == 1 else "f64", "data": "synthetic",
        "config": {"workload": w.name, "grid": [dom.nx, dom.ny, dom.nz], "fluid_nodes": dom.n_fluid,
                   "vertices": mesh.n_vertices, "faces": mesh.n_faces, "tau": dom.tau,
                   "alpha": list(mesh.alpha), "positions": "f64", "launch": "hipGraph, 16 steps per replay"},
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
