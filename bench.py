#!/usr/bin/env python3
"""Throughput of the state-vector gate path on one MI355X.

Workload: the 30-qubit supremacy-style random circuit on a 5 x 6 grid, depth
20 (U3 on every qubit per layer, then one of four CZ patterns), 845 gates, in
complex64 (8 GiB state).  One step applies the whole circuit to the state,
which stays resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--fuse-k F] [--tile-m M]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "gate-apps/s + HBM GB/s (30q c64); adjoint grads/s and batched circuits/s"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=30, help="qubits (grid 5 x n/5)")
    ap.add_argument("--dtype", default="c64")
    ap.add_argument("--fuse-k", type=int, default=0)
    ap.add_argument("--tile-m", type=int, default=0)
    ap.add_argument("--modes", default="", help="comma list of extra fuse_k:tile_m variants to time")
    ap.add_argument("--cpu-gates", type=int, default=4, help="gates of the circuit the oracle times")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def cpu_baseline(circ, ngates: int):
    """The CPU oracle (complex128, one thread) on the first `ngates` gates of
    the same circuit at full width."""
    import numpy as np
    import oracle as O
    import workloads as W
    sub = W.Circuit(circ.n, circ.ops[:ngates], 0, circ.name + f"_first{ngates}")
    psi = O.basis_state(circ.n)
    t0 = time.perf_counter()
    O.apply_circuit(sub, psi)
    dt = time.perf_counter() - t0
    del psi
    return {"value": ngates / dt, "unit": "gate-apps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {ngates} gates of the {circ.n}-qubit circuit, complex128, 1 thread, "
                      f"{dt:.1f} s"}


def time_mode(q, torch, s, circ, steps, warmup, fuse_k, tile_m):
    for _ in range(warmup):
        s.apply_circuit(circ, fuse_k=fuse_k, tile_m=tile_m)
    torch.cuda.synchronize()
    s.profile(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        s.apply_circuit(circ, fuse_k=fuse_k, tile_m=tile_m)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = start.elapsed_time(stop)
    stats = {}
    for cls in ("sweep_dense", "sweep_diag", "tile", "mfma"):
        n, ms, by = s.profile_read(cls)
        if n:
            stats[cls] = (n, ms, by)
    s.profile(False)
    return wall, ev_ms, stats


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2106_13995_amd as q
    import workloads as W

    rows = 5
    cols = a.n // rows
    circ = W.random_grid_circuit(rows, cols, depth=20, seed=2)
    ngates = len(circ.ops)
    s = q.State(circ.n, a.dtype)

    wall, ev_ms, stats = time_mode(q, torch, s, circ, a.steps, a.warmup, a.fuse_k, a.tile_m)
    ms_per_step = ev_ms / a.steps
    value = ngates * a.steps / (ev_ms / 1e3)

    # dominant kernel class by total time
    dom = max(stats.items(), key=lambda kv: kv[1][1])
    dname, (dn, dms, dby) = dom
    achieved = dby / (dms / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": dname, "launches": dn, "avg_launch_ms": round(dms / dn, 4),
                "bytes_per_launch": dby / dn}
    total_bytes = sum(v[2] for v in stats.values())

    # norm check: <psi|psi> (unitary circuit from |0>)
    norm = s.expectation(W.PauliSum(circ.n, [1.0], [0], [0]))

    extra = {}
    for m in [x for x in a.modes.split(",") if x]:
        fk, tm = (int(v) for v in m.split(":"))
        s.set_basis(0)
        w2, e2, st2 = time_mode(q, torch, s, circ, max(1, a.steps // 2), 1, fk, tm)
        extra[m] = {"ms_per_step": round(e2 / max(1, a.steps // 2), 3),
                    "gate_apps_per_s": round(ngates * max(1, a.steps // 2) / (e2 / 1e3), 1),
                    "passes_per_step": sum(v[0] for v in st2.values()) // max(1, a.steps // 2)}

    s.close()
    del s
    torch.cuda.empty_cache()

    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(circ, a.cpu_gates)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "gate-apps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex64" if a.dtype == "c64" else "complex128",
        "data": "synthetic",
        "config": {"workload": f"random supremacy-style circuit, {rows}x{cols} grid, {circ.n} qubits, depth 20, "
                               f"{ngates} gates (U3 + CZ), |0...0> input, state resident in HBM",
                   "n": circ.n, "gates": ngates, "fuse_k": a.fuse_k, "tile_m": a.tile_m},
        "hbm_gbs_algorithmic": round(total_bytes / (ev_ms / 1e3) / 1e9, 1),
        "passes_per_step": sum(v[0] for v in stats.values()) // a.steps,
        "wall_s": round(wall, 3),
        "norm": norm,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if extra:
        out["variants"] = extra
    print(json.dumps(out))


if __name__ == "__main__":
    main()
