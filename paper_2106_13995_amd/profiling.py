"""Summaries of rocprofv3 output for the committed performance records.

* ``kernel_stats``: per-kernel call count and average duration from a
  ``--kernel-trace --stats --output-format csv`` run;
* ``pmc_traffic``: HBM bytes per dispatch of one kernel from two ``--pmc``
  runs (FETCH_SIZE, then WRITE_SIZE, both in KiB per dispatch), each scaled by
  what the same counter reads for a plain device copy of known size.

    python -m paper_2106_13995_amd.profiling stats <kernel_stats.csv>
    python -m paper_2106_13995_amd.profiling traffic --fetch F.csv --write W.csv \
        --calib-fetch CF.csv --calib-write CW.csv --calib-bytes B --kernel SUBSTR \
        --cls tile --config KEY --out profiles/pmc_traffic.json [--skip S --take T]
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {
    "tile": ["kernels_reg.hip", "kernels.hip"],
    "tile_jit": ["jit.cpp", "stages.cpp", "gates.cpp"],
    "sweep_dense": ["kernels.hip"],
    "sweep_diag": ["kernels.hip"],
}


def source_hash(cls: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(cls, []):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_stats(path: str):
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            out.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_ms": float(r["AverageNs"]) / 1e6,
                        "total_ms": float(r["TotalDurationNs"]) / 1e6, "pct": float(r["Percentage"])})
    return out


def counter_per_dispatch(path: str, kernel_substr: str, skip: int = 0, take: int = 0):
    """Mean counter value per dispatch of kernels whose name contains
    `kernel_substr` (values of one dispatch are summed over instances).
    `skip` and `take` select, in dispatch order, the dispatches that count:
    the first `skip` are left out, then `take` are kept (0: all the rest)."""
    per = defaultdict(float)
    with open(path) as f:
        for r in csv.DictReader(f):
            if kernel_substr not in r.get("Kernel_Name", ""):
                continue
            per[int(r.get("Dispatch_Id") or r.get("Correlation_Id"))] += float(r["Counter_Value"])
    ids = sorted(per)[skip:]
    if take:
        ids = ids[:take]
    if not ids or (take and len(ids) < take):
        raise ValueError(f"too few dispatches of {kernel_substr!r} in {path}: {len(per)}, skip {skip}, take {take}")
    return sum(per[i] for i in ids) / len(ids), len(ids)


def pmc_traffic(a):
    fetch, nf = counter_per_dispatch(a.fetch, a.kernel, a.skip, a.take)
    write, nw = counter_per_dispatch(a.write, a.kernel, a.skip, a.take)
    cf, _ = counter_per_dispatch(a.calib_fetch, a.calib_kernel)
    cw, _ = counter_per_dispatch(a.calib_write, a.calib_kernel)
    kib = float(a.calib_bytes) / 1024.0
    sf, sw = kib / cf, kib / cw
    rec = {
        "kernel": a.kernel, "dispatches": nf, "skipped_dispatches": a.skip,
        "fetch_kib_raw": fetch, "write_kib_raw": write,
        "calib_fetch_kib_raw": cf, "calib_write_kib_raw": cw, "calib_bytes_each_way": int(a.calib_bytes),
        "fetch_scale": sf, "write_scale": sw,
        "bytes_per_launch": (fetch * sf + write * sw) * 1024.0,
        "source_hash": source_hash(a.cls),
        "commands": a.commands,
    }
    data = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            data = json.load(f)
    data.setdefault(a.config, {})[a.cls] = rec
    with open(a.out, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write", "kernel", "cls", "config", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--calib-bytes", required=True, type=int)
    t.add_argument("--calib-kernel", default="copy")
    t.add_argument("--commands", default="")
    t.add_argument("--skip", type=int, default=0, help="dispatches of the kernel left out at the start")
    t.add_argument("--take", type=int, default=0, help="dispatches counted after those (0: all the rest)")
    a = ap.parse_args()
    if a.cmd == "stats":
        for r in kernel_stats(a.csv):
            print(f"{r['calls']:6d}  {r['avg_ms']:10.4f} ms avg  {r['total_ms']:10.2f} ms total  {r['pct']:6.2f}%  {r['name']}")
    else:
        pmc_traffic(a)


if __name__ == "__main__":
    main()
