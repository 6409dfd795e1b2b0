"""HBM traffic of the filter pass kernels from rocprofv3 counter runs.

rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) over a ``bench.py
--profile-filter`` run reports KiB per dispatch for the pass kernels and for a
plain device copy of known size (the calibration: the copy moves exactly
``copy_bytes`` each way).  ``summarise`` turns the two counter CSVs into bytes
per pass launch (complex64 and complex128 passes separately), scaled by the
copy's known / measured ratio, and records the hash of the kernel source so
that a stale measurement is never reported for a changed kernel.  Family
``ki`` is the kicked-Ising Horner pass (one launch per Horner step), family
``bw`` the brickwork passes (two launches per Horner step: right block, then
left block with +psi).

Usage:
  python -m paper_2102_05054_amd.traffic FETCH.csv WRITE.csv COPY_BYTES OUT.json [ki|bw]
  python -m paper_2102_05054_amd.traffic --launches KERNEL_TRACE.csv OUT.json

The second form averages the durations of a ``rocprofv3 --kernel-trace`` run
per kernel and grid size: a solve launches the same pass kernel over 4 or 2
vectors (and the tile autotuner over fewer), and the launches over all the
vectors of a filter are the ones a roofline figure describes.
"""

from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
FAMILIES = {
    "ki": {"kernels": ("ki_pass_kernel", "ki_pass3_kernel"),
           "sources": ["csrc/ki_kernels_impl.h", "csrc/tile_engine.h", "csrc/ki_kernels.h"],
           "launches_per_step": 1},
    # (bw_pipe_kernel: the persistent brickwork pass of earlier traces)
    "bw": {"kernels": ("bw_pass_kernel", "bw_pipe_kernel", "bw_pass_split_kernel"),
           "sources": ["csrc/bw_kernels.hip", "csrc/tile_engine.h", "csrc/bw_kernels.h"],
           "launches_per_step": 2},
}
KERNEL_SOURCES = FAMILIES["ki"]["sources"]


def kernel_hash(family: str = "ki") -> str:
    h = hashlib.sha256()
    for rel in FAMILIES[family]["sources"]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _per_kernel(path):
    """Average counter value and dispatch count per kernel, over the
    dispatches of the kernel's largest grid: the launches over all vectors of
    the profiled filter (the autotuner also times sub-batches of fewer
    vectors, whose launches move fewer bytes)."""
    acc = defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            acc[r["Kernel_Name"]].append((int(r.get("Grid_Size") or 0), float(r["Counter_Value"])))
    avg, cnt = {}, {}
    for k, v in acc.items():
        gmax = max(g for g, _ in v)
        vals = [x for g, x in v if g == gmax]
        avg[k] = sum(vals) / len(vals)
        cnt[k] = len(vals)
    return avg, cnt


def summarise(fetch_csv, write_csv, copy_bytes, family="ki"):
    fetch, nf = _per_kernel(fetch_csv)
    write, _ = _per_kernel(write_csv)
    copy_names = [k for k in fetch if ("copyBuffer" in k or "elementwise" in k or "vectorized" in k)
                  and "_pass" not in k and "_pipe" not in k and fetch[k] * 1024.0 > 0.05 * copy_bytes]
    if not copy_names:
        raise RuntimeError("no copy kernel in the counter runs")
    for k in copy_names:
        print(f"calibration {k[:70]}: fetch factor {copy_bytes / (fetch[k] * 1024.0):.3f}, "
              f"write factor {copy_bytes / (write[k] * 1024.0):.3f}", file=sys.stderr)
    # the plain elementwise copy uses the same global load/store instructions as
    # the pass kernel; the runtime's blit kernel reads differently and is only
    # reported
    plain = [k for k in copy_names if "elementwise" in k or "vectorized" in k]
    cname = plain[0] if plain else copy_names[0]
    factors = {k: {"fetch": copy_bytes / (fetch[k] * 1024.0), "write": copy_bytes / (write[k] * 1024.0)}
               for k in copy_names}
    f_factor = copy_bytes / (fetch[cname] * 1024.0)
    w_factor = copy_bytes / (write[cname] * 1024.0)
    fam = FAMILIES[family]

    def real_of(name):
        # the precision of a pass kernel from its first template argument
        # (traces of the plane-split brickwork pass from before it took one,
        # when it was complex128 only, have an integer there)
        for t in fam["kernels"]:
            for r in ("float", "double"):
                if f"{t}<{r}" in name:
                    return r
            if "split" in t and f"{t}<" in name:
                return "double"
        return None

    passes = {}
    for k in fetch:
        if real_of(k):
            passes[k] = {
                "fetch_bytes": fetch[k] * 1024.0 * f_factor,
                "write_bytes": write.get(k, 0.0) * 1024.0 * w_factor,
                "dispatches": nf[k],
                "real": real_of(k),
            }

    def per_pass(real):
        sel = [v for v in passes.values() if v["real"] == real]
        n = sum(v["dispatches"] for v in sel)
        if n == 0:
            return None
        return sum((v["fetch_bytes"] + v["write_bytes"]) * v["dispatches"] for v in sel) / n

    def dominant(real):
        # the kernels of the tuned passes: those with at least half the
        # dispatches of the most frequent one (the two tile groups of a plan
        # alternate), dispatch-weighted
        sel = {k: v for k, v in passes.items() if v["real"] == real}
        if not sel:
            return None
        top = max(v["dispatches"] for v in sel.values())
        main = {k: v for k, v in sel.items() if v["dispatches"] * 2 >= top}
        n = sum(v["dispatches"] for v in main.values())
        return {"kernels": sorted(main), "dispatches": n,
                "bytes_per_launch": sum((v["fetch_bytes"] + v["write_bytes"]) * v["dispatches"]
                                        for v in main.values()) / n}

    def per_step(real):
        b = per_pass(real)
        return None if b is None else b * fam["launches_per_step"]

    c64 = per_pass("float")
    return {
        "family": family,
        # the kernel with the most dispatches (the tuned pass of the workload)
        "dominant_c64": dominant("float"),
        "dominant_c128": dominant("double"),
        "bytes_per_horner_step_c64": per_step("float"),
        "bytes_per_horner_step_c128": per_step("double"),
        "kernel_hash": kernel_hash(family),
        "copy_kernel": cname,
        "calibration_factors": factors,
        "copy_bytes": copy_bytes,
        "fetch_factor": f_factor,
        "write_factor": w_factor,
        "per_kernel": passes,
        "bytes_per_pass": c64,
        "bytes_per_pass_c64": c64,
        "bytes_per_pass_c128": per_pass("double"),
    }


def launch_durations(path):
    """Per kernel name: {grid size: (dispatches, average microseconds)},
    from a rocprofv3 kernel-trace CSV (Start/End timestamps in ns)."""
    acc = defaultdict(lambda: defaultdict(list))
    with open(path) as f:
        for r in csv.DictReader(f):
            if "Grid_Size" in r and r["Grid_Size"]:
                grid = int(r["Grid_Size"])
            else:
                grid = 1
                for ax in ("X", "Y", "Z"):
                    grid *= int(r.get(f"Grid_Size_{ax}") or 1)
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
            acc[r["Kernel_Name"]][grid].append(dur)
    return {k: {g: (len(v), sum(v) / len(v)) for g, v in sorted(per.items())} for k, per in acc.items()}


if __name__ == "__main__" and len(sys.argv) > 1 and sys.argv[1] == "--launches":
    table = launch_durations(sys.argv[2])
    rows = {k: {str(g): {"dispatches": n, "avg_us": a} for g, (n, a) in per.items()} for k, per in table.items()}
    with open(sys.argv[3], "w") as f:
        json.dump(rows, f, indent=1)
    for k, per in table.items():
        if any(x in k for x in FAMILIES["ki"]["kernels"] + FAMILIES["bw"]["kernels"]):
            for g, (n, a) in per.items():
                m = re.search(r"(\w+<[^>]*>)", k)
                print(f"{m.group(1) if m else k}  grid {g}: {n} dispatches, {a:.2f} us")
elif __name__ == "__main__":
    out = summarise(sys.argv[1], sys.argv[2], float(sys.argv[3]), sys.argv[5] if len(sys.argv) > 5 else "ki")
    with open(sys.argv[4], "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
