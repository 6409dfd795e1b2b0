"""Benchmark: time to the 100 eigenpairs closest to z = 1 of a kicked-Ising
chain of L = 20 qubits on one MI355X, complex64 filter + FP64 refinement
versus plain complex128, with U-applications/s and the filter kernel's
bandwidth against the HBM roofline.

Workload: kicked Ising, L = 20 (d = 1,048,576), J ~ U[0.8, 1.2],
h ~ U[-1, 1], g = 0.9, periodic, seed 3000, target phi = 0, nev = 100,
ncv = 220, tol = 1e-10.  The filter order follows the paper's rule
k = 0.8 * 2^{L+1} / ncv (Sec. 5) = 7626; at the nominal k = 400 with
ncv = 220 the apple-line ratio 2d/((k+1) ncv) is 24 and Krylov-Schur
stagnates (the worst Ritz estimate stays near 5e-2 over 200 restarts), so
no time-to-solution exists there.

Other modes: --workload ki_batched (the 1024-problem disorder workload in one
batched call), --workload bw_L24 (the brickwork filter at L = 24),
--workload bw_paper --L L (the paper's brickwork benchmark problem at L),
--scan-L L (an (ncv, k) runtime scan), --profile-filter (for counter runs).

One step = one complete arnoldi_eigs solve (filter, CGS2, restart, Ritz
vectors, FP64 residuals, refinement) in complex64 + FP64 refinement, block
Krylov-Schur with 4 vectors per filter launch (--block); the complex128
comparison solve uses 2 (--block-c128), the faster setting of each path.
value = U-applications per second over the timed steps (whole job).
The default run also reports, beside the headline, one timed call of the
batched disorder workload (batched_workload; --no-batched skips it).
roofline = the pass kernel that takes most of the timed solve (the FP64
refinement's complex128 pass, or the complex64 pass), timed with HIP events
in the launch configuration the solve uses (block vectors per launch).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--k K] [--no-c128] [--no-cpu]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--L", type=int, default=20)
    ap.add_argument("--k", type=int, default=None, help="filter order (default: paper rule)")
    ap.add_argument("--nev", type=int, default=100)
    ap.add_argument("--ncv", type=int, default=220)
    ap.add_argument("--W", type=float, default=1.0)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-restarts", type=int, default=60)
    ap.add_argument("--block", type=int, default=4,
                    help="vectors filtered per Krylov step of the complex64 + FP64 solve (1, 2, 4, 8)")
    ap.add_argument("--block-c128", type=int, default=2,
                    help="vectors filtered per Krylov step of the complex128 comparison solve")
    ap.add_argument("--no-c128", action="store_true", help="skip the complex128 comparison solve")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true",
                    help="default run: skip the batched disorder workload (one timed arnoldi_eigs_batched call)")
    ap.add_argument("--roofline-steps", type=int, default=2000)
    ap.add_argument("--scan-sizes", type=int, nargs="+", default=[20, 22, 24],
                    help="pass_scan: chain lengths")
    ap.add_argument("--policy", default="auto", choices=["auto", "tile", "pipe"],
                    help="pass_scan: kernel policy of the multi-vector passes (fq_set_kernel_policy)")
    ap.add_argument("--budget", type=float, default=400.0,
                    help="wall-clock budget in seconds of the default run: timed solves stop early so that the "
                         "comparison solve, the roofline passes and the JSON line fit in it")
    ap.add_argument("--scan-L", type=int, default=None,
                    help="(n_cv, k) scan of the brickwork circuit at this L (n_ev=50, z=1, complex128)")
    ap.add_argument("--workload", default="ki_L20", choices=["ki_L20", "ki_batched", "bw_L24", "bw_paper", "nominal", "pass_scan"],
                    help="ki_batched: 256 realisations x 4 targets, L in 12..16, one batched call; "
                         "bw_L24: the brickwork filter (k=300) at L=24")
    ap.add_argument("--filter-steps", type=int, default=0,
                    help="bw_paper: time only the block filter (--block-c128 vectors per launch, this many Horner "
                         "steps) instead of the solve")
    ap.add_argument("--graphs", type=int, default=1, choices=[0, 1],
                    help="ki_batched: replay the lockstep filters from captured HIP graphs (fq_set_graph_capture)")
    ap.add_argument("--profile-gemm", action="store_true",
                    help="only solves with filter order 1 (two restarts each), for counter runs of the FP64 "
                         "matrix-core basis rotation")
    ap.add_argument("--profile-filter", action="store_true",
                    help="only the Horner filters (k=200, complex64 then complex128, --block vectors per launch) "
                         "and the calibration copies, for counter runs; with --workload bw_L24 or bw_paper "
                         "--filter-steps, the calibration copies after that workload's filter")
    return ap.parse_args()


def filter_roofline(op, L, steps, nvec=1, dtype="c64"):
    """Average duration of the Horner pass kernel from HIP events on the
    launch stream, with nvec vectors per launch (apply_filter_many) as in a
    block solve; algorithmic bytes per pass = nvec * 3 * (8 or 16) * 2^L
    (read w and psi, write w)."""
    import torch
    d = 2 ** L
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    esize = 8 if dtype == "c64" else 16
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        psi = torch.randn((nvec, d), dtype=tdt, device="cuda")
        out = torch.empty_like(psi)

        def run(kk):
            if nvec == 1:
                op.apply_filter(psi[0], kk, 0.0, out=out[0], stream=s)
            else:
                op.apply_filter_many(psi, kk, 0.0, out=out, stream=s)

        run(steps)  # warm: tables, plans and the tile tuner for this k
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        run(steps)
        e1.record(s)
    s.synchronize()
    ms = e0.elapsed_time(e1)
    launches = steps + 1  # k Horner passes + the prologue kick pass
    avg_s = ms * 1e-3 / launches
    bytes_per_launch = nvec * 3 * esize * d
    real = "float" if dtype == "c64" else "double"
    return {
        "kernel": f"kicked-Ising Horner pass <{real}> ({nvec} vector(s) per launch: "
                  f"{'ki_pass3_kernel / ki_pass_kernel, autotuned' if nvec > 1 else 'ki_pass3_kernel where the tile has 16 amplitudes per thread, else ki_pass_kernel'}; "
                  f"kick, phase, +psi, kick)",
        "dtype": dtype,
        "vectors_per_launch": nvec,
        "avg_launch_us": avg_s * 1e6,
        "bytes_per_launch": bytes_per_launch,
        "achieved_GBs": bytes_per_launch / avg_s / 1e9,
        "U_apps_per_s": nvec / avg_s,
    }


COPY_BYTES = 2 ** 30


def profile_filter(op, L, nvec):
    """Workload of the counter runs: 200 Horner passes in complex64, then 200
    in complex128, nvec vectors per launch, and the calibration copies."""
    import torch
    for tdt in (torch.complex64, torch.complex128):
        psi = torch.randn((nvec, 2 ** L), dtype=tdt, device="cuda")
        out = torch.empty_like(psi)
        if nvec == 1:
            op.apply_filter(psi[0], 200, 0.0, out=out[0])
        else:
            op.apply_filter_many(psi, 200, 0.0, out=out)
        torch.cuda.synchronize()
        del psi, out
    calibration_copies()
    print(json.dumps({"profile_filter": True, "L": L, "vectors_per_launch": nvec, "copy_bytes": COPY_BYTES}))


def calibration_copies():
    """Two plain device copies of COPY_BYTES (1 GiB, source evicted from L2 and
    the Infinity Cache by a second 1 GiB write) that calibrate FETCH_SIZE /
    WRITE_SIZE in bytes."""
    import torch
    torch.cuda.synchronize()
    a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda").fill_(1)
    c = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda").fill_(2)
    b = torch.empty_like(a)
    b.copy_(a)
    # second calibration copy through torch's elementwise kernel (float32 view)
    torch.mul(c.view(torch.float32), 1.0, out=a.view(torch.float32))
    torch.cuda.synchronize()
    del a, b, c


def profile_gemm(op, L, ncv, nev, block):
    """Workload of the matrix-core counter runs: complex128 Krylov-Schur at
    filter order 1 for two restarts (block 1 and the given block), so that the
    restart rotation V_m Z_p (d x m by m x p, complex FP64) and the Ritz products
    dominate the few other kernels.  Prints the rotation's algorithmic flops."""
    import torch
    for b in sorted({1, block}):
        op.arnoldi_eigs(nev, 0.0, k=1, ncv=ncv, tol=1e-10, max_restarts=2, filter_dtype="c128", seed=1,
                        want_vectors=False, allow_not_converged=True, block=b)
    torch.cuda.synchronize()
    d = 2 ** L
    m = ncv
    p = min(m - 1, max(nev + 1, nev + (m - nev) // 2))
    print(json.dumps({"profile_gemm": True, "L": L, "m": m, "p": p,
                      "rotation_flop": 8 * d * m * p, "rotation_bytes": 16 * d * (m + p)}))


def traffic_file(nvec, L=20):
    if L == 20:
        name = "ki_pass_kernel_L20_traffic.json" if nvec == 1 else f"ki_pass_kernel_L20_block{nvec}_traffic.json"
    else:
        name = f"ki_pass_kernel_L{L}_traffic.json"
    return os.path.join(ROOT, "profiles", name)


def traffic_per_pass(nvec, dtype, L=20):
    """Calibrated HBM bytes per pass launch (nvec vectors) from the committed
    counter summary, only when it was measured on the current kernel source."""
    try:
        from paper_2102_05054_amd.traffic import kernel_hash
        with open(traffic_file(nvec, L)) as f:
            rec = json.load(f)
        if rec.get("kernel_hash") == kernel_hash():
            dom = rec.get(f"dominant_{dtype}")
            if dom:
                return dom["bytes_per_launch"]
            return rec.get(f"bytes_per_pass_{dtype}", rec["bytes_per_pass"] if dtype == "c64" else None)
    except (OSError, ValueError, KeyError):
        pass
    return None


def traffic_per_pass_L24(dtype):
    return traffic_per_pass(1, dtype, L=24)


def scan(L, nev=50, block=1):
    """Runtime over a grid of (n_cv, k) for the brickwork random circuit (the
    setting of the paper's Fig. "bench": n_ev = 50, z = 1).  Each line gives
    time, U-applications and restarts; the rule n_cv = 0.8 * 2^(L+1) / k is
    printed next to it.  From L = 16 on, n_cv stays at most 256 (the FP64
    basis of 2^L x n_cv amplitudes outgrows the Infinity Cache beyond, and
    its orthogonalisation then dominates) and the solves use blocks of
    `block` vectors."""
    import torch

    from paper_2102_05054_amd import brickwork, paper_parameters
    from workloads import brickwork as bw_params
    p = bw_params(L, 5000 + L)
    op = brickwork(L, p.gates)
    d = 2 ** L
    ncv0, k0 = paper_parameters(L, nev)
    cap = 256 if L >= 16 else d - 1
    if ncv0 > cap:
        ncv0 = cap
        k0 = int(math.floor(0.8 * 2 ** (L + 1) / ncv0))
    ks = sorted({max(4, int(k0 * f)) for f in (0.25, 0.5, 1.0, 2.0, 4.0)})
    ncvs = sorted({min(cap, max(2 * nev + 2, int(ncv0 * f))) for f in (0.5, 0.7, 1.0, 1.4, 2.0)})
    blk = block if L >= 16 else 1
    rows = []
    for ncv in ncvs:
        for k in ks:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, _, res, st, status = op.arnoldi_eigs(nev, 0.0, k=k, ncv=ncv, tol=1e-10, max_restarts=60,
                                                     seed=1, want_vectors=False, allow_not_converged=True,
                                                     block=blk)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rows.append({"L": L, "ncv": ncv, "k": k, "block": blk, "time_s": dt, "U_apps": st["n_U_apps"],
                         "restarts": st["n_restarts"], "nconv": st["nconv"], "status": int(status),
                         "max_residual": float(res.max()), "rule_ncv_0.8": 0.8 * 2 ** (L + 1) / k,
                         "apple_ncv": 2 ** (L + 1) / (k + 1)})
            print(json.dumps(rows[-1]), flush=True)
    ok = [r for r in rows if r["status"] == 0]
    best = min(ok, key=lambda r: r["time_s"]) if ok else None
    print(json.dumps({"scan_L": L, "paper_rule_at_ncv": {"ncv": ncv0, "k": k0}, "fastest": best}))
    op.close()


def batched(args):
    """The disorder-averaged workload on its own (--workload ki_batched)."""
    print(json.dumps(batched_workload(args.steps, max(1, args.warmup), not args.no_c128, True, bool(args.graphs))))


def batched_workload(steps, warmup, with_c128, one_by_one, graphs):
    """The disorder-averaged workload: 256 kicked-Ising realisations with L
    uniform in {12..16}, each at the 4 targets phi in {0, pi/2, pi, 3pi/2},
    nev = 20, ncv = 60, complex64 filter + FP64 refinement, tol 1e-10, in one
    arnoldi_eigs_batched call.  The filter order per chain length follows the
    paper's rule k = 0.8 * 2^(L+1) / ncv (at the nominal k = 150 the L = 16
    problems do not converge within 200 restarts).  The first call (warm-up)
    also runs the tile-shape autotuner.  Returns the bench line as a dict."""
    import numpy as np
    import torch

    from paper_2102_05054_amd import arnoldi_eigs_batched, kicked_ising, set_graph_capture
    from workloads import CONFIGS, config_kicked_ising
    set_graph_capture(graphs)
    c = CONFIGS["ki_batched"]
    nev, ncv = c["nev"], c["ncv"]
    ops, ks = [], []
    for r in range(c["n_real"]):
        p = config_kicked_ising("ki_batched", realisation=r)
        ops.append(kicked_ising(p.L, p.J, p.h, p.g, p.periodic))
        ks.append(int(math.floor(0.8 * 2 ** (p.L + 1) / ncv)))
    phis = list(c["phis"])
    nprob = len(ops) * len(phis)

    def run(dtype):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, res, stats, st = arnoldi_eigs_batched(ops, phis, nev, k=ks, ncv=ncv, tol=c["tol"], filter_dtype=dtype,
                                                  seed=1, max_restarts=200, allow_not_converged=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ev, res, stats, st

    for _ in range(max(1, warmup)):
        run("c64")
    t_total, uapps = 0.0, 0
    for _ in range(steps):
        dt, ev, res, stats, st = run("c64")
        t_total += dt
        uapps += sum(x["n_U_apps"] for x in stats)
    c128 = None
    if with_c128:
        run("c128")  # tunes the complex128 shapes
        dt2, ev2, res2, stats2, st2 = run("c128")
        c128 = {"time_s": dt2, "status": int(st2), "max_residual": float(res2.max()),
                "nconv": int(sum(x["nconv"] for x in stats2))}
    # one problem per chain length one by one, scaled by the counts
    seq = 0.0
    seq_detail = {}
    for L in (sorted({o.L for o in ops}) if one_by_one else []):
        i = next(i for i, o in enumerate(ops) if o.L == L)
        cnt = sum(1 for o in ops if o.L == L) * len(phis)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ops[i].arnoldi_eigs(nev, 0.0, k=ks[i], ncv=ncv, tol=c["tol"], filter_dtype="c64", seed=1,
                            want_vectors=False, allow_not_converged=True)
        torch.cuda.synchronize()
        one = time.perf_counter() - t0
        seq += one * cnt
        seq_detail[str(L)] = {"problems": cnt, "s_per_problem": one}
    line = {
        "metric": "U-applications/s and time to all eigenpairs of the batched workload (1024 problems)",
        "value": uapps / t_total,
        "unit": "U-applications/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(1, warmup),
        "ms_per_step": 1e3 * t_total / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 filter + f64",
        "data": "synthetic (seeded kicked-Ising couplings)",
        "config": {"workload": f"kicked Ising, 256 realisations, L uniform in 12..16, 4 targets, nev={nev}, "
                               f"ncv={ncv}, k per L by the paper rule, tol={c['tol']}",
                   "problems": nprob, "k_per_L": {str(o.L): k for o, k in zip(ops, ks)},
                   "graph_capture": graphs},
        "time_to_all_eigenpairs_s": {"batched c64+refine": t_total / steps,
                                     "batched c128": c128["time_s"] if c128 else None,
                                     "one by one c64+refine (estimated)": seq if one_by_one else None},
        "eigenpairs_per_s": nprob * nev / (t_total / steps),
        "solve": {"status": int(st), "max_residual": float(res.max()),
                  "nconv": int(sum(x["nconv"] for x in stats)), "pairs": nprob * nev,
                  "max_restarts_used": int(max(x["n_restarts"] for x in stats))},
        "c128_solve": c128,
        "one_by_one": seq_detail,
        "per_L": {},
    }
    for L in sorted({o.L for o in ops}):
        idx = [i * len(phis) + j for i, o in enumerate(ops) if o.L == L for j in range(len(phis))]
        line["per_L"][str(L)] = {
            "problems": len(idx),
            "k": ks[next(i for i, o in enumerate(ops) if o.L == L)],
            "mean_filter_apps": float(np.mean([stats[i]["n_filter_apps"] for i in idx])),
            "mean_U_apps_c64": float(np.mean([stats[i]["n_U_apps_c64"] for i in idx])),
            "mean_U_apps": float(np.mean([stats[i]["n_U_apps"] for i in idx])),
            "batch_time_s": float(max(stats[i]["t_total"] for i in idx)),
        }
    for o in ops:
        o.close()
    return line


def brickwork_filter(args):
    """Filter throughput of the brickwork circuit at L = 24 (d = 16,777,216),
    the size of the circuit workload: k = 300 Horner steps of g_k(U) psi in
    complex64 (timed steps) and complex128.  One Horner step is two tile
    passes (right block: read + write w; left block: read w and psi, write w),
    5 * d * s algorithmic bytes, and 32 * L * d real flops (each of the L
    two-site gates acts on all d amplitudes as 4x4 complex products).  The
    roofline is the FP32 vector rate without packed instructions, 256 CUs x 4
    SIMDs x 16 lanes x 2 flop x 2.4 GHz = 78.6 TFLOP/s.  The
    full eigen-solve at this size is out of reach at any converging filter
    order (the paper's rule gives k = 268,435 with ncv = 100)."""
    import numpy as np
    import torch

    from paper_2102_05054_amd import brickwork
    from workloads import CONFIGS
    from workloads import brickwork as bw_params
    c = CONFIGS["bw_L24"]
    L, k = c["L"], c["k"]
    d = 2 ** L
    p = bw_params(L, c["seed"])
    op = brickwork(L, p.gates)
    s = torch.cuda.Stream()
    out = {}
    for name, dt, size in (("c64", torch.complex64, 8), ("c128", torch.complex128, 16)):
        with torch.cuda.stream(s):
            x = torch.randn(d, dtype=dt, device="cuda")
            y = torch.empty_like(x)
            for _ in range(max(1, args.warmup)):
                op.apply_filter(x, 4, 0.0, out=y, stream=s)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            steps = args.steps if name == "c64" else 1
            e0.record(s)
            for _ in range(steps):
                op.apply_filter(x, k, 0.0, out=y, stream=s)
            e1.record(s)
            s.synchronize()
        ms = e0.elapsed_time(e1)
        us_step = 1e3 * ms / (steps * k)
        out[name] = {"us_per_horner_step": us_step, "U_apps_per_s": 1e6 / us_step,
                     "alg_GBs": 5 * d * size / (us_step * 1e3),
                     "TFLOPs": 32 * L * d / (us_step * 1e6), "filter_apps": steps, "ms": ms}
        del x, y
    op.close()
    if args.profile_filter:
        calibration_copies()
    c64 = out["c64"]
    line = {
        "metric": "U-applications/s and HBM GB/s of the brickwork filter at L=24",
        "value": c64["U_apps_per_s"],
        "unit": "U-applications/s",
        "n_gpus": 1, "steps": args.steps, "warmup": max(1, args.warmup),
        "ms_per_step": c64["ms"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic (seeded Haar-random two-site gates)",
        "config": {"workload": f"brickwork Haar circuit L={L} (d={d}), filter k={k}, phi=0, one step = one "
                               f"filter application", "L": L, "k": k},
        # 32*L flop per amplitude against 40 B moved: above the ridge of the
        # FP32 units without packed instructions (78.6 TFLOP/s / 8 TB/s = 9.8)
        "roofline": {"bound": "alu", "achieved": c64["TFLOPs"], "peak": 78.6, "unit": "TFLOP/s",
                     "frac": c64["TFLOPs"] / 78.6, "traffic": None,
                     "kernel": "bw_pass_split_kernel (complex64; bw_pass_kernel for complex128), right block + left block per Horner step",
                     "hbm_GBs": c64["alg_GBs"], "hbm_frac": c64["alg_GBs"] / 8000.0},
        "c128": out["c128"],
    }
    print(json.dumps(line))


# Time to the 50 eigenpairs closest to z = 1 of the brickwork Haar circuit on
# 16 cores of an AMD EPYC 7H12, complex FP64, n_cv = floor(2^(L/2+1)) and
# k = 0.8 * 2^(L+1) / n_cv (Sec. 5, Table "bench"), in seconds.
PAPER_BW_SECONDS = {10: 0.3, 11: 0.7, 12: 2.3, 13: 6.6, 14: 26.0, 15: 46.8, 16: 193.3, 17: 903.6, 18: 4965.2,
                    19: 16579.0, 20: 97706.9}


def brickwork_paper(args):
    """The paper's own benchmark problem: the 50 eigenpairs closest to z = 1
    of a brickwork Haar circuit of L sites, complex128 (the paper's precision),
    tol 1e-10, block Krylov-Schur with --block-c128 vectors per filter launch.
    n_cv = min(floor(2^(L/2+1)), 256) and k by the paper's rule
    0.8 * 2^(L+1) / n_cv for that n_cv: the (n_cv, k) scans at L = 12, 14 find
    smaller n_cv faster than the paper's, and n_cv in the thousands would make
    the host Schur step of each restart the bottleneck.  The paper's time for
    the same L (16-core CPU, its own n_cv and k) is quoted as context."""
    import torch

    from paper_2102_05054_amd import brickwork
    from workloads import brickwork as bw_params
    L = args.L
    nev = 50
    ncv = min(int(math.floor(2 ** (L / 2 + 1))), 256)
    k = int(math.floor(0.8 * 2 ** (L + 1) / ncv))
    p = bw_params(L, 5000 + L)
    op = brickwork(L, p.gates)
    if args.filter_steps > 0:
        brickwork_block_filter(args, op, L)
        return
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, _, res, st, status = op.arnoldi_eigs(nev, 0.0, k=k, ncv=ncv, tol=1e-10, max_restarts=args.max_restarts,
                                             filter_dtype="c128", seed=1, want_vectors=False, allow_not_converged=True,
                                             block=args.block_c128)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    op.close()
    paper = PAPER_BW_SECONDS.get(L)
    line = {
        "metric": "time to the 50 eigenpairs closest to z=1 of the brickwork Haar circuit (the paper's benchmark)",
        "value": dt, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * dt,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic (seeded Haar-random two-site gates)",
        "config": {"workload": f"brickwork Haar circuit L={L} (d={2 ** L}), nev=50, z=1, ncv={ncv}, k={k} "
                               f"(0.8*2^(L+1)/ncv), tol=1e-10, complex128", "L": L, "ncv": ncv, "k": k,
                   "block": args.block_c128},
        "solve": {"status": int(status), "nconv": st["nconv"], "max_residual": float(res.max()),
                  "n_restarts": st["n_restarts"], "n_U_apps": st["n_U_apps"], "t_filter_s": st["t_filter"],
                  "t_restart_s": st["t_restart"]},
        "paper_16core_cpu_s": paper,
        "ratio_paper_cpu_over_this": (paper / dt) if paper else None,
    }
    print(json.dumps(line))


def brickwork_block_filter(args, op, L):
    """The filter of the paper's benchmark solve alone: apply_filter_many on
    --block-c128 complex128 vectors (one launch per pass for all of them),
    --filter-steps Horner steps, timed with HIP events on the stream the
    passes run on.  Flops as for the L = 24 filter (32 * L * d per U); the FP64
    vector peak is 78.6 TFLOP/s."""
    import torch

    from workloads import random_state
    d, b, k = 2 ** L, args.block_c128, args.filter_steps
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x = torch.from_numpy(random_state(d, 7, b)).to("cuda", torch.complex128).contiguous()
        y = torch.empty_like(x)
        op.apply_filter_many(x, 2, 0.0, out=y, stream=s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        op.apply_filter_many(x, k, 0.0, out=y, stream=s)
        e1.record(s)
        s.synchronize()
    op.close()
    if args.profile_filter:
        calibration_copies()
    us_u = 1e3 * e0.elapsed_time(e1) / (k * b)
    tf = 32 * L * d / (us_u * 1e6)
    print(json.dumps({
        "metric": "U-applications/s of the block brickwork filter of the paper's benchmark",
        "value": 1e6 / us_u, "unit": "U-applications/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": e0.elapsed_time(e1), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128", "data": "synthetic (seeded Haar-random two-site gates)",
        "config": {"workload": f"brickwork Haar circuit L={L}, {b} vectors per launch, {k} Horner steps",
                   "L": L, "block": b, "k": k},
        "us_per_U": us_u,
        "roofline": {"bound": "alu", "achieved": tf, "peak": 78.6, "unit": "TFLOP/s", "frac": tf / 78.6,
                     "traffic": None, "hbm_GBs": 5 * d * 16 / (us_u * 1e3)},
    }))


def _cpu_worker(L, J, h, g, periodic, seconds, seed):
    """One host process: the oracle's matrix-free complex128 U applied
    repeatedly for about ``seconds``; returns (applications, wall, CPU time)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import models
    from workloads import KickedIsingParams, start_vector
    import numpy as np
    p = KickedIsingParams(L=L, J=np.asarray(J), h=np.asarray(h), g=g, periodic=periodic, phi=0.0)
    x = start_vector(2 ** L, seed)
    ru0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    n = 0
    while True:
        x = models.ki_apply(p, x)
        n += 1
        if time.perf_counter() - t0 > seconds:
            break
    wall = time.perf_counter() - t0
    ru1 = resource.getrusage(resource.RUSAGE_SELF)
    return n, wall, (ru1.ru_utime - ru0.ru_utime) + (ru1.ru_stime - ru0.ru_stime)


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    # a one-GPU job gets a 16-CPU share of the host, whatever the machine shows
    return max(1, min(n, 16))


def cpu_baseline(p, seconds=12.0):
    """The oracle's matrix-free U (complex128 NumPy, single-threaded as
    written) on every host core: one process per core, each applying U to
    its own state for a bounded time.  Runs before the GPU is initialised."""
    import concurrent.futures as cf
    import multiprocessing as mp
    workers = host_cores()
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(_cpu_worker, p.L, list(map(float, p.J)), list(map(float, p.h)), float(p.g),
                          bool(p.periodic), seconds, 3000 + i) for i in range(workers)]
        res = [f.result() for f in futs]
    wall_all = time.perf_counter() - t0
    n = sum(r[0] for r in res)
    rate = sum(r[0] / r[1] for r in res)
    cpu = sum(r[2] for r in res)
    busy = max(r[1] for r in res)
    return {
        "value": rate, "unit": "U-applications/s", "cores": round(cpu / busy, 2), "kind": "oracle",
        "sample": f"{n} matrix-free complex128 U applications of the oracle at L={p.L}, {workers} host processes "
                  f"x ~{seconds:.0f} s each ({wall_all:.1f} s wall with start-up, {cpu:.1f} s CPU; the host shows "
                  f"{os.cpu_count()} logical CPUs, of which {workers} were used)",
    }


def pass_roofline_L24(seconds_cap=20.0):
    """The kicked-Ising Horner pass at L = 24 (d = 16,777,216), where w and psi
    (2 x 128 MiB complex64, 2 x 256 MiB complex128) exceed the 256 MB
    Infinity Cache (complex64 only just: part of its reads may still hit
    there), one vector per launch: average pass duration from HIP events on
    the launch stream, 3 * d * s algorithmic bytes per pass."""
    from paper_2102_05054_amd import kicked_ising
    from workloads import config_kicked_ising
    q = config_kicked_ising("ki_L20", W=1.0, L=24)
    out = {}
    with kicked_ising(q.L, q.J, q.h, q.g, q.periodic) as op24:
        for dt in ("c64", "c128"):
            r = filter_roofline(op24, 24, 200, 1, dt)
            out[dt] = {"kernel": r["kernel"], "avg_launch_us": r["avg_launch_us"],
                       "bytes_per_launch": r["bytes_per_launch"], "achieved": r["achieved_GBs"],
                       "peak": 8000.0, "unit": "GB/s", "frac": r["achieved_GBs"] / 8000.0,
                       "traffic": traffic_per_pass_L24(dt)}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 (multi-GPU sharding is a design note only)"}))
        sys.exit(2)
    t_start = time.perf_counter()
    if args.scan_L is not None:
        scan(args.scan_L, block=args.block)
        return
    if args.workload == "ki_batched":
        batched(args)
        return
    if args.workload == "bw_L24":
        brickwork_filter(args)
        return
    if args.workload == "bw_paper":
        brickwork_paper(args)
        return
    if args.workload == "nominal":
        nominal(args)
        return
    if args.workload == "pass_scan":
        pass_scan(args)
        return
    from workloads import config_kicked_ising
    L = args.L
    k = args.k if args.k is not None else int(math.floor(0.8 * 2 ** (L + 1) / args.ncv))
    p = config_kicked_ising("ki_L20", W=args.W, L=L)
    # the host baseline runs first, before anything touches the GPU (its
    # worker processes are started from a process without a HIP context)
    cpu = None
    if not (args.no_cpu or args.profile_gemm or args.profile_filter):
        try:
            cpu = cpu_baseline(p)
        except Exception as e:  # reported, never fatal for the GPU measurement
            cpu = {"error": f"{type(e).__name__}: {e}"}
        log(f"cpu baseline: {cpu.get('value', 0):.2f} U-applications/s")

    import torch

    from paper_2102_05054_amd import kicked_ising
    op = kicked_ising(p.L, p.J, p.h, p.g, p.periodic)
    d = 2 ** L

    if args.profile_gemm:
        profile_gemm(op, L, args.ncv, args.nev, args.block)
        op.close()
        return
    if args.profile_filter:
        profile_filter(op, L, args.block)
        op.close()
        return

    def solve(dtype, block):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, _, res, st, status = op.arnoldi_eigs(args.nev, 0.0, k=k, ncv=args.ncv, tol=args.tol,
                                                 max_restarts=args.max_restarts, filter_dtype=dtype,
                                                 refine=True, seed=1, want_vectors=False,
                                                 allow_not_converged=True, block=block)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, ev, res, st, status

    # Wall budget: one warm-up solve at most (it also runs the tile tuner),
    # then timed solves while the rest still fits: the complex128 comparison
    # solve, the roofline passes and the JSON line need about one more solve,
    # the batched workload (a warm-up call with the tuner and a timed call)
    # about 90 s.
    batched_reserve = 0.0 if args.no_batched else 90.0
    warm = min(args.warmup, 1)
    for _ in range(warm):
        dt, *_ = solve("c64", args.block)
        log(f"warm-up c64+refine solve: {dt:.1f} s")
    t_total = 0.0
    uapps = 0
    runs = []
    for i in range(args.steps):
        dt, ev, res, st, status = solve("c64", args.block)
        log(f"c64+refine solve {i + 1}: {dt:.1f} s, status {int(status)}")
        t_total += dt
        uapps += st["n_U_apps"]
        runs.append((dt, ev, res, st, status))
        elapsed = time.perf_counter() - t_start
        if elapsed + dt * (1.0 + 2.2) + 30.0 + batched_reserve > args.budget:
            break
    last_dt, last_ev, last_res, last_st, last_status = runs[-1]
    steps_done = len(runs)

    c128 = None
    if not args.no_c128:
        dt2, ev2, res2, st2, status2 = solve("c128", args.block_c128)
        log(f"c128 solve: {dt2:.1f} s, status {int(status2)}")
        # the two precisions must return the same eigenvalue set
        a = np.sort_complex(np.asarray(last_ev))
        b = np.sort_complex(np.asarray(ev2))
        c128 = {"time_s": dt2, "status": int(status2), "nconv": st2["nconv"], "max_residual": float(res2.max()),
                "n_U_apps": st2["n_U_apps"], "n_restarts": st2["n_restarts"], "t_filter_s": st2["t_filter"],
                "block": args.block_c128,
                "max_eigenvalue_difference_to_c64_refine": float(np.max(np.abs(a - b))) if a.shape == b.shape
                else None}

    # the refinement's complex128 passes or the complex64 passes: whichever
    # phase took longer in the timed solve bounds it
    t_ref = last_st["t_refine"]
    dom = "c128" if t_ref > 0.5 * last_dt else "c64"
    roof = filter_roofline(op, L, args.roofline_steps, args.block, dom)
    other = filter_roofline(op, L, args.roofline_steps, args.block, "c64" if dom == "c128" else "c128")
    log(f"roofline: {roof['avg_launch_us']:.2f} us per {dom} pass")
    op.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    try:
        hbm = pass_roofline_L24()
        log(f"L=24 passes: c64 {hbm['c64']['avg_launch_us']:.1f} us, c128 {hbm['c128']['avg_launch_us']:.1f} us")
    except Exception as e:
        hbm = {"error": f"{type(e).__name__}: {e}"}
    # the disorder-averaged batched workload, reported beside (never fatal)
    batched_line = None
    if not args.no_batched:
        try:
            b = batched_workload(1, 1, False, False, True)
            batched_line = {"workload": b["config"]["workload"], "problems": b["config"]["problems"],
                            "time_to_all_eigenpairs_s": b["time_to_all_eigenpairs_s"]["batched c64+refine"],
                            "U_apps_per_s": b["value"], "eigenpairs_per_s": b["eigenpairs_per_s"],
                            "solve": b["solve"], "graph_capture": True,
                            "batch_time_s_per_L": {L: v["batch_time_s"] for L, v in b["per_L"].items()}}
            log(f"batched workload: {batched_line['time_to_all_eigenpairs_s']:.1f} s for {b['solve']['pairs']} pairs")
        except Exception as e:
            batched_line = {"error": f"{type(e).__name__}: {e}"}

    value = uapps / t_total
    line = {
        "metric": "U-applications/s (whole c64+FP64-refine solve) & filter HBM GB/s; time to 100 eigenpairs at L=20",
        "value": value,
        "unit": "U-applications/s",
        "n_gpus": 1,
        "steps": steps_done,
        "warmup": warm,
        "ms_per_step": 1e3 * t_total / steps_done,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 filter + f64",
        "data": "synthetic (seeded kicked-Ising couplings)",
        "config": {
            "workload": f"kicked Ising L={L} (d={d}), W={args.W}, nev={args.nev}, ncv={args.ncv}, "
                        f"k={k} (paper rule 0.8*2^(L+1)/ncv), phi=0, tol={args.tol}, "
                        f"block Krylov-Schur with {args.block} vectors per filter launch; one step = one "
                        f"complete solve",
            "L": L, "nev": args.nev, "ncv": args.ncv, "k": k, "phi": 0.0, "block": args.block,
        },
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "budget_s": args.budget,
        "time_to_eigenpairs_s": {"c64+refine": t_total / steps_done, "c128": c128["time_s"] if c128 else None},
        "eigenpairs_per_s": {"c64+refine": args.nev * steps_done / t_total,
                             "c128": (args.nev / c128["time_s"]) if c128 else None},
        # why the mixed form is not the faster one at this filter order
        "precision_note": ("the FP64 refinement needs about one full FP64 Krylov cycle whatever its start "
                           "(the Ritz vectors must be separated in FP64 from the eigenvectors next to the wanted "
                           "set inside the filter's main lobe), so the complex64 phase adds to the FP64 cost"),
        "solve": {"status": int(last_status), "nconv": last_st["nconv"], "max_residual": float(last_res.max()),
                  "n_restarts": last_st["n_restarts"], "n_U_apps": last_st["n_U_apps"],
                  "n_U_apps_c64": last_st["n_U_apps_c64"], "t_refine_s": last_st["t_refine"],
                  "t_filter_s": last_st["t_filter"], "t_orth_s": last_st["t_orth"],
                  "t_restart_s": last_st["t_restart"], "step_times_s": [r[0] for r in runs]},
        "c128_solve": c128,
        "roofline": {
            "bound": "hbm",
            "achieved": roof["achieved_GBs"],
            "peak": 8000.0,
            "unit": "GB/s",
            "frac": roof["achieved_GBs"] / 8000.0,
            "traffic": traffic_per_pass(args.block, dom),
            "kernel": roof["kernel"],
            "avg_launch_us": roof["avg_launch_us"],
            "bytes_per_launch": roof["bytes_per_launch"],
            "filter_U_apps_per_s": roof["U_apps_per_s"],
            "share_of_solve": (t_ref if dom == "c128" else last_dt - t_ref) / last_dt,
        },
        "roofline_other_pass": {
            "kernel": other["kernel"],
            "achieved": other["achieved_GBs"],
            "frac": other["achieved_GBs"] / 8000.0,
            "avg_launch_us": other["avg_launch_us"],
            "bytes_per_launch": other["bytes_per_launch"],
            "traffic": traffic_per_pass(args.block, other["dtype"]),
        },
        "roofline_L24_hbm_resident": hbm,
        "batched_workload": batched_line,
        "cpu_baseline": cpu,
        "wall_s": time.perf_counter() - t_start,
    }
    print(json.dumps(line), flush=True)


def pass_scan(args):
    """Horner pass of the kicked-Ising filter at L = 20, 22, 24 with 1, 2 and 4
    vectors per launch, complex64 and complex128: average pass duration (HIP
    events on the launch stream) and algorithmic GB/s (3 * n * d * s bytes
    per pass).  One vector per launch is the single-vector filter; more
    vectors go through apply_filter_many (autotuned tile shapes)."""
    import torch

    from paper_2102_05054_amd import kicked_ising
    from paper_2102_05054_amd._lib import FQ_POLICY_AUTO, FQ_POLICY_PIPE, FQ_POLICY_TILE, lib
    from workloads import config_kicked_ising
    policy = {"auto": FQ_POLICY_AUTO, "tile": FQ_POLICY_TILE, "pipe": FQ_POLICY_PIPE}[args.policy]
    assert lib().fq_set_kernel_policy(policy) == 0
    rows = []
    for L in args.scan_sizes:
        q = config_kicked_ising("ki_L20", W=1.0, L=L)
        with kicked_ising(q.L, q.J, q.h, q.g, q.periodic) as op:
            for dt in ("c64", "c128"):
                for n in (1, 2, 4):
                    if n * (2 ** L) * (16 if dt == "c128" else 8) * 2 > (24 << 30):
                        continue
                    steps = max(50, min(2000, int(2e8 / (n * 2 ** L))))
                    r = filter_roofline(op, L, steps, n, dt)
                    row = {"L": L, "dtype": dt, "vectors": n, "policy": args.policy, "avg_pass_us": r["avg_launch_us"],
                           "us_per_vector_pass": r["avg_launch_us"] / n, "alg_GBs": r["achieved_GBs"],
                           "frac": r["achieved_GBs"] / 8000.0, "steps": steps}
                    rows.append(row)
                    print(json.dumps(row), flush=True)
                    torch.cuda.empty_cache()
    print(json.dumps({"pass_scan": rows}))


def nominal(args):
    """The configurations at their nominal filter orders, reported as they
    end (converged or not): L = 16 complex128, k = 200, nev = 50, ncv = 120,
    phi drawn, one vector per step; L = 20, k = 400, nev = 100, ncv = 220,
    W in {1, 3}, complex64 + FP64 refinement (block 4) and complex128
    (block 2); the brickwork circuit at L = 24, k = 300, nev = 40, ncv = 100,
    complex64 + FP64 (block 4, at most 3 restarts).  Each solve stops after
    --max-restarts restarts; status, converged pairs and the largest FP64
    residual are printed per solve."""
    import torch

    from paper_2102_05054_amd import kicked_ising
    from workloads import CONFIGS, config_kicked_ising
    rows = []

    def run(name, p, nev, ncv, k, dtype, block, phi):
        with kicked_ising(p.L, p.J, p.h, p.g, p.periodic) as op:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, _, res, st, status = op.arnoldi_eigs(nev, phi, k=k, ncv=ncv, tol=1e-10,
                                                     max_restarts=args.max_restarts, filter_dtype=dtype,
                                                     seed=1, want_vectors=False, allow_not_converged=True,
                                                     block=block)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        r = {"case": name, "L": p.L, "k": k, "nev": nev, "ncv": ncv, "dtype": dtype, "block": block,
             "status": int(status), "nconv": st["nconv"], "max_residual": float(res.max()),
             "n_restarts": st["n_restarts"], "n_U_apps": st["n_U_apps"], "time_s": dt}
        rows.append(r)
        print(json.dumps(r), flush=True)

    c2 = CONFIGS["ki_L16"]
    p2 = config_kicked_ising("ki_L16")
    run("ki_L16 nominal", p2, c2["nev"], c2["ncv"], c2["k"], "c128", 1, p2.phi)
    c3 = CONFIGS["ki_L20"]
    for W in c3["W"]:
        p3 = config_kicked_ising("ki_L20", W=W)
        for dtype, block in (("c64", 4), ("c128", 2)):
            run(f"ki_L20 W={W:g} nominal", p3, c3["nev"], c3["ncv"], c3["k"], dtype, block, 0.0)
    # the brickwork circuit at L = 24: three restart cycles at most (each
    # cycle is ~3 s of filter, the first ~10 s), then one FP64 cycle
    from paper_2102_05054_amd import brickwork
    from workloads import brickwork as bw_params
    c5 = CONFIGS["bw_L24"]
    p5 = bw_params(c5["L"], c5["seed"])
    with brickwork(p5.L, p5.gates) as op:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, _, res, st, status = op.arnoldi_eigs(c5["nev"], 0.0, k=c5["k"], ncv=c5["ncv"], tol=c5["tol"],
                                                 max_restarts=min(args.max_restarts, 3), filter_dtype="c64",
                                                 seed=1, want_vectors=False, allow_not_converged=True, block=4)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    r = {"case": "bw_L24 nominal", "L": p5.L, "k": c5["k"], "nev": c5["nev"], "ncv": c5["ncv"], "dtype": "c64",
         "block": 4, "status": int(status), "nconv": st["nconv"], "max_residual": float(res.max()),
         "n_restarts": st["n_restarts"], "n_U_apps": st["n_U_apps"], "time_s": dt}
    rows.append(r)
    print(json.dumps(r), flush=True)
    print(json.dumps({"nominal": rows, "max_restarts": args.max_restarts}))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
