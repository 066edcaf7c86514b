#!/usr/bin/env python3
"""Benchmark: HEOM Liouvillian apply (matvec) GB/s on one MI355X.

Workload: two-orbital Anderson model, d = 16, 48 fermionic exponents,
tier 4 -> 213,053 ADOs (1.745 GB per FP64 ADO vector).  A step is one
apply y = M x of the full ADO vector.  value = algorithmic bytes per apply
(read x once, write y once, plus the neighbour/decay tables) / wall time
per step; roofline.achieved uses the average kernel time measured with HIP
events on the launch stream.  The oracle (assembled CSR, row-sampled at the
same tier) is timed on the host cores beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic per apply measured with rocprofv3 FETCH_SIZE / WRITE_SIZE,
# calibrated on a plain device copy (profiles/apply_wave_fp64_two_orbital_tier4.md).
# Valid only for the apply source it was measured on: reported as null otherwise.
MEASURED_TRAFFIC = {
    ("fp64", "untiled"): {"apply_sha256_prefix": "b4282ebb32f23ee1", "bytes": 7_589_248_000},
}


def _apply_source_sha():
    import hashlib
    with open(os.path.join(ROOT, "paper_2306_07522_amd", "csrc", "apply.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    p.add_argument("--tiled", type=int, default=-1, help="-1: untiled apply; 0: default chunks; k: k chunks")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--calib", action="store_true",
                   help="also run one plain device copy of the ADO vector (HBM counter calibration)")
    return p.parse_args()


def algorithmic_bytes(h, w, n_rhs=1):
    """Compulsory HBM bytes of one apply: x read once, y written once, plus
    row pointers (8 B/ADO), edges (8 B/edge) and decay (w B/ADO)."""
    N, d = h.N, h.d
    return 2 * N * d * d * w * n_rhs + 8 * (N + 1) + 8 * h.info.n_edges + w * N


def gpu_apply_bench(args):
    import torch
    from paper_2306_07522_amd import api, workloads as wl

    cfg = wl.two_orbital_anderson()
    h = api.Hierarchy(cfg["H"], cfg["baths"], cfg["m_max"], cfg["n_max"], parity_op=cfg["parity_op"])
    dtype = torch.complex128 if args.precision == "fp64" else torch.complex64
    w = 16 if args.precision == "fp64" else 8
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((h.N, h.d, h.d), dtype=dtype, device="cuda", generator=g)
    y = torch.empty_like(x)
    tiled = None if args.tiled < 0 else args.tiled
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        h.apply(x, y, tiled=tiled, stream=stream)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        evs[s][0].record(stream)
        h.apply(x, y, tiled=tiled, stream=stream)
        evs[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if args.calib:
        z = torch.empty_like(x)
        z.copy_(x)
        torch.cuda.synchronize()
        del z
    kern_ms = sorted(a.elapsed_time(b) for a, b in evs)
    avg_ms = sum(kern_ms) / len(kern_ms)
    nbytes = algorithmic_bytes(h, w)
    return dict(h=h, cfg=cfg, wall=wall, avg_kernel_ms=avg_ms, median_kernel_ms=kern_ms[len(kern_ms) // 2],
                bytes=nbytes)


def cpu_baseline(seconds):
    """Oracle apply on the host: the assembled HEOMLS restricted to a seeded
    sample of block rows of the same tier-4 hierarchy, multiplied with the
    C OpenMP CSR SpMV on every host core; throughput is scaled to GB/s with
    the same per-ADO algorithmic bytes as the GPU."""
    import numpy as np
    from oracle import exponents as ox, spmv_c
    from oracle.liouvillian import OracleHEOM
    from paper_2306_07522_amd import workloads as wl

    cfg = wl.two_orbital_anderson()
    om = OracleHEOM(cfg["H"], ox.exponent_records(cfg["baths"]), cfg["m_max"], cfg["n_max"])
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(om.N, 1500, replace=False))
    A = om.assemble(rows=rows).tocsr()
    x = rng.standard_normal(A.shape[1]) + 1j * rng.standard_normal(A.shape[1])
    spmv_c.spmv(A, x)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        spmv_c.spmv(A, x)
        n += 1
    dt = (time.perf_counter() - t0) / n
    d = om.d
    rows_per_s = len(rows) / dt
    gbs = rows_per_s * (2 * d * d * 16) / 1e9
    return dict(value=gbs, unit="GB/s", cores=spmv_c.threads(), kind="oracle",
                sample=f"{len(rows)} seeded block rows of the 213,053-ADO tier-4 HEOMLS (CSR, {A.nnz} nonzeros), "
                       f"C OpenMP SpMV, {n} reps in {seconds:.0f} s; GB/s = rows/s x 2 d^2 x 16 B")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    r = gpu_apply_bench(args)
    h = r["h"]
    ms_step = r["wall"] * 1e3 / args.steps
    value = r["bytes"] / (ms_step * 1e-3) / 1e9
    achieved = r["bytes"] / (r["avg_kernel_ms"] * 1e-3) / 1e9
    rec = MEASURED_TRAFFIC.get((args.precision, "untiled" if args.tiled < 0 else "tiled"))
    traffic = rec["bytes"] if rec and rec["apply_sha256_prefix"] == _apply_source_sha() else None
    out = {
        "metric": "HEOM matvec GB/s; solve s @1e-8 resid, plain vs NN-preconditioned",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if args.precision == "fp64" else "c64",
        "data": "synthetic",
        "config": {"workload": "two-orbital Anderson HEOMLS apply, d=16, 48 fermionic exponents, tier 4",
                   "n_ado": h.N, "d": h.d, "n_edges": h.info.n_edges, "precision": args.precision,
                   "apply": "untiled" if args.tiled < 0 else f"tiled({args.tiled})"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "kernel_ms": {"avg": round(r["avg_kernel_ms"], 4), "median": round(r["median_kernel_ms"], 4)},
        "bytes_per_step": r["bytes"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
