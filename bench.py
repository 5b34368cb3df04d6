"""Benchmark: HOOI sweeps of sparse Tucker on one MI355X.

One step = one full sweep of the hot path: for every mode the sparse TTMc, the FP64 QRP that
refreshes U_n, then the core and the fit, on the order-3 low-rank workload
(10,000^3, 10M nonzeros, ranks 16, FP32 TTMc / FP64 QRP).  Inputs are resident in HBM before
timing starts.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3


def alg_bytes_ttmc(ctx, info, nnz, mode, val_bytes, fac_bytes, y_bytes):
    """Compulsory HBM bytes of one TTMc launch: the mode-sorted stream (N-1 int32 indices and the
    value per nonzero), row ids and pointers, the chunk table, each other factor read once, and
    Y_(n) written once."""
    N = ctx.order
    S = info["rows"][mode]
    C = info["chunks"][mode]
    b = nnz * ((N - 1) * 4 + val_bytes)
    b += S * 4 + (S + 1) * 4 + C * 3 * 4
    b += sum(ctx.dims[t] * ctx.ranks[t] * fac_bytes for t in range(N) if t != mode)
    b += ctx.dims[mode] * ctx.K(mode) * y_bytes
    return b


def cpu_baseline(w, budget_s=10.0):
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    sweeps = 0
    U = w.U_init
    while sweeps == 0 or (time.perf_counter() - t0 < budget_s and sweeps < 3):
        U, _, _, _ = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, U, 1)
        sweeps += 1
    dt = time.perf_counter() - t0
    upd = sum(w.nnz * _K(w.ranks, n) for n in range(len(w.dims))) * sweeps
    return dict(value=upd / dt, unit="updates/s", cores=1, kind="oracle",
                sample=f"{sweeps} full HOOI sweep(s) of the same tensor (all modes: TTMc + QRP + core), "
                       f"single-threaded FP64 C oracle, {dt:.1f} s")


def _K(ranks, n):
    k = 1
    for t, r in enumerate(ranks):
        if t != n:
            k *= r
    return k


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true", help="small tensor (for profiling dry runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (calibrates FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the TTMc and QRP would shard).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 128 << 20                      # 128 Mi float32 = 512 MiB read + 512 MiB written per copy
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": True, "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                          "copies": 3}), flush=True)
        return

    import paper_2010_10638_amd as tk
    import synth

    t_gen = time.perf_counter()
    if args.small:
        w = synth.lowrank_f32(dims=(2000, 2000, 2000), nnz=1_000_000)
    else:
        w = synth.lowrank_f32()
    print(f"# generated {w.name} in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    coords = torch.from_numpy(w.coords).cuda()
    vals = torch.from_numpy(w.vals).cuda()
    ctx = tk.tucker_init(coords, vals, w.dims, w.ranks, dtype=w.dtype)
    del coords, vals
    info = tk.tucker_get_info(ctx)
    U = [torch.from_numpy(u).cuda() for u in w.U_init]
    G = torch.empty(w.ranks, dtype=torch.float64, device="cuda")
    fit = torch.empty(1, dtype=torch.float64, device="cuda")

    for _ in range(args.warmup):
        tk.hooi_sweep(ctx, U, G, fit)
    torch.cuda.synchronize()
    tk.tucker_profile(ctx, args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tk.hooi_sweep(ctx, U, G, fit)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = tk.tucker_profile_read(ctx)
    tk.tucker_profile(ctx, 0)
    print(f"# timed {args.steps} sweeps in {t1 - t0:.3f} s", file=sys.stderr, flush=True)

    N = len(w.dims)
    nnz = info["nnz"]
    upd_per_sweep = sum(nnz * _K(w.ranks, n) for n in range(N))
    sweep_s = (t1 - t0) / args.steps
    value = upd_per_sweep / sweep_s

    # dominant kernel: the TTMc (one launch per mode per sweep)
    val_bytes = {"f64": 8, "f32": 4, "bf16": 2}[w.dtype]
    fac_bytes = val_bytes
    y_bytes = 8 if w.dtype == "f64" else 4
    ttmc_s = sum(prof["ttmc_ms"]) / 1e3 / prof["sweeps"]          # per sweep, all modes
    launches = N
    flops = sum(2 * nnz * _K(w.ranks, n) for n in range(N)) / launches
    bytes_ = sum(alg_bytes_ttmc(ctx, info, nnz, n, val_bytes, fac_bytes, y_bytes) for n in range(N)) / launches
    t_launch = ttmc_s / launches
    tflops = flops / t_launch / 1e12
    gbs = bytes_ / t_launch / 1e9
    qrp_s = sum(prof["qrp_ms"]) / 1e3 / prof["sweeps"]
    core_s = prof["core_ms"] / 1e3 / prof["sweeps"]

    out = {
        "metric": "TTMc nnz*prod(R) updates/s over whole HOOI sweeps (TTMc + FP64 QRP + core)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sweep_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "dims": w.dims, "ranks": w.ranks, "nnz": nnz,
                   "ttmc": w.dtype, "qrp": "f64", "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / PEAK_FP32_MFMA_TFLOPS, "traffic": None,
                     "kernel": "k_ttmc3_mfma<float,float>",
                     "flops_per_launch": flops, "alg_bytes_per_launch": bytes_,
                     "avg_launch_ms": t_launch * 1e3,
                     "hbm_gbs_alg": gbs, "hbm_frac_alg": gbs / PEAK_HBM_GBS},
        "breakdown_ms_per_sweep": {"ttmc": ttmc_s * 1e3, "qrp": qrp_s * 1e3, "core_fit": core_s * 1e3,
                                   "ttmc_per_mode": [x / prof["sweeps"] for x in prof["ttmc_ms"]],
                                   "qrp_per_mode": [x / prof["sweeps"] for x in prof["qrp_ms"]]},
        "ttmc_updates_per_s": upd_per_sweep / ttmc_s,
        "fit": float(fit.item()),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        out["cpu_baseline"]["host"] = platform.processor() or platform.machine()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
