"""Benchmark: HOOI sweeps of sparse Tucker on one MI355X.

One step = one full sweep of the hot path: for every mode the sparse TTMc, the FP64 QRP that
refreshes U_n, then the core and the fit.  The default workload is the recommendation-shaped
order-3 tensor (500,000 x 100,000 x 365, 50M nonzeros with Zipf(1.2) indices on the first two
modes, log-normal values, ranks 10, FP32 TTMc / FP64 QRP, 5 sweeps from the seeded factors).
Inputs are resident in HBM before timing starts.  Prints one JSON line; besides the metric it
carries the roofline of the TTMc kernel, the same sweeps with the BF16-operand TTMc, the time to
reach the FP64 oracle's final fit (stored by tests/golden/make_fullsize_fits.py), the low-rank
10,000^3 workload's sweep, and the oracle timed on the host's cores.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--no-cpu-baseline] [--workload ...]
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
# rocprofv3 FETCH_SIZE / WRITE_SIZE counters of the dominant kernel on the default workload, with
# the source hash of the kernel file they were taken on (traffic is reported only while it matches)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_ttmc3_lds_f32_zipf_500000x100000x365_50M_r10.md")
TTMC_SOURCE = os.path.join(ROOT, "paper_2010_10638_amd", "csrc", "ttmc.hip")
# the FP64 oracle's fit sequences on the full-size workloads (written by a script that calls only
# the oracle and the input generator)
ORACLE_FITS = os.path.join(ROOT, "tests", "golden", "fullsize_fits.json")
FIT_TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}


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


def host_info():
    """CPU model and the host threads this process may use (OMP_NUM_THREADS caps them)."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0))
    omp = int(os.environ.get("OMP_NUM_THREADS") or avail)
    return model, avail, max(1, min(avail, omp))


def cpu_baseline(w):
    """The FP64 oracle on the host, on a bounded sample of the same workload: one TTMc per mode
    on all usable cores (row-partitioned, same arithmetic as the single-threaded oracle), the QRP
    of each mode's Y_(n) (on a row sample for modes above 100,000 rows, scaled by the row count:
    Householder QRP with R_n steps costs rows x K_n x R_n), the core, and one TTMc single-threaded.
    Value: nnz * K_n updates per second of the resulting all-core sweep."""
    import numpy as np
    import oracle
    oracle.build()
    model, avail, threads = host_info()
    N = len(w.dims)
    t_ttmc, t_qrp, qrp_note = [], [], []
    Y = None
    for n in range(N):
        t0 = time.perf_counter()
        Y = oracle.ttmc(w.coords, w.vals, w.dims, w.ranks, n, w.U_init, threads=threads)
        t_ttmc.append(time.perf_counter() - t0)
        rows = Y.shape[0]
        m = rows if rows <= 100_000 else 50_000
        t0 = time.perf_counter()
        oracle.factor(np.ascontiguousarray(Y[:m]), int(w.ranks[n]))
        t_qrp.append((time.perf_counter() - t0) * rows / m)
        qrp_note.append("all rows" if m == rows else f"{m} of {rows} rows, scaled")
    t0 = time.perf_counter()
    oracle.core(Y, w.U_init[N - 1], w.ranks)
    t_core = time.perf_counter() - t0
    # single-threaded TTMc of the last mode
    t0 = time.perf_counter()
    oracle.ttmc(w.coords, w.vals, w.dims, w.ranks, N - 1, w.U_init)
    t_single = time.perf_counter() - t0
    upd = [w.nnz * _K(w.ranks, n) for n in range(N)]
    sweep_s = sum(t_ttmc) + sum(t_qrp) + t_core
    return dict(value=sum(upd) / sweep_s, unit="updates/s", cores=threads, kind="oracle",
                sample=f"one FP64 oracle sweep of the same tensor from the seeded factors: TTMc of every "
                       f"mode on {threads} threads (row-partitioned), QRP per mode ({'; '.join(qrp_note)}), core; "
                       f"plus one single-threaded TTMc of mode {N - 1}",
                cpu_model=model, cpus_visible=avail, sweep_s=sweep_s,
                ttmc_s_per_mode=t_ttmc, qrp_s_per_mode=t_qrp, core_s=t_core,
                single_thread={"mode": N - 1, "ttmc_s": t_single, "ttmc_updates_per_s": upd[N - 1] / t_single})


def _sha256(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic():
    """HBM bytes per TTMc launch from the committed counter summary, or None when the summary is
    missing or was taken on another version of the kernel source."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    sha = traffic = None
    with open(TRAFFIC_PROFILE) as f:
        for line in f:
            if line.startswith("ttmc.hip sha256:"):
                sha = line.split(":", 1)[1].strip()
            elif line.startswith("traffic bytes per launch:"):
                traffic = float(line.split(":", 1)[1].strip())
    if sha is None or traffic is None or sha != _sha256(TTMC_SOURCE):
        return None
    return traffic


def _csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def summarize_trace(d):
    """Markdown table of a rocprofv3 --kernel-trace --stats output directory (run_kernel_stats.csv)."""
    rows = _csv(os.path.join(d, "run_kernel_stats.csv"))
    out = ["| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in rows[:30]:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def _counter_mean(d, counter, name_sub):
    vals = [float(r["Counter_Value"]) for r in _csv(os.path.join(d, "run_counter_collection.csv"))
            if r["Counter_Name"] == counter and name_sub in r["Kernel_Name"]]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def summarize_pmc(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, kernel):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE of `kernel`, calibrated by a 512 MiB device copy."""
    fk, nf = _counter_mean(fetch_dir, "FETCH_SIZE", kernel)
    wk, nw = _counter_mean(write_dir, "WRITE_SIZE", kernel)
    cf, _ = _counter_mean(copy_fetch_dir, "FETCH_SIZE", "copyBuffer")
    cw, _ = _counter_mean(copy_write_dir, "WRITE_SIZE", "copyBuffer")
    copy_kib = (128 << 20) * 4 / 1024
    ff, fw = copy_kib / cf, copy_kib / cw
    traffic = (fk * ff + wk * fw) * 1024
    return "\n".join([
        f"FETCH_SIZE per dispatch (KiB): {fk:.1f} over {nf} dispatches",
        f"WRITE_SIZE per dispatch (KiB): {wk:.1f} over {nw} dispatches",
        f"copy calibration: 524288 KiB read and written per copy; FETCH_SIZE reads {cf:.1f} KiB "
        f"(factor {ff:.3f}), WRITE_SIZE reads {cw:.1f} KiB (factor {fw:.3f})",
        f"traffic bytes per launch: {traffic:.0f}",
        f"ttmc.hip sha256: {_sha256(TTMC_SOURCE)}",
    ])


def oracle_fits(name):
    """The oracle's stored fit sequence for a workload name (its TTMc-type suffix dropped)."""
    if not os.path.exists(ORACLE_FITS):
        return None
    base = name.rsplit("_", 1)[0] if name.endswith(("_f32", "_bf16", "_f64")) else name
    with open(ORACLE_FITS) as f:
        data = json.load(f)["workloads"]
    for key in (name, base):
        if key in data:
            return data[key]["fits"]
    return None


def ttmc_kernel_name(w):
    if len(w.dims) == 3 and max(w.ranks) <= 16:
        return {"f64": "k_ttmc3_mfma<double,double>", "f32": "k_ttmc3_lds<float, false>",
                "bf16": "k_ttmc3_bf"}[w.dtype]
    if len(w.dims) >= 4:
        return "k_ttmc_fiber"
    return "k_ttmc_generic"


def roofline(w, N, flops, bytes_, t_launch, default):
    """Roofline object of the dominant kernel (the TTMc, one launch per mode; figures averaged over
    the modes).  Intensity = 2 K_n flops per nonzero over the stream bytes: the recommendation-shaped
    tensor (K_n = 100, about 14 flop/B) sits below the FP32 ridge of 19.7 flop/B and is reported
    against HBM; the low-rank tensor (K_n = 256, about 39 flop/B) against FP32 MFMA; the FP64 200^3
    case against FP64 MFMA (it is latency-bound)."""
    gbs = bytes_ / t_launch / 1e9
    tflops = flops / t_launch / 1e12
    common = {"kernel": ttmc_kernel_name(w), "flops_per_launch": flops, "alg_bytes_per_launch": bytes_,
              "avg_launch_ms": t_launch * 1e3, "hbm_gbs_alg": gbs, "hbm_frac_alg": gbs / PEAK_HBM_GBS,
              "tflops": tflops}
    if w.dtype == "f64":
        return {"bound": "mfma", "achieved": tflops, "peak": 78.6, "unit": "TFLOP/s", "frac": tflops / 78.6,
                "traffic": None, **common}
    if flops / bytes_ > PEAK_FP32_MFMA_TFLOPS / (PEAK_HBM_GBS / 1e3) and N == 3:
        return {"bound": "mfma", "achieved": tflops, "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / PEAK_FP32_MFMA_TFLOPS, "traffic": None, **common}
    return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "traffic": measured_traffic() if default else None, **common}


def compare_precisions(args, w, tk, torch):
    """The same sweeps (same initial factors) with each TTMc precision; the FP64 path is the
    reference for the fit error.  Sweep times are wall-clock per sweep (synchronised), median over
    the timed sweeps after one warm-up sweep."""
    import statistics
    coords = torch.from_numpy(w.coords).cuda()
    vals = torch.from_numpy(w.vals).cuda()
    res = {}
    for dt in ("f64", "f32", "bf16"):
        ctx = tk.tucker_init(coords, vals, w.dims, w.ranks, dtype=dt)
        U = [torch.from_numpy(u).cuda() for u in w.U_init]
        G = torch.empty(w.ranks, dtype=torch.float64, device="cuda")
        fit = torch.empty(1, dtype=torch.float64, device="cuda")
        fits, times, all_times = [], [], []
        for k in range(args.steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tk.hooi_sweep(ctx, U, G, fit)
            torch.cuda.synchronize()
            all_times.append(time.perf_counter() - t0)
            if k > 0:
                times.append(all_times[-1])
            fits.append(float(fit.item()))
        res[dt] = {"sweep_ms_median": statistics.median(times) * 1e3, "fits": fits, "_times": all_times}
        del ctx
    ref = res["f64"]["fits"]
    target = ref[-1]
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}
    for dt in ("f64", "f32", "bf16"):
        r = res[dt]
        if dt != "f64":
            r["fit_rel_err_vs_f64"] = max(abs(a - b) / abs(b) for a, b in zip(r["fits"], ref) if b != 0)
        # time to reach the FP64 path's final fit within this precision's tolerance (sweeps run
        # back to back, warm-up sweep included)
        hit = next((k for k, f in enumerate(r["fits"]) if target != 0 and abs(f - target) <= tol[dt] * abs(target)),
                   None)
        r["sweeps_to_final_fit"] = None if hit is None else hit + 1
        r["ms_to_final_fit"] = None if hit is None else sum(r["_times"][:hit + 1]) * 1e3
        del r["_times"]
    out = {"workload": w.name, "dims": w.dims, "ranks": w.ranks, "nnz": int(w.nnz), "sweeps": args.steps + 1,
           "qrp": "f64", "results": res}
    print(json.dumps(out), flush=True)


def run_completion(args, w, tk, torch):
    """One step = the completion loss and its gradients (adjoint TTMc over every mode) and one
    Adam update of the core and the factors, on the 30M-entry workload."""
    coords = torch.from_numpy(w.coords).cuda()
    vals = torch.from_numpy(w.vals).cuda()
    ctx = tk.tucker_init(coords, vals, w.dims, w.ranks, dtype="f32")
    del coords, vals
    nnz = tk.tucker_get_info(ctx)["nnz"]
    G = torch.from_numpy(w.G_init).float().cuda().requires_grad_()
    U = [torch.from_numpy(u).float().cuda().requires_grad_() for u in w.U_init]
    opt = torch.optim.Adam([G] + U, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)

    def step():
        opt.zero_grad()
        loss = tk.completion_loss(ctx, G, U)
        loss.backward()
        opt.step()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    N = len(w.dims)
    upd = sum(nnz * _K(w.ranks, n) for n in range(N))
    dt = (t1 - t0) / args.steps
    out = {"metric": "adjoint TTMc nnz*prod(R) updates/s over whole completion steps (loss, gradients, Adam)",
           "value": upd / dt, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "dims": w.dims, "ranks": w.ranks, "nnz": nnz, "optimizer": "adam",
                      "parallelism": "single-gpu"},
           "loss": float(loss.item())}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_completion(w, upd)
    print(json.dumps(out), flush=True)


def cpu_baseline_completion(w, upd_per_step, sample=100000):
    """The FP64 oracle's completion loss and gradients (every core entry per observed entry, one
    host thread) on the first `sample` observed entries, scaled to all entries, plus one Adam
    update of the parameters in numpy: the time of one completion step on the host."""
    import numpy as np
    import oracle
    oracle.build()
    model, avail, _ = host_info()
    c = np.ascontiguousarray(w.coords[:, :sample])
    v = np.ascontiguousarray(w.vals[:sample])
    t0 = time.perf_counter()
    loss, gG, gU = oracle.completion(w.G_init, w.U_init, c, v, w.dims)
    t_grad = (time.perf_counter() - t0) * w.nnz / sample
    params = [w.G_init] + list(w.U_init)
    grads = [gG] + gU
    m = [np.zeros_like(x) for x in params]
    s2 = [np.zeros_like(x) for x in params]
    t0 = time.perf_counter()
    for x, g, mm, ss in zip(params, grads, m, s2):
        mm[...] = 0.9 * mm + 0.1 * g
        ss[...] = 0.999 * ss + 0.001 * g * g
        _ = x - 1e-2 * (mm / 0.1) / (np.sqrt(ss / 0.001) + 1e-8)
    t_adam = time.perf_counter() - t0
    step_s = t_grad + t_adam
    return dict(value=upd_per_step / step_s, unit="updates/s", cores=1, kind="oracle",
                sample=f"FP64 oracle loss and gradients on the first {sample} of {w.nnz} observed entries, "
                       f"scaled to all of them ({t_grad:.1f} s), plus one numpy Adam update ({t_adam * 1e3:.1f} ms)",
                cpu_model=model, cpus_visible=avail, step_s=step_s)


def _K(ranks, n):
    k = 1
    for t, r in enumerate(ranks):
        if t != n:
            k *= r
    return k


def run_sweeps(args, w, tk, torch, profile=True):
    """Layout build, warm-up, then args.steps timed HOOI sweeps (and the same number again with
    region events for the breakdown).  Returns the measurements and the context."""
    coords = torch.from_numpy(w.coords).cuda()
    vals = torch.from_numpy(w.vals).cuda()
    ctx = tk.tucker_init(coords, vals, w.dims, w.ranks, dtype=w.dtype, svd=args.factor == "svd",
                         memo=not args.no_memo)
    del coords, vals
    info = tk.tucker_get_info(ctx)
    U = [torch.from_numpy(u).cuda() for u in w.U_init]
    G = torch.empty(w.ranks, dtype=torch.float64, device="cuda")
    fit = torch.empty(1, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        tk.hooi_sweep(ctx, U, G, fit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tk.hooi_sweep(ctx, U, G, fit)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = {"ctx": ctx, "info": info, "sweep_s": (t1 - t0) / args.steps, "fit": float(fit.item())}
    if profile:
        # the same number of sweeps again with HIP events on the sweep's stream around every
        # region and around each main TTMc kernel (breakdown and roofline; not the timed value)
        tk.tucker_profile(ctx, args.steps)
        for _ in range(args.steps):
            tk.hooi_sweep(ctx, U, G, fit)
        out["prof"] = tk.tucker_profile_read(ctx)
        tk.tucker_profile(ctx, 0)
    return out


def fits_from_start(w, ctx, tk, torch):
    """w.sweeps synchronised sweeps from the seeded factors: per-sweep wall time and fit, and the
    time to reach the FP64 oracle's final fit (stored) within the TTMc type's tolerance."""
    U = [torch.from_numpy(u).cuda() for u in w.U_init]
    G = torch.empty(w.ranks, dtype=torch.float64, device="cuda")
    fit = torch.empty(1, dtype=torch.float64, device="cuda")
    fits, times = [], []
    for _ in range(w.sweeps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tk.hooi_sweep(ctx, U, G, fit)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        fits.append(float(fit.item()))
    res = {"sweeps": w.sweeps, "fits": fits, "sweep_ms": [t * 1e3 for t in times]}
    ref = oracle_fits(w.name)
    if ref is not None and len(ref) == len(fits):
        tol = FIT_TOL[w.dtype]
        target = ref[-1]
        res["oracle_fits"] = ref
        res["fit_rel_err_vs_oracle"] = [abs(a - b) / abs(b) for a, b in zip(fits, ref)]
        res["tolerance"] = tol
        hit = next((k for k, f in enumerate(fits) if abs(f - target) <= tol * abs(target)), None)
        res["sweeps_to_oracle_final_fit"] = None if hit is None else hit + 1
        res["ms_to_oracle_final_fit"] = None if hit is None else sum(times[:hit + 1]) * 1e3
    return res


def ttmc_roofline(w, r):
    """Algorithmic bytes and flops per TTMc launch (averaged over the modes) and the main kernel's
    average duration from the region events."""
    ctx, info, prof = r["ctx"], r["info"], r["prof"]
    N = len(w.dims)
    nnz = info["nnz"]
    val_bytes = {"f64": 8, "f32": 4, "bf16": 2}[w.dtype]
    y_bytes = 8 if w.dtype == "f64" else 4
    kern_s = sum(prof["ttmc_kernel_ms"]) / 1e3 / prof["sweeps"]
    flops = sum(2 * nnz * _K(w.ranks, n) for n in range(N)) / N
    bytes_ = sum(alg_bytes_ttmc(ctx, info, nnz, n, val_bytes, val_bytes, y_bytes) for n in range(N)) / N
    return flops, bytes_, kern_s / N


def breakdown(r):
    prof = r["prof"]
    ns = prof["sweeps"]
    return {"ttmc": sum(prof["ttmc_ms"]) / ns, "qrp": sum(prof["qrp_ms"]) / ns, "core_fit": prof["core_ms"] / ns,
            "ttmc_per_mode": [x / ns for x in prof["ttmc_ms"]],
            "ttmc_kernel_per_mode": [x / ns for x in prof["ttmc_kernel_ms"]],
            "qrp_per_mode": [x / ns for x in prof["qrp_ms"]]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the workload's own sweeps (no BF16 rerun, no low-rank line, no fits from the start)")
    ap.add_argument("--small", action="store_true", help="small tensor (for profiling dry runs)")
    ap.add_argument("--workload", default="skewed-f32",
                    choices=["skewed-f32", "skewed-bf16", "lowrank", "hooi200", "order4-f32", "order4-bf16",
                             "image", "completion"],
                    help="skewed-* (default FP32): 500,000 x 100,000 x 365, 50M Zipf nnz, R 10; lowrank: "
                    "10,000^3, 10M nnz, R 16, FP32 TTMc; hooi200: 200^3, 20,000 nnz, R 8, FP64; order4-*: "
                    "50,000 x 50,000 x 5,000 x 100, 20M nnz, R 8; image: order 2, 130 x 150 image-shaped, R 30, "
                    "FP64; completion: 100,000 x 100,000 x 1,000, "
                    "30M entries, R 16, one Adam step of the completion loss per step")
    ap.add_argument("--no-memo", action="store_true",
                    help="order >= 4: form the last two modes' TTMc from the nonzeros (no shared fiber sums)")
    ap.add_argument("--factor", default="qrp", choices=["qrp", "svd"],
                    help="factor update of the HOOI sweeps: qrp (Alg. 2, default) or svd (Alg. 1, the "
                    "leading left singular vectors; not the bench line)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (calibrates FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--compare-precisions", action="store_true",
                    help="run the workload's HOOI sweeps with FP64, FP32 and BF16 TTMc (FP64 QRP in all) "
                    "and print per-precision sweep times, fits and the fit error against the FP64 path")
    ap.add_argument("--summarize-trace", metavar="DIR", help="print a markdown summary of a rocprofv3 "
                    "--kernel-trace --stats output directory and exit")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="print the calibrated per-launch HBM traffic of the TTMc kernel from four "
                    "rocprofv3 --pmc output directories and exit")
    args = ap.parse_args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.summarize_pmc:
        print(summarize_pmc(*args.summarize_pmc, kernel="k_ttmc3_lds<float, false>"))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the TTMc would "
              "shard by output rows, the QRP by an all-reduce of the Gram matrix).", file=sys.stderr)
        sys.exit(2)

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
    elif args.workload == "lowrank":
        w = synth.lowrank_f32()
    elif args.workload == "hooi200":
        w = synth.hooi_small_f64()
    elif args.workload.startswith("skewed"):
        w = synth.skewed(dtype=args.workload.split("-")[1])
    elif args.workload.startswith("order4"):
        w = synth.order4(dtype=args.workload.split("-")[1])
    elif args.workload == "image":
        w = synth.image_like()
    else:
        w = synth.completion()
    print(f"# generated {w.name} in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.set_device(0)
    if args.workload == "completion" and not args.small:
        return run_completion(args, w, tk, torch)
    if args.compare_precisions:
        return compare_precisions(args, w, tk, torch)

    r = run_sweeps(args, w, tk, torch)
    print(f"# timed {args.steps} sweeps: {r['sweep_s'] * 1e3:.3f} ms per sweep", file=sys.stderr, flush=True)
    N = len(w.dims)
    nnz = r["info"]["nnz"]
    upd_per_sweep = sum(nnz * _K(w.ranks, n) for n in range(N))
    flops, bytes_, t_launch = ttmc_roofline(w, r)
    default = args.workload == "skewed-f32" and not args.small and args.factor == "qrp"
    bd = breakdown(r)
    out = {
        "metric": "TTMc nnz*prod(R) updates/s over whole HOOI sweeps (TTMc + FP64 %s + core)" % args.factor.upper(),
        "value": upd_per_sweep / r["sweep_s"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["sweep_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "dims": w.dims, "ranks": w.ranks, "nnz": nnz,
                   "ttmc": w.dtype, "qrp": "f64", "factor_update": args.factor, "parallelism": "single-gpu"},
        "roofline": roofline(w, N, flops, bytes_, t_launch, default),
        "breakdown_ms_per_sweep": bd,
        "ttmc_updates_per_s": upd_per_sweep / (bd["ttmc"] / 1e3),
        "fit": r["fit"],
    }
    if not args.no_extras and not args.small:
        out["from_start"] = fits_from_start(w, r["ctx"], tk, torch)
        if args.workload.startswith("skewed") and args.factor == "qrp":
            # the same tensor and sweeps with the other TTMc type (BF16 operands / FP32 accumulation)
            other = "bf16" if w.dtype == "f32" else "f32"
            w2 = synth.Workload(w.name.rsplit("_", 1)[0] + "_" + other, w.dims, w.ranks, w.coords, w.vals,
                                w.U_init, sweeps=w.sweeps, dtype=other)
            del r["ctx"]
            r2 = run_sweeps(args, w2, tk, torch)
            f2, b2, t2 = ttmc_roofline(w2, r2)
            out[other] = {"ms_per_step": r2["sweep_s"] * 1e3, "value": upd_per_sweep / r2["sweep_s"],
                          "breakdown_ms_per_sweep": breakdown(r2), "hbm_frac_alg": b2 / t2 / 1e9 / PEAK_HBM_GBS,
                          "from_start": fits_from_start(w2, r2["ctx"], tk, torch)}
            del r2
        if default:
            # the low-rank 10,000^3 workload (10M nonzeros, ranks 16, FP32 TTMc) as a second line
            w3 = synth.lowrank_f32()
            r3 = run_sweeps(args, w3, tk, torch)
            f3, b3, t3 = ttmc_roofline(w3, r3)
            upd3 = sum(r3["info"]["nnz"] * _K(w3.ranks, n) for n in range(3))
            out["lowrank_f32"] = {"workload": w3.name, "ms_per_step": r3["sweep_s"] * 1e3,
                                  "value": upd3 / r3["sweep_s"], "ttmc_kernel_us": t3 * 1e6,
                                  "mfma_frac": f3 / t3 / 1e12 / PEAK_FP32_MFMA_TFLOPS,
                                  "hbm_frac_alg": b3 / t3 / 1e9 / PEAK_HBM_GBS,
                                  "from_start": fits_from_start(w3, r3["ctx"], tk, torch)}
            del r3
    if not args.no_cpu_baseline and default:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
