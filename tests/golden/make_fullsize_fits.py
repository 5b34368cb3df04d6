"""Writes fullsize_fits.json: the FP64 oracle's HOOI fit sequence (Alg. 2 sweeps from the seeded
initial factors) and pivot lists on the full-size synthetic workloads.

Calls only synth (seeded inputs) and oracle (the FP64 reference).  The TTMc runs row-partitioned
on the host's cores (bit-identical to the single-threaded oracle).  Run from the repository root:

    python tests/golden/make_fullsize_fits.py [workload names...]

With names, only those workloads are recomputed and the others kept from the existing file.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

WORKLOADS = {
    "hooi_200cube_r8_f64": lambda: synth.hooi_small_f64(),
    "lowrank_10000x10000x10000_nnz10000000_r16": lambda: synth.lowrank_f32(),
    "zipf_500000x100000x365_nnz50000000_r10": lambda: synth.skewed(dtype="f32"),
    "order4_50000x50000x5000x100_nnz20000000_r8": lambda: synth.order4(dtype="f32"),
    "image_130x150_r30_f64": lambda: synth.image_like(),
}


def main():
    threads = len(os.sched_getaffinity(0))
    path = os.path.join(HERE, "fullsize_fits.json")
    out = {"generator": "tests/golden/make_fullsize_fits.py", "threads": threads, "workloads": {}}
    names = sys.argv[1:] or list(WORKLOADS)
    if sys.argv[1:] and os.path.exists(path):
        with open(path) as f:
            out["workloads"] = json.load(f)["workloads"]
    for name in names:
        make = WORKLOADS[name]
        t0 = time.time()
        w = make()
        U, G, fits, pivs = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, w.U_init, w.sweeps, threads=threads)
        out["workloads"][name] = {
            "dims": list(map(int, w.dims)), "ranks": list(map(int, w.ranks)), "nnz": int(w.nnz),
            "sweeps": int(w.sweeps), "fits": [float(f) for f in fits],
            "pivots": [[[int(p) for p in pivs[s, n, :w.ranks[n]]] for n in range(len(w.dims))]
                       for s in range(w.sweeps)],
        }
        print(f"{name}: {w.sweeps} sweeps in {time.time() - t0:.1f} s, fits {list(fits)}", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
