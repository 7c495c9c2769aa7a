"""Throughput of the deconvolution iteration on one MI355X.

A step is one full iteration (Steps 1-3 of Sec. 3.1: forward transform, residual and lambda
search, both solves, inverse transforms, guided filter) over the 4096 x 4096 workload with
inputs resident in HBM.  Prints one JSON line (see the repository's bench contract).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mpixel-iters/s fwd & fwd+bwd at 4096² and batched mixed sizes; HBM GB/s"
# Algorithmic HBM bytes of each pass per launch, as multiples of P (pixels) and Q (half-spectrum
# bins, M * (N/2 + 1)); a lambda round reads q and |H|^2 once.
ALG_BYTES = {
    "row_fwd": (4, 8),          # read u_E (4P), write the row half spectra (8Q)
    "col_fwd_resid": (0, 36),   # read spectra, H, Y (24Q); write U_E (8Q) and q (4Q)
    "lambda_sweeps": (0, 8),    # per evaluation round: read q and |H|^2
    "col_inv_solve": (0, 36),   # read U_E, conj(H)Y (16Q), |H|^2 (4Q); write two spectra (16Q)
    "row_inv": (8, 16),         # read two spectra (16Q); write u_I, u_p (8P)
    "guided_filter": (12, 0),   # read u_I, u_p (8P); write u (4P)
}
KERNEL_SYMBOL = {
    "row_fwd": "k_row_fwd", "col_fwd_resid": "k_col_fwd_resid", "lambda_sweeps": "k_lam_sweep",
    "col_inv_solve": "k_col_inv", "row_inv": "k_row_inv", "guided_filter": "k_guided_filter",
}


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1609_01839_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(case, seconds_hint: float = 20.0) -> dict:
    """The FP64 oracle, as is, on a bounded sample: iterations of the same 4096^2 problem."""
    import numpy as np

    import oracle
    y = case.y.astype(np.float64)
    h = case.h.astype(np.float32).astype(np.float64)
    S = oracle.setup(y, h, case.sigma2)
    uE = np.zeros_like(y)
    t0 = time.perf_counter()
    n = 0
    while True:
        r = oracle.step(S, uE, case.w, float(np.float32(case.eps)))
        uE = r.u
        n += 1
        if time.perf_counter() - t0 > seconds_hint or n >= 3:
            break
    dt = time.perf_counter() - t0
    P = y.size
    return {"value": round(P * n / dt / 1e6, 4), "unit": "Mpixel-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} oracle iteration(s) of the same {case.shape[0]}x{case.shape[1]} problem from u_E = 0, "
                      f"{dt:.1f} s, numpy float64, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=4096, help="image side (default: the 4096^2 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the deconvolution of one frame runs on a single device "
              "(multi-GPU sharding is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1609_01839_amd as gfd
    import synth

    dev = torch.device("cuda:0")
    size = (args.size, args.size)
    case = synth.make_case(5, size=None if args.size == 4096 else size)
    M, N = case.shape
    P, Q = M * N, M * (N // 2 + 1)
    y = torch.from_numpy(case.y).to(dev)
    h = torch.from_numpy(case.h.astype(np.float32)).to(dev)
    g = gfd.GFDeconv(y, h, case.sigma2, case.w, case.eps)
    stream = torch.cuda.current_stream(dev)
    out = torch.empty((M, N), device=dev, dtype=torch.float32)
    lam = torch.empty((1,), device=dev, dtype=torch.float32)

    for _ in range(args.warmup):
        g.iterate(1, out, lam)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        g.iterate(1, out, lam)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    value = P * args.steps / (ms * 1e-3) / 1e6

    # per-pass device time from HIP events on the library's stream (eager launches)
    stages = g.profile(args.profile_iters)
    per_iter = {k: v / args.profile_iters for k, v in stages.items()}
    nsweep_launch = 6
    alg = {k: (a * P + b * Q) for k, (a, b) in ALG_BYTES.items()}
    dom = max((k for k in per_iter if k != "lambda_sweeps"), key=lambda k: per_iter[k])
    achieved = alg[dom] / (per_iter[dom] * 1e-3) / 1e9
    traffic = None
    pmc_path = os.path.join(ROOT, "profiles", f"pmc_{M}x{N}.json")
    if os.path.exists(pmc_path):
        pmc = json.load(open(pmc_path))
        if pmc.get("source_hash") == source_hash() and dom in pmc.get("bytes_per_launch", {}):
            traffic = pmc["bytes_per_launch"][dom]
    total_alg = sum(alg[k] for k in alg if k != "lambda_sweeps")
    roofline = {"bound": "hbm", "kernel": KERNEL_SYMBOL[dom], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": alg[dom], "avg_launch_us": round(per_iter[dom] * 1e3, 2)}

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{M}x{N} piecewise-constant synthetic image, Gaussian PSF std 2.5 on 31x31, "
                               f"sigma^2=4, w=17, eps=650.25, forward iteration (one step = one iteration)",
                   "M": M, "N": N, "iters_per_step": 1, "hip_graph": True},
        "roofline": roofline,
        "iteration": {"alg_bytes_per_px": round((total_alg + 8 * Q) / P, 2),
                      "alg_frac_of_hbm_roofline": round((total_alg / P) * P / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "stage_us": {k: round(v * 1e3, 2) for k, v in per_iter.items()},
                      "wall_s": round(wall, 4)},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case)
    g.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
