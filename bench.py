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
    "row_fwd": "k_row_fwd_r16<4096>", "col_fwd_resid": "k_col_fwd_r16<true, 4096>", "lambda_sweeps": "k_lam_sweep",
    "col_inv_solve": "k_col_inv_r16<4096>", "row_inv": "k_row_inv_r16<4096>", "guided_filter": "k_gf_g<8, false>",
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


def batch_leg(steps: int, warmup: int, n_images: int = 64) -> dict:
    """Mixed-size batch: one context (one launch per pass for all images, graph replay) against
    the one-image-per-launch path (a context per image, kernels launched one by one, images in
    sequence).  Both run the same kernels on the same inputs."""
    import numpy as np
    import torch

    import paper_1609_01839_amd as gfd
    import synth

    dev = torch.device("cuda:0")
    cases = synth.make_batch(n_images)
    probs = [dict(y=torch.from_numpy(c.y).to(dev), h=torch.from_numpy(c.h.astype(np.float32)).to(dev),
                  sigma2=c.sigma2, w=c.w, eps=c.eps) for c in cases]
    total_px = sum(c.y.size for c in cases)
    stream = torch.cuda.current_stream(dev)

    def timed(fn, n):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        fn(n)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / n

    # both paths run n iterations per deconv_iterate call and copy the estimates out once
    with gfd.GFDeconvBatch(probs) as gb:
        gb.autotune(4)
        out = torch.empty((gb.total,), device=dev, dtype=torch.float32)
        lam = torch.empty((gb.count, max(steps, warmup, 1)), device=dev, dtype=torch.float32)
        if warmup > 0:
            gb.iterate(warmup, out, lam[:, :warmup].contiguous())
        lam_s = torch.empty((gb.count, steps), device=dev, dtype=torch.float32)
        ms_batch = timed(lambda n: gb.iterate(n, out, lam_s), steps)
    singles = [gfd.GFDeconv(p["y"], p["h"], p["sigma2"], p["w"], p["eps"]) for p in probs]
    outs = [torch.empty(p["y"].shape, device=dev, dtype=torch.float32) for p in probs]
    n_single = max(2, steps // 4)
    lam1 = torch.empty((max(n_single, warmup, 1),), device=dev, dtype=torch.float32)
    for g in singles:
        g.set_graph(False)

    def run_singles(n):
        for g, o in zip(singles, outs):
            g.iterate(n, o, lam1[:n])

    run_singles(max(1, warmup // 2))
    ms_single = timed(run_singles, n_single)
    for g in singles:
        g.close()
    sizes = sorted({c.y.shape for c in cases})
    return {"workload": f"{n_images} piecewise-constant synthetic images of sizes drawn from "
                        f"{', '.join(f'{a}x{b}' for a, b in sizes)}, PSFs 9x9 box / 25x25 Gaussian / 15x15 "
                        f"1/(1+x^2+y^2), BSNR 20-40 dB, w in {{5, 7, 9}}, one step = one iteration of every image",
            "images": n_images, "pixels": total_px,
            "value": round(total_px / (ms_batch * 1e-3) / 1e6, 1), "unit": "Mpixel-iters/s",
            "ms_per_step": round(ms_batch, 4),
            "one_image_per_launch": {"value": round(total_px / (ms_single * 1e-3) / 1e6, 1),
                                     "ms_per_step": round(ms_single, 4)},
            "speedup_vs_one_image_per_launch": round(ms_single / ms_batch, 2)}


def fwd_bwd_leg(g, M: int, N: int, iters: int, repeats: int, u_ref) -> dict:
    """Forward iterations followed by the reverse mode (gradient of an MSE loss with respect
    to eps and the lambda scales, checkpoints every 5 iterations), on the same context."""
    import torch

    dev = u_ref.device
    stream = torch.cuda.current_stream(dev)
    out = torch.empty((M, N), device=dev, dtype=torch.float32)
    lam = torch.empty((iters,), device=dev, dtype=torch.float32)
    times = []
    for r in range(repeats + 1):
        g.reset()
        torch.cuda.synchronize()
        ev0, ev1, ev2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        ev0.record(stream)
        g.iterate(iters, out, lam)
        ev1.record(stream)
        gu = (2.0 / out.numel()) * (out - u_ref)
        g.backward(gu, 5)
        ev2.record(stream)
        torch.cuda.synchronize()
        if r > 0:                      # the first pass allocates the reverse-mode buffers
            times.append((ev0.elapsed_time(ev1), ev1.elapsed_time(ev2)))
    fwd = sorted(t[0] for t in times)[len(times) // 2]
    bwd = sorted(t[1] for t in times)[len(times) // 2]
    P = M * N
    return {"iterations": iters, "checkpoint_every": 5, "fwd_ms": round(fwd, 3), "bwd_ms": round(bwd, 3),
            "value": round(P * iters / ((fwd + bwd) * 1e-3) / 1e6, 1), "unit": "Mpixel-iters/s",
            "bwd_over_fwd": round(bwd / fwd, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=4096, help="image side (default: the 4096^2 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=10)
    ap.add_argument("--no-batch", action="store_true", help="skip the mixed-size batch leg")
    ap.add_argument("--no-bwd", action="store_true", help="skip the forward+adjoint leg")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--tuning", type=str, default="",
                    help="launch shapes instead of the autotuner: strip rows, forward row pairs, inverse rows")
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
    if args.tuning:
        vals = [int(x) for x in args.tuning.split(",")]
        if len(vals) != 3:
            raise SystemExit("--tuning takes three integers: strip rows, forward row pairs, inverse rows")
        g.set_tuning(*vals)
        tuning = dict(zip(("gf_strip_rows", "row_pairs_fwd", "rows_inv"), vals))
    else:
        tuning = None if args.no_autotune else g.autotune(16)
    stream = torch.cuda.current_stream(dev)
    out = torch.empty((M, N), device=dev, dtype=torch.float32)
    lam = torch.empty((max(args.steps, args.warmup, 1),), device=dev, dtype=torch.float32)

    # the K steps are one deconv_iterate call: K graph replays, then the estimate and the K
    # lambdas are copied out once (as a caller running K iterations would)
    if args.warmup > 0:
        g.iterate(args.warmup, out, lam[:args.warmup])
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    g.iterate(args.steps, out, lam[:args.steps])
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
                   "M": M, "N": N, "iters_per_step": 1, "hip_graph": True, "autotune": tuning},
        "roofline": roofline,
        "iteration": {"alg_bytes_per_px": round((total_alg + 8 * Q) / P, 2),
                      "alg_frac_of_hbm_roofline": round((total_alg / P) * P / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "stage_us": {k: round(v * 1e3, 2) for k, v in per_iter.items()},
                      "wall_s": round(wall, 4)},
    }
    if not args.no_bwd:
        u_ref = torch.from_numpy(case.u_orig.astype(np.float32)).to(dev)
        line["fwd_bwd"] = fwd_bwd_leg(g, M, N, 10, 3, u_ref)
        del u_ref
    g.close()
    del y, h, out
    if not args.no_batch:
        line["batch"] = batch_leg(max(args.steps // 2, 5), args.warmup)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
