"""Throughput of the deconvolution iteration on one MI355X.

A step is one full iteration (Steps 1-3 of Sec. 3.1: forward transform, residual and lambda
search, both solves, inverse transforms, guided filter) over the 4096 x 4096 workload with
inputs resident in HBM.  Prints one JSON line (see the repository's bench contract) with, besides
the headline rate: the roofline of the slowest pass, the forward+adjoint rate, the mixed-size
batch rate, each with its algorithmic bytes and fraction of the HBM roofline, the parity errors of
the timed results against the FP64 oracle, and the oracle's own rate on the host (one core for
the single frame, a process pool over all cores for the batch).

The CPU legs run first, before anything touches the GPU, so that the host pool (forked) never
inherits a GPU context and the GPU timings never share the host with it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batch] [--no-bwd]
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
    "row_fwd": "k_row_fwd_r16<4096>", "col_fwd_resid": "k_col_fwd_r16<true, 4096>", "lambda_sweeps": "k_lam_rounds",
    "col_inv_solve": "k_col_inv_r16<4096>", "row_inv": "k_row_inv_r16<4096>", "guided_filter": "k_gf_g<8, false, false>",
}
PARITY_ITERS = 3   # iterations of the single frame compared with the oracle (the CPU sample)


def iteration_bytes(P: int, Q: int) -> int:
    """Algorithmic bytes of one forward iteration (lambda rounds after the first excluded: in
    the steady state the first round, fused into the residual pass, decides)."""
    return sum(a * P + b * Q for k, (a, b) in ALG_BYTES.items() if k != "lambda_sweeps")


def backward_bytes(P: int, Q: int, K: int, c: int) -> int:
    """Algorithmic bytes of deconv_backward over K iterations with checkpoints every c, following
    its schedule: a replay of the forward from the starting estimate keeping every c-th
    pre-estimate, then per segment (last first) a replay of each iteration that writes u_I, u_p
    and U_E straight into that iteration's slot, with the filter that also writes the first box
    pass's results there, and the adjoint of each iteration in reverse, reading them there
    (windows that the strip filter holds, as in the benchmark's workload)."""
    replay = 12 * P + 76 * Q          # row_fwd 4P+8Q, column pass 16Q, column inverse 36Q, row inverse 8P+16Q
    gf = 12 * P                       # guided filter
    gf_save = 28 * P                  # the same, also writing a, the means of I and p, var + eps
    copy = 8 * P                      # an estimate copied to or from a checkpoint
    adjoint = 96 * P + 168 * Q        # box passes 44P+36P, transforms of g_I, g_p 8P+48Q,
    #                                   spectral adjoint 52Q, adjoint column pass 52Q, row inverse 8P+16Q
    nck = -(-K // c)
    total = copy + (nck - 1) * c * (replay + gf) + nck * copy
    for j in range(nck):
        n = min(c, K - j * c)
        total += (copy if j != nck - 1 else 0) + n * (replay + gf_save) + n * adjoint
    return total


def source_hash() -> str:
    """Hash of the kernel sources and the build script (its compiler flags)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1609_01839_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "paper_1609_01839_amd", "build.py"), "rb").read())
    return h.hexdigest()[:16]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ----------------------------------------------------------------------------- CPU legs (oracle)

def oracle_single(case, iters: int):
    """The FP64 oracle, as is, on the same frame: `iters` iterations from u_E = 0 (one process,
    numpy's single-threaded FFT).  Returns (timing dict, FP32 iterates, lambdas)."""
    import numpy as np

    import oracle
    y = case.y.astype(np.float64)
    h = case.h.astype(np.float32).astype(np.float64)
    S = oracle.setup(y, h, case.sigma2)
    uE = np.zeros_like(y)
    its, lams = [], []
    t0 = time.perf_counter()
    for _ in range(iters):
        r = oracle.step(S, uE, case.w, float(np.float32(case.eps)))
        uE = r.u
        its.append(r.u.astype(np.float32))
        lams.append(r.lam)
    dt = time.perf_counter() - t0
    return {"value": round(y.size * iters / dt / 1e6, 4), "unit": "Mpixel-iters/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{iters} oracle iterations of the same {case.shape[0]}x{case.shape[1]} frame from u_E = 0, "
                      f"{dt:.1f} s, numpy float64, one process"}, its, lams


def _oracle_batch_task(k: int):
    """One image of the batch: set-up and one oracle iteration from u_E = 0 (pool worker)."""
    import numpy as np

    import oracle
    import synth
    c = synth.batch_case(k)
    y = c.y.astype(np.float64)
    S = oracle.setup(y, c.h.astype(np.float32).astype(np.float64), c.sigma2)
    r = oracle.step(S, np.zeros_like(y), c.w, float(np.float32(c.eps)))
    return k, r.u.astype(np.float32), r.lam, y.size


def oracle_batch(n_images: int):
    """The oracle over the mixed-size batch on a process pool over every host core, one image per
    task (set-up and one iteration each).  Returns (timing dict, per-image FP32 iterates, lambdas)."""
    import multiprocessing as mp

    cores = len(os.sched_getaffinity(0))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(processes=cores) as pool:
        res = pool.map(_oracle_batch_task, range(n_images), chunksize=1)
    dt = time.perf_counter() - t0
    res.sort(key=lambda t: t[0])
    px = sum(r[3] for r in res)
    return {"value": round(px / dt / 1e6, 4), "unit": "Mpixel-iters/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"one oracle iteration (with its set-up) of each of the {n_images} batch images from "
                      f"u_E = 0, {dt:.1f} s wall-clock on a pool of {cores} processes"}, \
        [r[1] for r in res], [r[2] for r in res]


def rel_l2(a, b) -> float:
    import numpy as np
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def lam_err(g: float, o: float) -> float:
    if math.isinf(o) or math.isinf(g):
        return 0.0 if math.isinf(o) and math.isinf(g) else float("inf")
    return abs(g - o) / o


# ----------------------------------------------------------------------------- GPU legs

# launch shapes of the batch leg: strip rows, forward row pairs, inverse rows, mixed-radix rows,
# mixed-radix schedule (from a sweep of fixed shapes, one process each: 64-row strips and row
# pairs took 0.867 ms per step against 0.878 for 32 rows and single pairs, 0.870 for 64 rows with
# single pairs, 0.88-0.90 for 40, 48, 80, 96 and 128 rows)
BATCH_TUNING = (64, 2, 2, 2, 8)


def batch_leg(steps: int, warmup: int, n_images: int = 64, ref=None) -> dict:
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
    alg = sum(iteration_bytes(c.y.size, c.y.shape[0] * (c.y.shape[1] // 2 + 1)) for c in cases)
    stream = torch.cuda.current_stream(dev)

    def timed(fn, n):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        fn(n)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / n

    parity = None
    with gfd.GFDeconvBatch(probs) as gb:
        # fixed launch shapes (the autotuner's usual choice for this batch; the library does not
        # autotune multi-image contexts)
        gb.set_tuning(*BATCH_TUNING)
        tuning = dict(zip(("gf_strip_rows", "row_pairs_fwd", "rows_inv", "rows_lds", "radix"), BATCH_TUNING))
        tuning["fixed"] = True
        if ref is not None:  # the first iteration of every image against the oracle's
            us, lam = gb.iterate(1)
            lam = lam.cpu().numpy()
            errs = [rel_l2(u.cpu().numpy(), r) for u, r in zip(us, ref[0])]
            lerrs = [lam_err(float(lam[b, 0]), ref[1][b]) for b in range(len(cases))]
            parity = {"iterations": 1, "images": len(cases), "max_iterate_rel_l2": max(errs),
                      "max_lambda_rel_err": max(lerrs), "bar": {"iterate_rel_l2": 1e-5, "lambda_rel": 1e-4}}
        out = torch.empty((gb.total,), device=dev, dtype=torch.float32)
        lam = torch.empty((gb.count, max(steps, warmup, 1)), device=dev, dtype=torch.float32)
        if warmup > 0:
            gb.iterate(warmup, out, lam[:, :warmup].contiguous())
        lam_s = torch.empty((gb.count, steps), device=dev, dtype=torch.float32)
        ms_batch = timed(lambda n: gb.iterate(n, out, lam_s), steps)
        nprof = 5
        stage_us = {k: round(v / nprof * 1e3, 2) for k, v in gb.profile(nprof).items()}
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
    gbs = alg / (ms_batch * 1e-3) / 1e9
    out = {"workload": f"{n_images} piecewise-constant synthetic images of sizes drawn from "
                       f"{', '.join(f'{a}x{b}' for a, b in sizes)}, PSFs 9x9 box / 25x25 Gaussian / 15x15 "
                       f"1/(1+x^2+y^2), BSNR 20-40 dB, w in {{5, 7, 9}}, one step = one iteration of every image",
           "images": n_images, "pixels": total_px, "autotune": tuning,
           "value": round(total_px / (ms_batch * 1e-3) / 1e6, 1), "unit": "Mpixel-iters/s",
           "ms_per_step": round(ms_batch, 4), "stage_us": stage_us,
           "roofline": {"bound": "hbm", "alg_bytes_per_step": alg, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)},
           "one_image_per_launch": {"value": round(total_px / (ms_single * 1e-3) / 1e6, 1),
                                    "ms_per_step": round(ms_single, 4)},
           "speedup_vs_one_image_per_launch": round(ms_single / ms_batch, 2)}
    if parity is not None:
        out["parity_vs_oracle"] = parity
    return out


def fwd_bwd_leg(g, M: int, N: int, iters: int, repeats: int, u_ref, ckpt: int = 5) -> dict:
    """Forward iterations followed by the reverse mode (gradient of an MSE loss with respect
    to eps and the lambda scales, checkpoints every `ckpt` iterations), on the same context."""
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
        g.backward(gu, ckpt)
        ev2.record(stream)
        torch.cuda.synchronize()
        if r > 0:                      # the first pass allocates the reverse-mode buffers
            times.append((ev0.elapsed_time(ev1), ev1.elapsed_time(ev2)))
    fwd = sorted(t[0] for t in times)[len(times) // 2]
    bwd = sorted(t[1] for t in times)[len(times) // 2]
    P, Q = M * N, M * (N // 2 + 1)
    b_fwd = iters * iteration_bytes(P, Q)
    b_bwd = backward_bytes(P, Q, iters, ckpt)
    gbs = (b_fwd + b_bwd) / ((fwd + bwd) * 1e-3) / 1e9
    return {"iterations": iters, "checkpoint_every": ckpt, "fwd_ms": round(fwd, 3), "bwd_ms": round(bwd, 3),
            "value": round(P * iters / ((fwd + bwd) * 1e-3) / 1e6, 1), "unit": "Mpixel-iters/s",
            "bwd_over_fwd": round(bwd / fwd, 2),
            "roofline": {"bound": "hbm", "alg_bytes_per_px_iter": round((b_fwd + b_bwd) / (P * iters), 1),
                         "alg_bytes_per_px_iter_bwd": round(b_bwd / (P * iters), 1), "achieved": round(gbs, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "bwd_frac": round(b_bwd / (bwd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--size", type=int, default=4096, help="image side (default: the 4096^2 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle legs (and the parity report)")
    ap.add_argument("--profile-iters", type=int, default=10)
    ap.add_argument("--no-batch", action="store_true", help="skip the mixed-size batch leg")
    ap.add_argument("--no-bwd", action="store_true", help="skip the forward+adjoint leg")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--tuning", type=str, default="",
                    help="launch shapes instead of the autotuner: strip rows, forward row pairs, inverse rows"
                         "[, mixed-radix rows, mixed-radix schedule]")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the deconvolution of one frame runs on a single device "
              "(sharding over several GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth

    size = (args.size, args.size)
    case = synth.make_case(5, size=None if args.size == 4096 else size)
    M, N = case.shape
    P, Q = M * N, M * (N // 2 + 1)
    n_images = 64

    # ---- CPU legs first (no GPU context yet)
    cpu = single_ref = batch_ref = None
    if not args.no_cpu_baseline:
        cpu, its, lams = oracle_single(case, PARITY_ITERS)
        single_ref = (its, lams)
        if not args.no_batch:
            cpu_b, bits, blams = oracle_batch(n_images)
            cpu["batch"] = cpu_b
            batch_ref = (bits, blams)

    import torch

    import paper_1609_01839_amd as gfd

    dev = torch.device("cuda:0")
    y = torch.from_numpy(case.y).to(dev)
    h = torch.from_numpy(case.h.astype(np.float32)).to(dev)
    g = gfd.GFDeconv(y, h, case.sigma2, case.w, case.eps)
    if args.tuning:
        vals = [int(x) for x in args.tuning.split(",")]
        if len(vals) not in (3, 5):
            raise SystemExit("--tuning takes 3 or 5 integers: strip rows, forward row pairs, inverse rows"
                             "[, mixed-radix rows, mixed-radix schedule]")
        g.set_tuning(*vals)
        tuning = dict(zip(gfd.GFDeconv.TUNING_KEYS, vals))
    else:
        tuning = None if args.no_autotune else g.autotune(16)
    stream = torch.cuda.current_stream(dev)
    out = torch.empty((M, N), device=dev, dtype=torch.float32)
    lam = torch.empty((max(args.steps, args.warmup, PARITY_ITERS, 1),), device=dev, dtype=torch.float32)

    # parity of the timed configuration: the first iterations from u_E = 0 against the oracle's
    parity = None
    if single_ref is not None:
        errs, lerrs = [], []
        for k in range(PARITY_ITERS):
            g.iterate(1, out, lam[:1])
            errs.append(rel_l2(out.cpu().numpy(), single_ref[0][k]))
            lerrs.append(lam_err(float(lam[0].cpu()), single_ref[1][k]))
        parity = {"iterations": PARITY_ITERS, "iterate_rel_l2": [float(f"{e:.3g}") for e in errs],
                  "lambda_rel_err": [float(f"{e:.3g}") for e in lerrs],
                  "bar": {"iterate_rel_l2": 1e-5, "lambda_rel": 1e-4}}
        g.reset()

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
    alg = {k: (a * P + b * Q) for k, (a, b) in ALG_BYTES.items()}
    dom = max((k for k in per_iter if k != "lambda_sweeps"), key=lambda k: per_iter[k])
    achieved = alg[dom] / (per_iter[dom] * 1e-3) / 1e9
    traffic = None
    pmc_path = os.path.join(ROOT, "profiles", f"pmc_{M}x{N}.json")
    if os.path.exists(pmc_path):
        pmc = json.load(open(pmc_path))
        if pmc.get("source_hash") == source_hash() and dom in pmc.get("bytes_per_launch", {}):
            traffic = pmc["bytes_per_launch"][dom]
    total_alg = iteration_bytes(P, Q)
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
        "iteration": {"alg_bytes_per_px": round(total_alg / P, 2),
                      "alg_frac_of_hbm_roofline": round(total_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "stage_us": {k: round(v * 1e3, 2) for k, v in per_iter.items()},
                      "wall_s": round(wall, 4)},
    }
    if parity is not None:
        line["parity_vs_oracle"] = parity
    if not args.no_bwd:
        u_ref = torch.from_numpy(case.u_orig.astype(np.float32)).to(dev)
        line["fwd_bwd"] = fwd_bwd_leg(g, M, N, 10, 3, u_ref)
        del u_ref
    g.close()
    del y, h, out
    if not args.no_batch:
        line["batch"] = batch_leg(max(args.steps // 2, 5), args.warmup, n_images, batch_ref)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()
