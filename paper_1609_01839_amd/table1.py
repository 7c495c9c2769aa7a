"""The five degradation settings of Table 1 on seeded synthetic stand-in images.

    python -m paper_1609_01839_amd.table1 [--size 256] [--iters 30] [--seeds 0 1] [--json out.json]

Each setting (PSF and noise variance of Table 1, guided-filter parameters of Sec. 4: w = 3 and
eps = 7.5e-4 on the [0, 1] scale, i.e. 7.5e-4 * 255^2 on the [0, 255] scale used here) is run on
the GPU for the given number of iterations, once with rho from Eq.(12) and once with rho = 1.
Reported per run: the ISNR of the final estimate, the lambda trajectory and the branch flags.
The paper's own test images are not used (synthetic piecewise-constant images stand in), so the
numbers are not comparable to its Tables 2-3.
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np
import torch

import synth

from . import GFDeconv


def isnr(u, y, u_orig) -> float:
    """10 log10(||y - u_orig||^2 / ||u - u_orig||^2) in dB."""
    u, y, u_orig = (np.asarray(a, np.float64) for a in (u, y, u_orig))
    return 10.0 * math.log10(float(np.sum((y - u_orig) ** 2)) / float(np.sum((u - u_orig) ** 2)))


def run_setting(test: int, size: int = 256, iters: int = 30, seed: int = 0, rho=None, device="cuda:0") -> dict:
    c = synth.table1_case(test, size, size, seed=seed)
    dev = torch.device(device)
    y = torch.from_numpy(c.y).to(dev)
    h = torch.from_numpy(c.h.astype(np.float32)).to(dev)
    with GFDeconv(y, h, c.sigma2, c.w, c.eps, rho) as g:
        info = g.info()
        u, lam = g.iterate(iters)
        flags = g.status()
    u = u.cpu().numpy()
    lam = lam.cpu().numpy().astype(np.float64)
    return {"test": test, "seed": seed, "rho_mode": "Eq.(12)" if rho is None else f"fixed {rho}",
            "rho": info["rho"], "sigma2": c.sigma2, "eps": c.eps, "w": c.w, "iters": iters,
            "isnr_db": isnr(u, c.y, c.u_orig), "lambda": [float(v) for v in lam], "flags": int(flags)}


def run(size: int = 256, iters: int = 30, seeds=(0,), rho_choices=(None, 1.0)) -> list:
    return [run_setting(t, size, iters, s, r) for t in sorted(synth.TABLE1_SETTINGS) for s in seeds for r in rho_choices]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--seeds", type=int, nargs="+", default=[0])
    ap.add_argument("--json", default=None)
    args = ap.parse_args()
    res = run(args.size, args.iters, tuple(args.seeds))
    print("| test | PSF | sigma^2 | rho | ISNR dB | lambda_1 | lambda_K |")
    print("|---|---|---|---|---|---|---|")
    for r in res:
        psf = synth.TABLE1_SETTINGS[r["test"]][0]
        print(f"| {r['test']} | {psf} | {r['sigma2']:g} | {r['rho_mode']} ({r['rho']:.4f}) | {r['isnr_db']:.3f} | "
              f"{r['lambda'][0]:.4g} | {r['lambda'][-1]:.4g} |")
    if args.json:
        json.dump(res, open(args.json, "w"), indent=1)


if __name__ == "__main__":
    main()
