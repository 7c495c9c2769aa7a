"""Helpers of the GPU parity tests: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances come from the stated target: every iterate within 1e-5 relative L2 of the FP64
oracle, every lambda within 1e-4, the final ISNR within 0.01 dB.

Branch near-ties (Sec. 3.2: u_E in K when ||h*u_E - y||^2 <= T, a closed set): the GPU decides
the test in compensated FP32 and the oracle in FP64, so when E_inf / T is within 1e-5 of 1 the
two may take different branches.  ``run_trajectory`` then records a near-tie and checks that
step by rerunning it on the GPU with the oracle's branch and lambda injected (the stand-alone
spectral solve at the oracle's lambda, then the stand-alone guided filter), instead of failing.
A branch disagreement away from a near-tie is a failure.
"""
from __future__ import annotations

import math

import numpy as np
import torch

import oracle
import paper_1609_01839_amd as gfd
import synth

DEV = torch.device("cuda:0")
NEAR_TIE = 1e-5


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def problem(M, N, h, sigma2=None, bsnr=35.0, seed=0, textured=False):
    rng = np.random.default_rng(seed)
    u = synth.textured_image(M, N, rng) if textured else synth.piecewise_image(M, N, rng)
    b = synth.blur_periodic(u, h)
    if sigma2 is None:
        sigma2 = synth.sigma2_for_bsnr(b, bsnr)
    y = (b + math.sqrt(sigma2) * rng.standard_normal((M, N))).astype(np.float32)
    return u, y, float(sigma2)


def oracle_setup(y, h, sigma2, rho=None):
    return oracle.setup(y.astype(np.float64), h.astype(np.float32).astype(np.float64), sigma2, rho)


def gpu_step_with_lambda(g, uE, lam, w, eps):
    """One GPU iteration from u_E with lambda imposed (+inf: the u_E in K branch): the solves of
    Eqs.(8)-(9) at that lambda, then the guided filter of Eqs.(3)-(5)."""
    uI, up = g.spectral_solve(to_gpu(uE), lam)
    return gfd.guided_filter(uI, up, w, eps)


def run_trajectory(c, iters, rho=None, one_step=True, tuning=None, one_step_at=None, u0=None, log=print):
    """GPU trajectory of ``iters`` iterations against the oracle's, plus one-step checks (a GPU
    step started from the oracle's iterate k against the oracle's step from it).  ``u0`` (FP32
    values) replaces the zero starting estimate on both sides.

    Returns a dict: traj (rel L2 per iterate), lam (relative lambda error per iterate, 0 where
    both are +inf), steps (one-step rel L2), near_ties (list of iterations where the branches
    differed at a near-tie, checked with the oracle's branch injected), isnr_gpu, isnr_ref."""
    y, h = c.y, c.h.astype(np.float32)
    eps = float(np.float32(c.eps))
    if u0 is not None:
        u0 = np.asarray(u0, np.float32)
    ref_u, info = oracle.deconvolve(y.astype(np.float64), h.astype(np.float64), c.sigma2, c.w, eps, iters, rho=rho,
                                    u0=None if u0 is None else u0.astype(np.float64), keep_iterates=True)
    T = info["T"]
    errs, lam_errs, step_errs, ties = [], [], [], []
    with gfd.GFDeconv(to_gpu(y), to_gpu(h), c.sigma2, c.w, eps, rho) as g:
        if tuning is not None:
            g.set_tuning(*tuning)
        if u0 is not None:
            g.set_estimate(to_gpu(u0))
        u_last = None
        for k in range(iters):
            u, lam = g.iterate(1)
            lg, lo = float(lam.cpu()[0]), float(info["lam"][k])
            if math.isinf(lg) != math.isinf(lo):
                near = abs(info["E_inf"][k] / T - 1.0) < NEAR_TIE
                log(f"iteration {k}: branch differs (gpu lambda {lg:.6g}, oracle {lo:.6g}), "
                    f"E_inf/T - 1 = {info['E_inf'][k] / T - 1.0:.2e}, near-tie {near}")
                assert near, f"branch disagreement away from a near-tie at iteration {k}"
                if k > 0:
                    prev = info["iterates"][k - 1]
                else:
                    prev = np.zeros(c.y.shape) if u0 is None else u0
                inj = gpu_step_with_lambda(g, prev.astype(np.float32), lo, c.w, eps).cpu().numpy()
                e_inj = rel_l2(inj, info["iterates"][k])
                log(f"iteration {k}: oracle branch injected, rel L2 {e_inj:.2e}")
                ties.append((k, e_inj))
                # continue the trajectory from the oracle's iterate
                g.set_estimate(to_gpu(info["iterates"][k]))
                errs.append(e_inj)
                lam_errs.append(0.0)
                u_last = inj
                continue
            u_last = u.cpu().numpy()
            errs.append(rel_l2(u_last, info["iterates"][k]))
            lam_errs.append(0.0 if math.isinf(lo) else abs(lg - lo) / lo)
        isnr_gpu = oracle.isnr(u_last, y, c.u_orig)
        if one_step:
            S = oracle_setup(y, h, c.sigma2, rho)
            ks = range(iters - 1) if one_step_at is None else one_step_at
            for k in ks:
                g.set_estimate(to_gpu(info["iterates"][k]))
                u1, _ = g.iterate(1)
                ref = oracle.step(S, info["iterates"][k].astype(np.float32).astype(np.float64), c.w, eps)
                step_errs.append(rel_l2(u1.cpu().numpy(), ref.u))
    isnr_ref = oracle.isnr(ref_u, y, c.u_orig)
    return dict(traj=errs, lam=lam_errs, steps=step_errs, near_ties=ties, isnr_gpu=isnr_gpu, isnr_ref=isnr_ref,
                info=info)


def report(tag, r, log=print):
    log(f"{tag}: trajectory rel L2 " + " ".join(f"{e:.1e}" for e in r["traj"]))
    if r["steps"]:
        log(f"{tag}: one-step rel L2   " + " ".join(f"{e:.1e}" for e in r["steps"]))
    log(f"{tag}: lambda rel err    " + " ".join(f"{e:.1e}" for e in r["lam"]))
    log(f"{tag}: ISNR gpu {r['isnr_gpu']:.4f} dB, oracle {r['isnr_ref']:.4f} dB, near-ties {r['near_ties']}")


def assert_parity(r, tol=1e-5, lam_tol=1e-4, isnr_tol=0.01):
    assert max(r["traj"]) < tol, r["traj"]
    if r["steps"]:
        assert max(r["steps"]) < tol, r["steps"]
    assert max(r["lam"]) < lam_tol, r["lam"]
    assert abs(r["isnr_gpu"] - r["isnr_ref"]) < isnr_tol
