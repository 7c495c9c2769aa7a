"""Parity of the compile-time register-resident transforms below 4096 points against the FP64
oracle.

Every power-of-two side from 256 to 4096 takes a transform compiled for its length: the row
passes of an image that wide, and the column passes over tiles of the width the layout gives
that many rows (4 columns at 2048 rows, 8 at 1024, 16 at 512 and 256).  Narrow shapes reach each
length's column kernels (M x small N: the residual pass with the fused first lambda round, the
plain forward column pass, the column inverse with the solves, the adjoint column pass) and row
kernels (small M x N) cheaply; the other side takes the mixed-radix LDS transform.  2048 is the
length no other test reaches.

Bars: FFT round trip 1e-6; solves and every iterate 1e-5 relative L2; lambda 1e-5 for the
stand-alone search and 1e-4 along a trajectory; gradients 1e-4 of the oracle's adjoint.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
import paper_1609_01839_amd as gfd
import synth
from _parity import assert_parity, oracle_setup, problem, rel_l2, report, run_trajectory, to_gpu

pytestmark = pytest.mark.gpu

SHAPES = [(2048, 64), (64, 2048), (1024, 48), (48, 1024), (512, 40), (40, 512), (256, 24), (24, 256)]
H = synth.psf_gaussian(1.6, 9)


def log(msg):
    print(msg)
    sys.stdout.flush()


@pytest.mark.parametrize("M,N", SHAPES)
def test_round_trip_and_solves(M, N):
    """lambda = +inf (F^-1 F u_E through the forward and inverse passes), then the solves of
    Eqs.(8)-(9) at two lambdas."""
    u, y, s2 = problem(M, N, H, seed=M + N)
    S = oracle_setup(y, H, s2)
    rng = np.random.default_rng(21)
    uE = (u + 10 * rng.standard_normal((M, N))).astype(np.float32)
    UE = oracle.dft2(uE.astype(np.float64))
    with gfd.GFDeconv(to_gpu(y), to_gpu(H.astype(np.float32)), s2, 5, 650.25) as g:
        uI, up = g.spectral_solve(to_gpu(uE), math.inf)
        e1, e2 = rel_l2(uI.cpu().numpy(), uE), rel_l2(up.cpu().numpy(), uE)
        log(f"round trip {M}x{N}: {e1:.2e} {e2:.2e}")
        assert e1 < 1e-6 and e2 < 1e-6
        for lam in (0.02, 5.0):
            uI, up = g.spectral_solve(to_gpu(uE), lam)
            rI, rp = oracle.spectral_solve(S, UE, float(np.float32(lam)))
            eI, ep = rel_l2(uI.cpu().numpy(), rI), rel_l2(up.cpu().numpy(), rp)
            log(f"solve {M}x{N} lam={lam}: u_I {eI:.2e}, u_p {ep:.2e}")
            assert eI < 1e-5 and ep < 1e-5


@pytest.mark.parametrize("M,N", SHAPES)
def test_discrepancy_lambda(M, N):
    u, y, s2 = problem(M, N, H, seed=M + 3 * N)
    S = oracle_setup(y, H, s2)
    uE = (0.9 * u).astype(np.float32)
    with gfd.GFDeconv(to_gpu(y), to_gpu(H.astype(np.float32)), s2, 5, 650.25) as g:
        lam = float(g.discrepancy_lambda(to_gpu(uE)).cpu()[0])
    ref, flags = oracle.discrepancy_lambda(S, oracle.dft2(uE.astype(np.float64)))
    err = abs(lam - ref) / ref
    log(f"lambda {M}x{N}: gpu {lam:.9g} oracle {ref:.9g} rel {err:.2e}")
    assert flags == 0 and err < 1e-5


def strip_case(M, N, seed):
    rng = np.random.default_rng(seed)
    u = synth.piecewise_image(M, N, rng)
    b = synth.blur_periodic(u, H)
    s2 = float(synth.sigma2_for_bsnr(b, 30.0))
    y = (b + math.sqrt(s2) * rng.standard_normal((M, N))).astype(np.float32)
    return synth.Case(f"strip_{M}x{N}", u, H, y, s2, 5, synth.EPS_DEFAULT, 3)


@pytest.mark.parametrize("M,N", SHAPES)
def test_iteration_parity(M, N):
    c = strip_case(M, N, seed=7000 + M + N)
    r = run_trajectory(c, 3, log=log)
    report(f"{M}x{N} w=5", r, log)
    assert_parity(r)


@pytest.mark.parametrize("M,N", [(2048, 64), (64, 2048), (1024, 48)])
def test_adjoint_matches_oracle(M, N):
    c = strip_case(M, N, seed=8000 + M + N)
    eps, iters = float(np.float32(650.25)), 3
    scales = np.linspace(0.9, 1.1, iters).astype(np.float32)
    with gfd.GFDeconv(to_gpu(c.y), to_gpu(H.astype(np.float32)), c.sigma2, c.w, eps) as g:
        g.set_scales(scales)
        uk, _ = g.iterate(iters)
        gu = 2.0 * (uk - to_gpu(c.u_orig)) / uk.numel()
        ge, gs = g.backward(gu, 2)
    ge, gs = float(ge.cpu()[0]), gs.cpu().numpy()[0].astype(np.float64)
    y64, h64, s64 = c.y.astype(np.float64), H.astype(np.float32).astype(np.float64), scales.astype(np.float64)
    ref, _ = oracle.deconvolve(y64, h64, c.sigma2, c.w, eps, iters, scales=s64)
    re, rs, _ = adj.deconvolve_adjoint(y64, h64, c.sigma2, c.w, eps, iters, adj.mse_loss_grad(ref, c.u_orig)[1],
                                       scales=s64)
    e_eps = abs(ge - re) / abs(re)
    e_s = float(np.max(np.abs(gs - rs)) / np.max(np.abs(rs)))
    log(f"adjoint {M}x{N}: g_eps {ge:.6e} vs {re:.6e} ({e_eps:.1e}), g_s max rel {e_s:.1e}")
    assert e_eps < 1e-4 and e_s < 1e-4
