"""Parity of the 4096-point transforms against the FP64 oracle.

Sides of 4096 take compile-time transforms that no other size uses: the row passes of a
4096-wide image (forward rows and the inverse row gather) and the column passes over tiles of
two 4096-row columns (the residual pass with the fused first lambda round, the plain forward
column pass of the stand-alone solve and of the reverse mode, and the column inverse with the
solves of Eqs.(8)-(9)).  Narrow shapes reach each of them cheaply:

* 4096 x 64 and 4096 x 256: every column pass at 4096 rows (with the Nyquist column folded
  into tile 0), rows of 64 (mixed-radix LDS transform) and 256 (run-time register transform);
* 64 x 4096: both 4096-point row passes, columns of 64;
* 4096 x 4096 with the large-frame workload (Gaussian PSF std 2.5 on 31 x 31, sigma^2 = 4,
  w = 17, eps = 650.25) and the launch shapes the benchmark uses (104-row filter strips, two
  row pairs per forward row block, two rows per inverse row block).

Bars: FFT round trip 1e-6; solves and every iterate 1e-5 relative L2; lambda 1e-5 for the
stand-alone search and 1e-4 along a trajectory; final ISNR within 0.01 dB.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_1609_01839_amd as gfd
import synth
from _parity import assert_parity, oracle_setup, problem, rel_l2, report, run_trajectory, to_gpu

pytestmark = pytest.mark.gpu

SHAPES = [(4096, 64), (64, 4096), (4096, 256)]
H_LARGE = synth.psf_gaussian(2.5, 31)


def log(msg):
    print(msg)
    sys.stdout.flush()


@pytest.mark.parametrize("M,N", SHAPES)
def test_round_trip_4096(M, N):
    """lambda = +inf: u_I = u_p = F^-1 F u_E through the forward and inverse passes."""
    _, y, s2 = problem(M, N, H_LARGE, seed=M + N)
    rng = np.random.default_rng(11)
    uE = rng.uniform(0, 255, (M, N)).astype(np.float32)
    with gfd.GFDeconv(to_gpu(y), to_gpu(H_LARGE.astype(np.float32)), s2, 17, 650.25) as g:
        uI, up = g.spectral_solve(to_gpu(uE), math.inf)
        e1, e2 = rel_l2(uI.cpu().numpy(), uE), rel_l2(up.cpu().numpy(), uE)
    log(f"round trip {M}x{N}: {e1:.2e} {e2:.2e}")
    assert e1 < 1e-6 and e2 < 1e-6


@pytest.mark.parametrize("M,N", SHAPES)
def test_spectral_solve_4096(M, N):
    u, y, s2 = problem(M, N, H_LARGE, seed=M + 2 * N)
    S = oracle_setup(y, H_LARGE, s2)
    rng = np.random.default_rng(12)
    uE = (u + 10 * rng.standard_normal((M, N))).astype(np.float32)
    UE = oracle.dft2(uE.astype(np.float64))
    with gfd.GFDeconv(to_gpu(y), to_gpu(H_LARGE.astype(np.float32)), s2, 17, 650.25) as g:
        for lam in (1e-3, 0.05, 3.0, 1e4):
            uI, up = g.spectral_solve(to_gpu(uE), lam)
            rI, rp = oracle.spectral_solve(S, UE, float(np.float32(lam)))
            eI, ep = rel_l2(uI.cpu().numpy(), rI), rel_l2(up.cpu().numpy(), rp)
            log(f"solve {M}x{N} lam={lam}: u_I {eI:.2e}, u_p {ep:.2e}")
            assert eI < 1e-5 and ep < 1e-5


@pytest.mark.parametrize("M,N", SHAPES)
def test_discrepancy_lambda_4096(M, N):
    u, y, s2 = problem(M, N, H_LARGE, seed=M + 3 * N)
    S = oracle_setup(y, H_LARGE, s2)
    rng = np.random.default_rng(13)
    with gfd.GFDeconv(to_gpu(y), to_gpu(H_LARGE.astype(np.float32)), s2, 17, 650.25) as g:
        assert math.isclose(g.info()["rho"], S.rho, rel_tol=1e-9)
        for uE in (np.zeros((M, N)), 0.9 * u + 3 * rng.standard_normal((M, N))):
            uE = uE.astype(np.float32)
            lam = float(g.discrepancy_lambda(to_gpu(uE)).cpu()[0])
            ref, flags = oracle.discrepancy_lambda(S, oracle.dft2(uE.astype(np.float64)))
            err = abs(lam - ref) / ref
            log(f"lambda {M}x{N}: gpu {lam:.9g} oracle {ref:.9g} rel {err:.2e}")
            assert flags == 0 and err < 1e-5


def strip_case(M, N, seed):
    """The large-frame workload's PSF, noise and filter on a narrow frame."""
    rng = np.random.default_rng(seed)
    u = synth.piecewise_image(M, N, rng)
    b = synth.blur_periodic(u, H_LARGE)
    y = (b + 2.0 * rng.standard_normal((M, N))).astype(np.float32)
    return synth.Case(f"strip_{M}x{N}", u, H_LARGE, y, 4.0, 17, synth.EPS_DEFAULT, 5)


@pytest.mark.parametrize("M,N", SHAPES)
def test_iteration_parity_4096_sides(M, N):
    c = strip_case(M, N, seed=5000 + M + N)
    r = run_trajectory(c, 5, log=log)
    report(f"{M}x{N} w=17", r, log)
    assert_parity(r)


def test_iteration_parity_4096x4096_large_frame():
    """The large-frame workload itself, 3 iterations, with the benchmark's launch shapes:
    trajectory and one-step checks from the oracle's first two iterates."""
    c = synth.make_case(5)
    log(f"{c.name}: sigma^2 {c.sigma2}, w {c.w}, eps {c.eps}")
    r = run_trajectory(c, 3, tuning=(104, 2, 2), log=log)
    report("4096x4096", r, log)
    assert_parity(r)
