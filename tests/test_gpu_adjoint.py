"""GPU reverse mode (deconv_backward through the C ABI) against the FP64 oracle's adjoint.

The oracle's adjoint is pinned to central finite differences and to an independent float64
autograd (tests/test_oracle_adjoint.py); here the FP32 GPU gradients with respect to eps and
the lambda scales must agree with it within 1e-4 relative (scale gradients: relative to the
largest of them).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import adjoint as adj
import paper_1609_01839_amd as gfd
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = 1e-4


def to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def problem(M, N, h, bsnr=30.0, seed=0):
    rng = np.random.default_rng(seed)
    u = synth.piecewise_image(M, N, rng)
    b = synth.blur_periodic(u, h)
    s2 = synth.sigma2_for_bsnr(b, bsnr)
    y = (b + math.sqrt(s2) * rng.standard_normal((M, N))).astype(np.float32)
    return u, y, float(s2)


def gpu_grad(y, h, s2, w, eps, iters, u_orig, scales=None, rho=None, u0=None, ckpt=5):
    with gfd.GFDeconv(to_gpu(y), to_gpu(h), s2, w, eps, rho) as g:
        if scales is not None:
            g.set_scales(scales)
        if u0 is not None:
            g.set_estimate(to_gpu(u0))
        u, lam = g.iterate(iters)
        gu = 2.0 * (u - to_gpu(u_orig)) / u.numel()
        ge, gs = g.backward(gu, ckpt)
        return float(ge.cpu()[0]), gs.cpu().numpy()[0].astype(np.float64), u.cpu().numpy(), lam.cpu().numpy()


def oracle_grad(y, h, s2, w, eps, iters, u_orig, scales=None, rho=None, u0=None):
    y64, h64 = y.astype(np.float64), h.astype(np.float32).astype(np.float64)
    uK, info = oracle.deconvolve(y64, h64, s2, w, eps, iters, rho=rho, scales=scales, u0=u0)
    g_u = adj.mse_loss_grad(uK, u_orig)[1]
    ge, gs, _ = adj.deconvolve_adjoint(y64, h64, s2, w, eps, iters, g_u, rho=rho, scales=scales, u0=u0)
    return ge, gs, uK, info


def compare(tag, ge, gs, re, rs):
    e_eps = abs(ge - re) / abs(re)
    e_s = float(np.max(np.abs(gs - rs)) / np.max(np.abs(rs))) if len(rs) else 0.0
    print(f"{tag}: g_eps gpu {ge:.7e} oracle {re:.7e} rel {e_eps:.1e}; g_s max rel {e_s:.1e}")
    return e_eps, e_s


@pytest.mark.parametrize("M,N,w,kind", [(64, 80, 5, "box"), (96, 96, 3, "gauss"), (256, 256, 5, "box"),
                                        (75, 90, 7, "gauss")])
def test_adjoint_matches_oracle(M, N, w, kind):
    h = synth.psf_box(9) if kind == "box" else synth.psf_gaussian(1.6, 25 if min(M, N) > 30 else 9)
    u, y, s2 = problem(M, N, h, seed=M + N)
    eps = float(np.float32(650.25))
    iters = 6
    scales = np.linspace(0.9, 1.1, iters)
    ge, gs, _, _ = gpu_grad(y, h, s2, w, eps, iters, u, scales=scales)
    re, rs, _, _ = oracle_grad(y, h, s2, w, eps, iters, u, scales=np.float32(scales).astype(np.float64))
    e_eps, e_s = compare(f"{M}x{N} w={w} {kind}", ge, gs, re, rs)
    assert e_eps < TOL and e_s < TOL


def test_adjoint_checkpoint_interval_is_exact():
    h = synth.psf_box(5)
    u, y, s2 = problem(80, 64, h, seed=3)
    res = [gpu_grad(y, h, s2, 5, 650.25, 7, u, ckpt=c)[:2] for c in (1, 2, 3, 0, 7, 10)]
    for ge, gs in res[1:]:
        assert ge == res[0][0]
        assert np.array_equal(gs, res[0][1])


def test_adjoint_through_infinite_lambda_branch():
    h = synth.psf_gaussian(1.2, 7)
    u, y, s2 = problem(64, 64, h, bsnr=25.0, seed=5)
    s2b = 1.5 * s2
    iters = 4
    u0 = u.astype(np.float32).astype(np.float64)
    ge, gs, _, lam = gpu_grad(y, h, s2b, 3, 650.25, iters, u, rho=1.0, u0=u0)
    re, rs, _, info = oracle_grad(y, h, s2b, 3, float(np.float32(650.25)), iters, u, rho=1.0, u0=u0)
    assert np.isinf(lam[0]) and info["flags"][0] & oracle.FLAG_INF_BRANCH
    assert gs[0] == 0.0 and rs[0] == 0.0
    e_eps, e_s = compare("inf branch", ge, gs, re, rs)
    assert e_eps < TOL and e_s < TOL


def test_adjoint_gradient_config_4():
    """The gradient workload itself: 1024^2 piecewise image, Gaussian PSF std 1.6 on 25x25,
    BSNR 30 dB, 20 unrolled iterations, checkpoints every 5; gradient of MSE(u_20, u_orig) with
    respect to eps and the 20 lambda scales against the FP64 oracle's adjoint."""
    c = synth.make_case(4)
    iters = c.iters
    assert iters == 20 and c.shape == (1024, 1024)
    h = c.h.astype(np.float32)
    ge, gs, _, _ = gpu_grad(c.y, h, c.sigma2, c.w, c.eps, iters, c.u_orig, ckpt=5)
    re, rs, _, _ = oracle_grad(c.y, h, c.sigma2, c.w, float(np.float32(c.eps)), iters, c.u_orig)
    e_eps, e_s = compare("1024^2, 20 iterations, checkpoints every 5", ge, gs, re, rs)
    assert e_eps < TOL and e_s < TOL


@pytest.mark.parametrize("M,N", [(4096, 64), (64, 4096)])
def test_adjoint_4096_sides(M, N):
    """The reverse mode through the 4096-point transforms (column passes over 4096-row tiles,
    4096-point row passes), large-frame PSF and filter (Gaussian std 2.5 on 31x31, w = 17)."""
    h = synth.psf_gaussian(2.5, 31)
    u, y, s2 = problem(M, N, h, seed=M + 7 * N)
    iters = 4
    scales = np.linspace(0.95, 1.05, iters)
    ge, gs, _, _ = gpu_grad(y, h, s2, 17, 650.25, iters, u, scales=scales, ckpt=2)
    re, rs, _, _ = oracle_grad(y, h, s2, 17, float(np.float32(650.25)), iters, u,
                               scales=np.float32(scales).astype(np.float64))
    e_eps, e_s = compare(f"{M}x{N} w=17", ge, gs, re, rs)
    assert e_eps < TOL and e_s < TOL


def test_batch_backward_equals_single_contexts():
    cases = synth.make_batch(4, sizes=[(64, 80), (96, 96), (256, 256), (75, 90)], config=17)
    probs = [dict(y=to_gpu(c.y), h=to_gpu(c.h.astype(np.float32)), sigma2=c.sigma2, w=c.w, eps=c.eps) for c in cases]
    iters = 3
    singles = []
    for p, c in zip(probs, cases):
        with gfd.GFDeconv(p["y"], p["h"], p["sigma2"], p["w"], p["eps"]) as g:
            uu, _ = g.iterate(iters)
            ge, gs = g.backward(2.0 * (uu - to_gpu(c.u_orig)) / uu.numel())
            singles.append((ge.cpu().numpy(), gs.cpu().numpy()))
    with gfd.GFDeconvBatch(probs) as g:
        us, _ = g.iterate(iters)
        gu = torch.cat([(2.0 * (x - to_gpu(c.u_orig)) / x.numel()).reshape(-1) for x, c in zip(us, cases)])
        ge, gs = g.backward(gu)
        ge, gs = ge.cpu().numpy(), gs.cpu().numpy()
    for b, (se, ss) in enumerate(singles):
        assert ge[b] == se[0] and np.array_equal(gs[b], ss[0]), b


def test_autograd_function():
    h = synth.psf_box(5)
    u, y, s2 = problem(64, 64, h, seed=9)
    iters = 4
    eps = torch.tensor(650.25, device=DEV, requires_grad=True)
    s = torch.ones(iters, device=DEV, requires_grad=True)
    uK = gfd.deconvolve_autograd(to_gpu(y), to_gpu(h), s2, 5, eps, iters, scales=s)
    loss = ((uK - to_gpu(u)) ** 2).mean()
    loss.backward()
    ge, gs, _, _ = gpu_grad(y, h, s2, 5, 650.25, iters, u)
    assert float(eps.grad) == pytest.approx(ge, rel=1e-6)
    assert np.allclose(s.grad.cpu().numpy(), gs, rtol=1e-5, atol=1e-6 * np.max(np.abs(gs)))
