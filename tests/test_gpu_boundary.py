"""GPU parity of the boundary variants against the FP64 oracle (oracle.boundary): the guided
filter with clipped windows, the iteration with clipped windows and/or a padded non-circular
observation, batches mixing the variants, and their reverse mode.  Bounds as for the periodic
path: iterates within 1e-5 relative L2, lambdas within 1e-4, gradients within 1e-4."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import adjoint as adj
from oracle import boundary as bd
import paper_1609_01839_amd as gfd
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("M,N,w", [(64, 64, 3), (300, 517, 3), (129, 260, 5), (70, 300, 17), (33, 1000, 9),
                                   (17, 17, 17), (97, 61, 1), (256, 256, 7)])
def test_clipped_guided_filter_parity(M, N, w):
    rng = np.random.default_rng(M * 13 + N + w)
    I = synth.piecewise_image(M, N, rng, n_shapes=8) + 5.0 * rng.standard_normal((M, N))
    p = I + 20.0 * rng.standard_normal((M, N))
    I32, p32 = I.astype(np.float32), p.astype(np.float32)
    eps = float(np.float32(650.25))
    out = gfd.guided_filter(to_gpu(I32), to_gpu(p32), w, eps, clip=True).cpu().numpy()
    ref = bd.guided_filter_clipped(I32.astype(np.float64), p32.astype(np.float64), w, eps)
    e = rel_l2(out, ref)
    emax = float(np.max(np.abs(out - ref)) / np.max(np.abs(ref)))
    print(f"clipped GF {M}x{N} w={w}: rel L2 {e:.2e}, max {emax:.2e}")
    assert e < 2e-6 and emax < 2e-5


def test_clipped_guided_filter_special_cases():
    c = np.full((40, 50), 93.5, np.float32)
    out = gfd.guided_filter(to_gpu(c), to_gpu(c), 5, 650.25, clip=True).cpu().numpy()
    assert np.max(np.abs(out - c)) < 1e-4  # flat image: the constant (count-normalised means)
    rng = np.random.default_rng(5)
    I = rng.uniform(0, 255, (40, 50)).astype(np.float32)
    p = rng.uniform(0, 255, (40, 50)).astype(np.float32)
    out = gfd.guided_filter(to_gpu(I), to_gpu(p), 1, 650.25, clip=True).cpu().numpy()
    assert np.max(np.abs(out - p)) < 1e-3
    # away from the borders the clipped and the periodic filters agree
    a = gfd.guided_filter(to_gpu(I), to_gpu(p), 5, 650.25, clip=True).cpu().numpy()
    b = gfd.guided_filter(to_gpu(I), to_gpu(p), 5, 650.25).cpu().numpy()
    assert np.max(np.abs(a[4:-4, 4:-4] - b[4:-4, 4:-4])) < 1e-3
    assert np.max(np.abs(a - b)) > 1.0


def trajectory(y, h, s2, w, eps, iters, clip, pad, rho=None):
    """GPU iterates (observed shape) and lambdas, one iteration per call."""
    us, lams = [], []
    with gfd.GFDeconv(to_gpu(y), to_gpu(h), s2, w, eps, rho, clip=clip, pad=pad) as g:
        for _ in range(iters):
            u, lam = g.iterate(1)
            us.append(u.cpu().numpy())
            lams.append(float(lam.cpu()[0]))
        info, dom = g.info(), g.domain
    return us, np.array(lams), info, dom


@pytest.mark.parametrize("clip,pad,shape,psf", [(True, False, (96, 160), "gauss"), (False, True, (100, 120), "gauss"),
                                                (True, True, (90, 75), "box"), (False, True, (250, 256), "box")])
def test_boundary_iteration_matches_oracle(clip, pad, shape, psf):
    M, N = shape
    h = synth.psf_gaussian(1.6, 7) if psf == "gauss" else synth.psf_box(9)
    u, y, s2 = synth.nonperiodic_case(M, N, h, 35.0, seed=M + N)
    eps = float(np.float32(48.77))
    iters = 8
    us, lams, info, dom = trajectory(y, h, s2, 3, eps, iters, clip, pad)
    ref, rinfo = bd.deconvolve_boundary(y.astype(np.float64), h.astype(np.float32).astype(np.float64), s2, 3, eps,
                                        iters, clip=clip, pad=pad, keep_iterates=True)
    assert dom == rinfo["shape"]
    assert info["target"] == pytest.approx(rinfo["T"], rel=1e-9) and info["rho"] == pytest.approx(rinfo["rho"], rel=1e-9)
    errs = [rel_l2(us[k], rinfo["iterates"][k][:M, :N]) for k in range(iters)]
    lam_err = float(np.max(np.abs(lams / rinfo["lam"] - 1.0)))
    print(f"clip={clip} pad={pad} {M}x{N} domain {dom}: max iterate rel L2 {max(errs):.1e}, lambda {lam_err:.1e}")
    assert max(errs) < 1e-5 and lam_err < 1e-4


def test_padded_estimate_is_extended_like_the_observation():
    h = synth.psf_gaussian(1.2, 5)
    u, y, s2 = synth.nonperiodic_case(60, 72, h, 35.0, seed=3)
    eps = float(np.float32(300.0))
    u0 = (0.5 * y).astype(np.float32)
    with gfd.GFDeconv(to_gpu(y), to_gpu(h), s2, 3, eps, pad=True) as g:
        g.set_estimate(to_gpu(u0))
        got, _ = g.iterate(3)
    ref, _ = bd.deconvolve_boundary(y.astype(np.float64), h.astype(np.float32).astype(np.float64), s2, 3, eps, 3,
                                    pad=True, u0=u0.astype(np.float64))
    e = rel_l2(got.cpu().numpy(), ref)
    print(f"padded, set estimate: rel L2 {e:.1e}")
    assert e < 1e-5


def test_batch_mixing_boundary_variants_equals_single_contexts():
    cases = []
    for b, (M, N, clip, pad) in enumerate([(64, 64, False, False), (64, 64, True, False), (60, 70, False, True),
                                           (72, 80, True, True), (128, 96, True, False)]):
        h = synth.psf_gaussian(1.4, 7)
        _, y, s2 = synth.nonperiodic_case(M, N, h, 30.0, seed=40 + b)
        cases.append(dict(y=to_gpu(y), h=to_gpu(h), sigma2=s2, w=5, eps=650.25, clip=clip, pad=pad))
    with gfd.GFDeconvBatch(cases) as gb:
        outs, lams = gb.iterate(5)
        outs = [o.cpu().numpy() for o in outs]
        lams = lams.cpu().numpy()
    for b, c in enumerate(cases):
        with gfd.GFDeconv(c["y"], c["h"], c["sigma2"], c["w"], c["eps"], clip=c["clip"], pad=c["pad"]) as g:
            u, lam = g.iterate(5)
        assert outs[b].shape == tuple(c["y"].shape)
        assert np.array_equal(outs[b], u.cpu().numpy()), b
        assert np.array_equal(lams[b], lam.cpu().numpy()), b


@pytest.mark.parametrize("clip,pad", [(True, False), (False, True), (True, True)])
def test_boundary_adjoint_matches_oracle(clip, pad):
    h = synth.psf_gaussian(1.6, 9)
    M, N = (80, 96) if not pad else (70, 90)
    u, y, s2 = synth.nonperiodic_case(M, N, h, 30.0, seed=17)
    eps = float(np.float32(650.25))
    iters = 6
    scales = np.linspace(0.9, 1.1, iters).astype(np.float32)
    with gfd.GFDeconv(to_gpu(y), to_gpu(h), s2, 5, eps, clip=clip, pad=pad) as g:
        g.set_scales(scales)
        uk, _ = g.iterate(iters)
        gu = 2.0 * (uk - to_gpu(u)) / uk.numel()
        ge, gs = g.backward(gu, 4)
    ge, gs = float(ge.cpu()[0]), gs.cpu().numpy()[0].astype(np.float64)
    y64, h64 = y.astype(np.float64), h.astype(np.float32).astype(np.float64)
    ref, _ = bd.deconvolve_boundary(y64, h64, s2, 5, eps, iters, clip=clip, pad=pad, scales=scales.astype(np.float64))
    g_u = adj.mse_loss_grad(ref, u)[1]
    re, rs = bd.deconvolve_boundary_adjoint(y64, h64, s2, 5, eps, iters, g_u, clip=clip, pad=pad,
                                            scales=scales.astype(np.float64))
    e_eps = abs(ge - re) / abs(re)
    e_s = float(np.max(np.abs(gs - rs)) / np.max(np.abs(rs)))
    print(f"clip={clip} pad={pad}: g_eps {ge:.6e} vs {re:.6e} ({e_eps:.1e}), g_s max rel {e_s:.1e}")
    assert e_eps < 1e-4 and e_s < 1e-4
