"""GPU parity of the colour guided filter (three-channel guide) against the FP64 oracle.

Inputs are float32; the oracle runs in FP64 on the same float32 values.  The kernel forms the
window sums in compensated FP32 and solves each 3 x 3 system in FP64, so its error is that of
FP32 window means amplified by the conditioning of Sigma + eps U; with correlated channels
(natural-image-like guides) this stays within 1e-5 relative L2 and 1e-4 of the output's range
pixel by pixel.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1609_01839_amd as gfd
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
EPS_PAPER = 7.5e-4 * 255.0 ** 2  # Sec. 4's eps on the [0, 255] scale


def to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def colour_case(M, N, seed, spread=12.0):
    """A piecewise-constant luminance with three correlated channels and a noisy input p."""
    rng = np.random.default_rng(seed)
    base = synth.piecewise_image(M, N, rng, n_shapes=8)
    I3 = np.stack([0.9 * base + spread * rng.standard_normal((M, N)) + 10.0 * c for c in range(3)])
    p = base + 15.0 * rng.standard_normal((M, N))
    return I3.astype(np.float32), p.astype(np.float32)


def errors(out, ref):
    e = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    emax = float(np.max(np.abs(out - ref)) / (np.max(ref) - np.min(ref)))
    return e, emax


@pytest.mark.parametrize("M,N,w", [(64, 64, 3), (300, 517, 3), (129, 260, 5), (97, 61, 1), (70, 300, 17),
                                   (33, 1000, 9), (256, 256, 7)])
def test_guided_filter_color_parity(M, N, w):
    I3, p = colour_case(M, N, M * 31 + N + w)
    eps = float(np.float32(EPS_PAPER))
    out = gfd.guided_filter_color(to_gpu(I3), to_gpu(p), w, eps).cpu().numpy()
    ref = oracle.guided_filter_color(I3.astype(np.float64), p.astype(np.float64), w, eps)
    e, emax = errors(out, ref)
    print(f"colour GF {M}x{N} w={w}: rel L2 {e:.2e}, max {emax:.2e}")
    assert e < 1e-5 and emax < 1e-4


@pytest.mark.parametrize("eps", [1.0, 50.0, 1e4])
def test_guided_filter_color_eps_range(eps):
    I3, p = colour_case(200, 150, 7, spread=4.0)
    eps = float(np.float32(eps))
    out = gfd.guided_filter_color(to_gpu(I3), to_gpu(p), 5, eps).cpu().numpy()
    ref = oracle.guided_filter_color(I3.astype(np.float64), p.astype(np.float64), 5, eps)
    e, emax = errors(out, ref)
    print(f"colour GF eps={eps}: rel L2 {e:.2e}, max {emax:.2e}")
    assert e < 1e-5 and emax < 1e-4


def test_guided_filter_color_special_cases():
    rng = np.random.default_rng(3)
    p = rng.uniform(0, 255, (50, 70)).astype(np.float32)
    I3, _ = colour_case(50, 70, 4)
    # w = 1: a = 0, b = p
    out = gfd.guided_filter_color(to_gpu(I3), to_gpu(p), 1, 100.0).cpu().numpy()
    assert np.max(np.abs(out - p)) < 1e-3
    # constant guide: the output is the twice box-filtered input
    const = np.stack([np.full((50, 70), v, np.float32) for v in (10.0, 90.0, 200.0)])
    out = gfd.guided_filter_color(to_gpu(const), to_gpu(p), 5, 100.0).cpu().numpy()
    ref = oracle.box_mean(oracle.box_mean(p.astype(np.float64), 5), 5)
    assert np.max(np.abs(out - ref)) < 1e-3
    # flat input and guide: the constant comes back exactly
    c = np.full((40, 50), 93.5, np.float32)
    out = gfd.guided_filter_color(to_gpu(np.stack([c, c, c])), to_gpu(c), 5, 650.25).cpu().numpy()
    assert np.array_equal(out, c)
    # equal channels: the grey filter with eps / 3 (both from the oracle's definition)
    I, _ = colour_case(80, 90, 5)
    q = (I[0] + 10.0 * rng.standard_normal(I[0].shape)).astype(np.float32)
    out = gfd.guided_filter_color(to_gpu(np.stack([I[0]] * 3)), to_gpu(q), 3, 300.0).cpu().numpy()
    ref = oracle.guided_filter(I[0].astype(np.float64), q.astype(np.float64), 3, 100.0)
    e, emax = errors(out, ref)
    print(f"equal channels: rel L2 {e:.2e}, max {emax:.2e}")
    assert e < 1e-5 and emax < 1e-4


def test_guided_filter_color_4096_sampled():
    """4096 x 4096, w = 3: 32 x 32 patches gathered with periodic indices around sampled
    centres (corners included, so that the wrap is exercised); the oracle filters each patch
    periodically and its central 16 x 16 pixels, at least 2r from the patch's edges, are exact."""
    M = N = 4096
    w, r = 3, 1
    rng = np.random.default_rng(11)
    base = synth.piecewise_image(M, N, rng, n_shapes=40).astype(np.float32)
    noise = rng.standard_normal((4, M, N), dtype=np.float32)
    I3 = np.stack([0.9 * base + 12.0 * noise[c] + 10.0 * c for c in range(3)]).astype(np.float32)
    p = (base + 15.0 * noise[3]).astype(np.float32)
    del noise
    eps = float(np.float32(EPS_PAPER))
    out = gfd.guided_filter_color(to_gpu(I3), to_gpu(p), w, eps).cpu().numpy()
    centres = [(0, 0), (0, N - 1), (M - 1, 0), (M - 1, N - 1), (2048, 2048), (63, 64), (64, 251)]
    centres += [tuple(int(v) for v in rng.integers(0, 4096, 2)) for _ in range(9)]
    worst = 0.0
    for (cy, cx) in centres:
        ys = np.arange(cy - 16, cy + 16) % M
        xs = np.arange(cx - 16, cx + 16) % N
        Ip = I3[:, ys][:, :, xs].astype(np.float64)
        pp = p[ys][:, xs].astype(np.float64)
        ref = oracle.guided_filter_color(Ip, pp, w, eps)[8:24, 8:24]
        got = out[ys[8:24]][:, xs[8:24]]
        worst = max(worst, float(np.max(np.abs(got - ref))))
    print(f"4096^2 sampled: max abs error {worst:.2e}")
    assert worst < 1e-4 * 255.0
    assert 2 * r <= 8
