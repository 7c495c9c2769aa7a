"""Seeded synthetic inputs shaped like the paper's test workloads.

This module draws images, point-spread functions and noise, and applies the
degradation model of the paper's Eq.(1) (periodic blur plus white Gaussian
noise) to produce the observation y.  It contains none of the deconvolution
method's arithmetic: no spectral solve, no regularisation-parameter search and
no guided filter.  Both the FP64 oracle and the GPU library are fed from here.

The paper's own test images (Cameraman, House; Sec. 4) are not available, so
piecewise-constant stand-ins of the same kind of content (flat regions with
sharp edges over a smooth background) are drawn instead.  Seeds follow
``numpy.random.default_rng(1000 * config + image_index)``; the draw order is
image, then PSF parameters, then noise.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "piecewise_image", "textured_image", "psf_box", "psf_gaussian", "psf_inverse_quadratic",
    "psf_binomial", "blur_periodic", "sigma2_for_bsnr", "Case", "make_case", "make_batch", "batch_case",
    "BATCH_SIZES", "TABLE1_SETTINGS", "table1_case",
]


# ----------------------------------------------------------------------------- images

def piecewise_image(M: int, N: int, rng: np.random.Generator, n_shapes: int = 20) -> np.ndarray:
    """Linear-gradient background with ``n_shapes`` constant rectangles / disks, values in [0, 255]."""
    g0, g1 = rng.uniform(0.0, 255.0, size=2)
    theta = rng.uniform(0.0, 2.0 * math.pi)
    yy, xx = np.meshgrid(np.arange(M, dtype=np.float64), np.arange(N, dtype=np.float64), indexing="ij")
    proj = xx * math.cos(theta) + yy * math.sin(theta)
    t = (proj - proj.min()) / max(proj.max() - proj.min(), 1e-300)
    img = g0 + (g1 - g0) * t
    side = min(M, N)
    for _ in range(n_shapes):
        is_rect = rng.uniform() < 0.5
        val = rng.uniform(0.0, 255.0)
        cy, cx = rng.uniform(0, M), rng.uniform(0, N)
        if is_rect:
            hy, hx = rng.uniform(side / 16.0, side / 4.0, size=2) / 2.0
            mask = (np.abs(yy - cy) <= hy) & (np.abs(xx - cx) <= hx)
        else:
            rad = rng.uniform(side / 32.0, side / 8.0)
            mask = (yy - cy) ** 2 + (xx - cx) ** 2 <= rad * rad
        img[mask] = val
    return img


def _gaussian_lowpass_periodic(x: np.ndarray, std: float) -> np.ndarray:
    """Circular Gaussian low-pass (input texture synthesis only)."""
    M, N = x.shape
    ky = np.fft.fftfreq(M)[:, None]
    kx = np.fft.fftfreq(N)[None, :]
    g = np.exp(-2.0 * (math.pi * std) ** 2 * (ky ** 2 + kx ** 2))
    return np.real(np.fft.ifft2(np.fft.fft2(x) * g))


def textured_image(M: int, N: int, rng: np.random.Generator, texture_std: float = 10.0) -> np.ndarray:
    """Piecewise image plus band-limited Gaussian texture, clipped to [0, 255]."""
    img = piecewise_image(M, N, rng)
    tex = _gaussian_lowpass_periodic(rng.standard_normal((M, N)), 2.0)
    tex /= max(tex.std(), 1e-300)
    return np.clip(img + texture_std * tex, 0.0, 255.0)


# ----------------------------------------------------------------------------- PSFs

def psf_box(k: int) -> np.ndarray:
    """k x k uniform (boxcar) kernel."""
    return np.full((k, k), 1.0 / (k * k))


def psf_gaussian(std: float, k: int) -> np.ndarray:
    """k x k sampled Gaussian with standard deviation ``std`` (pixels), normalised to sum 1."""
    r = (k - 1) // 2
    i = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2.0 * std * std))
    return g / g.sum()


def psf_inverse_quadratic(k: int = 15, normalise: bool = True) -> np.ndarray:
    """h(i, j) = 1 / (1 + i^2 + j^2) for |i|, |j| <= (k-1)/2 (Table 1, tests 1-2)."""
    r = (k - 1) // 2
    i = np.arange(-r, r + 1, dtype=np.float64)
    h = 1.0 / (1.0 + i[:, None] ** 2 + i[None, :] ** 2)
    return h / h.sum() if normalise else h


def psf_binomial() -> np.ndarray:
    """[1 4 6 4 1]^T [1 4 6 4 1] / 256 (Table 1, test 4)."""
    v = np.array([1.0, 4.0, 6.0, 4.0, 1.0])
    return np.outer(v, v) / 256.0


# ----------------------------------------------------------------------------- degradation model

def blur_periodic(u: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Circular convolution h * u with a centred odd-sized kernel (Eq.(1) without noise)."""
    M, N = u.shape
    kh, kw = h.shape
    hp = np.zeros((M, N))
    rh, rw = (kh - 1) // 2, (kw - 1) // 2
    for i in range(kh):
        for j in range(kw):
            hp[(i - rh) % M, (j - rw) % N] += h[i, j]
    return np.real(np.fft.ifft2(np.fft.fft2(u) * np.fft.fft2(hp)))


def nonperiodic_case(M: int, N: int, h: np.ndarray, bsnr_db: float, seed: int, n_shapes: int = 12):
    """A scene larger than the frame, blurred, then cropped: y (float32, M x N) is a blurred
    view of u (M x N) whose blur reaches pixels outside the frame, i.e. not circular.
    Returns (u, y, sigma2)."""
    rng = np.random.default_rng(seed)
    kh, kw = h.shape
    mh, mw = kh, kw  # scene margin: at least the PSF's half-size on every side
    scene = piecewise_image(M + 2 * mh, N + 2 * mw, rng, n_shapes=n_shapes)
    b = blur_periodic(scene, h)[mh:mh + M, mw:mw + N]
    sigma2 = sigma2_for_bsnr(b, bsnr_db)
    y = (b + math.sqrt(sigma2) * rng.standard_normal((M, N))).astype(np.float32)
    return scene[mh:mh + M, mw:mw + N].copy(), y, float(sigma2)


def sigma2_for_bsnr(blurred: np.ndarray, bsnr_db: float) -> float:
    """Noise variance giving BSNR = 10 log10(var(h*u) / sigma^2) (population variance)."""
    return float(np.var(blurred) / (10.0 ** (bsnr_db / 10.0)))


@dataclasses.dataclass
class Case:
    """One deconvolution problem instance."""
    name: str
    u_orig: np.ndarray        # float64, M x N
    h: np.ndarray             # float64, kh x kw, odd sizes, centred
    y: np.ndarray             # float32, M x N (the FP32-rounded observation fed to both sides)
    sigma2: float
    w: int
    eps: float
    iters: int

    @property
    def shape(self):
        return self.u_orig.shape


EPS_DEFAULT = 1e-2 * 255.0 ** 2   # 650.25 on the [0, 255] scale

BATCH_SIZES = [(256, 256), (480, 640), (512, 512), (720, 1280), (1024, 1024)]


def _observe(u: np.ndarray, h: np.ndarray, rng: np.random.Generator, *, sigma2=None, bsnr_db=None):
    b = blur_periodic(u, h)
    if sigma2 is None:
        sigma2 = sigma2_for_bsnr(b, bsnr_db)
    y = b + math.sqrt(sigma2) * rng.standard_normal(u.shape)
    return y.astype(np.float32), float(sigma2)


def make_case(config: int, size=None, image_index: int = 0) -> Case:
    """Synthetic stand-in for one of the single-image workloads.

    config 1: 256^2 piecewise image, 9x9 box PSF, BSNR 40 dB, w=5, 10 iterations.
    config 2: 1024^2 textured image, 15x15 1/(1+x^2+y^2) PSF, sigma^2=2, w=7, 30 iterations.
    config 4: 1024^2 piecewise image, Gaussian std 1.6 on 25x25, BSNR 30 dB, w=7, 20 iterations.
    config 5: 4096^2 piecewise image, Gaussian std 2.5 on 31x31, sigma^2=4, w=17, 50 iterations.
    ``size`` overrides (M, N) keeping everything else (used for small test instances).
    """
    rng = np.random.default_rng(1000 * config + image_index)
    if config == 1:
        M, N = size or (256, 256)
        u = piecewise_image(M, N, rng)
        h = psf_box(9)
        y, s2 = _observe(u, h, rng, bsnr_db=40.0)
        return Case("c1_256_box9", u, h, y, s2, 5, EPS_DEFAULT, 10)
    if config == 2:
        M, N = size or (1024, 1024)
        u = textured_image(M, N, rng)
        h = psf_inverse_quadratic(15)
        y, s2 = _observe(u, h, rng, sigma2=2.0)
        return Case("c2_1024_invquad15", u, h, y, s2, 7, EPS_DEFAULT, 30)
    if config == 4:
        M, N = size or (1024, 1024)
        u = piecewise_image(M, N, rng)
        h = psf_gaussian(1.6, 25)
        y, s2 = _observe(u, h, rng, bsnr_db=30.0)
        return Case("c4_1024_gauss1.6", u, h, y, s2, 7, EPS_DEFAULT, 20)
    if config == 5:
        M, N = size or (4096, 4096)
        u = piecewise_image(M, N, rng)
        h = psf_gaussian(2.5, 31)
        y, s2 = _observe(u, h, rng, sigma2=4.0)
        return Case("c5_4096_gauss2.5", u, h, y, s2, 17, EPS_DEFAULT, 50)
    raise ValueError(f"no single-image workload for config {config}")


def batch_case(k: int, sizes=None, config: int = 3) -> Case:
    """Image k of the mixed-size batch: size, PSF, BSNR in [20, 40] dB and w in {5, 7, 9} drawn
    from its own seed (so any image can be made on its own)."""
    sizes = sizes or BATCH_SIZES
    rng = np.random.default_rng(1000 * config + k)
    M, N = sizes[int(rng.integers(len(sizes)))]
    u = piecewise_image(M, N, rng)
    kind = int(rng.integers(3))
    if kind == 0:
        h = psf_box(9)
    elif kind == 1:
        h = psf_gaussian(float(rng.uniform(1.0, 3.0)), 25)
    else:
        h = psf_inverse_quadratic(15)
    w = int(rng.choice([5, 7, 9]))
    bsnr = float(rng.uniform(20.0, 40.0))
    y, s2 = _observe(u, h, rng, bsnr_db=bsnr)
    return Case(f"b{k}_{M}x{N}_psf{kind}", u, h, y, s2, w, EPS_DEFAULT, 20)


def make_batch(n: int = 64, sizes=None, config: int = 3) -> list:
    """Mixed-size batch of n images (batch_case 0 .. n-1)."""
    return [batch_case(k, sizes, config) for k in range(n)]


# Table 1 of the paper: PSF and noise variance (on the [0, 255] scale) of the five settings.
TABLE1_SETTINGS = {
    1: ("inverse_quadratic_15", 2.0),
    2: ("inverse_quadratic_15", 8.0),
    3: ("box_9", 0.308),
    4: ("binomial_5", 49.0),
    5: ("gaussian_1.6", 4.0),
}


def table1_case(test: int, M: int = 256, N: int = 256, seed: int = 0) -> Case:
    """Stand-in image blurred and corrupted as in one of Table 1's settings (eps, w of Sec. 4)."""
    kind, s2 = TABLE1_SETTINGS[test]
    h = {"inverse_quadratic_15": lambda: psf_inverse_quadratic(15),
         "box_9": lambda: psf_box(9),
         "binomial_5": psf_binomial,
         "gaussian_1.6": lambda: psf_gaussian(1.6, 25)}[kind]()
    rng = np.random.default_rng(6000 + 10 * test + seed)
    u = piecewise_image(M, N, rng)
    y, s2 = _observe(u, h, rng, sigma2=s2)
    return Case(f"t{test}_{M}x{N}", u, h, y, s2, 3, 7.5e-4 * 255.0 ** 2, 30)
