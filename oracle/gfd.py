"""FP64 reference implementation of the deconvolution iteration (test infrastructure only).

Notation follows the paper: y observed image, h PSF, u_E pre-estimated image,
u_I guidance image (gradient-regularised solve), u_p filtering input
(identity-regularised solve), lambda regularisation parameter, w window side,
eps guided-filter regulariser, rho discrepancy factor.  Images are M x N and
P = M*N plays the role of the paper's N^2.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FLAG_INF_BRANCH = 1   # u_E already satisfied the discrepancy bound: lambda = +inf
FLAG_NO_ROOT = 2      # f(lambda) >= target even at the smallest lambda: lambda clamped


# ----------------------------------------------------------------------------- transforms

def dft2(x):
    """Unnormalised forward 2-D DFT, X[k,l] = sum x[m,n] exp(-2 pi i (km/M + ln/N)).

    Sec. 3.1: the two solves are carried out with the FFT under periodic convolution.
    """
    return np.fft.fft2(np.asarray(x, dtype=np.complex128))


def idft2(X):
    """Inverse of ``dft2`` (carries the 1/P factor)."""
    return np.fft.ifft2(np.asarray(X, dtype=np.complex128))


def embed_psf(h, M, N):
    """Periodic embedding of a centred odd-sized PSF, so that F(hp) F(u) = F(h * u).

    Eq.(1) models the blur as a convolution; with the FFT (Sec. 3.1) it is circular.
    Entry h[i + rh, j + rw] lands at ((i) mod M, (j) mod N).
    """
    h = np.asarray(h, dtype=np.float64)
    kh, kw = h.shape
    rh, rw = (kh - 1) // 2, (kw - 1) // 2
    hp = np.zeros((M, N))
    for i in range(kh):
        for j in range(kw):
            hp[(i - rh) % M, (j - rw) % N] += h[i, j]
    return hp


def grad_symbol(M, N):
    """|F(nabla)|^2 = |F(d_x)|^2 + |F(d_y)|^2 (Sec. 3.1, below Eqs.(8)-(9)).

    Reading: d_x and d_y are periodic forward differences, (d_x u)[m,n] = u[m,n+1] - u[m,n],
    written as convolution stencils and transformed with the same DFT.
    """
    kx = np.zeros((M, N))
    kx[0, 0] = -1.0
    kx[0, (-1) % N] += 1.0          # (k * u)[m,n] picks u[m, n+1] from k[0, -1]
    ky = np.zeros((M, N))
    ky[0, 0] = -1.0
    ky[(-1) % M, 0] += 1.0
    return np.abs(dft2(kx)) ** 2 + np.abs(dft2(ky)) ** 2


def rho_eq12(y, h, sigma2):
    """rho of Eq.(12): sqrt(1 - (||y - mean(y)||^2 - P sigma^2) / (||h||_1^2 ||y||^2)).

    Reading: the paper requires 0 < rho <= 1 (Sec. 3.2, definition of the set K), so the
    radicand is clipped to [1e-12, 1].
    """
    y = np.asarray(y, dtype=np.float64)
    P = y.size
    num = np.sum((y - y.mean()) ** 2) - P * sigma2
    den = np.sum(np.abs(h)) ** 2 * np.sum(y ** 2)
    return math.sqrt(min(max(1.0 - num / den, 1e-12), 1.0))


@dataclasses.dataclass
class Setup:
    """Per-image constants of the iteration (Step 0 plus the transforms of y and h)."""
    M: int
    N: int
    H: np.ndarray      # F(h), complex128 M x N
    Y: np.ndarray      # F(y)
    D2: np.ndarray     # |F(nabla)|^2
    rho: float
    sigma2: float
    T: float           # rho * P * sigma^2, the discrepancy target


def setup(y, h, sigma2, rho=None):
    """Constants for the iteration; ``rho=None`` takes Eq.(12)."""
    y = np.asarray(y, dtype=np.float64)
    M, N = y.shape
    H = dft2(embed_psf(h, M, N))
    Y = dft2(y)
    r = rho_eq12(y, h, sigma2) if rho is None else float(rho)
    return Setup(M, N, H, Y, grad_symbol(M, N), r, float(sigma2), r * M * N * float(sigma2))


# ----------------------------------------------------------------------------- lambda

def residual_energy(lam, S: Setup, UE):
    """||h * u_p - y||^2 as a function of lambda, Eq.(10), via Parseval.

    f(lam) = (1/P) sum |lam (H U_E - Y) / (|H|^2 + lam)|^2 ; lam = inf gives ||h * u_E - y||^2.
    Reading: with the unnormalised DFT, ||x||^2 = (1/P) sum |X|^2.
    """
    P = S.M * S.N
    R = S.H * UE - S.Y
    if math.isinf(lam):
        return float(np.sum(np.abs(R) ** 2) / P)
    return float(np.sum(np.abs(lam * R / (np.abs(S.H) ** 2 + lam)) ** 2) / P)


def discrepancy_lambda(S: Setup, UE, lam_floor=1e-30, max_steps=400):
    """lambda by the discrepancy principle (Sec. 3.2).

    If u_E lies in K = {u : ||h*u - y||^2 <= rho P sigma^2} the infinite branch is taken
    (reading: ties take the branch, as K is closed).  Otherwise the unique root of
    Eq.(11) is found by bisection, which the paper justifies by the monotonicity of the
    left-hand side.  Reading: the bisection runs on log(lambda) from a bracket grown by
    factors of 10 around lambda = 1, and stops when the bracket ratio is below 1 + 1e-14
    or f hits the target to 1e-13.  If even lambda_floor overshoots the target (possible
    only with exact spectral zeros of H or sigma^2 = 0), lambda_floor is returned with
    FLAG_NO_ROOT.  Returns (lambda_star, flags).
    """
    P = S.M * S.N
    R2 = np.abs(S.H * UE - S.Y) ** 2
    H2 = np.abs(S.H) ** 2
    T = S.T

    def f(lam):
        return float(np.sum(R2 * (lam / (H2 + lam)) ** 2) / P)

    if float(np.sum(R2) / P) <= T:
        return math.inf, FLAG_INF_BRANCH
    if f(lam_floor) >= T:
        return lam_floor, FLAG_NO_ROOT
    lo = hi = 1.0
    if f(1.0) > T:
        while f(lo) > T:
            lo = max(lo / 10.0, lam_floor)
        hi = min(lo * 10.0, 1.0)
    else:
        while f(hi) < T:
            hi *= 10.0
        lo = hi / 10.0
    for _ in range(max_steps):
        if hi / lo <= 1.0 + 1e-14:
            break
        mid = math.sqrt(lo * hi)
        fm = f(mid)
        if abs(fm / T - 1.0) <= 1e-13:
            return mid, 0
        if fm < T:
            lo = mid
        else:
            hi = mid
    return math.sqrt(lo * hi), 0


# ----------------------------------------------------------------------------- solves

def spectral_solve(S: Setup, UE, lam):
    """The two regularised least-squares solves, Eqs.(8)-(9), returning (u_I, u_p).

    F(u_I) = (conj(H) Y + lam |F(nabla)|^2 F(u_E)) / (|H|^2 + lam |F(nabla)|^2)   (Eq. 8)
    F(u_p) = (conj(H) Y + lam F(u_E)) / (|H|^2 + lam)                              (Eq. 9)
    lam = inf means u_I = u_p = u_E (Sec. 3.2).  Reading: one lambda serves both solves.
    """
    if math.isinf(lam):
        uE = np.real(idft2(UE))
        return uE.copy(), uE.copy()
    HY = np.conj(S.H) * S.Y
    H2 = np.abs(S.H) ** 2
    UI = (HY + lam * S.D2 * UE) / (H2 + lam * S.D2)
    Up = (HY + lam * UE) / (H2 + lam)
    uI, up = idft2(UI), idft2(Up)
    scale = max(np.max(np.abs(uI.real)), np.max(np.abs(up.real)), 1e-300)
    assert np.max(np.abs(uI.imag)) <= 1e-9 * scale and np.max(np.abs(up.imag)) <= 1e-9 * scale
    return uI.real.copy(), up.real.copy()


# ----------------------------------------------------------------------------- guided filter

def box_mean(x, w):
    """Mean of x over the w x w window centred at each pixel (Sec. 2, Eqs.(3)-(5)).

    Reading: windows wrap periodically, matching the periodic model of the solves, so every
    window holds exactly w^2 pixels and the paper's fixed 1/w^2 normaliser applies everywhere.
    The window sum is taken as a sum of column sums, one shift at a time.
    """
    x = np.asarray(x, dtype=np.float64)
    r = (w - 1) // 2
    rows = np.zeros_like(x)
    for dj in range(-r, r + 1):
        rows += np.roll(x, -dj, axis=1)          # rows[m, n] += x[m, n + dj]
    acc = np.zeros_like(x)
    for di in range(-r, r + 1):
        acc += np.roll(rows, -di, axis=0)        # acc[m, n] += rows[m + di, n]
    return acc / (w * w)


def guided_filter(uI, up, w, eps):
    """u = guidfilter(u_I, u_p, w, eps) (Sec. 2).

    a_k = (mean(u_I u_p) - mu_k pbar_k) / (sigma_k^2 + eps)       (Eq. 3)
    b_k = pbar_k - a_k mu_k                                          (Eq. 4)
    u(i) = abar_i u_I(i) + bbar_i, abar / bbar window means of a / b (Eq. 5)
    Reading: sigma_k^2 is the population variance (1/w^2) of u_I over the window.
    """
    mu = box_mean(uI, w)
    pbar = box_mean(up, w)
    var = box_mean(uI * uI, w) - mu * mu
    cov = box_mean(uI * up, w) - mu * pbar
    a = cov / (var + eps)
    b = pbar - a * mu
    return box_mean(a, w) * uI + box_mean(b, w)


def guided_filter_color(I3, up, w, eps):
    """Guided filter with a three-channel guide (the colour case of Sec. 3.1's complexity remark).

    Reading: the paper states that the filter has an exact linear-time algorithm for colour
    guidance images without writing it out; the multichannel generalisation of Eqs. (3)-(5) is
    taken: per window k, with the guide's channel means mu_k (3-vector) and window covariance
    Sigma_k (3x3, population), a_k = (Sigma_k + eps U)^-1 (mean(I p) - mu_k pbar_k),
    b_k = pbar_k - a_k . mu_k, and u(i) = abar_i . I(i) + bbar_i.  Each 3x3 system is solved by
    numpy.linalg.solve.
    """
    I3 = np.asarray(I3, dtype=np.float64)
    p = np.asarray(up, dtype=np.float64)
    mu = np.stack([box_mean(I3[c], w) for c in range(3)])
    pbar = box_mean(p, w)
    S = np.empty(p.shape + (3, 3))
    for c in range(3):
        for d in range(3):
            S[..., c, d] = box_mean(I3[c] * I3[d], w) - mu[c] * mu[d]
    S = S + eps * np.eye(3)
    cov = np.stack([box_mean(I3[c] * p, w) - mu[c] * pbar for c in range(3)], axis=-1)
    a = np.linalg.solve(S, cov[..., None])[..., 0]            # M x N x 3
    b = pbar - np.sum(a * np.moveaxis(mu, 0, -1), axis=-1)
    return sum(box_mean(a[..., c], w) * I3[c] for c in range(3)) + box_mean(b, w)


# ----------------------------------------------------------------------------- iteration

@dataclasses.dataclass
class StepResult:
    u: np.ndarray
    uI: np.ndarray
    up: np.ndarray
    lam: float          # lambda used in the solves (scale * lambda_star), inf on the branch
    lam_star: float
    flags: int
    E_inf: float        # ||h * u_E - y||^2


def step(S: Setup, uE, w, eps, scale=1.0):
    """One pass of Steps 1-3 of the algorithm (Sec. 3.1) from the pre-estimate u_E."""
    UE = dft2(uE)
    E_inf = residual_energy(math.inf, S, UE)
    lam_star, flags = discrepancy_lambda(S, UE)
    lam = lam_star if math.isinf(lam_star) else scale * lam_star
    uI, up = spectral_solve(S, UE, lam)
    u = guided_filter(uI, up, w, eps)
    return StepResult(u, uI, up, lam, lam_star, flags, E_inf)


def deconvolve(y, h, sigma2, w, eps, iters, rho=None, scales=None, u0=None, keep_iterates=False):
    """Steps 0-3 of the algorithm (Sec. 3.1) run for ``iters`` iterations from u_E^0 = 0.

    Returns (u, info) with info holding the lambda history, flags, E_inf history and,
    optionally, every iterate.  ``scales`` multiplies each iteration's lambda_star.
    """
    y = np.asarray(y, dtype=np.float64)
    S = setup(y, h, sigma2, rho)
    uE = np.zeros_like(y) if u0 is None else np.asarray(u0, dtype=np.float64).copy()
    lams, lam_stars, flags, Es, iterates = [], [], [], [], []
    for k in range(iters):
        s = 1.0 if scales is None else float(scales[k])
        r = step(S, uE, w, eps, s)
        lams.append(r.lam)
        lam_stars.append(r.lam_star)
        flags.append(r.flags)
        Es.append(r.E_inf)
        if keep_iterates:
            iterates.append(r.u)
        uE = r.u
    info = dict(lam=np.array(lams), lam_star=np.array(lam_stars), flags=np.array(flags),
                E_inf=np.array(Es), rho=S.rho, T=S.T, iterates=iterates)
    return uE, info


def isnr(u, y, u_orig):
    """Improvement in SNR, 10 log10(||y - u_orig||^2 / ||u - u_orig||^2) (dB)."""
    num = np.sum((np.asarray(y, np.float64) - u_orig) ** 2)
    den = np.sum((np.asarray(u, np.float64) - u_orig) ** 2)
    return 10.0 * math.log10(num / den)
