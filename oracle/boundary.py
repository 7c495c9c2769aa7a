"""Boundary variants of the iteration in FP64 (test infrastructure only).

The paper's solves (Eqs.(8)-(9)) diagonalise the blur with the DFT, i.e. they assume circular
convolution, and its guided filter (Eqs.(3)-(5)) divides every window sum by the fixed w^2.
Two variants for images that are not periodic:

* clipped windows: every box mean of the guided filter averages over the part of the w x w
  window that lies inside the image and divides by that part's pixel count.  The box operator
  becomes B = D^-1 S (S the clipped window sum, which is symmetric, D the counts), so its
  transpose is S D^-1, no longer B itself;
* padded observation: y (M x N, a non-circular blur) is placed in the top-left corner of an
  M' x N' domain, M' >= M + kh - 1 and N' >= N + kw - 1 the smallest sizes whose only prime
  factors are 2, 3 and 5, and the remaining pixels are filled so that the periodic extension is
  continuous: each row is first extended by a linear ramp from its last value towards its first,
  then each column of the widened image likewise.  The iteration runs on the padded domain, the
  discrepancy target counts only the observed pixels (T = rho M N sigma^2, rho of Eq.(12) from
  the observed y) and the estimate is cropped back to M x N.

Both are readings (the paper is silent on boundaries beyond its use of the DFT); each function
states the steps it takes.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .gfd import discrepancy_lambda, dft2, guided_filter, residual_energy, rho_eq12, setup, spectral_solve
from .adjoint import guided_filter_adjoint, solve_adjoint


# ----------------------------------------------------------------------------- clipped windows

def window_counts(M, N, w):
    """Pixels of the w x w window centred at each pixel that lie inside the M x N image."""
    r = (w - 1) // 2
    ny = np.array([min(m + r, M - 1) - max(m - r, 0) + 1 for m in range(M)], dtype=np.float64)
    nx = np.array([min(n + r, N - 1) - max(n - r, 0) + 1 for n in range(N)], dtype=np.float64)
    return np.outer(ny, nx)


def box_sum_clipped(x, w):
    """Sum of x over the part of the w x w window centred at each pixel inside the image."""
    x = np.asarray(x, dtype=np.float64)
    M, N = x.shape
    r = (w - 1) // 2
    z = np.zeros((M + 2 * r, N + 2 * r))
    z[r:r + M, r:r + N] = x
    acc = np.zeros_like(x)
    for di in range(w):
        for dj in range(w):
            acc += z[di:di + M, dj:dj + N]
    return acc


def box_mean_clipped(x, w):
    """B(x) = S(x) / counts: the mean over the window's pixels inside the image."""
    x = np.asarray(x, dtype=np.float64)
    return box_sum_clipped(x, w) / window_counts(*x.shape, w)


def box_mean_clipped_T(x, w):
    """Transpose of box_mean_clipped: S(x / counts)."""
    x = np.asarray(x, dtype=np.float64)
    return box_sum_clipped(x / window_counts(*x.shape, w), w)


def guided_filter_clipped(uI, up, w, eps):
    """Eqs.(3)-(5) with every window mean taken over the window's pixels inside the image."""
    B = lambda x: box_mean_clipped(x, w)
    I = np.asarray(uI, np.float64)
    p = np.asarray(up, np.float64)
    mu, pbar = B(I), B(p)
    var = B(I * I) - mu * mu
    cov = B(I * p) - mu * pbar
    a = cov / (var + eps)
    b = pbar - a * mu
    return B(a) * I + B(b)


def guided_filter_clipped_adjoint(uI, up, w, eps, g_u):
    """Reverse mode of guided_filter_clipped: the chain rule of Eqs.(3)-(5) with B^T = S D^-1
    wherever a gradient flows back through a window mean.  Returns (g_I, g_p, g_eps)."""
    B = lambda x: box_mean_clipped(x, w)
    Bt = lambda x: box_mean_clipped_T(x, w)
    I = np.asarray(uI, np.float64)
    p = np.asarray(up, np.float64)
    g_u = np.asarray(g_u, np.float64)
    mu, pbar = B(I), B(p)
    v = B(I * I) - mu * mu
    c = B(I * p) - mu * pbar
    a = c / (v + eps)
    # u = B(a) I + B(b)
    g_I = g_u * B(a)
    g_a = Bt(g_u * I)
    g_b = Bt(g_u)
    # b = pbar - a mu
    g_pbar = g_b.copy()
    g_a = g_a - g_b * mu
    g_mu = -g_b * a
    # a = c / (v + eps)
    g_c = g_a / (v + eps)
    g_v = -g_a * a / (v + eps)
    g_eps = float(np.sum(g_v))
    # c = B(I p) - mu pbar, v = B(I^2) - mu^2, mu = B(I), pbar = B(p)
    g_mu = g_mu - g_c * pbar - 2.0 * mu * g_v
    g_pbar = g_pbar - g_c * mu
    Btc = Bt(g_c)
    g_I = g_I + Bt(g_mu) + p * Btc + 2.0 * I * Bt(g_v)
    g_p = Bt(g_pbar) + I * Btc
    return g_I, g_p, g_eps


# ----------------------------------------------------------------------------- padding

def good_size(n):
    """The smallest m >= n whose only prime factors are 2, 3 and 5."""
    m = max(int(n), 1)
    while True:
        k = m
        for f in (2, 3, 5):
            while k % f == 0:
                k //= f
        if k == 1:
            return m
        m += 1


def padded_shape(M, N, kh, kw):
    return good_size(M + kh - 1), good_size(N + kw - 1)


def pad_observation(y, Mp, Np):
    """y in the top-left corner of an Mp x Np image whose periodic extension is continuous:
    columns N..Np-1 of row m ramp linearly from y[m, N-1] towards y[m, 0] (t / (Np - N + 1) of
    the way at column N - 1 + t), then rows M..Mp-1 ramp the same way between rows M-1 and 0 of
    the widened image."""
    y = np.asarray(y, dtype=np.float64)
    M, N = y.shape
    z = np.zeros((M, Np))
    z[:, :N] = y
    for t in range(1, Np - N + 1):
        z[:, N - 1 + t] = y[:, N - 1] + (y[:, 0] - y[:, N - 1]) * t / (Np - N + 1)
    out = np.zeros((Mp, Np))
    out[:M] = z
    for t in range(1, Mp - M + 1):
        out[M - 1 + t] = z[M - 1] + (z[0] - z[M - 1]) * t / (Mp - M + 1)
    return out


# ----------------------------------------------------------------------------- iteration

def boundary_setup(y, h, sigma2, rho=None, pad=False):
    """Constants of the iteration on the (possibly padded) domain, and the observed shape."""
    y = np.asarray(y, dtype=np.float64)
    M, N = y.shape
    if not pad:
        return setup(y, h, sigma2, rho), (M, N)
    kh, kw = np.asarray(h).shape
    Mp, Np = padded_shape(M, N, kh, kw)
    r = rho_eq12(y, h, sigma2) if rho is None else float(rho)
    S = setup(pad_observation(y, Mp, Np), h, sigma2, r)
    return dataclasses.replace(S, T=r * M * N * float(sigma2)), (M, N)


def boundary_step(S, uE, w, eps, clip, scale=1.0):
    """Steps 1-3 of Sec. 3.1 on the domain of S, with the periodic or the clipped filter."""
    UE = dft2(uE)
    lam_star, flags = discrepancy_lambda(S, UE)
    lam = lam_star if math.isinf(lam_star) else scale * lam_star
    uI, up = spectral_solve(S, UE, lam)
    u = (guided_filter_clipped if clip else guided_filter)(uI, up, w, eps)
    return u, uI, up, lam, lam_star, flags


def start_estimate(S, shape, u0, pad):
    """u_E^0: zeros, or u0 (y's shape) extended over the padding like y."""
    if u0 is None:
        return np.zeros((S.M, S.N))
    u0 = np.asarray(u0, np.float64)
    return pad_observation(u0, S.M, S.N) if pad else u0.copy()


def deconvolve_boundary(y, h, sigma2, w, eps, iters, rho=None, clip=False, pad=False, scales=None,
                        keep_iterates=False, u0=None):
    """The iteration from u_E = 0 (or u0) with clipped filter windows and/or a padded
    observation.  Returns (u cropped to y's shape, info with the lambda history and the
    iterates, uncropped)."""
    S, (M, N) = boundary_setup(y, h, sigma2, rho, pad)
    uE = start_estimate(S, (M, N), u0, pad)
    lams, flags_all, iterates, Es = [], [], [], []
    for k in range(iters):
        s = 1.0 if scales is None else float(scales[k])
        Es.append(residual_energy(math.inf, S, dft2(uE)))  # the E_inf of the branch test (reported only)
        uE, _, _, lam, _, flags = boundary_step(S, uE, w, eps, clip, s)
        lams.append(lam)
        flags_all.append(flags)
        if keep_iterates:
            iterates.append(uE)
    info = dict(lam=np.array(lams), flags=np.array(flags_all), rho=S.rho, T=S.T, shape=(S.M, S.N),
                iterates=iterates, E_inf=np.array(Es))
    return uE[:M, :N].copy(), info


def deconvolve_boundary_adjoint(y, h, sigma2, w, eps, iters, g_u, rho=None, clip=False, pad=False, scales=None,
                                u0=None):
    """Gradient of a loss through deconvolve_boundary given g_u = dLoss/du (observed shape):
    returns (g_eps, g_scales).  The crop's adjoint extends g_u by zeros; T and rho do not depend
    on eps or the scales, so the solves' adjoint is that of the periodic iteration."""
    S, (M, N) = boundary_setup(y, h, sigma2, rho, pad)
    s = np.ones(iters) if scales is None else np.asarray(scales, np.float64)
    pre = [start_estimate(S, (M, N), u0, pad)]
    steps = []
    for k in range(iters):
        r = boundary_step(S, pre[-1], w, eps, clip, float(s[k]))
        steps.append(r)
        pre.append(r[0])
    g = np.zeros((S.M, S.N))
    g[:M, :N] = np.asarray(g_u, np.float64)
    g_eps, g_s = 0.0, np.zeros(iters)
    gf_adj = guided_filter_clipped_adjoint if clip else guided_filter_adjoint
    for k in range(iters - 1, -1, -1):
        _, uI, up, lam, lam_star, flags = steps[k]
        g_I, g_p, ge = gf_adj(uI, up, w, eps, g)
        g_eps += ge
        g, g_s[k] = solve_adjoint(S, dft2(pre[k]), lam, lam_star, float(s[k]), flags, g_I, g_p)
    return g_eps, g_s
