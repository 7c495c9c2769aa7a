"""FP64 reverse-mode derivative of the unrolled iteration (test infrastructure only).

The forward map is ``gfd.deconvolve``: K passes of Steps 1-3 (Sec. 3.1) with lambda from the
discrepancy principle (Sec. 3.2) and the guided filter of Sec. 2.  Given the gradient of a
loss with respect to the final estimate u^K, the functions here return the gradient with
respect to the guided-filter regulariser eps (shared by all iterations) and to the
per-iteration lambda scales s_k (lambda_k = s_k lambda*_k).  Everything is written by hand
from the chain rule, in the reverse order of the forward steps:

* guided filter (Eqs.(3)-(5)): the box mean B is its own transpose for centred odd periodic
  windows, so every backward box sum is again B;
* inverse / forward DFT: with the real inner product Re sum conj(A) B, the adjoint of
  x = F^-1 X is (1/P) F and the adjoint of X = F x is P F^-1;
* the two solves (Eqs.(8)-(9)) are affine in F(u_E) for fixed lambda, with real multipliers
  lam / (|H|^2 + lam) and lam D2 / (|H|^2 + lam D2); their lambda-derivatives are
  conj(H) R / (|H|^2 + lam)^2 and D2 conj(H) R / (|H|^2 + lam D2)^2 with R = H U_E - Y;
* lambda*: f(lambda*, U_E) = T (Eq.(11)) defines lambda* implicitly; T depends on y only, so
  d lambda* = -(df/dU_E . dU_E) / f'(lambda*) with df/dU_E = (2/P) g conj(H) R,
  g = (lambda / (|H|^2 + lambda))^2 and f' = (1/P) sum |R|^2 2 lambda |H|^2 / (|H|^2 + lambda)^3;
* on the branch lambda = +inf (u_E in K) the solves return u_E itself and lambda has no
  derivative; when lambda* is clamped at its floor it is a constant.
The branch decisions themselves (E_inf <= T, the floor) are piecewise constant.
"""
from __future__ import annotations

import math

import numpy as np

from .gfd import FLAG_INF_BRANCH, FLAG_NO_ROOT, box_mean, dft2, idft2, setup, step


def guided_filter_adjoint(uI, up, w, eps, g_u):
    """Reverse mode of u = guidfilter(u_I, u_p, w, eps) (Sec. 2, Eqs.(3)-(5)).

    Forward: mu = B(I), pbar = B(p), v = B(I^2) - mu^2, c = B(I p) - mu pbar,
    a = c / (v + eps), b = pbar - a mu, u = B(a) I + B(b).
    Returns (g_I, g_p, g_eps) for the incoming gradient g_u.
    """
    I = np.asarray(uI, np.float64)
    p = np.asarray(up, np.float64)
    g_u = np.asarray(g_u, np.float64)
    mu = box_mean(I, w)
    pbar = box_mean(p, w)
    v = box_mean(I * I, w) - mu * mu
    c = box_mean(I * p, w) - mu * pbar
    a = c / (v + eps)
    # u = abar * I + bbar
    g_I = g_u * box_mean(a, w)
    g_abar = g_u * I
    g_bbar = g_u
    g_a = box_mean(g_abar, w)
    g_b = box_mean(g_bbar, w)
    # b = pbar - a mu
    g_pbar = g_b.copy()
    g_a = g_a - g_b * mu
    g_mu = -g_b * a
    # a = c / (v + eps)
    g_c = g_a / (v + eps)
    g_v = -g_a * a / (v + eps)
    g_eps = float(np.sum(g_v))
    # c = B(I p) - mu pbar ; v = B(I^2) - mu^2
    g_mu = g_mu - g_c * pbar - 2.0 * mu * g_v
    g_pbar = g_pbar - g_c * mu
    Bc = box_mean(g_c, w)
    g_I = g_I + box_mean(g_mu, w) + p * Bc + 2.0 * I * box_mean(g_v, w)
    g_p = box_mean(g_pbar, w) + I * Bc
    return g_I, g_p, g_eps


def lambda_slope(S, UE, lam):
    """f'(lambda) = (1/P) sum |R|^2 2 lambda |H|^2 / (|H|^2 + lambda)^3, f of Eq.(11)."""
    P = S.M * S.N
    R2 = np.abs(S.H * UE - S.Y) ** 2
    H2 = np.abs(S.H) ** 2
    return float(np.sum(R2 * 2.0 * lam * H2 / (H2 + lam) ** 3) / P)


def solve_adjoint(S, UE, lam, lam_star, scale, flags, g_I, g_p):
    """Reverse mode of Step 1 (Eqs.(8)-(9)) including lambda_k = scale * lambda*(U_E).

    Returns (g_uE, g_scale): the gradient with respect to the pre-estimate u_E and to the
    scale s_k of this iteration.
    """
    g_I = np.asarray(g_I, np.float64)
    g_p = np.asarray(g_p, np.float64)
    if flags & FLAG_INF_BRANCH or math.isinf(lam):
        return g_I + g_p, 0.0
    P = S.M * S.N
    H2 = np.abs(S.H) ** 2
    R = S.H * UE - S.Y
    HR = np.conj(S.H) * R
    # adjoint of u = Re F^-1(U) on real gradients: G_U = (1/P) F(g)
    G_I = dft2(g_I) / P
    G_p = dft2(g_p) / P
    dI = H2 + lam * S.D2
    dp = H2 + lam
    G_UE = G_p * (lam / dp) + G_I * (lam * S.D2 / dI)
    g_lam = float(np.sum(np.real(np.conj(G_p) * HR / dp ** 2))
                  + np.sum(np.real(np.conj(G_I) * S.D2 * HR / dI ** 2)))
    g_scale = g_lam * lam_star
    if not (flags & FLAG_NO_ROOT):
        g_lam_star = g_lam * scale
        g = (lam_star / (H2 + lam_star)) ** 2
        fprime = lambda_slope(S, UE, lam_star)
        G_UE = G_UE - (g_lam_star / fprime) * (2.0 / P) * g * HR
    # adjoint of U_E = F(u_E): g_uE = Re(P F^-1(G_UE))
    g_uE = np.real(idft2(G_UE)) * P
    return g_uE, g_scale


def deconvolve_adjoint(y, h, sigma2, w, eps, iters, g_u, rho=None, scales=None, u0=None, checkpoint_every=None):
    """Gradient of a loss through ``gfd.deconvolve`` given g_u = dLoss/du^K.

    With ``checkpoint_every = c`` only every c-th pre-estimate is kept from the forward run
    and each segment is recomputed before it is differentiated (same arithmetic, so the
    result does not depend on c).  Returns (g_eps, g_scales[iters], g_u0).
    """
    y = np.asarray(y, np.float64)
    S = setup(y, h, sigma2, rho)
    s = np.ones(iters) if scales is None else np.asarray(scales, np.float64)
    c = iters if not checkpoint_every else int(checkpoint_every)
    uE = np.zeros_like(y) if u0 is None else np.asarray(u0, np.float64).copy()
    checkpoints = {}
    for k in range(iters):
        if k % c == 0:
            checkpoints[k] = uE.copy()
        uE = step(S, uE, w, eps, float(s[k])).u
    g = np.asarray(g_u, np.float64).copy()
    g_eps = 0.0
    g_s = np.zeros(iters)
    for k0 in sorted(checkpoints, reverse=True):
        k1 = min(k0 + c, iters)
        pre = [checkpoints[k0]]
        results = []
        for k in range(k0, k1):
            r = step(S, pre[-1], w, eps, float(s[k]))
            results.append(r)
            pre.append(r.u)
        for k in range(k1 - 1, k0 - 1, -1):
            r = results[k - k0]
            g_I, g_p, ge = guided_filter_adjoint(r.uI, r.up, w, eps, g)
            g_eps += ge
            g, g_s[k] = solve_adjoint(S, dft2(pre[k - k0]), r.lam, r.lam_star, float(s[k]), r.flags, g_I, g_p)
    return g_eps, g_s, g


def mse_loss_grad(u, u_orig):
    """Loss MSE(u, u_orig) = mean((u - u_orig)^2) and its gradient with respect to u."""
    d = np.asarray(u, np.float64) - np.asarray(u_orig, np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size
