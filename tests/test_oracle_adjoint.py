"""Pins of the FP64 oracle's hand-written adjoint (reverse mode of the unrolled iteration).

The adjoint is checked against things it does not share code with: central finite
differences of the oracle's own forward map, an independent torch float64 autograd of the
same forward (with the implicit-function step for lambda), and special cases with known
gradients.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
import synth


def small_case(M=16, N=20, bsnr=30.0, seed=3, kind="gauss"):
    rng = np.random.default_rng(seed)
    u = synth.piecewise_image(M, N, rng, n_shapes=6)
    h = synth.psf_gaussian(1.2, 5) if kind == "gauss" else synth.psf_box(3)
    b = synth.blur_periodic(u, h)
    s2 = synth.sigma2_for_bsnr(b, bsnr)
    y = (b + math.sqrt(s2) * rng.standard_normal((M, N))).astype(np.float32).astype(np.float64)
    return u, y, h.astype(np.float64), s2


def test_guided_filter_adjoint_matches_central_differences():
    rng = np.random.default_rng(0)
    M, N, w, eps = 14, 17, 5, 300.0
    I = synth.piecewise_image(M, N, rng, n_shapes=4) + 8.0 * rng.standard_normal((M, N))
    p = I + 15.0 * rng.standard_normal((M, N))
    g_u = rng.standard_normal((M, N))
    dI, dp = rng.standard_normal((M, N)), rng.standard_normal((M, N))
    deps = 37.0
    gI, gp, geps = adj.guided_filter_adjoint(I, p, w, eps, g_u)
    lin = np.sum(gI * dI) + np.sum(gp * dp) + geps * deps

    def L(t):
        return np.sum(g_u * oracle.guided_filter(I + t * dI, p + t * dp, w, eps + t * deps))

    t = 1e-4
    fd = (L(t) - L(-t)) / (2 * t)
    assert abs(lin - fd) <= 1e-7 * abs(fd)
    # the eps component alone
    fe = (np.sum(g_u * oracle.guided_filter(I, p, w, eps + t)) - np.sum(g_u * oracle.guided_filter(I, p, w, eps - t))) / (2 * t)
    assert abs(geps - fe) <= 1e-7 * abs(fe)


def test_guided_filter_adjoint_w1_has_no_eps_gradient():
    rng = np.random.default_rng(1)
    I, p, g = rng.standard_normal((3, 9, 11))
    gI, gp, geps = adj.guided_filter_adjoint(I, p, 1, 2.0, g)
    assert geps == 0.0
    assert np.allclose(gp, g, rtol=0, atol=1e-15) and np.allclose(gI, 0.0, atol=1e-15)


def test_solve_adjoint_fixed_lambda_and_lambda_derivative():
    u, y, h, s2 = small_case()
    S = oracle.setup(y, h, s2)
    rng = np.random.default_rng(2)
    uE = u + 5.0 * rng.standard_normal(u.shape)
    gI, gp = rng.standard_normal((2,) + u.shape)
    lam = 0.37
    # flags = NO_ROOT: lambda is a constant of u_E, so only the affine solves are differentiated
    g_uE, g_s = adj.solve_adjoint(S, oracle.dft2(uE), lam, lam, 1.0, oracle.FLAG_NO_ROOT, gI, gp)

    def L(x, lm):
        a, b = oracle.spectral_solve(S, oracle.dft2(x), lm)
        return np.sum(gI * a) + np.sum(gp * b)

    d = rng.standard_normal(u.shape)
    t = 1e-3
    fd = (L(uE + t * d, lam) - L(uE - t * d, lam)) / (2 * t)
    assert abs(np.sum(g_uE * d) - fd) <= 1e-8 * abs(fd)
    tl = 1e-5 * lam
    fdl = (L(uE, lam + tl) - L(uE, lam - tl)) / (2 * tl)
    assert abs(g_s / lam - fdl) <= 1e-7 * abs(fdl)


def test_solve_adjoint_with_implicit_lambda():
    u, y, h, s2 = small_case()
    S = oracle.setup(y, h, s2)
    rng = np.random.default_rng(4)
    uE = u + 5.0 * rng.standard_normal(u.shape)
    gI, gp = rng.standard_normal((2,) + u.shape)
    scale = 0.8

    def L(x):
        UE = oracle.dft2(x)
        ls, fl = oracle.discrepancy_lambda(S, UE)
        assert fl == 0
        a, b = oracle.spectral_solve(S, UE, scale * ls)
        return np.sum(gI * a) + np.sum(gp * b)

    UE = oracle.dft2(uE)
    ls, fl = oracle.discrepancy_lambda(S, UE)
    g_uE, _ = adj.solve_adjoint(S, UE, scale * ls, ls, scale, fl, gI, gp)
    for seed in range(3):
        d = np.random.default_rng(10 + seed).standard_normal(u.shape)
        t = 1e-3          # truncation error ~ 4e-8 relative here, converging as t^2
        fd = (L(uE + t * d) - L(uE - t * d)) / (2 * t)
        assert abs(np.sum(g_uE * d) - fd) <= 3e-7 * abs(fd), (seed, np.sum(g_uE * d), fd)


def loss_of(case, eps, scales, iters, w=3, rho=None, u0=None):
    u, y, h, s2 = case
    uK, _ = oracle.deconvolve(y, h, s2, w, eps, iters, rho=rho, scales=scales, u0=u0)
    return adj.mse_loss_grad(uK, u)


@pytest.mark.parametrize("iters", [1, 4])
def test_full_adjoint_matches_central_differences(iters):
    """Relative step 1e-3 on eps and on every s_k; gradients within 1e-4 relative."""
    case = small_case()
    u, y, h, s2 = case
    eps = 650.25
    s = np.ones(iters)
    L0, g_u = loss_of(case, eps, s, iters)
    uK, _ = oracle.deconvolve(y, h, s2, 3, eps, iters, scales=s)
    g_eps, g_s, _ = adj.deconvolve_adjoint(y, h, s2, 3, eps, iters, adj.mse_loss_grad(uK, u)[1], scales=s)
    de = 1e-3 * eps
    fd_eps = (loss_of(case, eps + de, s, iters)[0] - loss_of(case, eps - de, s, iters)[0]) / (2 * de)
    print(f"g_eps {g_eps:.9e} fd {fd_eps:.9e}")
    assert abs(g_eps - fd_eps) <= 1e-4 * abs(fd_eps)
    for k in range(iters):
        sp, sm = s.copy(), s.copy()
        sp[k] += 1e-3
        sm[k] -= 1e-3
        fd = (loss_of(case, eps, sp, iters)[0] - loss_of(case, eps, sm, iters)[0]) / 2e-3
        print(f"g_s[{k}] {g_s[k]:.9e} fd {fd:.9e}")
        assert abs(g_s[k] - fd) <= 1e-4 * max(abs(fd), 1e-3 * np.max(np.abs(g_s)))


def test_adjoint_through_the_infinite_lambda_branch():
    """Start inside K (u_0 = original, target above the noise energy): iteration 0 takes the
    lambda = inf branch, later ones do not; the gradient still matches differences."""
    case = small_case(bsnr=25.0, seed=5)
    u, y, h, s2 = case
    s2b = 1.5 * s2
    iters = 3
    _, info = oracle.deconvolve(y, h, s2b, 3, 650.25, iters, rho=1.0, u0=u)
    assert info["flags"][0] & oracle.FLAG_INF_BRANCH
    assert not np.all(info["flags"] & oracle.FLAG_INF_BRANCH)
    c2 = (u, y, h, s2b)
    L0, g_u = loss_of(c2, 650.25, np.ones(iters), iters, rho=1.0, u0=u)
    g_eps, g_s, _ = adj.deconvolve_adjoint(y, h, s2b, 3, 650.25, iters, g_u, rho=1.0, u0=u)
    assert g_s[0] == 0.0
    de = 0.65025
    fd = (loss_of(c2, 650.25 + de, np.ones(iters), iters, rho=1.0, u0=u)[0]
          - loss_of(c2, 650.25 - de, np.ones(iters), iters, rho=1.0, u0=u)[0]) / (2 * de)
    assert abs(g_eps - fd) <= 1e-4 * abs(fd)


def test_checkpoint_interval_does_not_change_the_gradient():
    case = small_case(M=12, N=15)
    u, y, h, s2 = case
    iters = 6
    s = np.linspace(0.8, 1.2, iters)
    uK, _ = oracle.deconvolve(y, h, s2, 3, 650.25, iters, scales=s)
    g_u = adj.mse_loss_grad(uK, u)[1]
    ref = adj.deconvolve_adjoint(y, h, s2, 3, 650.25, iters, g_u, scales=s)
    for c in (1, 2, 4, 5):
        got = adj.deconvolve_adjoint(y, h, s2, 3, 650.25, iters, g_u, scales=s, checkpoint_every=c)
        assert got[0] == ref[0]
        assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])


def test_adjoint_matches_independent_torch_autograd():
    """torch float64 autograd of the same forward; lambda enters through one Newton step of
    f(lambda, U_E) = T at the (detached) root, which carries the implicit derivative."""
    torch = pytest.importorskip("torch")
    case = small_case(M=12, N=16, seed=7)
    u, y, h, s2 = case
    w, eps0, iters = 3, 650.25, 3
    S = oracle.setup(y, h, s2)
    P = y.size
    H = torch.from_numpy(S.H)
    Y = torch.from_numpy(S.Y)
    D2 = torch.from_numpy(S.D2)
    H2 = H.abs() ** 2
    eps = torch.tensor(eps0, dtype=torch.float64, requires_grad=True)
    s = torch.ones(iters, dtype=torch.float64, requires_grad=True)
    r = (w - 1) // 2

    def box(x):
        acc = torch.zeros_like(x)
        for di in range(-r, r + 1):
            for dj in range(-r, r + 1):
                acc = acc + torch.roll(x, shifts=(-di, -dj), dims=(0, 1))
        return acc / (w * w)

    def f_of(lam, UE):
        R2 = (H * UE - Y).abs() ** 2
        return (R2 * (lam / (H2 + lam)) ** 2).sum() / P

    uE = torch.zeros((12, 16), dtype=torch.float64)
    for k in range(iters):
        UE = torch.fft.fft2(uE.to(torch.complex128))
        ls, fl = oracle.discrepancy_lambda(S, UE.detach().numpy())
        assert fl == 0
        ls_t = torch.tensor(ls, dtype=torch.float64)
        fprime = adj.lambda_slope(S, UE.detach().numpy(), ls)
        lam_star = ls_t - (f_of(ls_t, UE) - S.T) / fprime
        lam = s[k] * lam_star
        HY = torch.conj(H) * Y
        uI = torch.fft.ifft2((HY + lam * D2 * UE) / (H2 + lam * D2)).real
        up = torch.fft.ifft2((HY + lam * UE) / (H2 + lam)).real
        mu, pb = box(uI), box(up)
        a = (box(uI * up) - mu * pb) / (box(uI * uI) - mu * mu + eps)
        b = pb - a * mu
        uE = box(a) * uI + box(b)
    loss = ((uE - torch.from_numpy(u)) ** 2).mean()
    loss.backward()
    g_u = adj.mse_loss_grad(uE.detach().numpy(), u)[1]
    g_eps, g_s, _ = adj.deconvolve_adjoint(y, h, s2, w, eps0, iters, g_u)
    print("torch", float(eps.grad), s.grad.numpy(), "oracle", g_eps, g_s)
    assert abs(g_eps - float(eps.grad)) <= 1e-8 * abs(float(eps.grad))
    assert np.allclose(g_s, s.grad.numpy(), rtol=1e-8, atol=1e-12 * np.max(np.abs(g_s)))
