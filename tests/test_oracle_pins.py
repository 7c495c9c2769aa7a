"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test compares the oracle with an independent computation (brute force, dense
linear algebra, a closed form or an invariant), chosen so that a plausible slip in
the oracle -- a flipped kernel, a wrong normaliser, a swapped guide/input, a missing
term -- fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.optimize

import oracle
import synth

rng0 = np.random.default_rng(12345)


# ----------------------------------------------------------------------------- brute-force helpers

def direct_dft2(x):
    """O(P^2) DFT from its definition (independent of any FFT algorithm)."""
    M, N = x.shape
    m = np.arange(M)
    n = np.arange(N)
    Wm = np.exp(-2j * np.pi * np.outer(m, m) / M)
    Wn = np.exp(-2j * np.pi * np.outer(n, n) / N)
    out = np.zeros((M, N), dtype=complex)
    for k in range(M):
        for l in range(N):
            out[k, l] = np.sum(x * Wm[k][:, None] * Wn[l][None, :])
    return out


def direct_circular_conv(h, u):
    """(h * u)[m, n] = sum_{i,j} h(i, j) u[(m - i) mod M, (n - j) mod N], h centred, by loops."""
    M, N = u.shape
    kh, kw = h.shape
    rh, rw = (kh - 1) // 2, (kw - 1) // 2
    out = np.zeros((M, N))
    for m in range(M):
        for n in range(N):
            s = 0.0
            for a in range(kh):
                for b in range(kw):
                    s += h[a, b] * u[(m - (a - rh)) % M, (n - (b - rw)) % N]
            out[m, n] = s
    return out


def brute_box_mean(x, w):
    M, N = x.shape
    r = (w - 1) // 2
    out = np.zeros((M, N))
    for m in range(M):
        for n in range(N):
            s = 0.0
            for di in range(-r, r + 1):
                for dj in range(-r, r + 1):
                    s += x[(m + di) % M, (n + dj) % N]
            out[m, n] = s / (w * w)
    return out


def circulant_matrix(h, M, N):
    """Dense P x P matrix A with (A u) = h * u (circular), built entry by entry."""
    P = M * N
    A = np.zeros((P, P))
    kh, kw = h.shape
    rh, rw = (kh - 1) // 2, (kw - 1) // 2
    for m in range(M):
        for n in range(N):
            for a in range(kh):
                for b in range(kw):
                    A[m * N + n, ((m - (a - rh)) % M) * N + (n - (b - rw)) % N] += h[a, b]
    return A


def forward_diff_matrices(M, N):
    P = M * N
    Dx = np.zeros((P, P))
    Dy = np.zeros((P, P))
    for m in range(M):
        for n in range(N):
            i = m * N + n
            Dx[i, i] -= 1.0
            Dx[i, m * N + (n + 1) % N] += 1.0
            Dy[i, i] -= 1.0
            Dy[i, ((m + 1) % M) * N + n] += 1.0
    return Dx, Dy


ASYM_H = np.array([[0.05, 0.10, 0.02], [0.20, 0.30, 0.08], [0.01, 0.15, 0.09]])  # catches flips


# ----------------------------------------------------------------------------- O1: DFT

@pytest.mark.parametrize("M,N", [(6, 10), (9, 8), (12, 15), (16, 20), (5, 3)])
def test_dft_equals_direct_definition(M, N):
    x = rng0.standard_normal((M, N))
    X = oracle.dft2(x)
    np.testing.assert_allclose(X, direct_dft2(x), rtol=0, atol=1e-11 * np.abs(X).max())
    np.testing.assert_allclose(oracle.idft2(X).real, x, atol=1e-13)
    # Parseval with the unnormalised forward transform
    assert math.isclose(np.sum(x ** 2), np.sum(np.abs(X) ** 2) / (M * N), rel_tol=1e-12)


@pytest.mark.parametrize("M,N,h", [(7, 9, ASYM_H), (10, 6, synth.psf_box(3)), (12, 15, synth.psf_gaussian(1.0, 5))])
def test_psf_embedding_gives_circular_convolution(M, N, h):
    u = rng0.uniform(0, 255, (M, N))
    via_fft = np.real(oracle.idft2(oracle.dft2(oracle.embed_psf(h, M, N)) * oracle.dft2(u)))
    np.testing.assert_allclose(via_fft, direct_circular_conv(h, u), rtol=0, atol=1e-10)


def test_psf_embedding_wraps_kernels_larger_than_half_the_image():
    h = rng0.uniform(0, 1, (5, 5))
    u = rng0.standard_normal((4, 6))
    via_fft = np.real(oracle.idft2(oracle.dft2(oracle.embed_psf(h, 4, 6)) * oracle.dft2(u)))
    np.testing.assert_allclose(via_fft, direct_circular_conv(h, u), atol=1e-12)


# ----------------------------------------------------------------------------- O3: gradient symbol

@pytest.mark.parametrize("M,N", [(8, 8), (6, 10), (15, 9)])
def test_gradient_symbol_closed_form_and_spatial_energy(M, N):
    D2 = oracle.grad_symbol(M, N)
    k = np.arange(M)[:, None]
    l = np.arange(N)[None, :]
    closed = 4 * np.sin(np.pi * k / M) ** 2 + 4 * np.sin(np.pi * l / N) ** 2
    np.testing.assert_allclose(D2, closed, atol=1e-12)
    u = rng0.standard_normal((M, N))
    gx = np.roll(u, -1, axis=1) - u
    gy = np.roll(u, -1, axis=0) - u
    spatial = np.sum(gx ** 2 + gy ** 2)
    assert math.isclose(spatial, np.sum(D2 * np.abs(oracle.dft2(u)) ** 2) / (M * N), rel_tol=1e-12)


# ----------------------------------------------------------------------------- O4: rho

def test_rho_hand_computed_value_and_clipping():
    y = np.array([[1.0, 2.0], [3.0, 4.0]])
    h = np.array([[1.0]])
    # ||y - mean||^2 = 5, P sigma^2 = 1, ||h||_1^2 ||y||^2 = 30  ->  rho = sqrt(1 - 4/30)
    assert math.isclose(oracle.rho_eq12(y, h, 0.25), math.sqrt(1 - 4 / 30), rel_tol=1e-15)
    # negative-PSF entries count through |h|: ||h||_1 = 2
    assert math.isclose(oracle.rho_eq12(y, np.array([[1.5, -0.5]]), 0.25), math.sqrt(1 - 4 / 120), rel_tol=1e-15)
    # noise power above the image variance: radicand > 1, clipped to 1
    assert oracle.rho_eq12(y, h, 10.0) == 1.0
    # huge variance against a tiny ||h||_1: radicand < 0, clipped to 1e-12
    assert math.isclose(oracle.rho_eq12(y, np.array([[1e-3]]), 0.0), 1e-6, rel_tol=1e-12)


def test_rho_scale_invariance():
    y = rng0.uniform(0, 255, (16, 12))
    h = synth.psf_box(3)
    r1 = oracle.rho_eq12(y, h, 3.0)
    r2 = oracle.rho_eq12(7.5 * y, h, 7.5 ** 2 * 3.0)
    assert math.isclose(r1, r2, rel_tol=1e-13)
    assert 0 < r1 <= 1


# ----------------------------------------------------------------------------- O5: lambda

def _small_problem(M=10, N=12, h=ASYM_H, sigma2=4.0, seed=3):
    rng = np.random.default_rng(seed)
    u = synth.piecewise_image(M, N, rng, n_shapes=3)
    y = direct_circular_conv(h, u) + math.sqrt(sigma2) * rng.standard_normal((M, N))
    return u, y


@pytest.mark.parametrize("rho", [1.0, None])
def test_lambda_meets_discrepancy_spatially(rho):
    h = ASYM_H
    u, y = _small_problem(h=h)
    S = oracle.setup(y, h, 4.0, rho)
    uE = 0.5 * u + 3.0                       # some pre-estimate outside K
    UE = oracle.dft2(uE)
    lam, flags = oracle.discrepancy_lambda(S, UE)
    assert flags == 0 and 0 < lam < math.inf
    _, up = oracle.spectral_solve(S, UE, lam)
    resid = np.sum((y - direct_circular_conv(h, up)) ** 2)
    assert math.isclose(resid, S.T, rel_tol=1e-10)


def test_residual_energy_monotone_and_bounded_by_lambda_infinity():
    h = ASYM_H
    u, y = _small_problem(h=h)
    S = oracle.setup(y, h, 4.0, 1.0)
    uE = np.zeros_like(y) + 10.0
    UE = oracle.dft2(uE)
    f_inf = oracle.residual_energy(math.inf, S, UE)
    assert math.isclose(f_inf, np.sum((direct_circular_conv(h, uE) - y) ** 2), rel_tol=1e-12)
    grid = np.logspace(-8, 8, 200)
    vals = np.array([oracle.residual_energy(l, S, UE) for l in grid])
    assert np.all(np.diff(vals) > 0)
    assert np.all(vals <= f_inf * (1 + 1e-14))                  # Eq.(10) inequality
    # the spectral formula of Eq.(10) equals the spatial residual of the solve at each lambda
    for lam in (1e-3, 0.7, 50.0):
        _, up = oracle.spectral_solve(S, UE, lam)
        spatial = np.sum((direct_circular_conv(h, up) - y) ** 2)
        assert math.isclose(oracle.residual_energy(lam, S, UE), spatial, rel_tol=1e-11)


@pytest.mark.parametrize("M,N,h", [(5, 6, ASYM_H), (6, 6, synth.psf_box(3)), (4, 5, synth.psf_gaussian(0.8, 3))])
def test_lambda_and_solves_equal_dense_normal_equations(M, N, h):
    rng = np.random.default_rng(M * 100 + N)
    u = rng.uniform(0, 255, (M, N))
    A = circulant_matrix(h, M, N)
    y = (A @ u.ravel()).reshape(M, N) + 2.0 * rng.standard_normal((M, N))
    uE = rng.uniform(0, 255, (M, N))
    T = 0.5 * np.sum((A @ uE.ravel() - y.ravel()) ** 2) + 1e-3   # a target strictly inside (0, f(inf))
    S = oracle.setup(y, h, 1.0, 1.0)
    S.T = T
    AtA = A.T @ A
    Aty = A.T @ y.ravel()
    I = np.eye(M * N)

    def dense_up(lam):
        return np.linalg.solve(AtA + lam * I, Aty + lam * uE.ravel())

    def g(lam_log):
        up = dense_up(math.exp(lam_log))
        return np.sum((A @ up - y.ravel()) ** 2) - T

    lam_dense = math.exp(scipy.optimize.brentq(g, -40, 40, xtol=1e-14, rtol=1e-14))
    UE = oracle.dft2(uE)
    lam, flags = oracle.discrepancy_lambda(S, UE)
    assert flags == 0
    assert math.isclose(lam, lam_dense, rel_tol=1e-8)
    # Eq.(9) equals the identity-regularised normal equations; Eq.(8) the gradient-regularised ones
    uI, up = oracle.spectral_solve(S, UE, lam)
    np.testing.assert_allclose(up.ravel(), dense_up(lam), atol=1e-9 * np.abs(up).max())
    Dx, Dy = forward_diff_matrices(M, N)
    L = Dx.T @ Dx + Dy.T @ Dy
    uI_dense = np.linalg.solve(AtA + lam * L, Aty + lam * L @ uE.ravel())
    np.testing.assert_allclose(uI.ravel(), uI_dense, atol=1e-8 * np.abs(uI).max())


# ----------------------------------------------------------------------------- O6: solves

def test_small_lambda_inverts_an_invertible_psf():
    M, N = 16, 20
    h = 0.4 * synth.psf_box(3)
    h[1, 1] += 0.6                            # |H| >= 0.46 everywhere
    u = rng0.uniform(0, 255, (M, N))
    y = direct_circular_conv(h, u)
    S = oracle.setup(y, h, 0.0, 1.0)
    uI, up = oracle.spectral_solve(S, oracle.dft2(rng0.uniform(0, 255, (M, N))), 1e-13)
    np.testing.assert_allclose(up, u, atol=1e-9)
    np.testing.assert_allclose(uI, u, atol=1e-9)


def test_solve_mean_and_large_lambda_limits():
    h = ASYM_H
    u, y = _small_problem(h=h)
    S = oracle.setup(y, h, 4.0, 1.0)
    uE = rng0.uniform(0, 255, y.shape)
    UE = oracle.dft2(uE)
    for lam in (1e-4, 1.0, 1e4):
        uI, _ = oracle.spectral_solve(S, UE, lam)
        assert math.isclose(uI.mean(), y.mean() / h.sum(), rel_tol=1e-12)
    _, up = oracle.spectral_solve(S, UE, 1e12)
    np.testing.assert_allclose(up, uE, atol=1e-6)
    uI, up = oracle.spectral_solve(S, UE, math.inf)
    np.testing.assert_array_equal(uI, up)
    np.testing.assert_allclose(up, uE, atol=1e-12)


# ----------------------------------------------------------------------------- O7: guided filter

@pytest.mark.parametrize("M,N,w", [(7, 9, 3), (8, 6, 5), (9, 9, 7), (6, 11, 1), (5, 7, 5)])
def test_box_mean_equals_brute_force_and_uniform_convolution(M, N, w):
    x = rng0.standard_normal((M, N))
    B = oracle.box_mean(x, w)
    np.testing.assert_allclose(B, brute_box_mean(x, w), atol=1e-14)
    via_fft = np.real(oracle.idft2(oracle.dft2(oracle.embed_psf(np.full((w, w), 1.0 / w ** 2), M, N)) * oracle.dft2(x)))
    np.testing.assert_allclose(B, via_fft, atol=1e-13)


def _gf_brute(I, p, w, eps):
    """Eqs.(3)-(5) pixel by pixel: a_k, b_k per window, then the average over covering windows."""
    M, N = I.shape
    r = (w - 1) // 2
    a = np.zeros((M, N))
    b = np.zeros((M, N))
    for m in range(M):
        for n in range(N):
            idx = [((m + di) % M, (n + dj) % N) for di in range(-r, r + 1) for dj in range(-r, r + 1)]
            Iw = np.array([I[q] for q in idx])
            pw = np.array([p[q] for q in idx])
            mu, pb = Iw.mean(), pw.mean()
            a[m, n] = (np.mean(Iw * pw) - mu * pb) / (np.mean((Iw - mu) ** 2) + eps)
            b[m, n] = pb - a[m, n] * mu
    out = np.zeros((M, N))
    for m in range(M):
        for n in range(N):
            ks = [((m + di) % M, (n + dj) % N) for di in range(-r, r + 1) for dj in range(-r, r + 1)]
            out[m, n] = np.mean([a[k] for k in ks]) * I[m, n] + np.mean([b[k] for k in ks])
    return out


@pytest.mark.parametrize("w", [1, 3, 5])
def test_guided_filter_equals_windowwise_definition(w):
    I = rng0.uniform(0, 255, (7, 8))
    p = I + 20 * rng0.standard_normal((7, 8))
    np.testing.assert_allclose(oracle.guided_filter(I, p, w, 30.0), _gf_brute(I, p, w, 30.0), atol=1e-9)


def test_guided_filter_identical_guide_small_eps_returns_input():
    p = rng0.uniform(0, 255, (24, 20))
    np.testing.assert_allclose(oracle.guided_filter(p, p, 5, 1e-10), p, rtol=1e-8)


def test_guided_filter_constant_image_and_unit_window_are_exact():
    c = np.full((9, 11), 37.25)
    assert np.array_equal(oracle.guided_filter(c, c, 5, 650.25), c)
    I = rng0.uniform(0, 255, (9, 11))
    p = rng0.uniform(0, 255, (9, 11))
    assert np.array_equal(oracle.guided_filter(I, p, 1, 3.0), p)


def test_guided_filter_infinite_eps_is_double_box_mean_of_input():
    I = rng0.uniform(0, 255, (12, 10))
    p = rng0.uniform(0, 255, (12, 10))
    np.testing.assert_allclose(oracle.guided_filter(I, p, 5, 1e30),
                               oracle.box_mean(oracle.box_mean(p, 5), 5), rtol=1e-12)


def test_guided_filter_affine_in_input_and_invariant_in_guide():
    I = rng0.uniform(0, 255, (14, 13))
    p = I + 15 * rng0.standard_normal((14, 13))
    base = oracle.guided_filter(I, p, 5, 40.0)
    np.testing.assert_allclose(oracle.guided_filter(I, 2.5 * p - 7.0, 5, 40.0), 2.5 * base - 7.0, atol=1e-9)
    np.testing.assert_allclose(oracle.guided_filter(-3.0 * I + 11.0, p, 5, 9.0 * 40.0), base, atol=1e-9)
    np.testing.assert_allclose(oracle.guided_filter(np.roll(I, (3, -2), (0, 1)), np.roll(p, (3, -2), (0, 1)), 5, 40.0),
                               np.roll(base, (3, -2), (0, 1)), atol=1e-10)


# ----------------------------------------------------------------------------- O8: whole iteration

def _case(M=24, N=20, seed=7):
    rng = np.random.default_rng(seed)
    u = synth.piecewise_image(M, N, rng, n_shapes=4)
    h = synth.psf_gaussian(1.2, 5)
    y = synth.blur_periodic(u, h) + 1.5 * rng.standard_normal((M, N))
    return u, h, y


def test_iteration_shift_equivariance():
    u, h, y = _case()
    out, info = oracle.deconvolve(y, h, 2.25, 5, 650.25, 4)
    sh = (5, -3)
    out2, info2 = oracle.deconvolve(np.roll(y, sh, (0, 1)), h, 2.25, 5, 650.25, 4)
    np.testing.assert_allclose(out2, np.roll(out, sh, (0, 1)), atol=1e-8)
    np.testing.assert_allclose(info2["lam"], info["lam"], rtol=1e-9)


def test_iteration_transpose_equivariance_for_symmetric_psf():
    u, h, y = _case(M=20, N=20)
    out, _ = oracle.deconvolve(y, h, 2.25, 3, 650.25, 3)
    outT, _ = oracle.deconvolve(y.T, h.T, 2.25, 3, 650.25, 3)
    np.testing.assert_allclose(outT, out.T, atol=1e-8)


def test_iteration_scale_covariance():
    u, h, y = _case()
    out, info = oracle.deconvolve(y, h, 2.25, 5, 650.25, 3)
    s = 0.01
    out2, info2 = oracle.deconvolve(s * y, h, s * s * 2.25, 5, s * s * 650.25, 3)
    np.testing.assert_allclose(out2, s * out, atol=1e-9)
    np.testing.assert_allclose(info2["lam"], info["lam"], rtol=1e-8)


def test_iteration_decreases_residual_and_improves_isnr():
    c = synth.make_case(1, size=(64, 64))
    out, info = oracle.deconvolve(c.y, c.h, c.sigma2, c.w, c.eps, 6)
    assert oracle.isnr(out, c.y, c.u_orig) > 1.0
    assert np.all(np.isfinite(info["lam"]))
    assert info["flags"][0] == 0


def test_infinite_branch_keeps_zero_estimate():
    u, h, y = _case()
    big = 10 * np.sum(y.astype(np.float64) ** 2) / y.size
    out, info = oracle.deconvolve(y, h, big, 5, 650.25, 3, rho=1.0)
    assert np.all(info["flags"] == oracle.FLAG_INF_BRANCH)
    assert np.all(np.isinf(info["lam"]))
    assert np.array_equal(out, np.zeros_like(out))


def test_zero_noise_hits_the_lambda_floor():
    u, h, y = _case()
    out, info = oracle.deconvolve(y, h, 0.0, 5, 650.25, 1)
    assert info["flags"][0] == oracle.FLAG_NO_ROOT
    assert info["lam"][0] == 1e-30


def test_lambda_scales_multiply_lambda_star():
    u, h, y = _case()
    _, info = oracle.deconvolve(y, h, 2.25, 5, 650.25, 3, scales=[1.0, 0.5, 2.0])
    np.testing.assert_allclose(info["lam"], info["lam_star"] * np.array([1.0, 0.5, 2.0]), rtol=1e-15)
