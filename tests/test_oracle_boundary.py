"""Pins of the oracle's boundary variants: clipped guided-filter windows (count-normalised
means, B^T != B) and the padded handling of a non-circularly blurred observation."""
import math

import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
from oracle import boundary as bd
import synth


def test_clipped_box_against_explicit_windows():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((7, 10))
    for w in (1, 3, 5, 7):
        r = (w - 1) // 2
        want_sum, want_cnt = np.zeros_like(x), np.zeros_like(x)
        for m in range(7):
            for n in range(10):
                for i in range(m - r, m + r + 1):
                    for j in range(n - r, n + r + 1):
                        if 0 <= i < 7 and 0 <= j < 10:
                            want_sum[m, n] += x[i, j]
                            want_cnt[m, n] += 1
        assert np.allclose(bd.box_sum_clipped(x, w), want_sum, rtol=0, atol=1e-12)
        assert np.array_equal(bd.window_counts(7, 10, w), want_cnt)
        assert np.allclose(bd.box_mean_clipped(x, w), want_sum / want_cnt, rtol=0, atol=1e-12)


def test_clipped_box_transpose_is_the_dense_transpose():
    M, N, w = 5, 6, 3
    P = M * N
    Bm = np.zeros((P, P))
    Bt = np.zeros((P, P))
    for k in range(P):
        e = np.zeros(P)
        e[k] = 1.0
        Bm[:, k] = bd.box_mean_clipped(e.reshape(M, N), w).ravel()
        Bt[:, k] = bd.box_mean_clipped_T(e.reshape(M, N), w).ravel()
    assert np.allclose(Bt, Bm.T, rtol=0, atol=1e-15)
    assert not np.allclose(Bm, Bm.T)  # clipping breaks the symmetry of the periodic box
    assert np.allclose(Bm.sum(axis=1), 1.0)  # rows of a mean sum to one


def test_clipped_box_interior_equals_the_periodic_box():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((20, 24))
    for w in (3, 5):
        r = (w - 1) // 2
        assert np.allclose(bd.box_mean_clipped(x, w)[r:-r, r:-r], oracle.box_mean(x, w)[r:-r, r:-r], atol=1e-12)


def test_clipped_guided_filter_window_by_window():
    rng = np.random.default_rng(2)
    M, N, w, eps, r = 8, 9, 3, 40.0, 1
    I = rng.uniform(0, 255, (M, N))
    p = I + 20 * rng.standard_normal((M, N))

    def window(m, n):
        return [(i, j) for i in range(m - r, m + r + 1) for j in range(n - r, n + r + 1) if 0 <= i < M and 0 <= j < N]

    A, B = np.zeros((M, N)), np.zeros((M, N))
    for m in range(M):
        for n in range(N):
            iv = np.array([I[q] for q in window(m, n)])
            pv = np.array([p[q] for q in window(m, n)])
            A[m, n] = np.mean((iv - iv.mean()) * (pv - pv.mean())) / (np.var(iv) + eps)
            B[m, n] = pv.mean() - A[m, n] * iv.mean()
    u = np.array([[np.mean([A[q] for q in window(m, n)]) * I[m, n] + np.mean([B[q] for q in window(m, n)])
                   for n in range(N)] for m in range(M)])
    assert np.max(np.abs(bd.guided_filter_clipped(I, p, w, eps) - u)) < 1e-10


def test_clipped_guided_filter_special_cases():
    rng = np.random.default_rng(3)
    I = rng.uniform(0, 255, (16, 18))
    p = I + 10 * rng.standard_normal(I.shape)
    c = np.full((16, 18), 77.0)
    assert np.allclose(bd.guided_filter_clipped(c, c, 5, 10.0), c, atol=1e-12)
    assert np.allclose(bd.guided_filter_clipped(I, p, 1, 10.0), p, atol=1e-12)
    # interior pixels (at least 2r from every border) agree with the periodic filter
    g1, g2 = bd.guided_filter_clipped(I, p, 3, 50.0), oracle.guided_filter(I, p, 3, 50.0)
    assert np.allclose(g1[2:-2, 2:-2], g2[2:-2, 2:-2], atol=1e-10)
    assert not np.allclose(g1, g2)


def test_clipped_guided_filter_adjoint_central_differences():
    rng = np.random.default_rng(4)
    M, N, w, eps = 11, 13, 5, 200.0
    I = rng.uniform(0, 255, (M, N))
    p = I + 15 * rng.standard_normal((M, N))
    g_u, dI, dp = rng.standard_normal((3, M, N))
    deps = 21.0
    gI, gp, ge = bd.guided_filter_clipped_adjoint(I, p, w, eps, g_u)

    def L(t):
        return np.sum(g_u * bd.guided_filter_clipped(I + t * dI, p + t * dp, w, eps + t * deps))

    t = 1e-4
    fd = (L(t) - L(-t)) / (2 * t)
    assert abs(np.sum(gI * dI) + np.sum(gp * dp) + ge * deps - fd) <= 1e-7 * abs(fd)


def test_good_size_and_padding():
    for n in range(1, 400):
        m = bd.good_size(n)
        k = m
        for f in (2, 3, 5):
            while k % f == 0:
                k //= f
        assert k == 1 and m >= n
        assert all(bd.good_size(q) != q for q in range(n, m))
    assert bd.padded_shape(256, 256, 31, 9) == (288, 270)
    # hand-computed: y = [[0, 3], [6, 9]] into 3 x 4 (column ramps of 2 steps, row ramp of 1 step)
    y = np.array([[0.0, 3.0], [6.0, 9.0]])
    want = np.array([[0.0, 3.0, 2.0, 1.0],
                     [6.0, 9.0, 8.0, 7.0],
                     [3.0, 6.0, 5.0, 4.0]])
    assert np.allclose(bd.pad_observation(y, 3, 4), want, atol=1e-15)
    # the periodic extension is continuous: from the last observed column on, and across the
    # wrap to column 0, every step is one ramp step
    rng = np.random.default_rng(5)
    y = np.cumsum(np.cumsum(rng.standard_normal((20, 30)), 0), 1)
    z = bd.pad_observation(y, 27, 40)
    assert np.array_equal(z[:20, :30], y)
    d = np.abs(z - np.roll(z, 1, axis=1))[:20]
    jump_x = max(np.max(d[:, 30:]), np.max(d[:, 0]))
    ramp = np.max(np.abs(y[:, -1] - y[:, 0])) / 11
    assert jump_x <= ramp + 1e-12


def test_unpadded_unclipped_variant_is_the_periodic_iteration():
    rng = np.random.default_rng(6)
    u = synth.piecewise_image(24, 30, rng, n_shapes=6)
    h = synth.psf_gaussian(1.2, 5)
    y = synth.blur_periodic(u, h) + 1.5 * rng.standard_normal(u.shape)
    a, ia = bd.deconvolve_boundary(y, h, 2.25, 3, 300.0, 4)
    b, ib = oracle.deconvolve(y, h, 2.25, 3, 300.0, 4)
    assert np.array_equal(a, b) and np.array_equal(ia["lam"], ib["lam"])


def test_padded_iteration_meets_the_observed_discrepancy_target():
    h = synth.psf_gaussian(1.5, 7)
    u, y, s2 = synth.nonperiodic_case(30, 36, h, 35.0, seed=7)
    uk, info = bd.deconvolve_boundary(y, h, s2, 3, 300.0, 3, pad=True)
    assert uk.shape == (30, 36) and info["shape"] == bd.padded_shape(30, 36, 7, 7)
    assert info["T"] == pytest.approx(oracle.rho_eq12(y, h, s2) * 30 * 36 * s2, rel=1e-15)
    # the lambda of the last iteration solves f(lambda) = T on the padded problem (Eq.(11))
    S, _ = bd.boundary_setup(y, h, s2, pad=True)
    uk2, info2 = bd.deconvolve_boundary(y, h, s2, 3, 300.0, 3, pad=True, keep_iterates=True)
    UE = oracle.dft2(info2["iterates"][-2])
    lam = info2["lam"][-1]
    assert math.isfinite(lam)
    assert oracle.residual_energy(lam, S, UE) == pytest.approx(S.T, rel=1e-8)


def test_padding_reduces_the_boundary_error_of_a_nonperiodic_blur():
    h = synth.psf_box(9)
    u, y, s2 = synth.nonperiodic_case(64, 64, h, 40.0, seed=8)
    per, _ = bd.deconvolve_boundary(y, h, s2, 3, 48.77, 10)
    pad, _ = bd.deconvolve_boundary(y, h, s2, 3, 48.77, 10, pad=True)
    band = np.ones(u.shape, bool)
    band[8:-8, 8:-8] = False
    e_per = np.sqrt(np.mean((per - u)[band] ** 2))
    e_pad = np.sqrt(np.mean((pad - u)[band] ** 2))
    print(f"border RMSE periodic {e_per:.2f}, padded {e_pad:.2f}")
    assert e_pad < 0.7 * e_per


@pytest.mark.parametrize("clip,pad", [(True, False), (False, True), (True, True)])
def test_boundary_adjoint_matches_central_differences(clip, pad):
    h = synth.psf_gaussian(1.2, 5)
    u, y, s2 = synth.nonperiodic_case(14, 16, h, 30.0, seed=9)
    y = y.astype(np.float64)
    iters, eps = 3, 650.25
    s = np.ones(iters)

    def loss(e, sc):
        uk, _ = bd.deconvolve_boundary(y, h, s2, 3, e, iters, clip=clip, pad=pad, scales=sc)
        return adj.mse_loss_grad(uk, u)

    _, g_u = loss(eps, s)
    g_eps, g_s = bd.deconvolve_boundary_adjoint(y, h, s2, 3, eps, iters, g_u, clip=clip, pad=pad, scales=s)
    de = 1e-3 * eps
    fd = (loss(eps + de, s)[0] - loss(eps - de, s)[0]) / (2 * de)
    assert abs(g_eps - fd) <= 1e-4 * abs(fd)
    for k in range(iters):
        sp, sm = s.copy(), s.copy()
        sp[k] += 1e-3
        sm[k] -= 1e-3
        fd = (loss(eps, sp)[0] - loss(eps, sm)[0]) / 2e-3
        assert abs(g_s[k] - fd) <= 1e-4 * max(abs(fd), 1e-3 * np.max(np.abs(g_s)))
