"""Pins of the oracle's colour guided filter (three-channel guide)."""
import numpy as np

import oracle
import synth


def rand_guide(M, N, seed):
    rng = np.random.default_rng(seed)
    base = synth.piecewise_image(M, N, rng, n_shapes=5)
    return np.stack([base + 10 * rng.standard_normal((M, N)) + 30 * c for c in range(3)]), rng


def test_equal_channels_reduce_to_the_grey_filter_with_eps_over_3():
    """I_r = I_g = I_b = I: Sigma = v 11^T, so a = c 1 / (3 v + eps) and a . I = c I / (v + eps/3)."""
    rng = np.random.default_rng(1)
    I = synth.piecewise_image(20, 23, rng, n_shapes=4) + 5 * rng.standard_normal((20, 23))
    p = I + 12 * rng.standard_normal(I.shape)
    for w, eps in ((3, 300.0), (5, 40.0)):
        got = oracle.guided_filter_color(np.stack([I, I, I]), p, w, eps)
        ref = oracle.guided_filter(I, p, w, eps / 3.0)
        assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_window_by_window_definition():
    """Brute force: every window's 3x3 system solved on its own, then the averages of a, b."""
    I3, rng = rand_guide(9, 11, 2)
    p = rng.uniform(0, 255, (9, 11))
    w, eps, r = 3, 50.0, 1
    M, N = p.shape
    A = np.zeros((M, N, 3))
    B = np.zeros((M, N))
    for m in range(M):
        for n in range(N):
            idx = [((m + i) % M, (n + j) % N) for i in range(-r, r + 1) for j in range(-r, r + 1)]
            G = np.array([[I3[c][q] for c in range(3)] for q in idx])      # w^2 x 3
            pv = np.array([p[q] for q in idx])
            mu = G.mean(axis=0)
            S = (G - mu).T @ (G - mu) / len(idx)
            cov = (G - mu).T @ (pv - pv.mean()) / len(idx)
            a = np.linalg.solve(S + eps * np.eye(3), cov)
            A[m, n] = a
            B[m, n] = pv.mean() - a @ mu
    u = np.zeros((M, N))
    for m in range(M):
        for n in range(N):
            idx = [((m + i) % M, (n + j) % N) for i in range(-r, r + 1) for j in range(-r, r + 1)]
            abar = np.mean([A[q] for q in idx], axis=0)
            bbar = np.mean([B[q] for q in idx])
            u[m, n] = abar @ np.array([I3[c][m, n] for c in range(3)]) + bbar
    got = oracle.guided_filter_color(I3, p, w, eps)
    assert np.max(np.abs(got - u)) <= 1e-9 * np.max(np.abs(u))


def test_constant_guide_and_w1_and_affine_input():
    I3, rng = rand_guide(12, 14, 3)
    p = rng.uniform(0, 255, (12, 14))
    const = np.stack([np.full((12, 14), v) for v in (10.0, 20.0, 30.0)])
    got = oracle.guided_filter_color(const, p, 5, 100.0)
    assert np.allclose(got, oracle.box_mean(oracle.box_mean(p, 5), 5), rtol=0, atol=1e-9)
    assert np.allclose(oracle.guided_filter_color(I3, p, 1, 3.0), p, rtol=0, atol=1e-9)
    g1 = oracle.guided_filter_color(I3, p, 3, 80.0)
    g2 = oracle.guided_filter_color(I3, 2.5 * p + 7.0, 3, 80.0)
    assert np.allclose(g2, 2.5 * g1 + 7.0, rtol=1e-12, atol=1e-9)
