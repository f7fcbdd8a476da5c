"""Pins of the FP64 references for the learned initial guess (CPU only)."""
import math

import numpy as np
import pytest

from oracle import learned as L


def test_bf16_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7  # BF16 spacing in [1, 2)
    assert L.bf16(np.array([one]))[0] == one
    assert L.bf16(np.array([one + ulp]))[0] == one + ulp  # representable
    assert L.bf16(np.array([one + 0.5 * ulp]))[0] == one  # tie -> even (mantissa 0)
    assert L.bf16(np.array([one + 1.5 * ulp]))[0] == one + 2 * ulp  # tie -> even (mantissa 2)
    assert L.bf16(np.array([one + 0.51 * ulp]))[0] == one + ulp
    assert L.bf16(np.array([-(one + 0.49 * ulp)]))[0] == -one
    assert L.bf16(np.array([3.0e-3]))[0] == pytest.approx(3.0e-3, rel=2.0 ** -8)


def test_gelu_and_derivative():
    z = np.linspace(-6, 6, 241)
    g = L.gelu(z)
    assert L.gelu(np.array([0.0]))[0] == 0.0
    # z * Phi(z): Phi(1) = 0.8413447460685429 (standard normal CDF)
    assert L.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert abs(L.gelu(np.array([-8.0]))[0]) < 1e-13
    assert L.gelu(np.array([8.0]))[0] == pytest.approx(8.0, rel=1e-14)
    h = 1e-5
    fd = (L.gelu(z + h) - L.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(L.gelu_grad(z), fd, atol=1e-9)
    assert np.all(np.diff(g[z > -0.75]) > 0)  # increasing right of the minimum


def test_fp64_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = L.init_params(7)
    X = rng.uniform(-1, 1, (16, L.IN))
    T = rng.standard_normal((16, L.OUT))
    _, loss, g = L.forward_backward(p, X, T, bf16_points=False)
    assert loss == pytest.approx(L.loss_fp64(p, X, T), rel=1e-14)
    idx = rng.choice(L.P, 40, replace=False)
    idx = np.concatenate([idx, [0, 2559, 2560, 2815, 2816, 76799, 76800, L.P - 1]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp = p.copy()
        pp[i] += h
        pm = p.copy()
        pm[i] -= h
        fd = (L.loss_fp64(pp, X, T) - L.loss_fp64(pm, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_bf16_points_gradient_near_fp64():
    rng = np.random.default_rng(3)
    p = L.init_params(9)
    X = rng.uniform(-1, 1, (64, L.IN))
    T = rng.standard_normal((64, L.OUT))
    _, _, g64 = L.forward_backward(p, X, T, bf16_points=False)
    _, _, gb = L.forward_backward(p, X, T, bf16_points=True)
    assert np.linalg.norm(gb - g64) <= 5e-2 * np.linalg.norm(g64)


def test_pod_orthonormal_and_eckart_young():
    rng = np.random.default_rng(4)
    n, m, r = 400, 60, 12
    # snapshots with a decaying spectrum
    U, _ = np.linalg.qr(rng.standard_normal((n, m)))
    W, _ = np.linalg.qr(rng.standard_normal((m, m)))
    S = U @ np.diag(2.0 ** -np.arange(m, dtype=float)) @ W.T
    Phi, lam, G = L.pod(S, r)
    np.testing.assert_allclose(Phi.T @ Phi, np.eye(r), atol=1e-10)
    resid = S - Phi @ (Phi.T @ S)
    all_lam = np.sort(np.linalg.eigvalsh(G))[::-1]
    assert np.sum(resid * resid) == pytest.approx(all_lam[r:].sum(), rel=1e-8)
    # columns are left singular vectors: S S^T Phi = Phi diag(lambda)
    np.testing.assert_allclose(S @ (S.T @ Phi), Phi * lam, atol=1e-10 * lam[0])
    for j in range(r):
        i = int(np.argmax(np.abs(Phi[:, j])))
        assert Phi[i, j] > 0


def test_adam_first_step_is_lr_times_the_gradient_sign():
    # t = 1: m = 0.1 g, v = 0.001 g^2, and the bias corrections 1 - 0.9 and
    # 1 - 0.999 give mhat = g, vhat = g^2, so every coordinate moves by
    # lr g / (|g| + eps), i.e. lr sign(g) once |g| >> eps
    g = np.array([3.0, -0.25, 1e-3, -40.0, 0.0])
    p0 = np.array([1.0, 2.0, -1.0, 0.5, 7.0])
    p, m, v = L.adam_step(p0, g, np.zeros(5), np.zeros(5), 1, 1e-3)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-13)
    np.testing.assert_allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert p[4] == 7.0


def test_adam_constant_gradient_closed_form():
    # with the same g every step, m_t = (1 - 0.9^t) g and v_t = (1 - 0.999^t)
    # g^2 (geometric series), so the bias-corrected step is the same each
    # time: after k steps p = p0 - k lr g / (|g| + eps)
    g = np.array([0.7, -2.0, 5e-4])
    p = np.array([0.1, 0.2, 0.3])
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 2e-3
    for t in range(1, 11):
        p, m, v = L.adam_step(p, g, m, v, t, lr)
        np.testing.assert_allclose(m, (1 - 0.9 ** t) * g, rtol=1e-13)
        np.testing.assert_allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)
    np.testing.assert_allclose(p, np.array([0.1, 0.2, 0.3]) - 10 * lr * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_eps_is_added_outside_the_square_root():
    # |g| = eps: the first step is lr g / (|g| + eps) = lr / 2 (3 eps: 3/4);
    # with eps inside the square root it would be lr / sqrt 2 (3/sqrt 10)
    p, _, _ = L.adam_step(np.zeros(1), np.array([1e-8]), np.zeros(1), np.zeros(1), 1, 1.0)
    assert p[0] == pytest.approx(-0.5, rel=1e-12)
    p, _, _ = L.adam_step(np.zeros(1), np.array([3e-8]), np.zeros(1), np.zeros(1), 1, 1.0)
    assert p[0] == pytest.approx(-0.75, rel=1e-12)


def test_adam_two_steps_worked_by_hand():
    # g_1 = 1, g_2 = -1, lr = 1e-2:
    #   t=1: m = 0.1, v = 0.001, mhat = 1, vhat = 1: p1 = p0 - lr / (1 + eps)
    #   t=2: m = 0.09 - 0.1 = -0.01, v = 0.000999 + 0.001 = 0.001999,
    #        mhat = -0.01 / (1 - 0.81) = -1/19, vhat = 0.001999 / (1 - 0.998001) = 1:
    #        p2 = p1 + (lr / 19) / (1 + eps)
    lr, eps = 1e-2, 1e-8
    p, m, v = L.adam_step(np.array([0.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr)
    assert p[0] == pytest.approx(-lr / (1 + eps), rel=1e-14)
    p, m, v = L.adam_step(p, np.array([-1.0]), m, v, 2, lr)
    assert m[0] == pytest.approx(-0.01, rel=1e-13)
    assert v[0] == pytest.approx(0.001999, rel=1e-13)
    assert p[0] == pytest.approx(-lr / (1 + eps) + (lr / 19) / (1 + eps), rel=1e-12)


def test_adam_zero_gradient_only_decays_the_moments():
    p, m, v = L.adam_step(np.array([1.5]), np.array([0.0]), np.array([0.2]), np.array([0.04]), 7, 1e-3)
    assert m[0] == pytest.approx(0.18, rel=1e-15) and v[0] == pytest.approx(0.03996, rel=1e-15)
    mhat, vhat = 0.18 / (1 - 0.9 ** 7), 0.03996 / (1 - 0.999 ** 7)
    assert p[0] == pytest.approx(1.5 - 1e-3 * mhat / (math.sqrt(vhat) + 1e-8), rel=1e-14)
