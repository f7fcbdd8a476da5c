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
