"""GPU parity of the learned initial guess: BF16-MFMA network kernels and the
FP64 POD kernels against the FP64 references of oracle/learned.py, and an
end-to-end check that the predicted guess seeds CG to the same tolerance in
fewer iterations.

Tolerances (Frobenius-relative): network outputs 5e-3 and gradients 2e-2 --
the reference evaluates in FP64 on the same BF16-rounded operands, and an
FP32-accumulated pre-activation occasionally rounds to the neighbouring
BF16 value; POD Gram 1e-13, eigenvalues 1e-9, basis 1e-8.
"""
import numpy as np
import pytest
import torch

from oracle import learned as L
from workloads import draw_xi

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def E():
    from paper_1511_03703_amd import ens
    ens.lib()
    assert ens.mlp_param_count() == L.P
    return ens


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _f32(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32), device=DEV)


@pytest.mark.parametrize("B", [32, 256, 1024])
def test_mlp_forward_and_gradient_match_reference(E, B):
    rng = np.random.default_rng(B)
    p = L.init_params(11).astype(np.float32)
    X = rng.uniform(-1, 1, (B, L.IN)).astype(np.float32)
    T = rng.standard_normal((B, L.OUT)).astype(np.float32)
    y, g, loss = E.mlp_grad(_f32(p), _f32(X), _f32(T))
    yo, lo, go = L.forward_backward(p.astype(np.float64), X, T, bf16_points=True)
    assert _rel(y.cpu().numpy(), yo) <= 5e-3
    assert abs(float(loss.item()) - lo) <= 5e-3 * lo
    gg = g.cpu().numpy()
    off = 0
    for name, shape in L.SIZES:
        k = int(np.prod(shape))
        assert _rel(gg[off:off + k], go[off:off + k]) <= 2e-2, name
        off += k
    y2 = E.mlp_forward(_f32(p), _f32(X))
    assert torch.equal(y2, y)


def test_mlp_training_reduces_loss_deterministically(E):
    rng = np.random.default_rng(5)
    N, B, steps = 512, 64, 300
    X = rng.uniform(-1, 1, (N, L.IN)).astype(np.float32)
    # smooth synthetic regression targets
    A = rng.standard_normal((L.IN, L.OUT)) / np.sqrt(L.IN)
    T = np.tanh(X @ A).astype(np.float32) + 0.1 * np.sin(3 * X[:, :1]).astype(np.float32)
    idx = np.concatenate([np.random.default_rng(100 + e).permutation(N) for e in range(steps * B // N + 1)])
    idx = torch.as_tensor(idx[:steps * B].astype(np.int32), device=DEV)
    results = []
    for rep in range(2):
        p = _f32(L.init_params(13))
        m = torch.zeros_like(p)
        v = torch.zeros_like(p)
        loss = torch.zeros(steps, dtype=torch.float32, device=DEV)
        E.mlp_train(p, m, v, 0, _f32(X), _f32(T), B, idx, 1e-3, loss=loss)
        torch.cuda.synchronize()
        results.append((p.cpu().numpy(), loss.cpu().numpy()))
    p1, l1 = results[0]
    p2, l2 = results[1]
    assert np.array_equal(p1, p2) and np.array_equal(l1, l2)
    assert l1[-20:].mean() < 0.1 * l1[:5].mean()
    # the GPU's reported batch loss matches the reference on its own parameters
    _, lo, _ = L.forward_backward(p1.astype(np.float64), X[:B], T[:B], bf16_points=True)
    y = E.mlp_forward(_f32(p1), _f32(X[:B])).cpu().numpy()
    assert abs(np.mean((y - T[:B]) ** 2) - lo) <= 1e-2 * lo


def _adam_ok(p, m, v, po, mo, vo, lr, t, tstep, mabs):
    # FP32 state after t steps against the FP64 reference started from the
    # same FP32 values (tstep: the Adam step index of the last step).  Each
    # FP32 operation rounds to a relative 6e-8 of its operands, so the bars
    # are relative to magnitudes, not to results that may cancel:
    #   m: to the moving average of |g| (mabs, the same recurrence on |g|),
    #      since terms of either sign may cancel;
    #   v: to v itself (no cancellation);
    #   p: to the rounding of p itself, plus the step's magnitude
    #      lr (mabs / c1) / (sqrt(vhat) + eps), which bounds both the step and
    #      what m's error does to it
    scale = np.maximum(mabs, np.abs(mo))
    assert (np.abs(m - mo) <= 2e-6 * t * scale + 1e-30).all(), float(np.max(np.abs(m - mo) / (scale + 1e-300)))
    np.testing.assert_allclose(v, vo, rtol=2e-6 * t, atol=1e-30)
    c1, c2 = 1.0 - 0.9 ** tstep, 1.0 - 0.999 ** tstep
    step = lr * (scale / c1) / (np.sqrt(vo / c2) + 1e-8)
    err = np.abs(p - po)
    bound = 1e-7 * t * np.abs(po) + 2e-6 * t * step + 1e-12
    assert (err <= bound).all(), float((err / bound).max())


@pytest.mark.parametrize("count", [L.P, 1000, 1])
def test_adam_step_matches_fp64_reference_on_fixed_gradients(E, count):
    # ens_mlp_adam (the kernel ens_mlp_train runs) against Algorithm 1 of
    # Kingma and Ba in FP64, on a seeded gradient sequence that mixes
    # magnitudes from 1e-8 (where eps matters) to 1e2, zeros and sign flips
    rng = np.random.default_rng(41 + count)
    lr = 1e-3
    p = rng.uniform(-1, 1, count).astype(np.float32)
    pt = _f32(p)
    mt = torch.zeros_like(pt)
    vt = torch.zeros_like(pt)
    po, mo, vo = p.astype(np.float64), np.zeros(count), np.zeros(count)
    mabs = np.zeros(count)
    for t in range(1, 11):
        scale = 10.0 ** rng.integers(-8, 3, count)
        g = (rng.standard_normal(count) * scale).astype(np.float32)
        g[rng.random(count) < 0.05] = 0.0
        E.mlp_adam(pt, _f32(g), mt, vt, t, lr)
        po, mo, vo = L.adam_step(po, g.astype(np.float64), mo, vo, t, lr)
        mabs = 0.9 * mabs + 0.1 * np.abs(g.astype(np.float64))
        if t in (1, 10):
            torch.cuda.synchronize()
            _adam_ok(pt.cpu().numpy(), mt.cpu().numpy(), vt.cpu().numpy(), po, mo, vo, lr, t, t, mabs)


@pytest.mark.parametrize("step0,steps", [(0, 1), (5, 1), (0, 10)])
def test_mlp_train_is_gradient_then_adam(E, step0, steps):
    # each step of ens_mlp_train = the network gradient of its mini-batch
    # (ens_mlp_grad, checked against the reference above) followed by the
    # FP64 Adam step of the reference at t = step0 + k + 1, from the same FP32
    # state; moments start from a state as after step0 steps.  A run of
    # `steps` in one call equals the same steps taken one call at a time.
    rng = np.random.default_rng(7 + step0 + steps)
    N, B, lr = 256, 64, 2e-3
    X = rng.uniform(-1, 1, (N, L.IN)).astype(np.float32)
    T = rng.standard_normal((N, L.OUT)).astype(np.float32)
    p0 = L.init_params(17).astype(np.float32)
    m0 = (1e-3 * rng.standard_normal(L.P) * (step0 > 0)).astype(np.float32)
    v0 = (1e-6 * rng.random(L.P) * (step0 > 0)).astype(np.float32)
    idx = rng.integers(0, N, steps * B).astype(np.int32)
    Xt, Tt = _f32(X), _f32(T)
    pa, ma, va = _f32(p0), _f32(m0), _f32(v0)
    E.mlp_train(pa, ma, va, step0, Xt, Tt, B, torch.as_tensor(idx, device=DEV), lr)
    p, m, v = _f32(p0), _f32(m0), _f32(v0)
    for k in range(steps):
        rows = idx[k * B:(k + 1) * B]
        _, g, _ = E.mlp_grad(p, _f32(X[rows]), _f32(T[rows]))
        po, mo, vo = L.adam_step(p.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64),
                                 m.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64),
                                 step0 + k + 1, lr)
        mabs = 0.9 * np.abs(m.cpu().numpy().astype(np.float64)) + 0.1 * np.abs(g.cpu().numpy().astype(np.float64))
        E.mlp_train(p, m, v, step0 + k, Xt, Tt, B, torch.as_tensor(rows, device=DEV), lr)
        torch.cuda.synchronize()
        _adam_ok(p.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy(), po, mo, vo, lr, 1, step0 + k + 1, mabs)
    assert torch.equal(p, pa) and torch.equal(m, ma) and torch.equal(v, va)


def test_pod_kernels_match_reference(E):
    rng = np.random.default_rng(6)
    n, m, r, k = 20000, 96, 16, 48
    U, _ = np.linalg.qr(rng.standard_normal((n, m)))
    W, _ = np.linalg.qr(rng.standard_normal((m, m)))
    S = U @ np.diag(1.5 ** -np.arange(m, dtype=float)) @ W.T
    Phi_o, lam_o, G_o = L.pod(S, r)
    St = torch.as_tensor(S, device=DEV)
    G = E.pod_gram(St)
    assert _rel(G.cpu().numpy(), G_o) <= 1e-13
    start = torch.as_tensor(rng.standard_normal((m, k)), device=DEV)
    V, lam = E.pod_eig(G, r, start, 12)
    np.testing.assert_allclose(lam.cpu().numpy(), lam_o, rtol=1e-9)
    Phi = E.pod_basis(St, V, lam)
    Pn = Phi.cpu().numpy()
    assert _rel(Pn, Phi_o) <= 1e-8
    np.testing.assert_allclose(Pn.T @ Pn, np.eye(r), atol=1e-10)
    X = rng.standard_normal((n, 8))
    C = E.pod_project(Phi, torch.as_tensor(X, device=DEV)).cpu().numpy()
    assert _rel(C, X.T @ Pn) <= 1e-13
    mu, sd, Tt = E.pod_standardize(torch.as_tensor(C, device=DEV))
    c32 = Tt.cpu().numpy()
    np.testing.assert_allclose(mu.cpu().numpy(), C.mean(0), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(sd.cpu().numpy(), C.std(0), rtol=1e-12)
    x0 = E.pod_reconstruct(Phi, Tt, mu, sd).cpu().numpy()
    cre = mu.cpu().numpy() + sd.cpu().numpy() * c32.astype(np.float64)
    assert _rel(x0, Pn @ cre.T) <= 1e-13
    # one common scale: the largest coefficient deviation for every column,
    # the targets keep the coefficients' relative sizes
    mu2, sd2, T2 = E.pod_standardize(torch.as_tensor(C, device=DEV), common=True)
    np.testing.assert_array_equal(mu2.cpu().numpy(), mu.cpu().numpy())
    big = C.std(0).max()
    np.testing.assert_allclose(sd2.cpu().numpy(), np.full(r, big), rtol=1e-12)
    np.testing.assert_allclose(T2.cpu().numpy(), ((C - C.mean(0)) / big).astype(np.float32), rtol=1e-6,
                               atol=1e-7)


def test_learned_guess_saves_iterations(E):
    """Small instance of the learned-guess workflow: 128 training solves on a
    12^3 mesh, POD r = 32, 400 Adam steps, 64 held-out samples."""
    N, M, sigma, s, rtol = 12, 10, 0.2, 32, 1e-8
    g = E.graph_build(N)
    kl = E.kl_build(N, M)
    train_xi = draw_xi(1005, 128, M)
    test_xi = draw_xi(1006, 64, M)
    n = g.n
    Sm = torch.zeros((n, 128), dtype=torch.float64, device=DEV)
    for j in range(4):
        xi = torch.as_tensor(train_xi[32 * j:32 * j + 32], device=DEV)
        v, _, b = E.assemble(g, kl, xi, M, sigma)
        x, st, rc = E.cg(g, v, b, opts=E.cg_opts(rtol=1e-10))
        assert rc == E.ENS_OK
        E.pod_collect(x, Sm, 32 * j)
    G = E.pod_gram(Sm)
    start = torch.as_tensor(np.random.default_rng(1007).standard_normal((128, 64)), device=DEV)
    V, lam = E.pod_eig(G, 32, start, 10)
    Phi = E.pod_basis(Sm, V, lam)
    C = E.pod_project(Phi, Sm)
    mu, sd, T = E.pod_standardize(C)
    p = _f32(L.init_params(1007))
    am, av = torch.zeros_like(p), torch.zeros_like(p)
    steps, B = 400, 32
    idx = np.concatenate([np.random.default_rng(2000 + e).permutation(128) for e in range(steps * B // 128)])
    E.mlp_train(p, am, av, 0, _f32(train_xi), T, B, torch.as_tensor(idx.astype(np.int32), device=DEV), 1e-3)
    saved, err0 = [], []
    for j in range(2):
        xi_np = test_xi[32 * j:32 * j + 32]
        xi = torch.as_tensor(xi_np, device=DEV)
        v, _, b = E.assemble(g, kl, xi, M, sigma)
        x_zero, st0, rc0 = E.cg(g, v, b, opts=E.cg_opts(rtol=rtol))
        c = E.mlp_forward(p, _f32(xi_np))
        x0 = E.pod_reconstruct(Phi, c, mu, sd)
        guess = x0.clone()
        x_l, st1, rc1 = E.cg(g, v, b, x=x0, opts=E.cg_opts(rtol=rtol))
        assert rc0 == E.ENS_OK and rc1 == E.ENS_OK
        xz, gl = x_zero.cpu().numpy(), guess.cpu().numpy()
        for e in range(32):
            assert st1[e]["rel_res"] <= rtol * (1 + 1e-6)
            saved.append(st0[e]["iters"] - st1[e]["iters"])
            err0.append(_rel(gl[:, e], xz[:, e]))
    print(f"iterations saved: mean {np.mean(saved):.1f} median {np.median(saved)}; "
          f"initial-guess error median {np.median(err0):.2e}", flush=True)
    assert np.median(err0) < 0.05
    assert np.mean(saved) > 2


def test_learned_guess_driver(E):
    """The package's learned-guess driver: basis from solver snapshots,
    staged-learning-rate training, guesses that CG accepts and improves on."""
    from paper_1511_03703_amd.learned import LearnedGuess
    N, M, sigma, s = 10, 10, 0.2, 32
    g = E.graph_build(N)
    kl = E.kl_build(N, M)
    train_xi = draw_xi(1310, 256, M)
    Sm = torch.zeros((g.n, 256), dtype=torch.float64, device=DEV)
    for j in range(8):
        v, _, b = E.assemble(g, kl, torch.as_tensor(train_xi[32 * j:32 * j + 32], device=DEV), M, sigma)
        x, _, rc = E.cg(g, v, b, opts=E.cg_opts(rtol=1e-10))
        assert rc == E.ENS_OK
        E.pod_collect(x, Sm, 32 * j)
    lg = LearnedGuess(r=32, device=DEV)
    T = lg.fit_basis(Sm, eig_seed=1311)
    lam = lg.lam.cpu().numpy()
    assert np.all(np.diff(lam) <= 0) and lam[-1] > 0
    loss = lg.fit_network(_f32(train_xi), T, steps=600, init_seed=1312, order_seed=1313, batch=64, halvings=2)
    ln = loss.cpu().numpy()
    assert np.all(np.isfinite(ln)) and ln[-30:].mean() < 0.1 * ln[:5].mean()
    test_xi = draw_xi(1314, s, M)
    v, _, b = E.assemble(g, kl, torch.as_tensor(test_xi, device=DEV), M, sigma)
    x0 = lg.guess(_f32(test_xi))
    x1, st1, rc1 = E.cg(g, v, b, x=x0.clone(), opts=E.cg_opts(rtol=1e-8))
    xz, st0, rc0 = E.cg(g, v, b, opts=E.cg_opts(rtol=1e-8))
    assert rc1 == E.ENS_OK and rc0 == E.ENS_OK
    assert np.mean([a["iters"] - c["iters"] for a, c in zip(st0, st1)]) > 2
    assert _rel(x0.cpu().numpy(), xz.cpu().numpy()) < 0.05
