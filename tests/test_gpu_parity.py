"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars (from the method and its arithmetic):
  - graph and index arrays: bit-exact;
  - assembled values: Frobenius-relative <= 1e-13 (summation order and FMA
    contraction differ), GPU matrix bitwise symmetric;
  - FP64 SpMV: relative <= 1e-14 per sample; FP32 SpMV vs FP64: <= 1e-6;
  - FP64 CG: at the GPU's per-sample iteration count the oracle's iterate
    agrees to relative 1e-9; the oracle's own stopping count is within +-1;
  - mixed-precision refinement: true FP64 residual <= 1e-8 per sample.
"""
import numpy as np
import pytest
import torch

from workloads import SMALL, draw_xi, draw_vector

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def E():
    from paper_1511_03703_amd import ens
    ens.lib()
    assert torch.cuda.is_available()
    return ens


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


# ------------------------------------------------------------------ graph

@pytest.mark.parametrize("N", [1, 2, 3, 5, 16, 33])
def test_graph_bit_exact(E, orc, N):
    g = E.graph_build(N)
    rp, ci = orc.graph(N)
    assert np.array_equal(_np(g.row_ptr), rp)
    assert np.array_equal(_np(g.col_idx), ci)


# --------------------------------------------------------------------- KL

@pytest.mark.parametrize("M", [1, 3, 10, 16])
def test_kl_table_matches_oracle(E, orc, M):
    N = 7
    kl = E.kl_parse(E.kl_build(N, M, 1.0), N, M)
    w, lam, nrm, par = orc.kl_1d(M, 1.0)
    tr, lam3 = orc.kl_modes(M, 1.0)
    np.testing.assert_allclose(kl["omega"], w, rtol=1e-14)
    np.testing.assert_allclose(kl["lam1"], lam, rtol=1e-14)
    np.testing.assert_allclose(kl["norm1"], nrm, rtol=1e-14)
    assert np.array_equal(kl["parity"], par)
    assert np.array_equal(kl["triple"], tr)
    np.testing.assert_allclose(kl["lam3"], lam3, rtol=1e-14)
    # table products reproduce sqrt(lambda_m) phi_m at every quadrature point
    pts = orc.qp_coords(N)
    for m in range(M):
        xi = np.zeros(M)
        xi[m] = 1.0
        ref = orc.kl_coef_points(M, 1.0, 0.0, 1.0, xi, pts.reshape(-1, 3)).reshape(N ** 3, 8)
        t = kl["triple"][m]
        got = np.zeros((N ** 3, 8))
        for e in range(N ** 3):
            ex, ey, ez = e % N, (e // N) % N, e // (N * N)
            for q in range(8):
                got[e, q] = (kl["sqrt_lam3"][m] * kl["phi"][t[0], 2 * ex + (q & 1)]
                             * kl["phi"][t[1], 2 * ey + ((q >> 1) & 1)] * kl["phi"][t[2], 2 * ez + ((q >> 2) & 1)])
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


# --------------------------------------------------------------- assembly

def _gpu_system(E, N, s, M, sigma, xi, want32=False, f=1.0):
    g = E.graph_build(N)
    kl = E.kl_build(N, M, 1.0)
    vals, v32, rhs = E.assemble(g, kl, _t(xi), M, sigma, f=f, want32=want32)
    return g, vals, v32, rhs


@pytest.mark.parametrize("N,s,M,sigma", [(16, 4, 3, 0.1), (5, 8, 10, 0.3), (6, 16, 10, 0.2), (3, 32, 16, 0.3),
                                         (1, 4, 10, 0.2), (9, 32, 10, 0.3), (2, 32, 10, 0.3)])
def test_assembly_matches_oracle(E, orc, N, s, M, sigma):
    xi = draw_xi(100 + N, s, M)
    g, vals, v32, rhs = _gpu_system(E, N, s, M, sigma, xi, want32=True)
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    gv, gb = _np(vals), _np(rhs)
    for e in range(s):
        assert _rel(gv[:, e], ov[:, e]) <= 1e-13
        assert _rel(gb[:, e], ob[:, e]) <= 1e-14
    # bitwise symmetry of the GPU matrix, every sample
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    key = rows.astype(np.int64) * n + ci
    tkey = ci.astype(np.int64) * n + rows
    order = np.argsort(key)
    perm = order[np.searchsorted(key[order], tkey)]
    assert np.array_equal(gv, gv[perm])
    # FP32 copy is the round-to-nearest of the FP64 values
    assert np.array_equal(_np(v32), gv.astype(np.float32))


def test_assembly_deterministic(E):
    N, s, M = 8, 16, 10
    xi = draw_xi(7, s, M)
    a = _np(_gpu_system(E, N, s, M, 0.3, xi)[1])
    b = _np(_gpu_system(E, N, s, M, 0.3, xi)[1])
    assert np.array_equal(a, b)


# -------------------------------------------------------------------- SpMV

def _random_crs(rng, n, maxlen, ncols):
    lens = rng.integers(0, min(maxlen, ncols) + 1, n)
    lens[rng.integers(0, n, max(1, n // 10))] = 0  # some empty rows
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([np.sort(rng.choice(ncols, L, replace=False)) for L in lens]).astype(np.int32)
    return rp, ci


@pytest.mark.parametrize("s", [4, 8, 16, 32])
@pytest.mark.parametrize("n", [1, 37, 1000, 4099])
def test_spmv_random_graphs(E, orc, s, n):
    rng = np.random.default_rng(n * 100 + s)
    rp, ci = _random_crs(rng, n, 64, n)
    nnz = int(rp[-1])
    vals = rng.standard_normal((nnz, s))
    x = rng.standard_normal((n, s))
    ref = orc.ens_spmv(rp, ci, vals, x)
    g = E.graph_from_arrays(_t(rp, torch.int32), _t(ci, torch.int32))
    y = _np(E.spmv(g, _t(vals), _t(x)))
    scale = max(np.abs(vals).max(initial=0.0) * np.abs(x).max(), 1.0) * 64
    assert np.max(np.abs(y - ref)) <= 1e-15 * scale
    y32 = _np(E.spmv(g, _t(vals, torch.float32), _t(x, torch.float32)))
    assert np.max(np.abs(y32 - ref)) <= 2e-6 * scale


@pytest.mark.parametrize("s", [4, 32])
@pytest.mark.parametrize("lo,hi", [(40, 64), (0, 8)])
def test_spmv_row_tiles_staged_and_not(E, orc, s, lo, hi):
    # a workgroup stages its rows' indices in LDS when they average at most
    # 32 per row and reads them from global memory otherwise: rows of 40-64
    # entries take the second path in every tile, rows of 0-8 the first
    rng = np.random.default_rng(lo * 1000 + s)
    n = 2000
    lens = rng.integers(lo, hi + 1, n)
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([np.sort(rng.choice(n, L, replace=False)) for L in lens]).astype(np.int32)
    vals = rng.standard_normal((int(rp[-1]), s))
    x = rng.standard_normal((n, s))
    ref = orc.ens_spmv(rp, ci, vals, x)
    g = E.graph_from_arrays(_t(rp, torch.int32), _t(ci, torch.int32))
    scale = max(np.abs(vals).max(initial=0.0) * np.abs(x).max(), 1.0) * 64
    for dt, tol in ((torch.float64, 1e-15), (torch.float32, 2e-6)):
        y = _np(E.spmv(g, _t(vals, dt), _t(x, dt)))
        assert np.max(np.abs(y - ref)) <= tol * scale


@pytest.mark.parametrize("lanes", [0, 4, 8, 16, 32, 64])
def test_scalar_spmv(E, orc, lanes):
    rng = np.random.default_rng(lanes)
    n = 3001
    rp, ci = _random_crs(rng, n, 70, n)
    vals = rng.standard_normal(int(rp[-1]))
    x = rng.standard_normal(n)
    ref = orc.spmv(rp, ci, vals, x)
    g = E.graph_from_arrays(_t(rp, torch.int32), _t(ci, torch.int32))
    y = _np(E.scalar_spmv(g, _t(vals), _t(x), lanes_per_row=lanes))
    assert np.max(np.abs(y - ref)) <= 1e-13 * (1 + np.abs(ref).max())


def _ascending_sum(rp, ci, vals, x, dt):
    # each product rounded once, then added in ascending entry order, in dt
    vals, x = vals.astype(dt), x.astype(dt)
    y = np.zeros(len(rp) - 1, dt)
    for r in range(len(rp) - 1):
        s = dt(0)
        for k in range(rp[r], rp[r + 1]):
            s = dt(s + dt(vals[k] * x[ci[k]]))
        y[r] = s
    return y


@pytest.mark.parametrize("n,maxlen", [(1, 5), (64, 27), (65, 27), (1000, 20), (777, 70), (3001, 40)])
def test_scalar_spmv_row_tiles(E, orc, n, maxlen):
    # the row-tile product (lanes_per_row 0): tiles whose entries fit in LDS
    # (short rows), tiles that read global memory (long rows), both in one
    # matrix (maxlen 70 puts tiles on either side), ragged last tiles, empty
    # rows; against the oracle within rounding, and bitwise against the
    # ascending sum of singly rounded products the header states
    print(f"scalar row tiles n={n} maxlen={maxlen}", flush=True)
    rng = np.random.default_rng(7000 + n + maxlen)
    rp, ci = _random_crs(rng, n, maxlen, n)
    vals = rng.standard_normal(int(rp[-1]))
    x = rng.standard_normal(n)
    ref = orc.spmv(rp, ci, vals, x)
    g = E.graph_from_arrays(_t(rp, torch.int32), _t(ci, torch.int32))
    for dt, tdt, tol in ((np.float64, torch.float64, 1e-13), (np.float32, torch.float32, 2e-5)):
        y = _np(E.scalar_spmv(g, _t(vals, tdt), _t(x, tdt), lanes_per_row=0))
        assert np.max(np.abs(y - ref)) <= tol * (1 + np.abs(ref).max())
        assert np.array_equal(y, _ascending_sum(rp, ci, vals, x, dt))


def test_spmv_on_assembled_matrix(E, orc):
    N, s, M = 12, 16, 10
    xi = draw_xi(5, s, M)
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, 0.2, 1.0, xi)
    x = draw_vector(6, ((N + 1) ** 3, s))
    ref = orc.ens_spmv(rp, ci, ov, x)
    g = E.graph_build(N)
    y = _np(E.spmv(g, _t(ov), _t(x)))
    for e in range(s):
        assert _rel(y[:, e], ref[:, e]) <= 1e-14


# ---------------------------------------------------------------------- CG

def _check_cg_against_oracle(orc, rp, ci, ov, ob, x_gpu, stats, rtol, x0=None):
    s = ov.shape[1]
    iters = np.array([st["iters"] for st in stats], np.int32)
    xo, ito, relo, sto = orc.ens_pcg(rp, ci, ov, ob, x0=x0, fixed_iters=iters)
    xt, itt, relt, stt = orc.ens_pcg(rp, ci, ov, ob, x0=x0, rtol=rtol)
    true_res = orc.ens_true_residual(rp, ci, ov, ob, x_gpu)
    for e in range(s):
        assert stats[e]["status"] == 0, stats[e]
        assert _rel(x_gpu[:, e], xo[:, e]) <= 1e-9, (e, _rel(x_gpu[:, e], xo[:, e]))
        assert abs(int(itt[e]) - int(iters[e])) <= 1, (e, itt[e], iters[e])
        assert true_res[e] <= rtol * (1 + 1e-6), (e, true_res[e])
        assert abs(stats[e]["rel_res"] - true_res[e]) <= 1e-6 * rtol + 1e-3 * true_res[e]


def test_cg_small_config(E, orc):
    """16^3 elements, s=4, M=3, sigma=0.1, Jacobi-CG to 1e-10 (FP64)."""
    w = SMALL
    xi = w.xi()
    g, vals, _, rhs = _gpu_system(E, w.N, w.s, w.M, w.sigma, xi)
    x, stats, st = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=w.rtol))
    assert st == E.ENS_OK
    rp, ci = orc.graph(w.N)
    ov, ob = orc.assemble_ensemble(w.N, rp, ci, w.M, 1.0, 1.0, w.sigma, 1.0, xi)
    _check_cg_against_oracle(orc, rp, ci, ov, ob, _np(x), stats, w.rtol)


@pytest.mark.parametrize("s", [4, 8, 16, 32])
def test_cg_every_ensemble_size(E, orc, s):
    N, M, sigma, rtol = 7, 10, 0.3, 1e-10
    xi = draw_xi(40 + s, s, M)
    g, vals, _, rhs = _gpu_system(E, N, s, M, sigma, xi)
    x, stats, st = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=rtol, check_every=3))
    assert st == E.ENS_OK
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    _check_cg_against_oracle(orc, rp, ci, ov, ob, _np(x), stats, rtol)


def test_cg_nonzero_initial_guess(E, orc):
    N, s, M, rtol = 9, 8, 10, 1e-10
    xi = draw_xi(3, s, M)
    g, vals, _, rhs = _gpu_system(E, N, s, M, 0.2, xi)
    x0 = draw_vector(8, ((N + 1) ** 3, s), 0.0, 0.05)
    x, stats, st = E.cg(g, vals, rhs, x=_t(x0), opts=E.cg_opts(rtol=rtol))
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, 0.2, 1.0, xi)
    _check_cg_against_oracle(orc, rp, ci, ov, ob, _np(x), stats, rtol, x0=x0)


def test_ensemble_equals_scalar_solves(E, orc):
    N, s, M, rtol = 10, 8, 10, 1e-10
    xi = draw_xi(12, s, M)
    g, vals, _, rhs = _gpu_system(E, N, s, M, 0.3, xi)
    x, stats, _ = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=rtol))
    vsm = E.relayout(vals, True)
    bsm = E.relayout(rhs, True)
    for lanes in (0, 4, 16):
        xs, sstats, st = E.scalar_cg(g, vsm, bsm, opts=E.cg_opts(rtol=rtol), lanes_per_row=lanes)
        assert st == E.ENS_OK
        xe = _np(x)
        xsn = _np(xs)
        for e in range(s):
            d = _rel(xsn[e], xe[:, e])
            assert abs(sstats[e]["iters"] - stats[e]["iters"]) <= 1
            assert d <= (1e-10 if sstats[e]["iters"] == stats[e]["iters"] else 1e-6), (e, d)
    back = _np(E.relayout(vsm, False))
    assert np.array_equal(back, _np(vals))
    # the concurrent one-sample baseline runs the same kernels per sample, so
    # its results equal the sequential baseline's bitwise
    for lanes in (8, 0):
        xs1, st1, _ = E.scalar_cg(g, vsm, bsm, opts=E.cg_opts(rtol=rtol, check_every=5), lanes_per_row=lanes)
        for streams in (1, 3, 8):
            xc, stc, rc = E.scalar_cg_concurrent(g, vsm, bsm, opts=E.cg_opts(rtol=rtol, check_every=5),
                                                 lanes_per_row=lanes, streams=streams)
            assert rc == E.ENS_OK
            assert torch.equal(xc, xs1) and stc == st1


def test_shutdown_releases_and_state_comes_back(E):
    # the library's own state (device context, side streams, profiling
    # events) is released and rebuilt on demand; results are unchanged
    N, s, M, rtol = 6, 4, 3, 1e-10
    g, vals, _, rhs = _gpu_system(E, N, s, M, 0.2, draw_xi(41, s, M))
    vsm, bsm = E.relayout(vals, True), E.relayout(rhs, True)
    E.prof_enable(True)
    E.prof_reset()
    x0, st0, _ = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=rtol))
    xc0, stc0, _ = E.scalar_cg_concurrent(g, vsm, bsm, opts=E.cg_opts(rtol=rtol), lanes_per_row=8, streams=3)
    E.shutdown()
    assert E.prof_query(E.K_SPMV_F64)["launches"] > 0  # timings taken before survive
    E.shutdown()  # a second call finds nothing to release
    x1, st1, _ = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=rtol))
    xc1, stc1, _ = E.scalar_cg_concurrent(g, vsm, bsm, opts=E.cg_opts(rtol=rtol), lanes_per_row=8, streams=3)
    assert torch.equal(x0, x1) and st0 == st1
    assert torch.equal(xc0, xc1) and stc0 == stc1
    E.prof_enable(False)


def test_cg_edge_cases(E, orc):
    N, s, M = 6, 4, 3
    xi = draw_xi(2, s, M)
    g, vals, _, rhs = _gpu_system(E, N, s, M, 0.1, xi)
    # zero right-hand side with a nonzero start: x = 0, no iterations
    x, stats, st = E.cg(g, vals, torch.zeros_like(rhs), x=torch.ones_like(rhs))
    assert st == E.ENS_OK and not _np(x).any()
    assert all(t["iters"] == 0 and t["status"] == 0 for t in stats)
    # starting at the solution: no iterations
    xs, _, _ = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=1e-13))
    x, stats, st = E.cg(g, vals, rhs, x=xs.clone(), opts=E.cg_opts(rtol=1e-8))
    assert all(t["iters"] == 0 and t["status"] == 0 for t in stats)
    # iteration cap
    x, stats, st = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=1e-12, max_iter=1))
    assert st == E.ENS_W_NOT_CONVERGED
    assert all(t["iters"] == 1 and t["status"] == E.SAMPLE_MAXITER for t in stats)
    # negative definite: breakdown at the first p.Ap
    x, stats, st = E.cg(g, -vals, rhs)
    assert all(t["status"] == E.SAMPLE_BREAKDOWN and t["iters"] == 0 for t in stats)
    # one NaN sample does not disturb the others
    xi2 = xi.copy()
    xi2[1, 0] = np.nan
    g2, v2, _, b2 = _gpu_system(E, N, s, M, 0.1, xi2)
    x, stats, st = E.cg(g2, v2, b2)
    assert stats[1]["status"] == E.SAMPLE_NONFINITE
    assert all(stats[e]["status"] == 0 for e in (0, 2, 3))


def test_cg_masks_freeze_converged_samples(E, orc):
    # samples with very different conditioning converge at different
    # iterations; each must match the oracle at its own count
    N, s, M = 10, 8, 10
    xi = draw_xi(77, s, M)
    xi[::2] *= 0.0  # half the samples have constant coefficient
    g, vals, _, rhs = _gpu_system(E, N, s, M, 0.3, xi)
    x, stats, st = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=1e-10, check_every=5))
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, 0.3, 1.0, xi)
    _check_cg_against_oracle(orc, rp, ci, ov, ob, _np(x), stats, 1e-10)


# ---------------------------------------------------------- mixed precision

@pytest.mark.parametrize("N,s,sigma", [(16, 4, 0.1), (12, 32, 0.3), (20, 16, 0.3)])
def test_mixed_refinement_reaches_fp64_residual(E, orc, N, s, sigma):
    M, rtol = 10, 1e-8
    xi = draw_xi(200 + N, s, M)
    g, vals, v32, rhs = _gpu_system(E, N, s, M, sigma, xi, want32=True)
    x, stats, st = E.cg(g, vals, rhs, values32=v32, opts=E.cg_opts(rtol=rtol, mixed=True))
    assert st == E.ENS_OK, stats
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    xg = _np(x)
    true_res = orc.ens_true_residual(rp, ci, ov, ob, xg)
    xref, _, _, _ = orc.ens_pcg(rp, ci, ov, ob, rtol=1e-12)
    for e in range(s):
        assert stats[e]["status"] == 0 and stats[e]["outer_iters"] >= 1
        assert true_res[e] <= rtol * (1 + 1e-6), (e, true_res[e])
        assert abs(stats[e]["rel_res"] - true_res[e]) <= 1e-3 * true_res[e] + 1e-14
        # error against the FP64 solve is stated, bounded by kappa * rtol
        assert _rel(xg[:, e], xref[:, e]) <= 1e-5


# ---------------------------------------------------- coupled ensemble CG

@pytest.mark.parametrize("N,s", [(7, 8), (12, 32), (5, 4)])
def test_coupled_cg_matches_oracle(E, orc, N, s):
    """Coupled solve (one alpha, beta and stopping test for the ensemble)
    against the oracle's CG on the block-diagonal system at the GPU's
    iteration count."""
    M, sigma, rtol = 10, 0.3, 1e-10
    xi = draw_xi(300 + N, s, M)
    g, vals, _, rhs = _gpu_system(E, N, s, M, sigma, xi)
    x, stats, st = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=rtol, coupled=True, check_every=4))
    assert st == E.ENS_OK
    its = {t["iters"] for t in stats}
    assert len(its) == 1
    k = its.pop()
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    xo, _, _, _ = orc.ens_pcg_coupled(rp, ci, ov, ob, fixed_iters=k)
    _, ko, relo, sto = orc.ens_pcg_coupled(rp, ci, ov, ob, rtol=rtol)
    xg = _np(x)
    assert _rel(xg, xo) <= 1e-9, _rel(xg, xo)
    assert abs(ko - k) <= 1 and sto == orc.CONVERGED
    per = orc.ens_true_residual(rp, ci, ov, ob, xg)
    total = np.sqrt(np.sum(per ** 2 * np.sum(ob * ob, axis=0)) / np.sum(ob * ob))
    assert total <= rtol * (1 + 1e-6)
    for e in range(s):
        assert abs(stats[e]["rel_res"] - per[e]) <= 1e-6 * rtol + 1e-3 * per[e]
    _, st_ps, _ = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=rtol))
    print(f"coupled iterations {k}; per-sample {min(t['iters'] for t in st_ps)}..{max(t['iters'] for t in st_ps)}")


def test_coupled_cg_of_identical_samples(E):
    N, s, M = 9, 16, 10
    xi = np.repeat(draw_xi(77, 1, M), s, axis=0)
    g, vals, _, rhs = _gpu_system(E, N, s, M, 0.3, xi)
    xc, stc, _ = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=1e-10, coupled=True))
    xp, stp, _ = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=1e-10))
    assert [t["iters"] for t in stc] == [t["iters"] for t in stp]
    assert _rel(_np(xc), _np(xp)) <= 1e-12


def test_coupled_mixed_is_refused(E):
    N, s, M = 4, 4, 3
    g, vals, v32, rhs = _gpu_system(E, N, s, M, 0.1, draw_xi(1, s, M), want32=True)
    with pytest.raises(E.EnsError) as ex:
        E.cg(g, vals, rhs, values32=v32, opts=E.cg_opts(mixed=True, coupled=True))
    assert ex.value.status == E.ENS_E_UNSUPPORTED


def test_stream_read_folds_every_word(E):
    # the read-only bandwidth kernel reads every 16-byte chunk exactly once:
    # the XOR of its per-workgroup words is the XOR of the buffer's words
    rng = np.random.default_rng(77)
    for nbytes in (16, 4096 * 3 + 16 * 7, 64 << 20):
        words = rng.integers(0, 2 ** 32, nbytes // 4, dtype=np.uint64).astype(np.uint32)
        src = torch.as_tensor(words.view(np.int32), device=DEV)
        out = E.stream_read(src)
        pieces = -(-nbytes // E.STREAM_READ_CHUNK_BYTES)
        assert out.numel() == pieces
        got = _np(out).view(np.uint32)
        assert np.bitwise_xor.reduce(got) == np.bitwise_xor.reduce(words), nbytes
        # each word folds exactly its own 16 KB piece
        per = E.STREAM_READ_CHUNK_BYTES // 4
        want = [np.bitwise_xor.reduce(words[k * per:(k + 1) * per]) for k in range(min(pieces, 64))]
        assert np.array_equal(got[:len(want)], np.array(want, np.uint32)), nbytes


def test_stream_copy_and_triad(E):
    # the copy moves every 16-byte chunk, the triad forms a = b + q c per
    # element (one rounding of the fused multiply-add or two: within an
    # FP64 rounding of |b| + |q c| of each other), ragged sizes included
    rng = np.random.default_rng(78)
    for n in (1, 255, 257 * 256 + 3, 1 << 22):
        b = rng.standard_normal(n)
        c = rng.standard_normal(n)
        tb, tc = _t(b), _t(c)
        ta = torch.full((n + 32,), 5.0, dtype=torch.float64, device=DEV)
        E.stream_triad(ta[:n], tb, tc, 0.75)
        got = _np(ta)
        assert (np.abs(got[:n] - (b + 0.75 * c)) <= 2.0 ** -52 * (np.abs(b) + np.abs(0.75 * c))).all(), n
        assert (got[n:] == 5.0).all()
        if n % 2 == 0:
            dst = torch.full((n + 32,), -1.0, dtype=torch.float64, device=DEV)
            E.stream_copy(tb, dst[:n])
            got = _np(dst)
            assert np.array_equal(got[:n], b) and (got[n:] == -1.0).all(), n


def test_stream_write_sets_every_chunk(E):
    # the write-only bandwidth kernel writes every 16-byte chunk, and only
    # those of the buffer it is given (a guard region after it is untouched)
    for nbytes in (16, 4096 * 3 + 16 * 7, 64 << 20):
        buf = torch.full((nbytes // 4 + 64,), -7, dtype=torch.int32, device=DEV)
        E.stream_write(buf[: nbytes // 4], 0x5A5A0000)
        got = _np(buf).view(np.uint32)
        want = np.tile(np.array([0x5A5A0000, 0x5A5A0001, 0x5A5A0002, 0x5A5A0003], np.uint32), nbytes // 16)
        assert np.array_equal(got[: nbytes // 4], want), nbytes
        assert (got[nbytes // 4:] == np.uint32(0xFFFFFFF9)).all(), nbytes
