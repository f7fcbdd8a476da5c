"""GPU parity of the grouping predictor and of grouped batches (Sec. 3.7).
The per-sample coefficient extremes over the Gauss points equal the
oracle's (1e-13 of their size; NaN for a non-finite sample).  Regrouping
the samples of a batch by the predictor's order leaves every sample's
Jacobi-CG bitwise unchanged (per-sample scalars and masks: a sample's solve
does not depend on the samples beside it), and only the ensembles'
iteration maxima change."""
import numpy as np
import pytest
import torch

from workloads import draw_xi

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def E():
    from paper_1511_03703_amd import ens
    ens.lib()
    assert torch.cuda.is_available()
    return ens


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("N,s,M", [(5, 1, 3), (16, 37, 10), (9, 4, 0), (24, 64, 10)])
def test_kl_extrema_match_oracle(E, orc, N, s, M):
    sigma = 0.4
    xi = draw_xi(5200 + N + s, s, max(M, 1))[:, :max(M, 1)]
    kl = E.kl_build(N, M)
    kmin, kmax = E.kl_extrema(N, kl, torch.as_tensor(xi, device=DEV), M, sigma)
    omin, omax = orc.sample_extrema(N, M, 1.0, 1.0, sigma, xi)
    for got, want in ((_np(kmin), omin), (_np(kmax), omax)):
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    if M == 0:
        assert (_np(kmin) == 1.0).all() and (_np(kmax) == 1.0).all()


def test_kl_extrema_of_a_non_finite_sample(E, orc):
    N, s, M = 8, 6, 10
    xi = draw_xi(5210, s, M)
    xi[2, 4] = np.nan
    kl = E.kl_build(N, M)
    kmin, kmax = E.kl_extrema(N, kl, torch.as_tensor(xi, device=DEV), M, 0.3)
    kmin, kmax = _np(kmin), _np(kmax)
    assert np.isnan(kmin[2]) and np.isnan(kmax[2])
    ok = np.arange(s) != 2
    omin, omax = orc.sample_extrema(N, M, 1.0, 1.0, 0.3, xi[ok])
    assert np.abs(kmin[ok] - omin).max() <= 1e-13 and np.abs(kmax[ok] - omax).max() <= 1e-13
    assert E.group_order(kmax / kmin)[-1] == 2


def test_regrouped_batch_gives_each_sample_the_same_solve(E):
    N, s, G, M, sigma, rtol = 10, 8, 4, 10, 0.5, 1e-10
    xi = draw_xi(5220, G * s, M)
    g, kl = E.graph_build(N), E.kl_build(N, M)
    xt = torch.as_tensor(xi, device=DEV)
    kmin, kmax = E.kl_extrema(N, kl, xt, M, sigma)
    perm = E.group_order(_np(kmax) / _np(kmin))
    assert sorted(perm.tolist()) == list(range(G * s))

    def solve(order):
        groups = []
        for k in range(G):
            v, _, b = E.assemble(g, kl, xt[torch.as_tensor(order[k * s:(k + 1) * s], device=DEV)].contiguous(), M,
                                 sigma)
            groups.append([g, v, b, torch.zeros_like(b)])
        stats, rc, _ = E.solve_batch(groups, s, E.batch_opts(rtol=rtol, check_every=5))
        assert rc == E.ENS_OK
        x = np.concatenate([_np(gr[3]) for gr in groups], 1)
        it = np.array([t["iters"] for st in stats for t in st])
        out_x, out_it = np.empty_like(x), np.empty_like(it)
        out_x[:, order], out_it[order] = x, it
        return out_x, out_it, sum(max(t["iters"] for t in st) for st in stats)

    x0, it0, m0 = solve(np.arange(G * s))
    x1, it1, m1 = solve(perm)
    assert np.array_equal(x0, x1) and np.array_equal(it0, it1)
    # the ensembles' summed maxima never exceed the per-sample total, and
    # sorting by the exact counts would give the smallest sum
    ideal = sum(np.sort(it0)[k * s:(k + 1) * s].max() for k in range(G))
    assert ideal <= min(m0, m1) <= it0.sum()
    print("summed ensemble maxima: draw order", m0, "grouped by contrast", m1, "ideal", ideal)


def test_pool_regroups_each_mesh_size_by_contrast(E):
    from paper_1511_03703_amd import batchpool
    meshes, s, M, sigma = [8, 12, 8, 12, 8], 4, 10, 0.3
    xi = torch.as_tensor(draw_xi(5230, len(meshes) * s, M).reshape(len(meshes), s, M), device=DEV)
    pool = batchpool.BatchPool(E, meshes, s, M, 64 << 20)
    xg, order = pool.group_by_contrast(xi, sigma)
    assert sorted(order.tolist()) == list(range(len(meshes) * s))
    flat, gflat = _np(xi).reshape(-1, M), _np(xg).reshape(-1, M)
    assert np.array_equal(gflat, flat[order])
    for N in (8, 12):
        pos = np.concatenate([np.arange(g * s, (g + 1) * s) for g, m in enumerate(meshes) if m == N])
        assert (np.asarray(meshes)[order[pos] // s] == N).all()   # samples stay on their mesh size
        kl = pool.graphs[N][1]
        kmin, kmax = E.kl_extrema(N, kl, xg.reshape(-1, M)[torch.as_tensor(pos, device=DEV)].contiguous(), M, sigma)
        c = _np(kmax) / _np(kmin)
        assert (np.diff(c) >= 0).all()
