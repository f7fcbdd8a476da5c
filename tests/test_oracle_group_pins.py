"""Pins of the grouping predictor (Sec. 3.7: the variation of a sample's
parameters over the domain predicts its iteration count): the oracle's
per-sample coefficient extremes against an evaluation at explicitly listed
Gauss points by the separately pinned point evaluator, the constant cases,
and the predictor's relation to actual Jacobi-CG iteration counts."""
import numpy as np

from workloads import draw_xi


def test_extrema_are_those_of_the_pointwise_coefficient(orc):
    N, M, sigma = 6, 10, 0.3
    xi = draw_xi(5100, 3, M)
    kmin, kmax = orc.sample_extrema(N, M, 1.0, 1.0, sigma, xi)
    pts = orc.qp_coords(N).reshape(-1, 3)
    for e in range(3):
        k = orc.kl_coef_points(M, 1.0, 1.0, sigma, xi[e], pts)
        assert abs(kmin[e] - k.min()) <= 1e-14 and abs(kmax[e] - k.max()) <= 1e-14
        assert kmin[e] < 1.0 < kmax[e]


def test_extrema_of_a_constant_coefficient(orc):
    xi = draw_xi(5101, 2, 4)
    for M, sigma in ((0, 0.3), (4, 0.0)):
        kmin, kmax = orc.sample_extrema(5, M, 1.0, 1.7, sigma, xi[:, :max(M, 1)])
        assert (kmin == 1.7).all() and (kmax == 1.7).all()
    # doubling sigma doubles the excursions about kappa0
    k1 = orc.sample_extrema(5, 4, 1.0, 1.0, 0.1, xi)
    k2 = orc.sample_extrema(5, 4, 1.0, 1.0, 0.2, xi)
    assert np.allclose(k2[0] - 1.0, 2 * (k1[0] - 1.0), rtol=1e-12, atol=1e-15)
    assert np.allclose(k2[1] - 1.0, 2 * (k1[1] - 1.0), rtol=1e-12, atol=1e-15)


def test_contrast_predicts_iteration_counts(orc):
    # the contrast kmax / kmin ranks samples by Jacobi-CG iteration count
    # (Spearman correlation well above zero), which is what grouping by it
    # relies on
    N, M, sigma, s = 12, 10, 0.5, 48
    xi = draw_xi(5102, s, M)
    kmin, kmax = orc.sample_extrema(N, M, 1.0, 1.0, sigma, xi)
    rp, ci = orc.graph(N)
    vals, b = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    _, it, _, st = orc.ens_pcg(rp, ci, vals, b, rtol=1e-8)
    assert (st == orc.CONVERGED).all()
    rank = lambda a: np.argsort(np.argsort(a, kind="stable"), kind="stable")
    rho = np.corrcoef(rank(kmax / kmin), rank(it))[0, 1]
    assert rho > 0.3, rho
