"""GPU parity of the multigrid-preconditioned ensemble CG against the
oracle's per-sample MG-PCG (same hierarchy, transfers, smoother and coarse
solve).  Bars: at each sample's GPU iteration count the oracle's iterate
agrees to relative 1e-9; the oracle's own count is within +-1; the true
residual meets the tolerance."""
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


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _system(E, N, s, M, sigma, xi):
    g = E.graph_build(N)
    kl = E.kl_build(N, M)
    xt = torch.as_tensor(xi, device=DEV)
    vals, _, rhs = E.assemble(g, kl, xt, M, sigma)
    mg = E.Multigrid(N, M, s).setup(g, vals, xt, sigma)
    return g, vals, rhs, mg


@pytest.mark.parametrize("N,s", [(8, 4), (12, 8), (16, 32), (6, 16), (20, 8)])
def test_mg_cg_matches_oracle(E, orc, N, s):
    M, sigma, rtol = 10, 0.3, 1e-10
    xi = draw_xi(1400 + N, s, M)
    g, vals, rhs, mg = _system(E, N, s, M, sigma, xi)
    x, stats, st = E.cg_mg(g, vals, rhs, mg, opts=E.cg_opts(rtol=rtol, check_every=4))
    assert st == E.ENS_OK, stats
    iters = np.array([t["iters"] for t in stats], np.int32)
    xo, _, _, _, _ = orc.ens_mg_pcg(N, M, 1.0, 1.0, sigma, 1.0, xi, fixed_iters=iters)
    _, ito, _, sto, _ = orc.ens_mg_pcg(N, M, 1.0, 1.0, sigma, 1.0, xi, rtol=rtol)
    xg = _np(x)
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    true_res = orc.ens_true_residual(rp, ci, ov, ob, xg)
    for e in range(s):
        assert stats[e]["status"] == 0
        assert _rel(xg[:, e], xo[:, e]) <= 1e-9, (e, _rel(xg[:, e], xo[:, e]))
        assert abs(int(ito[e]) - int(iters[e])) <= 1, (e, ito[e], iters[e])
        assert true_res[e] <= rtol * (1 + 1e-6)
        assert abs(stats[e]["rel_res"] - true_res[e]) <= 1e-6 * rtol + 1e-3 * true_res[e]
    # far fewer iterations than Jacobi-CG on the same samples
    _, stj, _ = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=rtol))
    assert max(iters) < min(t["iters"] for t in stj)


def test_single_level_is_an_exact_solve(E):
    # an odd mesh has no coarser level: the preconditioner is A^-1 itself
    N, s, M = 7, 8, 10
    g, vals, rhs, mg = _system(E, N, s, M, 0.3, draw_xi(1450, s, M))
    x, stats, st = E.cg_mg(g, vals, rhs, mg, opts=E.cg_opts(rtol=1e-12))
    assert st == E.ENS_OK and all(t["iters"] == 1 for t in stats)


def test_mg_edge_cases_and_errors(E):
    N, s, M = 8, 8, 10
    xi = draw_xi(1460, s, M)
    g, vals, rhs, mg = _system(E, N, s, M, 0.2, xi)
    # zero right-hand side with a nonzero start: x = 0, no iterations
    x, stats, st = E.cg_mg(g, vals, torch.zeros_like(rhs), mg, x=torch.ones_like(rhs))
    assert st == E.ENS_OK and not _np(x).any() and all(t["iters"] == 0 for t in stats)
    # iteration cap
    x, stats, st = E.cg_mg(g, vals, rhs, mg, opts=E.cg_opts(rtol=1e-15, max_iter=2))
    assert st == E.ENS_W_NOT_CONVERGED and all(t["iters"] == 2 and t["status"] == E.SAMPLE_MAXITER for t in stats)
    # a NaN sample does not disturb the others
    xi2 = xi.copy()
    xi2[2, 0] = np.nan
    g2, v2, b2, mg2 = _system(E, N, s, M, 0.2, xi2)
    x, stats, st = E.cg_mg(g2, v2, b2, mg2)
    assert stats[2]["status"] == E.SAMPLE_NONFINITE
    assert all(stats[e]["status"] == 0 for e in range(s) if e != 2)
    # refusals
    with pytest.raises(E.EnsError):
        E.cg_mg(g, vals, rhs, mg, opts=E.cg_opts(mixed=True))
    with pytest.raises(E.EnsError):
        E.cg_mg(g, vals, rhs, mg, opts=E.cg_opts(coupled=True))
    g9 = E.graph_build(9)
    v9, _, b9 = E.assemble(g9, E.kl_build(9, M), torch.as_tensor(xi, device=DEV), M, 0.2)
    with pytest.raises(E.EnsError):
        E.cg_mg(g9, v9, b9, mg)
    with pytest.raises(E.EnsError) as ex:
        E.Multigrid(11, M, s)  # odd 11: a 1000-unknown coarse block
    assert ex.value.status == E.ENS_E_UNSUPPORTED
    # a buffer that was never built or set up is refused before any launch
    import ctypes
    raw = torch.empty(mg.buffer.numel(), dtype=torch.uint8, device=DEV)
    desc = E.ens_mg(N, M, s, 0, raw.data_ptr(), raw.numel())
    prob = E.ens_problem(M, 1.0, 1.0, 0.2, 1.0)
    gc = g.c()
    xt = torch.as_tensor(xi, device=DEV)
    assert E.lib().ens_mg_setup(ctypes.byref(desc), ctypes.byref(gc), ctypes.c_void_p(vals.data_ptr()), None,
                                ctypes.byref(prob), ctypes.c_void_p(xt.data_ptr()), None) == E.ENS_E_ARG
    # a built buffer set up for another correlation length is refused too
    prob2 = E.ens_problem(M, 0.5, 1.0, 0.2, 1.0)
    assert E.lib().ens_mg_setup(ctypes.byref(mg.desc), ctypes.byref(gc), ctypes.c_void_p(vals.data_ptr()), None,
                                ctypes.byref(prob2), ctypes.c_void_p(xt.data_ptr()), None) == E.ENS_E_ARG
    ws = torch.empty(E.cg_workspace_bytes(g, s, E.cg_opts()), dtype=torch.uint8, device=DEV)
    st_ = (E.ens_cg_stat * s)()
    xx = torch.zeros_like(rhs)
    assert E.lib().ens_cg_mg(ctypes.byref(gc), s, ctypes.c_void_p(vals.data_ptr()), None,
                             ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(xx.data_ptr()),
                             ctypes.byref(E.cg_opts()), ctypes.byref(desc), ctypes.c_void_p(ws.data_ptr()),
                             ws.numel(), st_, None) == E.ENS_E_ARG


def test_mg_is_deterministic(E):
    N, s, M = 16, 16, 10
    xi = draw_xi(1470, s, M)
    out = []
    for _ in range(2):
        g, vals, rhs, mg = _system(E, N, s, M, 0.3, xi)
        x, stats, _ = E.cg_mg(g, vals, rhs, mg, opts=E.cg_opts(rtol=1e-10))
        out.append((_np(x), stats))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


@pytest.mark.parametrize("N,s", [(16, 32), (12, 8), (24, 16)])
def test_mixed_refinement_with_fp32_multigrid(E, orc, N, s):
    """FP32 inner CG preconditioned by the FP32 cycle inside the FP64
    refinement: every sample reaches the FP64 true residual; the error
    against an FP64 solve is stated and bounded by kappa * rtol."""
    M, sigma, rtol = 10, 0.3, 1e-8
    xi = draw_xi(1480 + N, s, M)
    g = E.graph_build(N)
    kl = E.kl_build(N, M)
    xt = torch.as_tensor(xi, device=DEV)
    vals, v32, rhs = E.assemble(g, kl, xt, M, sigma, want32=True)
    mg = E.Multigrid(N, M, s, fp32=True).setup(g, vals, xt, sigma, values32=v32)
    x, stats, st = E.cg_mg(g, vals, rhs, mg, values32=v32, opts=E.cg_opts(rtol=rtol, mixed=True, check_every=4))
    assert st == E.ENS_OK, stats
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    xg = _np(x)
    true_res = orc.ens_true_residual(rp, ci, ov, ob, xg)
    xref, _, _, _, _ = orc.ens_mg_pcg(N, M, 1.0, 1.0, sigma, 1.0, xi, rtol=1e-12)
    for e in range(s):
        assert stats[e]["status"] == 0 and stats[e]["outer_iters"] >= 1
        assert true_res[e] <= rtol * (1 + 1e-6), (e, true_res[e])
        assert abs(stats[e]["rel_res"] - true_res[e]) <= 1e-3 * true_res[e] + 1e-14
        assert _rel(xg[:, e], xref[:, e]) <= 1e-5
    assert max(t["iters"] for t in stats) <= 20
    # an FP64 cycle is refused for the mixed solve, and the FP32 cycle for FP64 CG
    mg64 = E.Multigrid(N, M, s).setup(g, vals, xt, sigma)
    with pytest.raises(E.EnsError):
        E.cg_mg(g, vals, rhs, mg64, values32=v32, opts=E.cg_opts(mixed=True))
    with pytest.raises(E.EnsError):
        E.cg_mg(g, vals, rhs, mg, opts=E.cg_opts())


@pytest.mark.parametrize("N,s,fp32", [(16, 32, True), (12, 8, False), (8, 4, True), (20, 16, False)])
def test_fused_assembly_and_setup_equal_the_two_calls(E, N, s, fp32):
    # the fine level's D^-1 and bound formed inside the assembly are the
    # separate pass's bitwise: the same matrices, loads and solve
    M, sigma = 10, 0.3
    xi = draw_xi(1490 + N, s, M)
    g = E.graph_build(N)
    kl = E.kl_build(N, M)
    xt = torch.as_tensor(xi, device=DEV)
    vals, v32, rhs = E.assemble(g, kl, xt, M, sigma, want32=fp32)
    mg1 = E.Multigrid(N, M, s, fp32=fp32).setup(g, vals, xt, sigma, values32=v32)
    vals2 = torch.full_like(vals, float("nan"))
    v322 = torch.full_like(v32, float("nan")) if fp32 else None
    rhs2 = torch.full_like(rhs, float("nan"))
    mg2 = E.Multigrid(N, M, s, fp32=fp32).assemble_setup(g, kl, xt, sigma, vals2, rhs2, values32=v322)
    assert torch.equal(vals, vals2) and torch.equal(rhs, rhs2)
    if fp32:
        assert torch.equal(v32, v322)
    opts = E.cg_opts(rtol=1e-8 if fp32 else 1e-10, mixed=fp32, check_every=4)
    x1, st1, _ = E.cg_mg(g, vals, rhs, mg1, values32=v32, opts=opts)
    x2, st2, _ = E.cg_mg(g, vals2, rhs2, mg2, values32=v322, opts=opts)
    assert torch.equal(x1, x2) and st1 == st2
