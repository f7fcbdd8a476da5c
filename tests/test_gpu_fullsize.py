"""Full-size GPU parity at the mid and headline workloads, in the launch
configuration bench.py times, on samples the oracle can afford one by one.

  64^3, s = 16, FP64 Jacobi-CG to 1e-10: samples 0-3 compared at the GPU's
      iteration counts (relative 1e-9), iteration counts within +-1, values
      of those samples against the oracle's scalar assembly (1e-13).
  128^3, s = 32, FP32 CG in FP64 refinement to 1e-8, with Jacobi and with
      the FP32 multigrid cycle of the timed step: samples 0 and 31 -- the
      oracle assembles each sample from scratch and checks the true FP64
      residual of both GPU solutions (<= 1e-8) and the assembled values
      (1e-13).
  128^3, s = 32, FP64 CG with the FP64 multigrid cycle to 1e-8 (coarse
      levels rediscretized; and Galerkin): samples 0 and 31 (0) against the
      oracle's MG-PCG at the GPU's iteration counts (relative 1e-9), its own
      counts within +-1, the true residual <= 1e-8.
  The one-sample baseline at 64^3 (the mid workload's 16 samples in the
      sample-major layout, 16 lanes per row as timed): samples 0 and 15
      against the oracle at the GPU's iteration counts (relative 1e-9), its
      own counts within +-1.
  The learned guess at 64^3, s = 32 (a reduced training set of 256
      snapshots): held-out samples 0 and 31 solved by FP64 Jacobi-CG from the
      network's guess, against the oracle started from the same guess at the
      GPU's iteration counts (relative 1e-9), its own counts within +-1, the
      true residual <= 1e-8.
  The batch: one group of the drawn batch per mesh size (32^3 .. 96^3,
      s = 32, tile 4), FP64 Jacobi-CG to 1e-8: samples 0 and 31 of each
      against the oracle at the GPU's iteration counts (relative 1e-9), the
      oracle's own counts within +-1, the true residual <= 1e-8.
"""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

from workloads import HEADLINE, MID

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1511_03703_amd import ens
    ens.lib()
    return ens


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle_sample(orc, rp, ci, w, xi_e):
    ac = orc.kl_coef_qp(w.N, w.M, w.L, w.kappa0, w.sigma, xi_e)
    return orc.assemble_scalar(w.N, rp, ci, ac, fconst=w.f)


def test_mid_workload_fp64(E, orc):
    w = MID
    xi = w.xi()
    g = E.graph_build(w.N)
    kl = E.kl_build(w.N, w.M, w.L)
    vals, _, rhs = E.assemble(g, kl, torch.as_tensor(xi, device="cuda"), w.M, w.sigma)
    x, stats, st = E.cg(g, vals, rhs, opts=E.cg_opts(rtol=w.rtol))
    assert st == E.ENS_OK
    check = [0, 1, 2, 3]
    gv = {e: vals[:, e].cpu().numpy() for e in check}
    xg = x.cpu().numpy()
    print(f"GPU done: iterations {[s['iters'] for s in stats]}", flush=True)
    rp, ci = orc.graph(w.N)

    def one(e):
        v, b = _oracle_sample(orc, rp, ci, w, xi[e])
        xo = orc.pcg(rp, ci, v, b, fixed_iters=stats[e]["iters"])[0]
        _, it_tol, _, _ = orc.pcg(rp, ci, v, b, rtol=w.rtol)
        res = np.linalg.norm(b - orc.spmv(rp, ci, v, xg[:, e])) / np.linalg.norm(b)
        return e, _rel(gv[e], v), _rel(xg[:, e], xo), it_tol, res

    with cf.ThreadPoolExecutor(4) as ex:
        for e, dv, dx, it_tol, res in ex.map(one, check):
            print(f"sample {e}: values {dv:.2e} x {dx:.2e} iters gpu {stats[e]['iters']} oracle {it_tol} "
                  f"true residual {res:.2e}", flush=True)
            assert dv <= 1e-13
            assert dx <= 1e-9
            assert abs(it_tol - stats[e]["iters"]) <= 1
            assert res <= w.rtol * (1 + 1e-6)


def test_headline_workload_refinement(E, orc):
    w = HEADLINE
    xi = w.xi()
    g = E.graph_build(w.N)
    kl = E.kl_build(w.N, w.M, w.L)
    vals, v32, rhs = E.assemble(g, kl, torch.as_tensor(xi, device="cuda"), w.M, w.sigma, want32=True)
    opts = E.cg_opts(rtol=w.rtol, mixed=True, inner_rtol=1e-4, check_every=16)
    x, stats, st = E.cg(g, vals, rhs, values32=v32, opts=opts)
    assert st == E.ENS_OK
    assert all(s["status"] == 0 and s["rel_res"] <= w.rtol * (1 + 1e-6) for s in stats)
    check = [0, w.s - 1]
    gv = {e: vals[:, e].cpu().numpy() for e in check}
    xg = {e: x[:, e].cpu().numpy() for e in check}
    g32 = v32[:, check[0]].cpu().numpy()
    assert np.array_equal(g32, gv[check[0]].astype(np.float32))
    print(f"GPU done: inner iterations {[s['iters'] for s in stats]}", flush=True)
    # the timed step: the same refinement with the FP32 multigrid cycle, its
    # fine matrix formed by the fused assembly and set-up
    mg = E.Multigrid(w.N, w.M, w.s, fp32=True, L=w.L)
    mg.assemble_setup(g, kl, torch.as_tensor(xi, device="cuda"), w.sigma, vals, rhs, values32=v32)
    opts_mg = E.cg_opts(rtol=w.rtol, mixed=True, inner_rtol=1e-4, check_every=4)
    xm, stats_mg, st = E.cg_mg(g, vals, rhs, mg, values32=v32, opts=opts_mg)
    assert st == E.ENS_OK
    xmg = {e: xm[:, e].cpu().numpy() for e in check}
    print(f"GPU done: multigrid inner iterations {[s['iters'] for s in stats_mg]}", flush=True)
    del vals, v32, mg, xm
    torch.cuda.empty_cache()
    rp, ci = orc.graph(w.N)

    def one(e):
        v, b = _oracle_sample(orc, rp, ci, w, xi[e])
        nb = np.linalg.norm(b)
        res = np.linalg.norm(b - orc.spmv(rp, ci, v, xg[e])) / nb
        res_mg = np.linalg.norm(b - orc.spmv(rp, ci, v, xmg[e])) / nb
        return e, _rel(gv[e], v), res, res_mg

    with cf.ThreadPoolExecutor(2) as ex:
        for e, dv, res, res_mg in ex.map(one, check):
            print(f"sample {e}: values {dv:.2e} true residual {res:.3e} (GPU reported {stats[e]['rel_res']:.3e}), "
                  f"multigrid {res_mg:.3e} (GPU reported {stats_mg[e]['rel_res']:.3e})", flush=True)
            assert dv <= 1e-13
            assert res <= w.rtol * (1 + 1e-6)
            assert abs(res - stats[e]["rel_res"]) <= 1e-3 * res
            assert res_mg <= w.rtol * (1 + 1e-6)
            assert abs(res_mg - stats_mg[e]["rel_res"]) <= 1e-3 * res_mg


@pytest.mark.parametrize("galerkin", [False, True])
def test_headline_fp64_multigrid_equal_iterations(E, orc, galerkin):
    # bench.py --workload mg --mg-fp64: FP64 CG with the FP64 V-cycle (levels
    # 128 .. 4) on the headline samples to 1e-8.  Samples 0 and 31 (sample 0
    # alone for Galerkin levels) against the oracle's MG-PCG with the same
    # kind of coarse levels at the GPU's iteration counts (relative 1e-9),
    # the oracle's own counts within +-1, the true residual <= 1e-8.
    w = HEADLINE
    xi = w.xi()
    g = E.graph_build(w.N)
    kl = E.kl_build(w.N, w.M, w.L)
    xt = torch.as_tensor(xi, device="cuda")
    vals = torch.empty((w.nnz, w.s), dtype=torch.float64, device="cuda")
    rhs = torch.empty((w.n, w.s), dtype=torch.float64, device="cuda")
    mg = E.Multigrid(w.N, w.M, w.s, L=w.L)
    mg.assemble_setup(g, kl, xt, w.sigma, vals, rhs, kappa0=w.kappa0, f=w.f, galerkin=galerkin)
    x, stats, st = E.cg_mg(g, vals, rhs, mg, opts=E.cg_opts(rtol=w.rtol, check_every=4))
    assert st == E.ENS_OK
    check = [0] if galerkin else [0, w.s - 1]
    iters = np.array([stats[e]["iters"] for e in check], np.int32)
    xg = x.cpu().numpy()[:, check]
    print(f"GPU done (galerkin={galerkin}): iterations {[t['iters'] for t in stats]}", flush=True)
    del vals, rhs, mg, x
    torch.cuda.empty_cache()
    sub = np.ascontiguousarray(xi[check])
    xo, _, _, _, _ = orc.ens_mg_pcg(w.N, w.M, w.L, w.kappa0, w.sigma, w.f, sub, fixed_iters=iters,
                                    galerkin=galerkin)
    _, ito, rro, sto, _ = orc.ens_mg_pcg(w.N, w.M, w.L, w.kappa0, w.sigma, w.f, sub, rtol=w.rtol,
                                         galerkin=galerkin)
    rp, ci = orc.graph(w.N)
    for j, e in enumerate(check):
        v, b = _oracle_sample(orc, rp, ci, w, xi[e])
        res = np.linalg.norm(b - orc.spmv(rp, ci, v, xg[:, j])) / np.linalg.norm(b)
        err = _rel(xg[:, j], xo[:, j])
        print(f"sample {e}: GPU {iters[j]} iterations, oracle {ito[j]}; rel. error at equal count {err:.2e}; "
              f"true residual {res:.3e}", flush=True)
        assert err <= 1e-9
        assert abs(int(ito[j]) - int(iters[j])) <= 1 and sto[j] == 0
        assert res <= w.rtol * (1 + 1e-6)


def test_newton_workload(E, orc):
    """128^3, s = 32, Newton with adaptive forcing and GMRES on the FP32
    Jacobian preconditioned by the FP32 V-cycle of D + alpha C, as bench.py
    times it.  Samples 0 and 31: the oracle evaluates the nonlinear residual
    of the GPU solution (<= 1e-8 |load|), the GPU residual and Jacobian at
    that solution element by element (1e-12 of the load, 1e-13 of the
    Jacobian's scale), and the fine matrix of the hierarchy against its
    Jacobian at u = 0 without reaction (1e-13)."""
    import workloads as W
    w = W.NEWTON
    xi = w.xi()
    dev = "cuda"
    g = E.graph_build(w.N)
    kl = E.kl_build(w.N, w.M, w.L)
    xt = torch.as_tensor(xi, device=dev)
    prob = E.nl_problem(w.M, w.sigma, W.NEWTON_ALPHA, W.NEWTON_BETA, W.NEWTON_VEL)
    K = torch.empty((w.nnz, w.s), dtype=torch.float64, device=dev)
    K32 = torch.empty((w.nnz, w.s), dtype=torch.float32, device=dev)
    rhs = torch.empty((w.n, w.s), dtype=torch.float64, device=dev)
    mg = E.Multigrid(w.N, w.M, w.s, fp32=True).assemble_setup_adv(g, kl, xt, prob, K, rhs, values32=K32)
    u, stats, st = E.newton(g, kl, xt, prob, opts=E.newton_opts(rtol=w.rtol, lin_rtol=W.NEWTON_ETA_MAX,
                                                                restart=W.NEWTON_RESTART, jac32=True,
                                                                forcing=E.FORCING_EW),
                            mg=mg, mg_values=K32)
    assert st == E.ENS_OK, stats
    print(f"GPU done: Newton steps {[t['newton_iters'] for t in stats]}, "
          f"GMRES {[t['lin_iters'] for t in stats]}", flush=True)
    check = [0, 31]
    kg = {e: K[:, e].cpu().numpy() for e in check}
    del mg, K, K32
    Fg, Jg, _ = E.nl_assemble(g, kl, xt, prob, u)
    ug = u.cpu().numpy()
    fg = {e: Fg[:, e].cpu().numpy() for e in check}
    jg = {e: Jg[:, e].cpu().numpy() for e in check}
    del Fg, Jg
    rp, ci = orc.graph(w.N)

    def one(e):
        ac = orc.kl_coef_qp(w.N, w.M, w.L, w.kappa0, w.sigma, xi[e])
        F, J, ld = orc.nl_assemble_scalar(w.N, rp, ci, ac, w.f, W.NEWTON_ALPHA, np.array(W.NEWTON_VEL),
                                          W.NEWTON_BETA, ug[:, e])
        # F nearly cancels at the root, so its error is measured against the
        # size of its terms (the load)
        _, J0, _ = orc.nl_assemble_scalar(w.N, rp, ci, ac, w.f, W.NEWTON_ALPHA, np.array(W.NEWTON_VEL), 0.0,
                                          np.zeros(w.n))
        return e, np.linalg.norm(F) / np.linalg.norm(ld), np.abs(fg[e] - F).max() / np.abs(ld).max(), \
            np.abs(jg[e] - J).max() / np.abs(J).max(), np.abs(kg[e] - J0).max() / np.abs(J0).max()

    with cf.ThreadPoolExecutor(2) as ex:
        for e, res, dF, dJ, dK in ex.map(one, check):
            print(f"sample {e}: |F|/|load| {res:.3e}, F {dF:.2e}, J {dJ:.2e}, D + alpha C {dK:.2e}", flush=True)
            assert res <= w.rtol * (1 + 1e-6)
            assert abs(stats[e]["rel_res"] - res) <= 1e-3 * res + 1e-14
            assert dF <= 1e-12 and dJ <= 1e-13 and dK <= 1e-13


def test_batch_workload_sampled(E, orc):
    import workloads as W
    meshes = W.batch_meshes()
    s, M, sigma, rtol = 32, W.BATCH_M, W.BATCH_SIGMA, W.BATCH_RTOL
    xi_all = W.draw_xi(W.BATCH_XI_SEED, len(meshes) * s, M).reshape(len(meshes), s, M)
    picks = [int(np.flatnonzero(meshes == N)[0]) for N in W.BATCH_MESHES]
    groups = []
    for gi in picks:
        N = int(meshes[gi])
        g, kl = E.graph_build(N), E.kl_build(N, M)
        v, _, b = E.assemble(g, kl, torch.as_tensor(xi_all[gi], device="cuda"), M, sigma)
        groups.append([g, v, b, torch.zeros_like(b)])
    stats, rc, _ = E.solve_batch(groups, s, E.batch_opts(rtol=rtol, check_every=16, tile=4))
    assert rc == E.ENS_OK
    xs = [gr[3][:, [0, s - 1]].cpu().numpy() for gr in groups]
    del groups
    torch.cuda.empty_cache()
    print(f"GPU done: iterations {[[st[0]['iters'], st[-1]['iters']] for st in stats]}", flush=True)
    for gi, st, x in zip(picks, stats, xs):
        N = int(meshes[gi])
        rp, ci = orc.graph(N)
        xi = xi_all[gi][[0, s - 1]]
        ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
        iters = np.array([st[0]["iters"], st[-1]["iters"]], np.int32)
        xo, _, _, _ = orc.ens_pcg(rp, ci, ov, ob, fixed_iters=iters)
        _, itt, _, _ = orc.ens_pcg(rp, ci, ov, ob, rtol=rtol)
        true = orc.ens_true_residual(rp, ci, ov, ob, x)
        for k in range(2):
            print(f"N={N} sample {k}: iters {iters[k]} (oracle {itt[k]}), rel diff "
                  f"{_rel(x[:, k], xo[:, k]):.2e}, true residual {true[k]:.2e}", flush=True)
            assert _rel(x[:, k], xo[:, k]) <= 1e-9
            assert abs(int(itt[k]) - int(iters[k])) <= 1
            assert true[k] <= rtol * (1 + 1e-6)


def test_learned_workload_sampled(E, orc):
    import workloads as W
    from paper_1511_03703_amd.learned import LearnedGuess
    w = W.LEARNED
    g, kl = E.graph_build(w.N), E.kl_build(w.N, w.M, w.L)
    train_xi = W.draw_xi(W.LEARNED_TRAIN_SEED, 256, w.M)
    Sm = torch.zeros((g.n, 256), dtype=torch.float64, device="cuda")
    for j in range(256 // w.s):
        v, _, b = E.assemble(g, kl, torch.as_tensor(train_xi[w.s * j:w.s * (j + 1)], device="cuda"), w.M, w.sigma)
        x, _, rc = E.cg(g, v, b, opts=E.cg_opts(rtol=1e-10))
        assert rc == E.ENS_OK
        E.pod_collect(x, Sm, w.s * j)
    lg = LearnedGuess(r=32, device="cuda")
    T = lg.fit_basis(Sm, eig_seed=W.LEARNED_INIT_SEED)
    lg.fit_network(torch.as_tensor(train_xi, dtype=torch.float32, device="cuda"), T, steps=600,
                   init_seed=W.LEARNED_INIT_SEED + 1, order_seed=W.LEARNED_INIT_SEED + 2, batch=64, halvings=2)
    test_xi = W.draw_xi(W.LEARNED_TEST_SEED, w.s, w.M)
    v, _, b = E.assemble(g, kl, torch.as_tensor(test_xi, device="cuda"), w.M, w.sigma)
    x0 = lg.guess(torch.as_tensor(test_xi, dtype=torch.float32, device="cuda"))
    x, st, rc = E.cg(g, v, b, x=x0.clone(), opts=E.cg_opts(rtol=w.rtol))
    assert rc == E.ENS_OK
    pick = [0, w.s - 1]
    xg, x0g = x[:, pick].cpu().numpy(), x0[:, pick].cpu().numpy()
    iters = np.array([st[e]["iters"] for e in pick], np.int32)
    print(f"GPU done: iterations {[t['iters'] for t in st]}", flush=True)
    rp, ci = orc.graph(w.N)
    ov, ob = orc.assemble_ensemble(w.N, rp, ci, w.M, w.L, w.kappa0, w.sigma, w.f, test_xi[pick])
    xo, _, _, _ = orc.ens_pcg(rp, ci, ov, ob, x0=x0g, fixed_iters=iters)
    _, itt, _, _ = orc.ens_pcg(rp, ci, ov, ob, x0=x0g, rtol=w.rtol)
    true = orc.ens_true_residual(rp, ci, ov, ob, xg)
    for k in range(2):
        print(f"sample {pick[k]}: iters {iters[k]} (oracle {itt[k]}), rel diff {_rel(xg[:, k], xo[:, k]):.2e}, "
              f"true residual {true[k]:.2e}", flush=True)
        assert _rel(xg[:, k], xo[:, k]) <= 1e-9
        assert abs(int(itt[k]) - int(iters[k])) <= 1
        assert true[k] <= w.rtol * (1 + 1e-6)


def test_one_sample_baseline_at_64_cubed(E, orc):
    w = MID
    xi = w.xi()
    g = E.graph_build(w.N)
    kl = E.kl_build(w.N, w.M, w.L)
    vals, _, rhs = E.assemble(g, kl, torch.as_tensor(xi, device="cuda"), w.M, w.sigma)
    vsm, bsm = E.relayout(vals, True), E.relayout(rhs, True)
    del vals
    xs, stats, st = E.scalar_cg(g, vsm, bsm, opts=E.cg_opts(rtol=w.rtol), lanes_per_row=16)
    assert st == E.ENS_OK
    check = [0, w.s - 1]
    xg = {e: xs[e].cpu().numpy() for e in check}
    print(f"GPU done: iterations {[t['iters'] for t in stats]}", flush=True)
    rp, ci = orc.graph(w.N)

    def one(e):
        v, b = _oracle_sample(orc, rp, ci, w, xi[e])
        xo = orc.pcg(rp, ci, v, b, fixed_iters=stats[e]["iters"])[0]
        _, it_tol, _, _ = orc.pcg(rp, ci, v, b, rtol=w.rtol)
        return e, _rel(xg[e], xo), it_tol

    with cf.ThreadPoolExecutor(2) as ex:
        for e, dx, it_tol in ex.map(one, check):
            print(f"sample {e}: x {dx:.2e} iters gpu {stats[e]['iters']} oracle {it_tol}", flush=True)
            assert dx <= 1e-9
            assert abs(int(it_tol) - stats[e]["iters"]) <= 1
