"""Pins of the oracle's nonlinear problem (Sec. 4, Eq. diffusion_sys), its
Jacobian (Eq. fenl_lin_sys), the right-preconditioned GMRES and Newton's
method, each against something other than the oracle itself: the pinned
linear assembly, closed-form Galerkin integrals of linear and constant
fields, central differences (exact for a quadratic residual), the
antisymmetry of the advection form, brute-force least squares over an
explicit Krylov basis, a dense solve, and an independent nonlinear solver
(MINPACK via scipy) that uses neither the Jacobian nor the Krylov solver."""
import numpy as np
import pytest

from workloads import draw_xi, draw_vector

VEL = np.array([0.3, -0.5, 0.8])


def _coords(orc, N):
    n1 = N + 1
    i = np.arange(orc.num_nodes(N))
    return np.stack([i % n1, (i // n1) % n1, i // (n1 * n1)], 1) / N


def _boundary(N):
    n1 = N + 1
    i = np.arange(n1 ** 3)
    c = np.stack([i % n1, (i // n1) % n1, i // (n1 * n1)], 1)
    return ((c == 0) | (c == N)).any(1)


def _acoef(orc, N, kappa0=1.0, sigma=0.0, xi=None, M=0):
    return orc.kl_coef_qp(N, M, 1.0, kappa0, sigma, np.zeros(max(M, 1)) if xi is None else xi)


def test_linear_case_is_the_pinned_assembly(orc):
    # alpha = beta = 0: J is the stiffness matrix and F(u) = K u - b for a u
    # that vanishes on the boundary
    N, M, s = 6, 5, 3
    rp, ci = orc.graph(N)
    xi = draw_xi(3001, s, M)
    bnd = _boundary(N)
    u = draw_vector(3002, (orc.num_nodes(N), s))
    u[bnd] = 0.0
    F, J, ld = orc.ens_nl_assemble(N, rp, ci, M, 1.0, 1.0, 0.3, 1.0, 0.0, VEL, 0.0, xi, u)
    K, b = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, 0.3, 1.0, xi)
    assert np.allclose(J, K, rtol=0, atol=1e-14 * np.abs(K).max())
    assert np.allclose(ld, b, rtol=0, atol=1e-16)
    Ku = orc.ens_spmv(rp, ci, K, u)
    assert np.allclose(F, Ku - b, rtol=0, atol=1e-14)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_closed_form_for_a_linear_field(orc, d):
    # kappa constant, u = x_d at every node (boundary included): the
    # diffusion term of an interior row vanishes, the advection term is
    # alpha v_d h^3 and the reaction term beta h^3 (c_i^2 + h^2/6), all
    # integrated exactly by the 2x2x2 Gauss rule
    N, alpha, beta, f = 5, 2.5, 1.5, 0.7
    h = 1.0 / N
    rp, ci = orc.graph(N)
    X = _coords(orc, N)
    u = X[:, d].copy()
    F, _, ld = orc.nl_assemble_scalar(N, rp, ci, _acoef(orc, N, kappa0=1.7), f, alpha, VEL, beta, u)
    bnd = _boundary(N)
    want = h ** 3 * (alpha * VEL[d] + beta * (X[:, d] ** 2 + h * h / 6.0) - f)
    assert np.allclose(F[~bnd], want[~bnd], rtol=1e-12, atol=1e-15)
    assert np.array_equal(F[bnd], u[bnd])
    assert np.allclose(ld[~bnd], f * h ** 3, rtol=1e-13) and not ld[bnd].any()


def test_closed_form_for_a_constant_field(orc):
    # u = c everywhere: F_i = (beta c^2 - f) h^3 on interior rows; the
    # reaction part of J has row sums 2 beta c h^3 on rows away from the
    # boundary (whose columns are all kept)
    N, beta, f, c = 6, 3.0, 0.4, 0.35
    h = 1.0 / N
    rp, ci = orc.graph(N)
    ac = _acoef(orc, N, kappa0=1.0, sigma=0.3, xi=draw_xi(3003, 1, 4)[0], M=4)
    n = orc.num_nodes(N)
    u = np.full(n, c)
    F, J, _ = orc.nl_assemble_scalar(N, rp, ci, ac, f, 0.0, VEL, beta, u)
    F0, K, _ = orc.nl_assemble_scalar(N, rp, ci, ac, f, 0.0, VEL, 0.0, u)
    bnd = _boundary(N)
    assert np.allclose(F[~bnd], (beta * c * c - f) * h ** 3, rtol=1e-11)
    X = _coords(orc, N) * N
    deep = ((X >= 2) & (X <= N - 2)).all(1)
    rs = np.add.reduceat(J - K, rp[:-1])
    assert np.allclose(rs[deep], 2 * beta * c * h ** 3, rtol=1e-11)


def test_jacobian_is_the_derivative_of_the_residual(orc):
    # F is quadratic in u, so central differences are exact up to rounding
    N, M = 4, 5
    rp, ci = orc.graph(N)
    ac = _acoef(orc, N, sigma=0.3, xi=draw_xi(3004, 1, M)[0], M=M)
    u = draw_vector(3005, orc.num_nodes(N), 0.0, 0.2)
    alpha, beta, f = 4.0, 20.0, 1.0
    F, J, _ = orc.nl_assemble_scalar(N, rp, ci, ac, f, alpha, VEL, beta, u)
    Jd = orc.crs_to_dense(rp, ci, J)
    bnd = _boundary(N)
    inner = np.flatnonzero(~bnd)
    d = 1e-3
    for j in inner:
        up, um = u.copy(), u.copy()
        up[j] += d
        um[j] -= d
        Fp, _, _ = orc.nl_assemble_scalar(N, rp, ci, ac, f, alpha, VEL, beta, up, want_jac=False)
        Fm, _, _ = orc.nl_assemble_scalar(N, rp, ci, ac, f, alpha, VEL, beta, um, want_jac=False)
        col = (Fp - Fm) / (2 * d)
        assert np.allclose(col[inner], Jd[inner, j], rtol=0, atol=1e-10 * np.abs(Jd).max()), j
    # boundary rows are identity rows; interior rows keep no boundary column
    assert np.array_equal(Jd[bnd], np.eye(len(u))[bnd])
    assert not Jd[np.ix_(inner, np.flatnonzero(bnd))].any()


def test_advection_form_is_antisymmetric(orc):
    # int phi_i v.grad phi_j = -int phi_j v.grad phi_i for interior pairs, so
    # with beta = 0 the symmetric part of J is the stiffness matrix
    N, M = 5, 4
    rp, ci = orc.graph(N)
    ac = _acoef(orc, N, sigma=0.3, xi=draw_xi(3006, 1, M)[0], M=M)
    u = draw_vector(3007, orc.num_nodes(N))
    _, J, _ = orc.nl_assemble_scalar(N, rp, ci, ac, 1.0, 6.0, VEL, 0.0, u)
    _, K, _ = orc.nl_assemble_scalar(N, rp, ci, ac, 1.0, 0.0, VEL, 0.0, u)
    Jd, Kd = orc.crs_to_dense(rp, ci, J), orc.crs_to_dense(rp, ci, K)
    inner = np.flatnonzero(~_boundary(N))
    Ji, Ki = Jd[np.ix_(inner, inner)], Kd[np.ix_(inner, inner)]
    assert np.allclose(0.5 * (Ji + Ji.T), Ki, rtol=0, atol=1e-14 * np.abs(Ki).max())
    assert np.abs(Ji - Ji.T).max() > 1e-3 * np.abs(Ki).max()


def _nl_system(orc, N, M=5, seed=3010, alpha=5.0, beta=30.0, s=1):
    rp, ci = orc.graph(N)
    xi = draw_xi(seed, s, M)
    u = draw_vector(seed + 1, (orc.num_nodes(N), s), 0.0, 0.1)
    u[_boundary(N)] = 0.0
    F, J, _ = orc.ens_nl_assemble(N, rp, ci, M, 1.0, 1.0, 0.3, 1.0, alpha, VEL, beta, xi, u)
    return rp, ci, xi, J, F


def _prec_dense(orc, N, M, xi, J, rp, ci, prec, alpha=5.0):
    n = orc.num_nodes(N)
    if prec == orc.PREC_JACOBI:
        d = J[[np.flatnonzero(ci[rp[i]:rp[i + 1]] == i)[0] + rp[i] for i in range(n)]]
        return np.diag(1.0 / d)
    if prec == orc.PREC_MG_ADV:
        return np.stack([orc.mg_apply_adv(N, M, 1.0, 1.0, 0.3, 1.0, alpha, VEL, xi, np.eye(n)[j]) for j in range(n)],
                        1)
    return np.stack([orc.mg_apply(N, M, 1.0, 1.0, 0.3, 1.0, xi, np.eye(n)[j]) for j in range(n)], 1)


def _adv_operator(orc, N, M, xi, alpha):
    # D + alpha C: the Jacobian at u = 0 of the problem without reaction
    rp, ci = orc.graph(N)
    ac = orc.kl_coef_qp(N, M, 1.0, 1.0, 0.3, xi)
    _, J, _ = orc.nl_assemble_scalar(N, rp, ci, ac, 1.0, alpha, VEL, 0.0, np.zeros(orc.num_nodes(N)))
    return rp, ci, J


def test_advection_vcycle_on_one_level_is_the_exact_solve(orc):
    # N = 4 has no coarser level: the cycle is the LU solve of D + alpha C
    # (identity boundary rows), against a dense solve
    N, M, alpha = 4, 5, 12.0
    xi = draw_xi(3080, 1, M)[0]
    assert orc.mg_levels(N) == [N]
    rp, ci, J = _adv_operator(orc, N, M, xi, alpha)
    A = orc.crs_to_dense(rp, ci, J)
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()   # nonsymmetric
    r = draw_vector(3081, orc.num_nodes(N))
    z = orc.mg_apply_adv(N, M, 1.0, 1.0, 0.3, 1.0, alpha, VEL, xi, r)
    zd = np.linalg.solve(A, r)
    assert np.abs(z - zd).max() <= 1e-12 * np.abs(zd).max()


def test_advection_vcycle_is_the_two_level_composition(orc):
    # N = 8 over N = 4: pre-smoothing, residual, restriction, exact coarse
    # solve, prolongation, post-smoothing, with D + alpha C rediscretized on
    # both meshes (a cycle that kept the diffusion matrix on either level
    # would differ), composed here from the pinned pieces
    Nf, Nc, M, alpha = 8, 4, 5, 10.0
    xi = draw_xi(3082, 1, M)[0]
    assert orc.mg_levels(Nf) == [Nf, Nc]
    rpf, cif, Jf = _adv_operator(orc, Nf, M, xi, alpha)
    rpc, cic, Jc = _adv_operator(orc, Nc, M, xi, alpha)
    Af, Ac = orc.crs_to_dense(rpf, cif, Jf), orc.crs_to_dense(rpc, cic, Jc)
    lmax = orc.gershgorin(rpf, cif, Jf)
    b = draw_vector(3083, orc.num_nodes(Nf))
    x = orc.mg_cheb2(rpf, cif, Jf, lmax, b)
    rc = orc.mg_restrict(Nf, b - Af @ x)
    x = orc.mg_prolong_add(Nc, np.linalg.solve(Ac, rc), x)
    x = orc.mg_cheb2(rpf, cif, Jf, lmax, b, x0=x)
    z = orc.mg_apply_adv(Nf, M, 1.0, 1.0, 0.3, 1.0, alpha, VEL, xi, b)
    assert np.abs(z - x).max() <= 1e-11 * np.abs(x).max()
    zd = orc.mg_apply(Nf, M, 1.0, 1.0, 0.3, 1.0, xi, b)
    assert np.abs(z - zd).max() > 1e-3 * np.abs(x).max()


def test_advection_vcycle_without_advection_is_the_diffusion_cycle(orc):
    N, M = 16, 5
    xi = draw_xi(3084, 1, M)[0]
    b = draw_vector(3085, orc.num_nodes(N))
    z0 = orc.mg_apply_adv(N, M, 1.0, 1.0, 0.3, 1.0, 0.0, VEL, xi, b)
    zd = orc.mg_apply(N, M, 1.0, 1.0, 0.3, 1.0, xi, b)
    assert np.abs(z0 - zd).max() <= 1e-12 * np.abs(zd).max()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_gmres_iterates_minimise_the_residual_over_the_krylov_space(orc, prec):
    # after k steps from x0, x_k = x0 + M K y with K = [r0, (AM) r0, ...] and
    # y the least-squares minimiser of |r0 - A M K y|: brute force with an
    # explicit (normalised) Krylov basis
    N, M = 4, 5
    rp, ci, xi, J, F = _nl_system(orc, N, M)
    A = orc.crs_to_dense(rp, ci, J[:, 0])
    b = F[:, 0]
    Pm = _prec_dense(orc, N, M, xi[0], J[:, 0], rp, ci, prec)
    x0 = draw_vector(3020, len(b), -0.01, 0.01)
    x0[_boundary(N)] = 0.0
    r0 = b - A @ x0
    for k in range(1, 6):
        xg, it, _, st = orc.ens_gmres(N, rp, ci, J, F, x0=x0[:, None], prec=prec, M=M, sigma=0.3, xi=xi,
                                      restart=8, fixed_iters=[k], alpha=5.0, vel=VEL)
        assert it[0] == k and st[0] == orc.CONVERGED
        Kb = [r0 / np.linalg.norm(r0)]
        for _ in range(k - 1):
            w = A @ (Pm @ Kb[-1])
            Kb.append(w / np.linalg.norm(w))
        Kb = np.stack(Kb, 1)
        y = np.linalg.lstsq(A @ Pm @ Kb, r0, rcond=None)[0]
        xb = x0 + Pm @ Kb @ y
        assert np.linalg.norm(xg[:, 0] - xb) <= 1e-9 * np.linalg.norm(xb), k


def test_gmres_reaches_the_dense_solution_with_and_without_restarts(orc):
    N, M = 4, 5
    rp, ci, xi, J, F = _nl_system(orc, N, M, s=2)
    for e in range(2):
        A = orc.crs_to_dense(rp, ci, J[:, e])
        xd = np.linalg.solve(A, F[:, e])
        for restart in (30, 3):
            x, it, rr, st = orc.ens_gmres(N, rp, ci, J[:, e:e + 1], F[:, e:e + 1], rtol=1e-13, restart=restart)
            assert st[0] == orc.CONVERGED and rr[0] <= 1e-13
            assert np.linalg.norm(x[:, 0] - xd) <= 1e-10 * np.linalg.norm(xd)
        _, it30, _, _ = orc.ens_gmres(N, rp, ci, J[:, e:e + 1], F[:, e:e + 1], rtol=1e-10, restart=30)
        _, it3, _, _ = orc.ens_gmres(N, rp, ci, J[:, e:e + 1], F[:, e:e + 1], rtol=1e-10, restart=3)
        assert it3[0] > it30[0]


def test_gmres_edge_cases(orc):
    N, M = 4, 5
    rp, ci, xi, J, F = _nl_system(orc, N, M)
    x, it, rr, st = orc.ens_gmres(N, rp, ci, J, np.zeros_like(F), x0=np.ones_like(F))
    assert not x.any() and it[0] == 0 and st[0] == orc.CONVERGED
    x, it, _, st = orc.ens_gmres(N, rp, ci, J, F, rtol=1e-15, max_iter=4)
    assert it[0] == 4 and st[0] == orc.MAXITER
    J2 = J.copy()
    J2[5, 0] = np.nan
    _, _, _, st = orc.ens_gmres(N, rp, ci, J2, F)
    assert st[0] == orc.NONFINITE


def test_newton_linear_case_takes_one_step(orc):
    # alpha = beta = 0: the discrete equations are linear and one Newton step
    # with an accurate inner solve is the linear solution (Sec. 4)
    N, M, s = 6, 5, 3
    xi = draw_xi(3030, s, M)
    u, ni, li, rr, st, _ = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, 0.0, VEL, 0.0, xi, rtol=1e-8, lin_rtol=1e-12)
    assert list(ni) == [1] * s and (st == orc.CONVERGED).all()
    rp, ci = orc.graph(N)
    K, b = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, 0.3, 1.0, xi)
    xc, _, _, _ = orc.ens_pcg(rp, ci, K, b, rtol=1e-13)
    assert np.abs(u - xc).max() <= 1e-9 * np.abs(xc).max()


def test_newton_converges_quadratically_to_the_root(orc):
    N, M, s = 6, 5, 2
    xi = draw_xi(3040, s, M)
    alpha, beta = 10.0, 100.0
    u, ni, li, rr, st, fn = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, alpha, VEL, beta, xi, rtol=1e-12,
                                           lin_rtol=1e-14)
    assert (st == orc.CONVERGED).all()
    for e in range(s):
        f = fn[e, :ni[e] + 1]
        assert (np.diff(f) < 0).all()
        # quadratic: F_{k+1} / F_k^2 stays bounded while F_k falls by orders
        q = f[1:-1] / f[:-2] ** 2
        assert q.max() < 10.0 * q.min() + 1.0, f
    rp, ci = orc.graph(N)
    F, _, ld = orc.ens_nl_assemble(N, rp, ci, M, 1.0, 1.0, 0.3, 1.0, alpha, VEL, beta, xi, u, want_jac=False)
    assert (np.linalg.norm(F, axis=0) <= 1e-12 * np.linalg.norm(ld, axis=0) * (1 + 1e-6)).all()


def test_newton_root_matches_an_independent_nonlinear_solver(orc):
    # MINPACK's hybrid method with its own difference Jacobian, on the
    # pinned residual: neither the analytic Jacobian, GMRES nor Newton's loop
    from scipy.optimize import root
    N, M = 4, 5
    xi = draw_xi(3050, 1, M)
    alpha, beta = 8.0, 200.0
    rp, ci = orc.graph(N)
    ac = orc.kl_coef_qp(N, M, 1.0, 1.0, 0.3, xi[0])
    fun = lambda v: orc.nl_assemble_scalar(N, rp, ci, ac, 1.0, alpha, VEL, beta, v, want_jac=False)[0]
    ref = root(fun, np.zeros(orc.num_nodes(N)), method="hybr", options={"xtol": 1e-13})
    # converged, or stopped at round-off: either way its residual is at noise level
    assert np.linalg.norm(fun(ref.x)) <= 1e-15
    for prec in (orc.PREC_JACOBI, orc.PREC_MG, orc.PREC_MG_ADV):
        u, ni, _, _, st, _ = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, alpha, VEL, beta, xi, prec=prec, rtol=1e-12,
                                            lin_rtol=1e-12)
        assert st[0] == orc.CONVERGED and ni[0] >= 2
        assert np.abs(u[:, 0] - ref.x).max() <= 1e-10 * np.abs(ref.x).max()


def test_newton_edge_cases(orc):
    N, M, s = 4, 5, 3
    xi = draw_xi(3060, s, M)
    # no source: u = 0 is the root, reached with no step
    u, ni, _, rr, st, _ = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 0.0, 5.0, VEL, 10.0, xi)
    assert not u.any() and not ni.any() and (st == orc.CONVERGED).all()
    # step cap
    _, ni, _, _, st, _ = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, 5.0, VEL, 100.0, xi, rtol=1e-15, max_newton=1)
    assert (ni == 1).all() and (st == orc.MAXITER).all()
    # a non-finite sample stops alone
    xi2 = xi.copy()
    xi2[1, 0] = np.nan
    _, _, _, _, st, _ = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, 5.0, VEL, 10.0, xi2, prec=orc.PREC_JACOBI)
    assert st[1] == orc.NONFINITE and st[0] == orc.CONVERGED and st[2] == orc.CONVERGED


def test_adaptive_forcing_reaches_the_same_root_with_fewer_krylov_steps(orc):
    # the forcing terms change only how accurately each Newton system is
    # solved: the root is the one MINPACK finds on the pinned residual, and
    # loose early solves save Krylov iterations
    from scipy.optimize import root
    N, M = 6, 5
    xi = draw_xi(3070, 2, M)
    alpha, beta = 10.0, 100.0
    rp, ci = orc.graph(N)
    uf, nif, lif, _, stf, _ = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, alpha, VEL, beta, xi, rtol=1e-11,
                                             lin_rtol=1e-3)
    ue, nie, lie, _, ste, fn = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, alpha, VEL, beta, xi, rtol=1e-11,
                                              lin_rtol=0.3, forcing=orc.FORCING_EW)
    assert (stf == orc.CONVERGED).all() and (ste == orc.CONVERGED).all()
    for e in range(2):
        ac = orc.kl_coef_qp(N, M, 1.0, 1.0, 0.3, xi[e])
        fun = lambda v: orc.nl_assemble_scalar(N, rp, ci, ac, 1.0, alpha, VEL, beta, v, want_jac=False)[0]
        ref = root(fun, np.zeros(orc.num_nodes(N)), method="hybr", options={"xtol": 1e-13}).x
        assert np.abs(ue[:, e] - ref).max() <= 1e-9 * np.abs(ref).max()
        assert np.abs(uf[:, e] - ref).max() <= 1e-9 * np.abs(ref).max()
        # each Newton step still reduces |F| (a loose first solve included)
        f = fn[e, :nie[e] + 1]
        assert (np.diff(f) < 0).all()
    assert lie.sum() < lif.sum()


def test_advection_cycle_saves_krylov_steps_where_advection_matters(orc):
    # the diffusion cycle misses the advection term, the D + alpha C cycle
    # does not: the same Newton iterates' systems need far fewer GMRES
    # steps, and the root is the same
    N, M = 16, 5
    xi = draw_xi(3090, 2, M)
    kw = dict(rtol=1e-10, lin_rtol=0.3, forcing=orc.FORCING_EW)
    u1, ni1, li1, _, st1, _ = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, 10.0, VEL, 100.0, xi, prec=orc.PREC_MG, **kw)
    u2, ni2, li2, _, st2, _ = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, 10.0, VEL, 100.0, xi, prec=orc.PREC_MG_ADV,
                                             **kw)
    assert (st1 == orc.CONVERGED).all() and (st2 == orc.CONVERGED).all()
    assert np.abs(u1 - u2).max() <= 1e-8 * np.abs(u1).max()
    assert li2.sum() <= 0.6 * li1.sum()


def _golden_rows(name):
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(t) for t in line.split()])
    return rows


def test_forcing_term_matches_the_hand_worked_values(orc):
    # tests/golden/ew_forcing.txt: each branch of Eisenstat-Walker choice 2
    # (plain ratio, safeguard used and unused, cap, floor, k = 0) worked by
    # hand from the published definition
    rows = _golden_rows("ew_forcing.txt")
    assert len(rows) >= 10
    for k, eta_prev, fn, fprev, eta_max, floor, want in rows:
        got = orc.ew_forcing(int(k), eta_prev, fn, fprev, eta_max, floor)
        assert got == pytest.approx(want, rel=1e-14, abs=0.0), (k, eta_prev, fn, fprev, eta_max, floor)


def test_newton_solves_each_system_to_its_forcing_term(orc):
    # the Newton loop feeds the pinned forcing function the right inputs:
    # eta_0 = eta_max, then |F_k|, |F_{k-1}|, eta_{k-1} and the floor
    # 0.5 rtol |load| / |F_k| (|load| = |F(u_0)| from u_0 = 0: boundary rows
    # are u_i = 0 there and interior rows are minus the load)
    N, M, s, rtol, eta_max = 6, 5, 3, 1e-11, 0.5
    xi = draw_xi(3075, s, M)
    _, ni, _, _, st, fn, eta = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, 10.0, VEL, 100.0, xi, rtol=rtol,
                                              lin_rtol=eta_max, forcing=orc.FORCING_EW, want_eta=True)
    assert (st == orc.CONVERGED).all()
    seen_below_cap = False
    for e in range(s):
        k_last = int(ni[e])
        assert k_last >= 3
        assert eta[e, 0] == eta_max
        for k in range(1, k_last):
            want = orc.ew_forcing(k, eta[e, k - 1], fn[e, k], fn[e, k - 1], eta_max, 0.5 * rtol * fn[e, 0] / fn[e, k])
            assert eta[e, k] == want, (e, k)
            seen_below_cap |= eta[e, k] < eta_max
        # no system is solved at the converged iterate
        assert (eta[e, k_last:] == 0.0).all()
    assert seen_below_cap
    # fixed forcing solves every system to lin_rtol
    _, ni2, _, _, _, _, eta2 = orc.ens_newton(N, M, 1.0, 1.0, 0.3, 1.0, 10.0, VEL, 100.0, xi, rtol=rtol,
                                              lin_rtol=1e-3, want_eta=True)
    for e in range(s):
        assert (eta2[e, :ni2[e]] == 1e-3).all()
