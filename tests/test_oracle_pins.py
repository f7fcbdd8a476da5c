"""Pins of the FP64 CPU oracle against what the mathematics fixes.

None of these checks re-types an oracle formula: each compares the oracle
with an independent construction (a Kronecker-sum discretisation, a Nystrom
eigen-solve, a Fourier series, a Galerkin projection on a Krylov basis, a
dense factorisation, a library routine) or with an invariant the method
must satisfy.  They run on the CPU only.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import draw_xi, draw_vector


# ------------------------------------------------------------------- graph

@pytest.mark.parametrize("N", [1, 2, 3, 5, 8])
def test_graph_closed_forms(orc, N):
    rp, ci = orc.graph(N)
    n = (N + 1) ** 3
    assert rp.shape[0] == n + 1
    assert rp[-1] == (3 * N + 1) ** 3
    lens = np.diff(rp)
    hist = {L: int((lens == L).sum()) for L in np.unique(lens)}
    expect = {27: (N - 1) ** 3, 18: 6 * (N - 1) ** 2, 12: 12 * (N - 1), 8: 8}
    expect = {k: v for k, v in expect.items() if v}
    assert hist == expect
    for i in range(n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)


@pytest.mark.parametrize("N", [2, 3])
def test_graph_matches_element_adjacency(orc, N):
    # independent construction: dense node adjacency from the element list
    n = (N + 1) ** 3
    adj = np.zeros((n, n), bool)
    nid = lambda i, j, k: i + (N + 1) * (j + (N + 1) * k)
    for ez, ey, ex in itertools.product(range(N), repeat=3):
        verts = [nid(ex + dx, ey + dy, ez + dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
        for a in verts:
            for b in verts:
                adj[a, b] = True
    rp, ci = orc.graph(N)
    dense = np.zeros((n, n), bool)
    for i in range(n):
        dense[i, ci[rp[i]:rp[i + 1]]] = True
    assert np.array_equal(dense, adj)


def test_elem_slot_points_at_element_pairs(orc):
    N = 3
    rp, ci = orc.graph(N)
    slot = orc.elem_slot(N, rp, ci)
    nid = lambda i, j, k: i + (N + 1) * (j + (N + 1) * k)
    for e in range(N ** 3):
        ex, ey, ez = e % N, (e // N) % N, e // (N * N)
        verts = [nid(ex + (a & 1), ey + ((a >> 1) & 1), ez + ((a >> 2) & 1)) for a in range(8)]
        for a in range(8):
            for b in range(8):
                k = slot[e, a, b]
                assert rp[verts[a]] <= k < rp[verts[a] + 1]
                assert ci[k] == verts[b]


# ---------------------------------------------------------------------- KL

def test_kl_1d_matches_nystrom(orc):
    # Nystrom (midpoint rule) discretisation of the integral operator with
    # kernel exp(-|x-x'|/L) on [0,1]; its top eigenvalues converge to the
    # operator's at O(h^2).
    # Richardson extrapolation of two resolutions removes the h^2 term.
    L = 1.0

    def nystrom(m):
        x = (np.arange(m) + 0.5) / m
        K = np.exp(-np.abs(x[:, None] - x[None, :]) / L) / m
        return np.sort(np.linalg.eigvalsh(K))[::-1][:8]

    ev = (4.0 * nystrom(3000) - nystrom(1500)) / 3.0
    w, lam, nrm, par = orc.kl_1d(8, L)
    assert np.all(np.diff(lam) < 0)
    np.testing.assert_allclose(lam, ev, rtol=1e-8)


@pytest.mark.parametrize("L", [0.5, 1.0, 2.0])
def test_kl_1d_eigen_equation_and_orthonormality(orc, L):
    K = 8
    w, lam, nrm, par = orc.kl_1d(K, L)

    def phi(k, x):
        t = x - 0.5
        return nrm[k] * (np.cos(w[k] * t) if par[k] == 0 else np.sin(w[k] * t))

    g, gw = np.polynomial.legendre.leggauss(60)
    xs = 0.5 * (g + 1.0)
    ws = 0.5 * gw
    G = np.array([[np.sum(ws * phi(i, xs) * phi(j, xs)) for j in range(K)] for i in range(K)])
    np.testing.assert_allclose(G, np.eye(K), atol=1e-12)
    # integral equation int_0^1 exp(-|x-x'|/L) phi(x') dx' = lambda phi(x),
    # split at x so each piece is smooth
    for x0 in (0.0, 0.13, 0.5, 0.77, 1.0):
        for k in range(K):
            tot = 0.0
            for lo, hi in ((0.0, x0), (x0, 1.0)):
                if hi <= lo:
                    continue
                xx = lo + (hi - lo) * 0.5 * (g + 1.0)
                tot += np.sum(0.5 * (hi - lo) * gw * np.exp(-np.abs(x0 - xx) / L) * phi(k, xx))
            assert abs(tot - lam[k] * phi(k, x0)) < 1e-12


def test_kl_1d_mercer_trace(orc):
    # sum of all eigenvalues = int_0^1 C(x,x) dx = 1 (unit variance)
    w, lam, nrm, par = orc.kl_1d(400, 1.0)
    tail = 2.0 / (np.pi * 401)  # lambda_k ~ 2c / w_k^2, w_k ~ k pi: tail sum bound
    assert 1.0 - tail - 1e-3 < lam.sum() < 1.0


def test_kl_3d_modes_order_and_orthonormality(orc):
    M = 13
    tr, lam3 = orc.kl_modes(M, 1.0)
    w, lam1, nrm, par = orc.kl_1d(M, 1.0)
    # descending, ties broken by ascending (ix, iy, iz)
    for m in range(M - 1):
        assert lam3[m] >= lam3[m + 1]
        if lam3[m] == lam3[m + 1]:
            assert tuple(tr[m]) < tuple(tr[m + 1])
    # permutations of one triple tie exactly
    assert lam3[1] == lam3[2] == lam3[3]
    # the ranking is a prefix of the full ranking of all triples by lambda
    allv = sorted((lam1[i] * lam1[j] * lam1[k] for i in range(M) for j in range(M) for k in range(M)),
                  reverse=True)
    np.testing.assert_allclose(lam3, allv[:M], rtol=1e-14)
    # orthogonality of the 3D fields sqrt(lambda_m) phi_m under tensor Gauss
    g, gw = np.polynomial.legendre.leggauss(24)
    x1 = 0.5 * (g + 1.0)
    w1 = 0.5 * gw
    X, Y, Z = np.meshgrid(x1, x1, x1, indexing="ij")
    W = (w1[:, None, None] * w1[None, :, None] * w1[None, None, :]).ravel()
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    fields = []
    for m in range(M):
        xi = np.zeros(M)
        xi[m] = 1.0
        fields.append(orc.kl_coef_points(M, 1.0, 0.0, 1.0, xi, pts))
    F = np.array(fields)
    Gm = (F * W) @ F.T
    np.testing.assert_allclose(Gm, np.diag(lam3), atol=1e-12)


def test_kl_3d_axis_assignment(orc):
    # the modes with one odd (sine) factor are odd about 1/2 along that
    # factor's axis and even along the other two
    M = 4
    tr, lam3 = orc.kl_modes(M, 1.0)
    rng = np.random.default_rng(3)
    base = rng.uniform(0, 1, (20, 3))
    for m in range(1, 4):
        xi = np.zeros(M)
        xi[m] = 1.0
        axis = int(np.argmax(tr[m]))
        a0 = orc.kl_coef_points(M, 1.0, 0.0, 1.0, xi, base)
        assert np.max(np.abs(a0)) > 1e-2
        for d in range(3):
            refl = base.copy()
            refl[:, d] = 1.0 - refl[:, d]
            a1 = orc.kl_coef_points(M, 1.0, 0.0, 1.0, xi, refl)
            np.testing.assert_allclose(a1, -a0 if d == axis else a0, atol=1e-14)


@pytest.mark.parametrize("M,sigma", [(3, 0.1), (10, 0.2), (10, 0.3)])
def test_kl_coefficient_positive_at_configs(orc, M, sigma):
    xi = draw_xi(77, 64, M)
    pts = orc.qp_coords(12).reshape(-1, 3)
    for e in range(xi.shape[0]):
        a = orc.kl_coef_points(M, 1.0, 1.0, sigma, xi[e], pts)
        assert a.min() > 0.2


# ---------------------------------------------------------------- assembly

def _q1_1d(N, wfun=None):
    """1D Q1 stiffness and mass on [0,1] with weight w(x), integrated with a
    4-point Gauss rule (exact for the polynomial weights used here)."""
    h = 1.0 / N
    K = np.zeros((N + 1, N + 1))
    Mm = np.zeros((N + 1, N + 1))
    g, gw = np.polynomial.legendre.leggauss(4)
    for e in range(N):
        xs = e * h + h * 0.5 * (g + 1.0)
        ws = h * 0.5 * gw
        wv = np.ones_like(xs) if wfun is None else wfun(xs)
        t = (xs - e * h) / h
        phi = [1.0 - t, t]
        dphi = [-1.0 / h, 1.0 / h]
        for a in range(2):
            for b in range(2):
                K[e + a, e + b] += np.sum(ws * wv * dphi[a] * dphi[b])
                Mm[e + a, e + b] += np.sum(ws * wv * phi[a] * phi[b])
    return K, Mm


def _dense(orc, rp, ci, vals):
    return orc.crs_to_dense(rp, ci, vals)


def test_element_matrix_closed_form(orc):
    # one element of side h at kappa = 1: K_e = (h/36) E with E_aa = 12,
    # 0 between vertices differing in one coordinate, -3 otherwise
    N = 1
    rp, ci = orc.graph(N)
    vals, rhs = orc.assemble_scalar(N, rp, ci, np.ones((1, 8)), dirichlet=False)
    A = _dense(orc, rp, ci, vals)
    E = np.zeros((8, 8))
    for a in range(8):
        for b in range(8):
            d = bin(a ^ b).count("1")
            E[a, b] = 12.0 if d == 0 else (0.0 if d == 1 else -3.0)
    np.testing.assert_allclose(A, E / 36.0, atol=1e-15)
    np.testing.assert_allclose(rhs, np.full(8, 1.0 / 8.0), atol=1e-16)


@pytest.mark.parametrize("N", [2, 3, 4])
def test_constant_coefficient_equals_kronecker_sum(orc, N):
    K1, M1 = _q1_1d(N)
    A_kron = (np.kron(np.kron(M1, M1), K1) + np.kron(np.kron(M1, K1), M1) + np.kron(np.kron(K1, M1), M1))
    rp, ci = orc.graph(N)
    vals, rhs = orc.assemble_scalar(N, rp, ci, np.ones((N ** 3, 8)), dirichlet=False)
    A = _dense(orc, rp, ci, vals)
    np.testing.assert_allclose(A, A_kron, atol=1e-14 * np.abs(A_kron).max())
    m = M1.sum(1)
    np.testing.assert_allclose(rhs, np.kron(np.kron(m, m), m), atol=1e-16)


@pytest.mark.parametrize("N", [2, 3])
def test_separable_variable_coefficient_equals_kronecker_sum(orc, N):
    # kappa = (1 + x)(1 + 2y)(1 + 3z): each 1D integrand is at most cubic, so
    # the 2x2x2 Gauss rule of the assembly is exact and must reproduce the
    # weighted Kronecker sum exactly (to rounding).
    fx = lambda x: 1.0 + x
    fy = lambda y: 1.0 + 2.0 * y
    fz = lambda z: 1.0 + 3.0 * z
    Kx, Mx = _q1_1d(N, fx)
    Ky, My = _q1_1d(N, fy)
    Kz, Mz = _q1_1d(N, fz)
    A_kron = np.kron(np.kron(Mz, My), Kx) + np.kron(np.kron(Mz, Ky), Mx) + np.kron(np.kron(Kz, My), Mx)
    pts = orc.qp_coords(N)
    acoef = fx(pts[..., 0]) * fy(pts[..., 1]) * fz(pts[..., 2])
    rp, ci = orc.graph(N)
    vals, rhs = orc.assemble_scalar(N, rp, ci, acoef, dirichlet=False)
    A = _dense(orc, rp, ci, vals)
    np.testing.assert_allclose(A, A_kron, atol=1e-13 * np.abs(A_kron).max())


@pytest.fixture(scope="module")
def kl_system(orc):
    N, M, sigma = 6, 10, 0.3
    rp, ci = orc.graph(N)
    xi = draw_xi(11, 3, M)
    out = []
    for e in range(3):
        ac = orc.kl_coef_qp(N, M, 1.0, 1.0, sigma, xi[e])
        raw, braw = orc.assemble_scalar(N, rp, ci, ac, dirichlet=False)
        bc, bbc = orc.assemble_scalar(N, rp, ci, ac, dirichlet=True)
        out.append((ac, raw, braw, bc, bbc))
    return N, rp, ci, out


def test_zero_row_sums_before_boundary_conditions(orc, kl_system):
    N, rp, ci, out = kl_system
    for ac, raw, braw, bc, bbc in out:
        rows = np.add.reduceat(raw, rp[:-1])
        diag = max(raw[k] for i in range(len(rp) - 1) for k in range(rp[i], rp[i + 1]) if ci[k] == i)
        assert np.max(np.abs(rows)) <= 64 * np.finfo(float).eps * diag
        assert abs(braw.sum() - 1.0) < 1e-14
        h = 1.0 / N
        interior = [i + (N + 1) * (j + (N + 1) * k) for k in range(1, N) for j in range(1, N) for i in range(1, N)]
        np.testing.assert_allclose(braw[interior], h ** 3, rtol=1e-14)


def test_bitwise_symmetry_and_spd(orc, kl_system):
    N, rp, ci, out = kl_system
    for ac, raw, braw, bc, bbc in out:
        for vals in (raw, bc):
            A = _dense(orc, rp, ci, vals)
            assert np.array_equal(A, A.T)
        A = _dense(orc, rp, ci, bc)
        assert np.linalg.eigvalsh(A).min() > 0
        x, ok = orc.cholesky_solve(A, bbc)
        assert ok
        np.testing.assert_allclose(x, np.linalg.solve(A, bbc), rtol=1e-12, atol=1e-15)


def test_dirichlet_rows_and_columns(orc, kl_system):
    N, rp, ci, out = kl_system
    nid = lambda i, j, k: i + (N + 1) * (j + (N + 1) * k)
    bnd = np.zeros((N + 1) ** 3, bool)
    for k, j, i in itertools.product(range(N + 1), repeat=3):
        bnd[nid(i, j, k)] = i in (0, N) or j in (0, N) or k in (0, N)
    for ac, raw, braw, bc, bbc in out:
        A = _dense(orc, rp, ci, bc)
        Araw = _dense(orc, rp, ci, raw)
        assert np.all(A[bnd][:, bnd] == np.eye(bnd.sum()))
        assert np.all(A[bnd][:, ~bnd] == 0) and np.all(A[~bnd][:, bnd] == 0)
        assert np.array_equal(A[~bnd][:, ~bnd], Araw[~bnd][:, ~bnd])
        assert np.all(bbc[bnd] == 0) and np.array_equal(bbc[~bnd], braw[~bnd])


def test_stencil_interior_row_constant_coefficient(orc):
    N, a = 6, 2.5
    rp, ci = orc.graph(N)
    vals, _ = orc.assemble_scalar(N, rp, ci, np.full((N ** 3, 8), a))
    h = 1.0 / N
    c = 3 + (N + 1) * (3 + (N + 1) * 3)
    row = dict(zip(ci[rp[c]:rp[c + 1]].tolist(), vals[rp[c]:rp[c + 1]].tolist()))
    nid = lambda i, j, k: i + (N + 1) * (j + (N + 1) * k)
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        d = abs(dx) + abs(dy) + abs(dz)
        expect = {0: 8.0 / 3.0, 1: 0.0, 2: -1.0 / 6.0, 3: -1.0 / 12.0}[d] * a * h
        assert abs(row[nid(3 + dx, 3 + dy, 3 + dz)] - expect) < 1e-15


# ------------------------------------------------------------------ solves

def _const_system(orc, N, a):
    rp, ci = orc.graph(N)
    vals, rhs = orc.assemble_scalar(N, rp, ci, np.full((N ** 3, 8), a))
    return rp, ci, vals, rhs


def test_single_interior_node_closed_form(orc):
    for a in (1.0, 0.5, 3.0):
        rp, ci, vals, rhs = _const_system(orc, 2, a)
        x, it, rel, st = orc.pcg(rp, ci, vals, rhs, rtol=1e-14)
        centre = 1 + 3 * (1 + 3 * 1)
        assert abs(x[centre] - 3.0 / (32.0 * a)) < 1e-15


def test_scaling_with_constant_coefficient(orc):
    rp, ci, v1, b1 = _const_system(orc, 6, 1.0)
    rp, ci, v3, b3 = _const_system(orc, 6, 3.0)
    x1 = orc.pcg(rp, ci, v1, b1, rtol=1e-14)[0]
    x3 = orc.pcg(rp, ci, v3, b3, rtol=1e-14)[0]
    np.testing.assert_allclose(x3, x1 / 3.0, rtol=1e-11, atol=1e-16)


def test_cube_symmetry(orc):
    N = 6
    rp, ci, vals, rhs = _const_system(orc, N, 1.0)
    x = orc.pcg(rp, ci, vals, rhs, rtol=1e-14)[0].reshape(N + 1, N + 1, N + 1)  # [k][j][i]
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product((False, True), repeat=3):
            y = np.transpose(x, perm)
            for ax, f in enumerate(flips):
                if f:
                    y = np.flip(y, ax)
            np.testing.assert_allclose(y, x, atol=1e-14)


@pytest.mark.parametrize("N", [2, 3, 4])
def test_cg_matches_dense_solve(orc, N):
    rp, ci = orc.graph(N)
    xi = draw_xi(5, 2, 10)
    for e in range(2):
        ac = orc.kl_coef_qp(N, 10, 1.0, 1.0, 0.3, xi[e])
        vals, rhs = orc.assemble_scalar(N, rp, ci, ac)
        A = orc.crs_to_dense(rp, ci, vals)
        xd, ok = orc.cholesky_solve(A, rhs)
        assert ok
        x, it, rel, st = orc.pcg(rp, ci, vals, rhs, rtol=1e-14)
        assert st == orc.CONVERGED and rel <= 1e-14 * (1 + 1e-6)
        assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


def test_pcg_iterates_are_krylov_galerkin(orc):
    # k steps of Jacobi-PCG from 0 give the A-orthogonal (Galerkin) projection
    # of the solution onto span{D^-1 r0, (D^-1 A) D^-1 r0, ...} (k terms).
    N = 3
    rp, ci = orc.graph(N)
    xi = draw_xi(9, 1, 10)[0]
    ac = orc.kl_coef_qp(N, 10, 1.0, 1.0, 0.3, xi)
    vals, b = orc.assemble_scalar(N, rp, ci, ac)
    A = orc.crs_to_dense(rp, ci, vals)
    Dinv = 1.0 / np.diag(A)
    v = Dinv * b
    basis = []
    for k in range(1, 6):
        basis.append(v)
        Q, _ = np.linalg.qr(np.array(basis).T)
        y = np.linalg.solve(Q.T @ A @ Q, Q.T @ b)
        xg = Q @ y
        xk = orc.pcg(rp, ci, vals, b, fixed_iters=k)[0]
        np.testing.assert_allclose(xk, xg, rtol=0, atol=1e-12 * np.abs(xg).max())
        v = Dinv * (A @ v)


def test_fixed_iterations_reproduce_tolerance_run(orc):
    rp, ci = orc.graph(8)
    xi = draw_xi(21, 1, 10)[0]
    ac = orc.kl_coef_qp(8, 10, 1.0, 1.0, 0.2, xi)
    vals, b = orc.assemble_scalar(8, rp, ci, ac)
    x, it, rel, st = orc.pcg(rp, ci, vals, b, rtol=1e-8)
    xf, itf, relf, stf = orc.pcg(rp, ci, vals, b, fixed_iters=it)
    assert itf == it and np.array_equal(x, xf)
    assert rel <= 1e-8 * (1 + 1e-6)
    xm, itm, relm, _ = orc.pcg(rp, ci, vals, b, fixed_iters=it - 1)
    assert relm > 1e-8 * 0.5


def _fourier_centre(K=301):
    i = np.arange(1, K + 1, 2, dtype=np.float64)
    s = (-1.0) ** ((np.arange(i.size)))  # sin(i pi / 2) for odd i
    I, J, Kk = np.meshgrid(i, i, i, indexing="ij")
    S = s[:, None, None] * s[None, :, None] * s[None, None, :]
    return float(np.sum(64.0 * S / (np.pi ** 5 * I * J * Kk * (I * I + J * J + Kk * Kk))))


def test_centre_value_converges_to_fourier_series(orc):
    # -Laplace u = 1 on the unit cube, u = 0 on the boundary; the continuum
    # centre value from the sine series, FE error O(h^2)
    exact = _fourier_centre()
    errs = []
    for N in (8, 16, 32):
        rp, ci, vals, rhs = _const_system(orc, N, 1.0)
        x = orc.pcg(rp, ci, vals, rhs, rtol=1e-13)[0]
        c = N // 2
        errs.append(abs(x[c + (N + 1) * (c + (N + 1) * c)] - exact))
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4
    assert errs[2] < 2e-3 * exact


def test_manufactured_solution_second_order(orc):
    errs = []
    for N in (8, 16, 32):
        rp, ci = orc.graph(N)
        vals, rhs = orc.assemble_scalar(N, rp, ci, np.ones((N ** 3, 8)), src_kind=1)
        x = orc.pcg(rp, ci, vals, rhs, rtol=1e-13)[0]
        g = np.arange(N + 1) / N
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        u = (np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)).ravel()
        errs.append(np.max(np.abs(x - u)))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


# --------------------------------------------------------------- products

def _random_crs(rng, n, maxlen, ncols):
    lens = rng.integers(0, maxlen + 1, n)
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([np.sort(rng.choice(ncols, L, replace=False)) for L in lens]).astype(np.int32)
    return rp, ci


def test_ensemble_product_layout_equals_scalar_products(orc):
    # Fig. ensemble_crs in the commuted layout against Fig. crs per sample:
    # both sum each row in entry order, so the results agree bit for bit.
    rng = np.random.default_rng(4)
    n, s = 97, 7
    rp, ci = _random_crs(rng, n, 40, n)
    vals = rng.standard_normal((rp[-1], s))
    x = rng.standard_normal((n, s))
    z = orc.ens_spmv(rp, ci, vals, x)
    for e in range(s):
        ze = orc.spmv(rp, ci, np.ascontiguousarray(vals[:, e]), np.ascontiguousarray(x[:, e]))
        assert np.array_equal(z[:, e], ze)
        A = sp.csr_matrix((vals[:, e], ci, rp), shape=(n, n))
        np.testing.assert_allclose(ze, A @ x[:, e], rtol=1e-13, atol=1e-13)


def test_ensemble_assembly_and_solve_equal_scalar_ones(orc):
    N, M, sigma = 5, 10, 0.3
    rp, ci = orc.graph(N)
    xi = draw_xi(31, 4, M)
    V, B = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    X, it, rel, st = orc.ens_pcg(rp, ci, V, B, rtol=1e-10)
    for e in range(4):
        ac = orc.kl_coef_qp(N, M, 1.0, 1.0, sigma, xi[e])
        v, b = orc.assemble_scalar(N, rp, ci, ac)
        assert np.array_equal(V[:, e], v) and np.array_equal(B[:, e], b)
        x, it1, rel1, st1 = orc.pcg(rp, ci, v, b, rtol=1e-10)
        assert np.array_equal(X[:, e], x) and it1 == it[e]


# ------------------------------------------------------ failure handling

def test_failure_statuses(orc):
    N = 4
    rp, ci, vals, rhs = _const_system(orc, N, 1.0)
    # negative definite: breakdown at the first p.Ap
    x, it, rel, st = orc.pcg(rp, ci, -vals, rhs)
    assert st == orc.BREAKDOWN and it == 0
    # iteration cap
    x, it, rel, st = orc.pcg(rp, ci, vals, rhs, max_iter=1, rtol=1e-12)
    assert st == orc.MAXITER and it == 1
    # zero right-hand side
    x, it, rel, st = orc.pcg(rp, ci, vals, np.zeros_like(rhs), x0=np.ones_like(rhs))
    assert st == orc.CONVERGED and it == 0 and not x.any()
    # NaN in the KL input propagates to a non-finite status
    ac = orc.kl_coef_qp(N, 3, 1.0, 1.0, 0.1, np.array([0.1, np.nan, 0.2]))
    v, b = orc.assemble_scalar(N, rp, ci, ac)
    x, it, rel, st = orc.pcg(rp, ci, v, b)
    assert st == orc.NONFINITE


def test_start_already_converged(orc):
    rp, ci, vals, rhs = _const_system(orc, 4, 1.0)
    xs = orc.pcg(rp, ci, vals, rhs, rtol=1e-14)[0]
    x, it, rel, st = orc.pcg(rp, ci, vals, rhs, x0=xs, rtol=1e-8)
    assert it == 0 and st == orc.CONVERGED and np.array_equal(x, xs)


# ----------------------------------------------- coupled ensemble CG (oracle)

def _block_system(orc, N, s, sigma, seed):
    rp, ci = orc.graph(N)
    xi = draw_xi(seed, s, 10)
    ov, ob = orc.assemble_ensemble(N, rp, ci, 10, 1.0, 1.0, sigma, 1.0, xi)
    blocks = [orc.crs_to_dense(rp, ci, np.ascontiguousarray(ov[:, e])) for e in range(s)]
    n = rp.shape[0] - 1
    A = np.zeros((n * s, n * s))
    for e, Ae in enumerate(blocks):
        A[e * n:(e + 1) * n, e * n:(e + 1) * n] = Ae
    b = ob.T.ravel()  # sample-major
    return rp, ci, ov, ob, A, b


def test_coupled_cg_iterates_are_block_krylov_galerkin(orc):
    # Coupled CG is CG on blockdiag(A_1..A_s): k steps from 0 give the
    # Galerkin projection onto the Jacobi-preconditioned Krylov space of the
    # whole block system (one space for all samples, not one per sample).
    N, s = 3, 3
    rp, ci, ov, ob, A, b = _block_system(orc, N, s, 0.3, 31)
    n = rp.shape[0] - 1
    Dinv = 1.0 / np.diag(A)
    v = Dinv * b
    basis = []
    for k in range(1, 7):
        basis.append(v)
        Q, _ = np.linalg.qr(np.array(basis).T)
        xg = Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ b)
        xk, it, _, _ = orc.ens_pcg_coupled(rp, ci, ov, ob, fixed_iters=k)
        assert it == k
        np.testing.assert_allclose(xk.T.ravel(), xg, rtol=0, atol=1e-12 * np.abs(xg).max())
        v = Dinv * (A @ v)
    # differs from the per-sample iteration, whose Krylov spaces are separate
    xs, _, _, _ = orc.ens_pcg(rp, ci, ov, ob, fixed_iters=np.full(s, 3, np.int32))
    xc, _, _, _ = orc.ens_pcg_coupled(rp, ci, ov, ob, fixed_iters=3)
    assert np.abs(xs - xc).max() > 1e-8 * np.abs(xs).max()
    # converged: every block solved; total residual within tolerance
    x, it, rel, st = orc.ens_pcg_coupled(rp, ci, ov, ob, rtol=1e-13)
    assert st == orc.CONVERGED and rel <= 1e-13 * (1 + 1e-6)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x.T.ravel() - xd) <= 1e-11 * np.linalg.norm(xd)
    assert 1 <= it <= n * s


def test_coupled_cg_of_identical_samples_is_the_scalar_cg(orc):
    # with s equal samples every ensemble sum is s times the sample's own, so
    # alpha, beta and the stopping test are those of the one-sample CG
    N, s = 6, 4
    rp, ci = orc.graph(N)
    xi = np.repeat(draw_xi(32, 1, 10), s, axis=0)
    ov, ob = orc.assemble_ensemble(N, rp, ci, 10, 1.0, 1.0, 0.3, 1.0, xi)
    x1, it1, rel1, _ = orc.pcg(rp, ci, np.ascontiguousarray(ov[:, 0]), np.ascontiguousarray(ob[:, 0]), rtol=1e-10)
    xc, itc, relc, stc = orc.ens_pcg_coupled(rp, ci, ov, ob, rtol=1e-10)
    assert itc == it1 and stc == orc.CONVERGED
    for e in range(s):
        np.testing.assert_allclose(xc[:, e], x1, rtol=0, atol=1e-12 * np.abs(x1).max())


# ------------------------------------------------------- multigrid (oracle)

def test_mg_hierarchy_levels(orc):
    assert orc.mg_levels(128) == [128, 64, 32, 16, 8, 4]
    assert orc.mg_levels(96) == [96, 48, 24, 12, 6, 3]
    assert orc.mg_levels(7) == [7] and orc.mg_levels(4) == [4]


def _coords(N):
    t = np.arange(N + 1) / N
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def test_mg_prolongation_interpolates_trilinear_functions(orc):
    # P is the coarse Q1 basis written in the fine one: a trilinear function
    # given at the coarse nodes is reproduced at every fine node whose parents
    # are interior; fine boundary nodes receive nothing
    Nc = 4
    Nf = 2 * Nc
    f = lambda x, y, z: 1 + x + 2 * y + 3 * z + x * y - 0.5 * y * z + 2 * x * y * z
    Xc, Yc, Zc = _coords(Nc)
    xc = f(Xc, Yc, Zc)
    Xf, Yf, Zf = _coords(Nf)
    base = np.random.default_rng(3).uniform(-1, 1, Xf.size)
    xf = orc.mg_prolong_add(Nc, xc, base) - base
    idx = np.arange(Xf.size)
    i, j, k = idx % (Nf + 1), (idx // (Nf + 1)) % (Nf + 1), idx // (Nf + 1) ** 2
    deep = (i >= 2) & (i <= Nf - 2) & (j >= 2) & (j <= Nf - 2) & (k >= 2) & (k <= Nf - 2)
    np.testing.assert_allclose(xf[deep], f(Xf, Yf, Zf)[deep], rtol=1e-14, atol=1e-14)
    bnd = (i == 0) | (j == 0) | (k == 0) | (i == Nf) | (j == Nf) | (k == Nf)
    assert not xf[bnd].any()


def test_mg_restriction_is_the_adjoint_of_prolongation(orc):
    rng = np.random.default_rng(4)
    for Nc in (2, 3, 5):
        u = rng.standard_normal((Nc + 1) ** 3)
        v = rng.standard_normal((2 * Nc + 1) ** 3)
        Pu = orc.mg_prolong_add(Nc, u, np.zeros(v.size))
        Rv = orc.mg_restrict(2 * Nc, v)
        assert abs(Pu @ v - u @ Rv) <= 1e-13 * np.abs(Pu).sum() * np.abs(v).max()


def _dense_P(orc, Nc):
    nc, nf = (Nc + 1) ** 3, (2 * Nc + 1) ** 3
    P = np.zeros((nf, nc))
    for c in range(nc):
        e = np.zeros(nc)
        e[c] = 1.0
        P[:, c] = orc.mg_prolong_add(Nc, e, np.zeros(nf))
    return P


def test_mg_galerkin_product_equals_coarse_assembly(orc):
    # nested Q1 spaces with an exactly integrated constant coefficient: the
    # Galerkin operator P^T A_f P is the matrix assembled on the coarse mesh
    Nc = 3
    Nf = 2 * Nc
    mats = []
    for N in (Nf, Nc):
        rp, ci = orc.graph(N)
        ac = orc.kl_coef_qp(N, 4, 1.0, 1.7, 0.0, np.zeros(4))
        vals, _ = orc.assemble_scalar(N, rp, ci, ac)
        mats.append(orc.crs_to_dense(rp, ci, vals))
    Af, Ac = mats
    P = _dense_P(orc, Nc)
    G = P.T @ Af @ P
    idx = np.arange((Nc + 1) ** 3)
    i, j, k = idx % (Nc + 1), (idx // (Nc + 1)) % (Nc + 1), idx // (Nc + 1) ** 2
    inner = (i > 0) & (j > 0) & (k > 0) & (i < Nc) & (j < Nc) & (k < Nc)
    np.testing.assert_allclose(G[np.ix_(inner, inner)], Ac[np.ix_(inner, inner)], rtol=0,
                               atol=1e-13 * np.abs(Ac).max())


def _hat_P(Nc):
    """Trilinear interpolation from interior coarse nodes to interior fine
    nodes built from the coarse hat functions: P[i, J] = prod over axes of
    max(0, 1 - Nc |x_i - X_J|) at the fine node coordinates x_i."""
    Nf = 2 * Nc

    def coords(N):
        idx = np.arange((N + 1) ** 3)
        c = np.stack([idx % (N + 1), (idx // (N + 1)) % (N + 1), idx // (N + 1) ** 2], 1)
        return c / N, ((c > 0) & (c < N)).all(1)

    xf, inf_ = coords(Nf)
    xc, inc = coords(Nc)
    P = np.prod(np.maximum(0.0, 1.0 - Nc * np.abs(xf[:, None, :] - xc[None, :, :])), axis=2)
    # at fine nodes the hat values are products of 1 and 1/2: remove the
    # rounding of the coordinates
    P = np.round(P * 8.0) / 8.0
    P[~inf_, :] = 0.0
    P[:, ~inc] = 0.0
    return P, inc


def _fine_matrix(orc, N, sigma, seed, M=10):
    rp, ci = orc.graph(N)
    xi = draw_xi(seed, 1, M)[0]
    ac = orc.kl_coef_qp(N, M, 1.0, 1.0, sigma, xi)
    vals, _ = orc.assemble_scalar(N, rp, ci, ac)
    return rp, ci, vals, xi


@pytest.mark.parametrize("Nc", [2, 3, 4])
def test_mg_galerkin_operator_is_the_dense_triple_product(orc, Nc):
    # Alg. vcycle forms A^{k+1} = R A^k P with R = P^T: at a variable
    # coefficient the oracle's product equals dense P^T A P, P built from the
    # coarse hat functions (not from the oracle's transfer code); boundary
    # rows are identities and interior rows have no boundary entries
    rp, ci, vals, _ = _fine_matrix(orc, 2 * Nc, 0.3, 5100 + Nc)
    P, inner = _hat_P(Nc)
    np.testing.assert_array_equal(P, _dense_P(orc, Nc))
    G = P.T @ orc.crs_to_dense(rp, ci, vals) @ P
    rpc, cic = orc.graph(Nc)
    Ac = orc.crs_to_dense(rpc, cic, orc.mg_galerkin(Nc, rp, ci, vals))
    scale = np.abs(G).max()
    np.testing.assert_allclose(Ac[np.ix_(inner, inner)], G[np.ix_(inner, inner)], rtol=0, atol=1e-14 * scale)
    bnd = ~inner
    np.testing.assert_array_equal(Ac[bnd], np.eye(inner.size)[bnd])
    assert (Ac[np.ix_(inner, bnd)] == 0.0).all()
    Ai = Ac[np.ix_(inner, inner)]
    np.testing.assert_allclose(Ai, Ai.T, rtol=0, atol=1e-15 * scale)
    assert np.linalg.eigvalsh(0.5 * (Ai + Ai.T)).min() > 0.0


def test_mg_galerkin_differs_from_rediscretization_only_at_variable_coefficient(orc):
    Nc = 4
    rpc, cic = orc.graph(Nc)
    for sigma, same in ((0.0, True), (0.3, False)):
        rp, ci, vals, xi = _fine_matrix(orc, 2 * Nc, sigma, 5200)
        g = orc.mg_galerkin(Nc, rp, ci, vals)
        ac = orc.kl_coef_qp(Nc, 10, 1.0, 1.0, sigma, xi)
        r, _ = orc.assemble_scalar(Nc, rpc, cic, ac)
        d = np.abs(g - r).max() / np.abs(r).max()
        assert (d <= 1e-14) if same else (d >= 1e-4), (sigma, d)


def test_mg_galerkin_coarse_correction_is_an_a_orthogonal_projection(orc):
    # with A_c = P^T A P the two-grid coarse correction E = I - P A_c^-1 P^T A
    # satisfies E^2 = E and A E = E^T A (an A-orthogonal projection): the
    # variational property Galerkin coarse operators are chosen for; the
    # rediscretized A_c of a variable coefficient has neither
    Nc = 4
    rp, ci, vals, xi = _fine_matrix(orc, 2 * Nc, 0.3, 5300)
    P, inner_c = _hat_P(Nc)
    Af = orc.crs_to_dense(rp, ci, vals)
    nf = Af.shape[0]
    idx = np.arange(nf)
    c = np.stack([idx % (2 * Nc + 1), (idx // (2 * Nc + 1)) % (2 * Nc + 1), idx // (2 * Nc + 1) ** 2], 1)
    inner_f = ((c > 0) & (c < 2 * Nc)).all(1)
    A = Af[np.ix_(inner_f, inner_f)]
    Pi = P[np.ix_(inner_f, inner_c)]
    rpc, cic = orc.graph(Nc)
    ac = orc.kl_coef_qp(Nc, 10, 1.0, 1.0, 0.3, xi)
    redisc, _ = orc.assemble_scalar(Nc, rpc, cic, ac)
    for vc, proj in ((orc.mg_galerkin(Nc, rp, ci, vals), True), (redisc, False)):
        Ac = orc.crs_to_dense(rpc, cic, vc)[np.ix_(inner_c, inner_c)]
        E = np.eye(A.shape[0]) - Pi @ np.linalg.solve(Ac, Pi.T @ A)
        d2 = np.abs(E @ E - E).max()
        dsym = np.abs(A @ E - E.T @ A).max() / np.abs(A).max()
        if proj:
            assert d2 <= 1e-12 and dsym <= 1e-12, (d2, dsym)
        else:
            assert d2 >= 1e-4, d2


def test_mg_galerkin_pcg_converges_to_the_dense_solution(orc):
    N, M, sigma = 8, 10, 0.3
    xi = draw_xi(42, 3, M)
    x, it, rr, st, lm = orc.ens_mg_pcg(N, M, 1.0, 1.0, sigma, 1.0, xi, rtol=1e-12, galerkin=True)
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    for e in range(3):
        A = orc.crs_to_dense(rp, ci, np.ascontiguousarray(ov[:, e]))
        xd = np.linalg.solve(A, ob[:, e])
        assert st[e] == orc.CONVERGED and rr[e] <= 1e-12 * (1 + 1e-6)
        assert np.linalg.norm(x[:, e] - xd) <= 1e-10 * np.linalg.norm(xd)
        assert it[e] <= 10
        # the coarse level's bound is that of the Galerkin matrix
        g = orc.mg_galerkin(4, rp, ci, np.ascontiguousarray(ov[:, e]))
        rpc, cic = orc.graph(4)
        assert lm[e, 1] == orc.gershgorin(rpc, cic, g)


def test_chebyshev_smoother_matches_its_polynomial(orc):
    # order-2 Chebyshev on [lmax/4, lmax] from x = 0: the error in each
    # eigenvector of D^-1 A is multiplied by T2((theta-l)/delta) / T2(theta/delta)
    n = 40
    rp = [0]
    ci, vals = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                vals.append(2.0 if i == j else -1.0)
        rp.append(len(ci))
    rp, ci, vals = np.array(rp, np.int32), np.array(ci, np.int32), np.array(vals)
    A = orc.crs_to_dense(rp, ci, vals)
    lmax = orc.gershgorin(rp, ci, vals)
    assert lmax == 2.0
    b = np.random.default_rng(5).standard_normal(n)
    xs = np.linalg.solve(A, b)
    x = orc.mg_cheb2(rp, ci, vals, lmax, b)
    lam, Q = np.linalg.eigh(A / 2.0)   # D^-1 A, D = 2 I
    hi, lo = lmax, lmax / 4.0
    th, de = (hi + lo) / 2, (hi - lo) / 2
    T2 = lambda t: 2 * t * t - 1
    R = T2((th - lam) / de) / T2(th / de)
    np.testing.assert_allclose(xs - x, Q @ (R * (Q.T @ xs)), rtol=0, atol=1e-12 * np.abs(xs).max())
    # a second application from the result continues with the same polynomial
    x2 = orc.mg_cheb2(rp, ci, vals, lmax, b, x0=x)
    np.testing.assert_allclose(xs - x2, Q @ (R * R * (Q.T @ xs)), rtol=0, atol=1e-12 * np.abs(xs).max())


def test_vcycle_is_spd_and_contracts(orc):
    N, M, sigma = 8, 10, 0.3
    xi = draw_xi(41, 1, M)[0]
    n = (N + 1) ** 3
    idx = np.arange(n)
    i, j, k = idx % (N + 1), (idx // (N + 1)) % (N + 1), idx // (N + 1) ** 2
    inner = np.flatnonzero((i > 0) & (j > 0) & (k > 0) & (i < N) & (j < N) & (k < N))
    Mop = np.zeros((n, inner.size))
    for c, t in enumerate(inner):
        e = np.zeros(n)
        e[t] = 1.0
        Mop[:, c] = orc.mg_apply(N, M, 1.0, 1.0, sigma, 1.0, xi, e)
    Mi = Mop[inner]
    np.testing.assert_allclose(Mi, Mi.T, rtol=0, atol=1e-13 * np.abs(Mi).max())
    assert np.linalg.eigvalsh(0.5 * (Mi + Mi.T)).min() > 0
    assert not Mop[np.setdiff1d(idx, inner)].any()   # no correction on the boundary
    rp, ci = orc.graph(N)
    ac = orc.kl_coef_qp(N, M, 1.0, 1.0, sigma, xi)
    vals, _ = orc.assemble_scalar(N, rp, ci, ac)
    Ai = orc.crs_to_dense(rp, ci, vals)[np.ix_(inner, inner)]
    ev = np.linalg.eigvals(np.eye(inner.size) - Mi @ Ai)
    assert np.abs(ev).max() < 0.15


def test_mg_pcg_converges_to_the_dense_solution(orc):
    N, M, sigma = 8, 10, 0.3
    xi = draw_xi(42, 3, M)
    x, it, rr, st, lm = orc.ens_mg_pcg(N, M, 1.0, 1.0, sigma, 1.0, xi, rtol=1e-12)
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    for e in range(3):
        A = orc.crs_to_dense(rp, ci, np.ascontiguousarray(ov[:, e]))
        xd = np.linalg.solve(A, ob[:, e])
        assert st[e] == orc.CONVERGED and rr[e] <= 1e-12 * (1 + 1e-6)
        assert np.linalg.norm(x[:, e] - xd) <= 1e-10 * np.linalg.norm(xd)
        assert it[e] <= 10
        assert lm[e, 0] == orc.gershgorin(rp, ci, np.ascontiguousarray(ov[:, e]))
    # fewer iterations than Jacobi, and the count does not grow with the mesh
    its = [orc.ens_mg_pcg(Nn, M, 1.0, 1.0, sigma, 1.0, xi[:1], rtol=1e-10)[1][0] for Nn in (8, 16, 32)]
    assert max(its) - min(its) <= 3
