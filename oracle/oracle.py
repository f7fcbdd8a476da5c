"""ctypes front end of the FP64 CPU oracle (``ens_oracle.c``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It never imports the GPU
package, and the GPU package never imports it.

Every function follows one passage of Phipps et al. (arXiv 1511.03703); the
C source names the passage next to each routine.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ens_oracle.c")
_LIB = os.path.join(_HERE, "libensoracle.so")

CONVERGED, MAXITER, BREAKDOWN, NONFINITE = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-Wall", "-Wno-unused-function", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        i32, i64, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.orc_num_nodes.restype = i64
        L.orc_num_nodes.argtypes = [ctypes.c_int]
        L.orc_num_elems.restype = i64
        L.orc_num_elems.argtypes = [ctypes.c_int]
        L.orc_graph_nnz.restype = i64
        L.orc_graph_nnz.argtypes = [ctypes.c_int]
        L.orc_graph.argtypes = [ctypes.c_int, vp, vp]
        L.orc_elem_slot.argtypes = [ctypes.c_int, vp, vp, vp]
        L.orc_kl_1d.argtypes = [ctypes.c_int, dbl, vp, vp, vp, vp]
        L.orc_kl_modes.argtypes = [ctypes.c_int, dbl, vp, vp]
        L.orc_kl_coef_points.argtypes = [ctypes.c_int, dbl, dbl, dbl, vp, i64, vp, vp]
        L.orc_qp_coords.argtypes = [ctypes.c_int, vp]
        L.orc_kl_coef_qp.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, vp, vp]
        L.orc_assemble_scalar.argtypes = [ctypes.c_int, vp, vp, vp, ctypes.c_int, dbl, ctypes.c_int, vp, vp]
        L.orc_assemble_ensemble.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int, dbl, dbl, dbl, dbl,
                                            ctypes.c_int, vp, vp, vp]
        L.orc_spmv.restype = None
        L.orc_spmv.argtypes = [i64, vp, vp, vp, vp, vp]
        L.orc_ens_spmv.restype = None
        L.orc_ens_spmv.argtypes = [i64, ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_pcg.argtypes = [i64, vp, vp, vp, vp, vp, dbl, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.orc_ens_pcg.argtypes = [i64, ctypes.c_int, vp, vp, vp, vp, vp, dbl, ctypes.c_int, vp, vp, vp, vp]
        L.orc_mg_levels.argtypes = [ctypes.c_int, vp]
        L.orc_mg_prolong_add.argtypes = [ctypes.c_int, vp, vp]
        L.orc_mg_restrict.argtypes = [ctypes.c_int, vp, vp]
        L.orc_gershgorin.restype = dbl
        L.orc_gershgorin.argtypes = [i64, vp, vp, vp]
        L.orc_mg_cheb2.argtypes = [i64, vp, vp, vp, dbl, vp, vp, ctypes.c_int, vp, vp, vp]
        L.orc_mg_apply.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, dbl, vp, vp, vp, ctypes.c_int]
        L.orc_mg_galerkin.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_mg_apply_adv.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, dbl, dbl, vp, vp, vp, vp]
        L.orc_mg_pcg.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, dbl, vp, vp, dbl, ctypes.c_int,
                                 ctypes.c_int, vp, vp, vp, vp, ctypes.c_int]
        L.orc_ens_mg_pcg.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, dbl, ctypes.c_int, vp, vp, dbl,
                                     ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_int]
        L.orc_ens_pcg_coupled.argtypes = [i64, ctypes.c_int, vp, vp, vp, vp, vp, dbl, ctypes.c_int, ctypes.c_int,
                                          vp, vp, vp]
        L.orc_solve_sample.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, dbl, vp, dbl,
                                       ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_solve_samples.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, dbl, ctypes.c_int,
                                        vp, dbl, ctypes.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_ens_true_residual.restype = None
        L.orc_ens_true_residual.argtypes = [i64, ctypes.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_crs_to_dense.restype = None
        L.orc_crs_to_dense.argtypes = [i64, vp, vp, vp, vp]
        L.orc_cholesky_solve.argtypes = [i64, vp, vp, vp]
        L.orc_nl_assemble_scalar.argtypes = [ctypes.c_int, vp, vp, vp, dbl, dbl, vp, dbl, vp, vp, vp, vp]
        L.orc_ens_nl_assemble.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int, dbl, dbl, dbl, dbl, dbl, vp, dbl,
                                          ctypes.c_int, vp, vp, vp, vp, vp]
        L.orc_gmres.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, vp,
                                dbl, vp, dbl, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.orc_ens_gmres.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, vp, ctypes.c_int, ctypes.c_int, dbl,
                                    dbl, dbl, vp, dbl, vp, dbl, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp]
        L.orc_newton.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, dbl, dbl, vp, dbl, vp, vp, ctypes.c_int,
                                 dbl, ctypes.c_int, dbl, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp,
                                 vp]
        L.orc_ens_newton.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl, dbl, dbl, dbl, vp, dbl, ctypes.c_int, vp,
                                     vp, ctypes.c_int, dbl, ctypes.c_int, dbl, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, vp, vp, vp, vp, vp, vp]
        L.orc_ew_forcing.restype = dbl
        L.orc_ew_forcing.argtypes = [ctypes.c_int, dbl, dbl, dbl, dbl, dbl]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle call failed with status {rc}")


# --------------------------------------------------------------------- mesh


def num_nodes(N: int) -> int:
    return int(lib().orc_num_nodes(N))


def num_elems(N: int) -> int:
    return int(lib().orc_num_elems(N))


def graph(N: int):
    """CRS graph of the Q1 stiffness matrix (Fig. crs), columns ascending."""
    n = num_nodes(N)
    nnz = int(lib().orc_graph_nnz(N))
    rp = np.zeros(n + 1, np.int32)
    ci = np.zeros(nnz, np.int32)
    _check(lib().orc_graph(N, _p(rp), _p(ci)))
    return rp, ci


def elem_slot(N: int, rp, ci):
    """ElemGraph map of Alg. assembly: CRS index of (node(e,a), node(e,b))."""
    out = np.zeros((num_elems(N), 8, 8), np.int64)
    _check(lib().orc_elem_slot(N, _p(rp), _p(ci), _p(out)))
    return out


# ----------------------------------------------------------------------- KL


def kl_1d(K: int, L: float = 1.0):
    """First K 1D eigenpairs of exp(-|t-t'|/L) on [0,1], lambda descending."""
    w = np.zeros(K)
    lam = np.zeros(K)
    nrm = np.zeros(K)
    par = np.zeros(K, np.int32)
    _check(lib().orc_kl_1d(K, L, _p(w), _p(lam), _p(nrm), _p(par)))
    return w, lam, nrm, par


def kl_modes(M: int, L: float = 1.0):
    tr = np.zeros((M, 3), np.int32)
    lam = np.zeros(M)
    _check(lib().orc_kl_modes(M, L, _p(tr), _p(lam)))
    return tr, lam


def kl_coef_points(M, L, kappa0, sigma, xi, pts):
    xi = _f64(xi).reshape(-1)
    pts = _f64(pts).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    _check(lib().orc_kl_coef_points(M, L, kappa0, sigma, _p(xi), pts.shape[0], _p(pts), _p(out)))
    return out


def qp_coords(N):
    out = np.zeros((num_elems(N), 8, 3))
    _check(lib().orc_qp_coords(N, _p(out)))
    return out


def kl_coef_qp(N, M, L, kappa0, sigma, xi):
    out = np.zeros((num_elems(N), 8))
    xi = _f64(xi).reshape(-1)
    _check(lib().orc_kl_coef_qp(N, M, L, kappa0, sigma, _p(xi), _p(out)))
    return out


def sample_extrema(N, M, L, kappa0, sigma, xi):
    """Per-sample minimum and maximum of the coefficient over the Gauss
    points of the N^3 mesh (the variation of a sample's parameters over the
    domain, Sec. 3.7's predictor of its iteration count), by evaluating it
    at every point: (kmin [s], kmax [s])."""
    xi = np.atleast_2d(_f64(xi))
    kmin, kmax = np.zeros(xi.shape[0]), np.zeros(xi.shape[0])
    for e in range(xi.shape[0]):
        a = kl_coef_qp(N, M, L, kappa0, sigma, xi[e])
        kmin[e], kmax[e] = (np.nan, np.nan) if not np.isfinite(a).all() else (a.min(), a.max())
    return kmin, kmax


# ----------------------------------------------------------------- assembly


def assemble_scalar(N, rp, ci, acoef, src_kind=0, fconst=1.0, dirichlet=True):
    """One sample's A (CRS values) and load vector f from the coefficient at
    the quadrature points, acoef[N^3][8] (Alg. assembly)."""
    n = num_nodes(N)
    vals = np.zeros(int(rp[-1]))
    rhs = np.zeros(n)
    acoef = _f64(acoef)
    _check(lib().orc_assemble_scalar(N, _p(rp), _p(ci), _p(acoef), src_kind, fconst, int(dirichlet),
                                     _p(vals), _p(rhs)))
    return vals, rhs


def assemble_ensemble(N, rp, ci, M, L, kappa0, sigma, fconst, xi):
    """values [nnz][s] and rhs [n][s] in the commuted layout."""
    xi = _f64(xi)
    s = xi.shape[0]
    n = num_nodes(N)
    vals = np.zeros((int(rp[-1]), s))
    rhs = np.zeros((n, s))
    _check(lib().orc_assemble_ensemble(N, _p(rp), _p(ci), M, L, kappa0, sigma, fconst, s, _p(xi),
                                       _p(vals), _p(rhs)))
    return vals, rhs


# ----------------------------------------------------------------- products


def spmv(rp, ci, vals, x):
    n = rp.shape[0] - 1
    x = _f64(x)
    z = np.zeros(n)
    lib().orc_spmv(n, _p(rp), _p(ci), _p(_f64(vals)), _p(x), _p(z))
    return z


def ens_spmv(rp, ci, vals, x):
    n = rp.shape[0] - 1
    s = vals.shape[1]
    z = np.zeros((n, s))
    lib().orc_ens_spmv(n, s, _p(rp), _p(ci), _p(_f64(vals)), _p(_f64(x)), _p(z))
    return z


# ------------------------------------------------------------------- solves


def pcg(rp, ci, vals, b, x0=None, rtol=1e-10, max_iter=10000, fixed_iters=-1):
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    it = np.zeros(1, np.int32)
    rr = np.zeros(1)
    st = np.zeros(1, np.int32)
    _check(lib().orc_pcg(n, _p(rp), _p(ci), _p(_f64(vals)), _p(_f64(b)), _p(x), rtol, max_iter,
                         fixed_iters, _p(it), _p(rr), _p(st)))
    return x, int(it[0]), float(rr[0]), int(st[0])


def ens_pcg(rp, ci, vals, b, x0=None, rtol=1e-10, max_iter=10000, fixed_iters=None):
    n = rp.shape[0] - 1
    s = vals.shape[1]
    x = np.zeros((n, s)) if x0 is None else _f64(x0).copy()
    it = np.zeros(s, np.int32)
    rr = np.zeros(s)
    st = np.zeros(s, np.int32)
    fi = None if fixed_iters is None else np.ascontiguousarray(fixed_iters, np.int32)
    _check(lib().orc_ens_pcg(n, s, _p(rp), _p(ci), _p(_f64(vals)), _p(_f64(b)), _p(x), rtol, max_iter,
                             None if fi is None else _p(fi), _p(it), _p(rr), _p(st)))
    return x, it, rr, st


def ens_pcg_coupled(rp, ci, vals, b, x0=None, rtol=1e-10, max_iter=10000, fixed_iters=-1):
    """Coupled ensemble CG (one system over all samples).  Returns (x [n][s],
    iters, rel_res over all samples, status)."""
    n = rp.shape[0] - 1
    s = vals.shape[1]
    x = np.zeros((n, s)) if x0 is None else _f64(x0).copy()
    it = np.zeros(1, np.int32)
    rr = np.zeros(1)
    st = np.zeros(1, np.int32)
    _check(lib().orc_ens_pcg_coupled(n, s, _p(rp), _p(ci), _p(_f64(vals)), _p(_f64(b)), _p(x), rtol, max_iter,
                                     int(fixed_iters), _p(it), _p(rr), _p(st)))
    return x, int(it[0]), float(rr[0]), int(st[0])


MG_MAX_LEVELS = 16


def mg_levels(N):
    Ns = np.zeros(MG_MAX_LEVELS, np.int32)
    k = lib().orc_mg_levels(N, _p(Ns))
    return [int(v) for v in Ns[:k]]


def mg_prolong_add(Nc, xc, xf):
    xf = _f64(xf).copy()
    lib().orc_mg_prolong_add(Nc, _p(_f64(xc)), _p(xf))
    return xf


def mg_restrict(Nf, rf):
    rc = np.zeros(num_nodes(Nf // 2))
    lib().orc_mg_restrict(Nf, _p(_f64(rf)), _p(rc))
    return rc


def gershgorin(rp, ci, vals):
    return float(lib().orc_gershgorin(rp.shape[0] - 1, _p(rp), _p(ci), _p(_f64(vals))))


def mg_cheb2(rp, ci, vals, lmax, b, x0=None):
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    r, d, ax = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_mg_cheb2(n, _p(rp), _p(ci), _p(_f64(vals)), lmax, _p(_f64(b)), _p(x), int(x0 is None), _p(r), _p(d),
                       _p(ax))
    return x


def mg_apply(N, M, L, kappa0, sigma, fconst, xi, r, galerkin=False):
    """z = M r, one V-cycle; coarse levels rediscretized, or with galerkin
    the products P^T A P of the level above."""
    z = np.zeros(num_nodes(N))
    _check(lib().orc_mg_apply(N, M, L, kappa0, sigma, fconst, _p(_f64(xi)), _p(_f64(r)), _p(z), int(galerkin)))
    return z


def mg_galerkin(Nc, rpf, cif, vf):
    """Values of the Galerkin coarse operator P^T A P (identity boundary
    rows) on orc_graph(Nc), from the fine matrix (rpf, cif, vf) on 2 Nc."""
    rpc, cic = graph(Nc)
    vc = np.zeros(cic.shape[0])
    _check(lib().orc_mg_galerkin(Nc, _p(rpf), _p(cif), _p(_f64(vf)), _p(rpc), _p(cic), _p(vc)))
    return vc


def mg_apply_adv(N, M, L, kappa0, sigma, fconst, alpha, vel, xi, r):
    """z = M r for the V-cycle of the advection-diffusion operator D + alpha C."""
    z = np.zeros(num_nodes(N))
    _check(lib().orc_mg_apply_adv(N, M, L, kappa0, sigma, fconst, alpha, _p(_f64(vel)), _p(_f64(xi)),
                                  _p(_f64(r)), _p(z)))
    return z


def max_threads():
    return int(lib().orc_max_threads())


def ens_mg_pcg(N, M, L, kappa0, sigma, fconst, xi, x0=None, rtol=1e-10, max_iter=10000, fixed_iters=None,
               galerkin=False):
    """Multigrid-preconditioned CG per sample (each sample its own hierarchy;
    coarse levels rediscretized, or Galerkin products with galerkin).
    Returns (x [n][s], iters, rel_res, status, lmax [s][levels])."""
    xi = _f64(xi)
    s = xi.shape[0]
    n = num_nodes(N)
    x = np.zeros((n, s)) if x0 is None else _f64(x0).copy()
    it = np.zeros(s, np.int32)
    rr = np.zeros(s)
    st = np.zeros(s, np.int32)
    lm = np.zeros((s, MG_MAX_LEVELS))
    fi = None if fixed_iters is None else np.ascontiguousarray(fixed_iters, np.int32)
    _check(lib().orc_ens_mg_pcg(N, M, L, kappa0, sigma, fconst, s, _p(xi), _p(x), rtol, max_iter,
                                None if fi is None else _p(fi), _p(it), _p(rr), _p(st), _p(lm), int(galerkin)))
    return x, it, rr, st, lm[:, :len(mg_levels(N))]


def solve_samples(N, M, L, kappa0, sigma, fconst, xi, rtol, max_iter=10000, want_x=True, timing=False):
    """Independent per-sample graph + KL + assembly + Jacobi-CG, one sample per
    OpenMP thread.  Returns (x [count][n] or None, iters, rel_res, status,
    threads) and, with timing=True, per-sample [set-up, solve] wall seconds."""
    xi = _f64(xi)
    count = xi.shape[0]
    n = num_nodes(N)
    x = np.zeros((count, n)) if want_x else None
    it = np.zeros(count, np.int32)
    rr = np.zeros(count)
    st = np.zeros(count, np.int32)
    th = np.zeros(1, np.int32)
    tm = np.zeros((count, 2))
    _check(lib().orc_solve_samples(N, M, L, kappa0, sigma, fconst, count, _p(xi), rtol, max_iter,
                                   None if x is None else _p(x), _p(it), _p(rr), _p(st), _p(th), _p(tm)))
    if timing:
        return x, it, rr, st, int(th[0]), tm
    return x, it, rr, st, int(th[0])


def ens_true_residual(rp, ci, vals, b, x):
    n = rp.shape[0] - 1
    s = vals.shape[1]
    rel = np.zeros(s)
    lib().orc_ens_true_residual(n, s, _p(rp), _p(ci), _p(_f64(vals)), _p(_f64(b)), _p(_f64(x)), _p(rel))
    return rel


def crs_to_dense(rp, ci, vals):
    n = rp.shape[0] - 1
    d = np.zeros((n, n))
    lib().orc_crs_to_dense(n, _p(rp), _p(ci), _p(_f64(vals)), _p(d))
    return d


def cholesky_solve(A, b):
    """Returns (x, ok): ok is False when a pivot is not positive (not SPD)."""
    A = _f64(A).copy()
    n = A.shape[0]
    x = np.zeros(n)
    rc = lib().orc_cholesky_solve(n, _p(A), _p(_f64(b)), _p(x))
    return x, rc == 0


# ------------------------------------------------------- nonlinear problem

PREC_JACOBI, PREC_MG, PREC_MG_ADV = 0, 1, 2


def nl_assemble_scalar(N, rp, ci, acoef, fconst, alpha, vel, beta, u, want_jac=True):
    """One sample's residual F(u), Jacobian values (or None) and load of the
    nonlinear problem (Sec. 4, Eq. diffusion_sys and fenl_lin_sys)."""
    n = num_nodes(N)
    F = np.zeros(n)
    ld = np.zeros(n)
    vals = np.zeros(int(rp[-1])) if want_jac else None
    _check(lib().orc_nl_assemble_scalar(N, _p(rp), _p(ci), _p(_f64(acoef)), fconst, alpha, _p(_f64(vel)), beta,
                                        _p(_f64(u)), _p(F), None if vals is None else _p(vals), _p(ld)))
    return F, vals, ld


def ens_nl_assemble(N, rp, ci, M, L, kappa0, sigma, fconst, alpha, vel, beta, xi, u, want_jac=True):
    """Ensemble residual F [n][s], Jacobian [nnz][s] (or None), load [n][s]."""
    xi = _f64(xi)
    s = xi.shape[0]
    n = num_nodes(N)
    F = np.zeros((n, s))
    ld = np.zeros((n, s))
    vals = np.zeros((int(rp[-1]), s)) if want_jac else None
    _check(lib().orc_ens_nl_assemble(N, _p(rp), _p(ci), M, L, kappa0, sigma, fconst, alpha, _p(_f64(vel)), beta, s,
                                     _p(xi), _p(_f64(u)), _p(F), None if vals is None else _p(vals), _p(ld)))
    return F, vals, ld


def ens_gmres(N, rp, ci, values, b, x0=None, prec=PREC_JACOBI, M=0, L=1.0, kappa0=1.0, sigma=0.0, xi=None,
              rtol=1e-10, restart=30, max_iter=10000, fixed_iters=None, alpha=0.0, vel=(0.0, 0.0, 0.0)):
    """Right-preconditioned restarted GMRES per sample (prec: Jacobi, the
    diffusion V-cycle, or the V-cycle of D + alpha C, which alone uses alpha
    and vel).  Returns (x [n][s], iters, rel_res, status)."""
    values = _f64(values)
    s = values.shape[1]
    n = num_nodes(N)
    x = np.zeros((n, s)) if x0 is None else _f64(x0).copy()
    xi = np.zeros((s, max(M, 1))) if xi is None else _f64(xi)
    it = np.zeros(s, np.int32)
    rr = np.zeros(s)
    st = np.zeros(s, np.int32)
    fi = None if fixed_iters is None else np.ascontiguousarray(fixed_iters, np.int32)
    _check(lib().orc_ens_gmres(N, _p(rp), _p(ci), s, _p(values), _p(_f64(b)), _p(x), prec, M, L, kappa0, sigma,
                               _p(xi), alpha, _p(_f64(vel)), rtol, restart, max_iter, None if fi is None else _p(fi),
                               _p(it), _p(rr), _p(st)))
    return x, it, rr, st


FORCING_FIXED, FORCING_EW = 0, 1


def ew_forcing(k, eta_prev, fn, fprev, lin_rtol, floor_tol):
    """The oracle's forcing term of Newton step k (Eisenstat-Walker choice 2
    with its safeguard, capped at lin_rtol, at least floor_tol)."""
    return lib().orc_ew_forcing(int(k), float(eta_prev), float(fn), float(fprev), float(lin_rtol), float(floor_tol))


def ens_newton(N, M, L, kappa0, sigma, fconst, alpha, vel, beta, xi, u0=None, prec=PREC_MG, rtol=1e-8,
               max_newton=20, lin_rtol=1e-4, restart=30, lin_max_iter=1000, forcing=FORCING_FIXED, want_eta=False):
    """Newton per sample (forcing: fixed lin_rtol, or Eisenstat-Walker with
    eta_0 = eta_max = lin_rtol).  Returns (u [n][s], newton_iters,
    lin_iters, rel_res, status, fnorm [s][max_newton + 1]), and with
    want_eta the tolerance of every Newton system solved, eta [s][max_newton
    + 1] (0 past the last system), as a seventh item."""
    xi = _f64(xi)
    s = xi.shape[0]
    n = num_nodes(N)
    u = np.zeros((n, s)) if u0 is None else _f64(u0).copy()
    ni = np.zeros(s, np.int32)
    li = np.zeros(s, np.int32)
    rr = np.zeros(s)
    st = np.zeros(s, np.int32)
    fn = np.zeros((s, max_newton + 1))
    eta = np.zeros((s, max_newton + 1))
    _check(lib().orc_ens_newton(N, M, L, kappa0, sigma, fconst, alpha, _p(_f64(vel)), beta, s, _p(xi), _p(u), prec,
                                rtol, max_newton, lin_rtol, restart, lin_max_iter, int(forcing), _p(ni), _p(li),
                                _p(rr), _p(st), _p(fn), _p(eta)))
    if want_eta:
        return u, ni, li, rr, st, fn, eta
    return u, ni, li, rr, st, fn
