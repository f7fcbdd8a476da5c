"""Thin ctypes binding of libens (include/ens.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream, every computation runs in the library's HIP kernels.
If the library is missing this module raises instead of falling back to
anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libens.so")

ENS_OK, ENS_W_NOT_CONVERGED = 0, 1
ENS_E_ARG, ENS_E_UNSUPPORTED, ENS_E_HIP, ENS_E_NOMEM, ENS_E_RANGE = -1, -2, -3, -4, -5
SAMPLE_CONVERGED, SAMPLE_MAXITER, SAMPLE_BREAKDOWN, SAMPLE_NONFINITE, SAMPLE_STAGNATED = 0, 1, 2, 3, 4
F64, F32 = 0, 1
K_SPMV_F64, K_SPMV_F32, K_ASSEMBLE, K_SCALAR_SPMV, K_MG_ROW, K_NL_ASSEMBLE, K_GM_SPMV, K_GM_ORTH = range(8)


class EnsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class ens_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class ens_mg(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("s", ctypes.c_int32), ("fp32", ctypes.c_int32),
                ("buffer", ctypes.c_void_p), ("bytes", ctypes.c_size_t)]


class ens_problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("L", ctypes.c_double), ("kappa0", ctypes.c_double),
                ("sigma", ctypes.c_double), ("f", ctypes.c_double)]


class ens_cg_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("mixed", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double), ("inner_max_iter", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("check_every", ctypes.c_int32), ("coupled", ctypes.c_int32),
                ("compact", ctypes.c_int32)]


class ens_cg_stat(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("compacted", ctypes.c_int32), ("rel_res", ctypes.c_double)]


class ens_group(ctypes.Structure):
    _fields_ = [("graph", ctypes.POINTER(ens_graph)), ("values", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("stats", ctypes.POINTER(ens_cg_stat))]


class ens_group_input(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("kl", ctypes.c_void_p), ("xi", ctypes.c_void_p)]


class ens_nl_problem(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("L", ctypes.c_double), ("kappa0", ctypes.c_double),
                ("sigma", ctypes.c_double), ("f", ctypes.c_double), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double)]


class ens_gmres_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32)]


class ens_newton_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_newton", ctypes.c_int32), ("lin_rtol", ctypes.c_double),
                ("restart", ctypes.c_int32), ("lin_max_iter", ctypes.c_int32), ("jac32", ctypes.c_int32),
                ("forcing", ctypes.c_int32)]


class ens_newton_stat(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("lin_iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rel_res", ctypes.c_double)]


class ens_batch_opts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


_lib = None

# (name, restype, argtypes)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_SZ = ctypes.c_size_t
_GP = ctypes.POINTER(ens_graph)
_SIGS = [
    ("ens_last_error", ctypes.c_char_p, []),
    ("ens_status_string", ctypes.c_char_p, [_I32]),
    ("ens_abi_version", _I32, []),
    ("ens_shutdown", _I32, []),
    ("ens_mesh_sizes", _I32, [_I32, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    ("ens_graph_build", _I32, [_I32, _P, _P, _P]),
    ("ens_kl_bytes", _I32, [_I32, _I32, ctypes.POINTER(_SZ)]),
    ("ens_kl_build", _I32, [_I32, _I32, _D, _P, _P]),
    ("ens_assemble", _I32, [_I32, _GP, _P, ctypes.POINTER(ens_problem), _I32, _P, _P, _P, _P, _P]),
    ("ens_nl_assemble", _I32, [_I32, _GP, _P, ctypes.POINTER(ens_nl_problem), _I32, _P, _P, _P, _P, _P, _P, _P]),
    ("ens_gmres_workspace_bytes", _I32, [_GP, _I32, _I32, ctypes.POINTER(_SZ)]),
    ("ens_gmres", _I32, [_GP, _I32, _P, _P, _P, ctypes.POINTER(ens_gmres_opts), ctypes.POINTER(ens_mg), _P, _P, _SZ,
                         ctypes.POINTER(ens_cg_stat), _P]),
    ("ens_newton_workspace_bytes", _I32, [_GP, _I32, ctypes.POINTER(ens_newton_opts), ctypes.POINTER(_SZ)]),
    ("ens_newton", _I32, [_I32, _GP, _P, ctypes.POINTER(ens_nl_problem), _I32, _P, _P, ctypes.POINTER(ens_newton_opts),
                          ctypes.POINTER(ens_mg), _P, _P, _SZ, ctypes.POINTER(ens_newton_stat), _P]),
    ("ens_spmv", _I32, [_GP, _I32, _I32, _P, _P, _P, _P]),
    ("ens_scalar_spmv", _I32, [_GP, _I32, _P, _P, _P, _I32, _P]),
    ("ens_cg_workspace_bytes", _I32, [_GP, _I32, ctypes.POINTER(ens_cg_opts), ctypes.POINTER(_SZ)]),
    ("ens_cg", _I32, [_GP, _I32, _P, _P, _P, _P, ctypes.POINTER(ens_cg_opts), _P, _SZ,
                      ctypes.POINTER(ens_cg_stat), _P]),
    ("ens_cg_noalloc", _I32, [_GP, _I32, _P, _P, _P, _P, ctypes.POINTER(ens_cg_opts), ctypes.POINTER(ens_cg_stat),
                              _P]),
    ("ens_scalar_cg", _I32, [_GP, _I32, _P, _P, _P, ctypes.POINTER(ens_cg_opts), _I32, _P, _SZ,
                             ctypes.POINTER(ens_cg_stat), _P]),
    ("ens_mg_bytes", _I32, [_I32, _I32, _I32, _I32, ctypes.POINTER(_SZ)]),
    ("ens_mg_build", _I32, [ctypes.POINTER(ens_mg), ctypes.c_double, _P]),
    ("ens_mg_setup", _I32, [ctypes.POINTER(ens_mg), _GP, _P, _P, ctypes.POINTER(ens_problem), _P, _P]),
    ("ens_mg_release", _I32, [ctypes.POINTER(ens_mg)]),
    ("ens_mg_assemble_setup", _I32, [ctypes.POINTER(ens_mg), _GP, _P, ctypes.POINTER(ens_problem), _P, _P, _P, _P,
                                     _P]),
    ("ens_mg_setup_galerkin", _I32, [ctypes.POINTER(ens_mg), _GP, _P, _P, _P]),
    ("ens_mg_assemble_setup_galerkin", _I32, [ctypes.POINTER(ens_mg), _GP, _P, ctypes.POINTER(ens_problem), _P, _P,
                                              _P, _P, _P]),
    ("ens_mg_level_values", _I32, [ctypes.POINTER(ens_mg), _I32, ctypes.POINTER(_I32), ctypes.POINTER(_P),
                                   ctypes.POINTER(_P)]),
    ("ens_kl_extrema", _I32, [_I32, _P, ctypes.POINTER(ens_problem), _I32, _P, _P, _P, _P]),
    ("ens_group_order", _I32, [ctypes.c_int64, _P, _P]),
    ("ens_mg_assemble_setup_adv", _I32, [ctypes.POINTER(ens_mg), _GP, _P, ctypes.POINTER(ens_nl_problem), _P, _P, _P,
                                         _P, _P]),
    ("ens_cg_mg", _I32, [_GP, _I32, _P, _P, _P, _P, ctypes.POINTER(ens_cg_opts), ctypes.POINTER(ens_mg), _P, _SZ,
                         ctypes.POINTER(ens_cg_stat), _P]),
    ("ens_scalar_cg_concurrent_workspace_bytes", _I32, [_GP, _I32, ctypes.POINTER(_SZ)]),
    ("ens_scalar_cg_concurrent", _I32, [_GP, _I32, _P, _P, _P, ctypes.POINTER(ens_cg_opts), _I32, _I32, _P, _SZ,
                                        ctypes.POINTER(ens_cg_stat), _P]),
    ("ens_relayout", _I32, [_P, _P, _I64, _I32, _I32, _P]),
    ("ens_batch_workspace_bytes", _I32, [ctypes.POINTER(ens_group), _I32, _I32, ctypes.POINTER(ens_batch_opts),
                                         ctypes.POINTER(_SZ)]),
    ("ens_assemble_solve_batch_workspace_bytes", _I32, [ctypes.POINTER(ens_group), ctypes.POINTER(ens_group_input),
                                                         _I32, _I32, ctypes.POINTER(ens_problem),
                                                         ctypes.POINTER(ens_batch_opts), ctypes.POINTER(_SZ)]),
    ("ens_assemble_solve_batch", _I32, [ctypes.POINTER(ens_group), ctypes.POINTER(ens_group_input), _I32, _I32,
                                        ctypes.POINTER(ens_problem), ctypes.POINTER(ens_batch_opts), _P, _SZ, _P]),
    ("ens_solve_batch", _I32, [ctypes.POINTER(ens_group), _I32, _I32, ctypes.POINTER(ens_batch_opts), _P, _SZ, _P]),
    ("ens_batch_autotune_workspace_bytes", _I32, [_P, _I32, ctypes.POINTER(ens_problem), _P, _I32, _P, _I32,
                                                  ctypes.POINTER(ens_batch_opts), ctypes.POINTER(_SZ)]),
    ("ens_batch_autotune", _I32, [_P, _I32, ctypes.POINTER(ens_problem), _P, _P, _I32, _P, _I32,
                                  ctypes.POINTER(ens_batch_opts), ctypes.c_char_p, ctypes.POINTER(_I32),
                                  ctypes.POINTER(_I32), _P, _P, _SZ, _P]),
    ("ens_stream_copy", _I32, [_P, _P, _SZ, _P]),
    ("ens_stream_triad", _I32, [_P, _P, _P, _D, _I64, _P]),
    ("ens_stream_read", _I32, [_P, _SZ, _P, _P]),
    ("ens_stream_write", _I32, [_P, _SZ, ctypes.c_uint32, _P]),
    ("ens_mlp_param_count", _I64, []),
    ("ens_mlp_workspace_bytes", _I32, [_I32, ctypes.POINTER(_SZ)]),
    ("ens_mlp_forward", _I32, [_P, _I32, _P, _P, _P, _SZ, _P]),
    ("ens_mlp_grad", _I32, [_P, _I32, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    ("ens_mlp_train", _I32, [_P, _P, _P, _I32, _P, _P, _I32, _I32, _I32, _P, ctypes.c_float, _P, _P, _SZ, _P]),
    ("ens_mlp_adam", _I32, [_P, _P, _P, _P, ctypes.c_int64, _I32, ctypes.c_float, _P]),
    ("ens_pod_collect", _I32, [_P, _I64, _I32, _P, _I32, _I32, _P]),
    ("ens_pod_gram_workspace_bytes", _I32, [_I64, _I32, ctypes.POINTER(_SZ)]),
    ("ens_pod_gram", _I32, [_P, _I64, _I32, _P, _P, _SZ, _P]),
    ("ens_pod_eig_workspace_bytes", _I32, [_I32, _I32, ctypes.POINTER(_SZ)]),
    ("ens_pod_eig", _I32, [_P, _I32, _I32, _I32, _P, _I32, _P, _P, _P, _SZ, _P]),
    ("ens_pod_basis", _I32, [_P, _I64, _I32, _P, _P, _I32, _P, _P]),
    ("ens_pod_project_workspace_bytes", _I32, [_I64, _I32, _I32, ctypes.POINTER(_SZ)]),
    ("ens_pod_project", _I32, [_P, _P, _I64, _I32, _I32, _P, _P, _SZ, _P]),
    ("ens_pod_standardize", _I32, [_P, _I32, _I32, _I32, _P, _P, _P, _P]),
    ("ens_pod_reconstruct", _I32, [_P, _I64, _I32, _P, _P, _P, _I32, _P, _P]),
    ("ens_prof_enable", _I32, [_I32]),
    ("ens_prof_reset", _I32, []),
    ("ens_prof_query", _I32, [_I32, ctypes.POINTER(_D), ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
]
EXPORTED = [s[0] for s in _SIGS]


def lib():
    """Load libens.so (built in-tree by build.py); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_1511_03703_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int, where: str, allow=(ENS_OK,)):
    if st not in allow:
        detail = lib().ens_last_error().decode(errors="replace")
        raise EnsError(st, where, detail or lib().ens_status_string(st).decode())
    return st


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ mesh


def mesh_sizes(N: int):
    n, nnz, ne = _I64(), _I64(), _I64()
    _check(lib().ens_mesh_sizes(N, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(ne)), "ens_mesh_sizes")
    return n.value, nnz.value, ne.value


@dataclass
class Graph:
    N: int
    n: int
    nnz: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor

    def c(self) -> ens_graph:
        return ens_graph(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr())


def graph_build(N: int, device="cuda", stream=None) -> Graph:
    n, nnz, _ = mesh_sizes(N)
    rp = torch.empty(n + 1, dtype=torch.int32, device=device)
    ci = torch.empty(nnz, dtype=torch.int32, device=device)
    _check(lib().ens_graph_build(N, _ptr(rp), _ptr(ci), _stream(stream)), "ens_graph_build")
    return Graph(N, n, nnz, rp, ci)


def graph_from_arrays(row_ptr: torch.Tensor, col_idx: torch.Tensor, N: int = 0) -> Graph:
    return Graph(N, row_ptr.numel() - 1, col_idx.numel(), row_ptr, col_idx)


# -------------------------------------------------------------------- KL


def kl_bytes(N: int, M: int) -> int:
    b = _SZ()
    _check(lib().ens_kl_bytes(N, M, ctypes.byref(b)), "ens_kl_bytes")
    return b.value


def kl_build(N: int, M: int, L: float = 1.0, device="cuda", stream=None) -> torch.Tensor:
    buf = torch.zeros(kl_bytes(N, M), dtype=torch.uint8, device=device)
    _check(lib().ens_kl_build(N, M, L, _ptr(buf), _stream(stream)), "ens_kl_build")
    return buf


def kl_parse(buf: torch.Tensor, N: int, M: int) -> dict:
    """Host view of the KL table layout documented in ens.h."""
    import numpy as np
    b = buf.cpu().numpy().tobytes()
    d = np.frombuffer(b, dtype=np.float64, count=5 * M)
    i = np.frombuffer(b, dtype=np.int32, count=4 * M, offset=5 * M * 8)
    off = (5 * M * 8 + 4 * M * 4 + 15) & ~15
    phi = np.frombuffer(b, dtype=np.float64, count=M * 2 * N, offset=off).reshape(M, 2 * N)
    return {"sqrt_lam3": d[0:M], "lam3": d[M:2 * M], "omega": d[2 * M:3 * M], "lam1": d[3 * M:4 * M],
            "norm1": d[4 * M:5 * M], "parity": i[0:M], "triple": i[M:4 * M].reshape(M, 3), "phi": phi}


# -------------------------------------------------------------- assembly


def assemble(g: Graph, kl: torch.Tensor, xi: torch.Tensor, M: int, sigma: float, L: float = 1.0,
             kappa0: float = 1.0, f: float = 1.0, values=None, values32=None, rhs=None, want32=False,
             stream=None):
    """values [nnz][s] FP64, optional values32 [nnz][s] FP32, rhs [n][s] FP64."""
    s = xi.shape[0]
    dev = xi.device
    if values is None:
        values = torch.empty((g.nnz, s), dtype=torch.float64, device=dev)
    if want32 and values32 is None:
        values32 = torch.empty((g.nnz, s), dtype=torch.float32, device=dev)
    if rhs is None:
        rhs = torch.empty((g.n, s), dtype=torch.float64, device=dev)
    prob = ens_problem(M, L, kappa0, sigma, f)
    gc = g.c()
    _check(lib().ens_assemble(g.N, ctypes.byref(gc), _ptr(kl), ctypes.byref(prob), s, _ptr(xi), _ptr(values),
                              _ptr(values32), _ptr(rhs), _stream(stream)), "ens_assemble")
    return values, values32, rhs


# ------------------------------------------------------ nonlinear problem

DEFAULT_VEL = (3 ** -0.5, 3 ** -0.5, 3 ** -0.5)


def kl_extrema(N: int, kl: torch.Tensor, xi: torch.Tensor, M: int, sigma: float, L: float = 1.0,
               kappa0: float = 1.0, stream=None):
    """Per-sample minimum and maximum of the coefficient over the N^3 mesh's
    Gauss points: (kmin [s], kmax [s]) device FP64."""
    s = xi.shape[0]
    kmin = torch.empty(s, dtype=torch.float64, device=xi.device)
    kmax = torch.empty(s, dtype=torch.float64, device=xi.device)
    prob = ens_problem(M, L, kappa0, sigma, 1.0)
    _check(lib().ens_kl_extrema(N, _ptr(kl), ctypes.byref(prob), s, _ptr(xi), _ptr(kmin), _ptr(kmax),
                                _stream(stream)), "ens_kl_extrema")
    return kmin, kmax


def group_order(key) -> np.ndarray:
    """Sample order for grouping into ensembles: ascending key, ties and
    non-finite keys in index order (non-finite last)."""
    key = np.ascontiguousarray(key, dtype=np.float64)
    perm = np.empty(key.shape[0], dtype=np.int32)
    _check(lib().ens_group_order(key.shape[0], key.ctypes.data_as(ctypes.c_void_p),
                                 perm.ctypes.data_as(ctypes.c_void_p)), "ens_group_order")
    return perm


def nl_problem(M: int, sigma: float, alpha: float, beta: float, vel=DEFAULT_VEL, L: float = 1.0,
               kappa0: float = 1.0, f: float = 1.0) -> ens_nl_problem:
    return ens_nl_problem(M, L, kappa0, sigma, f, alpha, beta, float(vel[0]), float(vel[1]), float(vel[2]))


def nl_assemble(g: Graph, kl: torch.Tensor, xi: torch.Tensor, prob: ens_nl_problem, u: torch.Tensor,
                want_jac=True, want_load=False, want_jac32=False, values=None, values32=None, F=None, load=None,
                stream=None):
    """Residual F [n][s], Jacobian values [nnz][s] (or None) and load [n][s]
    (or None) of the nonlinear problem at u [n][s]; with want_jac32 the
    FP32 Jacobian is returned too: (F, values, load, values32)."""
    s = xi.shape[0]
    dev = u.device
    if want_jac and values is None:
        values = torch.empty((g.nnz, s), dtype=torch.float64, device=dev)
    if want_jac32 and values32 is None:
        values32 = torch.empty((g.nnz, s), dtype=torch.float32, device=dev)
    if F is None:
        F = torch.empty((g.n, s), dtype=torch.float64, device=dev)
    if want_load and load is None:
        load = torch.empty((g.n, s), dtype=torch.float64, device=dev)
    gc = g.c()
    _check(lib().ens_nl_assemble(g.N, ctypes.byref(gc), _ptr(kl), ctypes.byref(prob), s, _ptr(xi), _ptr(u),
                                 _ptr(values if want_jac else None), _ptr(values32 if want_jac32 else None), _ptr(F),
                                 _ptr(load if want_load else None), _stream(stream)), "ens_nl_assemble")
    out = (F, (values if want_jac else None), (load if want_load else None))
    return out + (values32,) if want_jac32 else out


def gmres_opts(rtol=1e-10, restart=30, max_iter=1000) -> ens_gmres_opts:
    return ens_gmres_opts(rtol, restart, max_iter)


def gmres_workspace_bytes(g: Graph, s: int, restart: int) -> int:
    nb = _SZ()
    _check(lib().ens_gmres_workspace_bytes(ctypes.byref(g.c()), s, restart, ctypes.byref(nb)),
           "ens_gmres_workspace_bytes")
    return nb.value


def gmres(g: Graph, values, b, x=None, opts: ens_gmres_opts | None = None, mg=None, mg_values=None,
          workspace=None, stream=None):
    """Right-preconditioned restarted GMRES per sample (mg: a set-up FP64
    Multigrid whose fine matrix is mg_values; None: Jacobi).  Returns (x,
    stats, status)."""
    s = values.shape[1]
    if opts is None:
        opts = gmres_opts()
    if x is None:
        x = torch.zeros_like(b)
    nbytes = gmres_workspace_bytes(g, s, opts.restart)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    stats = (ens_cg_stat * s)()
    gc = g.c()
    st = _check(lib().ens_gmres(ctypes.byref(gc), s, _ptr(values), _ptr(b), _ptr(x), ctypes.byref(opts),
                                ctypes.byref(mg.desc) if mg is not None else None, _ptr(mg_values), _ptr(workspace),
                                workspace.numel(), stats, _stream(stream)),
                "ens_gmres", allow=(ENS_OK, ENS_W_NOT_CONVERGED))
    return x, _stats_list(stats, s), st


FORCING_FIXED, FORCING_EW = 0, 1


def newton_opts(rtol=1e-8, max_newton=20, lin_rtol=1e-4, restart=30, lin_max_iter=1000, jac32=False,
                forcing=FORCING_FIXED) -> ens_newton_opts:
    return ens_newton_opts(rtol, max_newton, lin_rtol, restart, lin_max_iter, int(jac32), int(forcing))


def newton_workspace_bytes(g: Graph, s: int, opts: ens_newton_opts) -> int:
    nb = _SZ()
    _check(lib().ens_newton_workspace_bytes(ctypes.byref(g.c()), s, ctypes.byref(opts), ctypes.byref(nb)),
           "ens_newton_workspace_bytes")
    return nb.value


def newton(g: Graph, kl: torch.Tensor, xi: torch.Tensor, prob: ens_nl_problem, u=None,
           opts: ens_newton_opts | None = None, mg=None, mg_values=None, workspace=None, stream=None):
    """Newton's method per sample with GMRES inner solves.  Returns (u,
    stats, status); stats[e] = dict(newton_iters, lin_iters, status,
    rel_res)."""
    s = xi.shape[0]
    if opts is None:
        opts = newton_opts()
    if u is None:
        u = torch.zeros((g.n, s), dtype=torch.float64, device=xi.device)
    nbytes = newton_workspace_bytes(g, s, opts)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=xi.device)
    stats = (ens_newton_stat * s)()
    gc = g.c()
    st = _check(lib().ens_newton(g.N, ctypes.byref(gc), _ptr(kl), ctypes.byref(prob), s, _ptr(xi), _ptr(u),
                                 ctypes.byref(opts), ctypes.byref(mg.desc) if mg is not None else None,
                                 _ptr(mg_values), _ptr(workspace), workspace.numel(), stats, _stream(stream)),
                "ens_newton", allow=(ENS_OK, ENS_W_NOT_CONVERGED))
    out = [dict(newton_iters=stats[e].newton_iters, lin_iters=stats[e].lin_iters, status=stats[e].status,
                rel_res=stats[e].rel_res) for e in range(s)]
    return u, out, st


# ------------------------------------------------------------------ SpMV


def spmv(g: Graph, values: torch.Tensor, x: torch.Tensor, y=None, stream=None):
    s = values.shape[1]
    dt = F64 if values.dtype == torch.float64 else F32
    if y is None:
        y = torch.empty_like(x)
    gc = g.c()
    _check(lib().ens_spmv(ctypes.byref(gc), s, dt, _ptr(values), _ptr(x), _ptr(y), _stream(stream)), "ens_spmv")
    return y


def scalar_spmv(g: Graph, values: torch.Tensor, x: torch.Tensor, y=None, lanes_per_row=0, stream=None):
    dt = F64 if values.dtype == torch.float64 else F32
    if y is None:
        y = torch.empty_like(x)
    gc = g.c()
    _check(lib().ens_scalar_spmv(ctypes.byref(gc), dt, _ptr(values), _ptr(x), _ptr(y), lanes_per_row,
                                 _stream(stream)), "ens_scalar_spmv")
    return y


# -------------------------------------------------------------------- CG


def cg_opts(rtol=1e-10, max_iter=10000, mixed=False, inner_rtol=1e-5, inner_max_iter=10000, max_outer=10,
            check_every=16, coupled=False, compact=False) -> ens_cg_opts:
    return ens_cg_opts(rtol, max_iter, int(mixed), inner_rtol, inner_max_iter, max_outer, check_every, int(coupled),
                       int(compact))


def cg_workspace_bytes(g: Graph, s: int, opts: ens_cg_opts) -> int:
    b = _SZ()
    gc = g.c()
    _check(lib().ens_cg_workspace_bytes(ctypes.byref(gc), s, ctypes.byref(opts), ctypes.byref(b)),
           "ens_cg_workspace_bytes")
    return b.value


def _stats_list(st, count):
    return [{"iters": st[e].iters, "outer_iters": st[e].outer_iters, "status": st[e].status,
             "compacted": st[e].compacted, "rel_res": st[e].rel_res} for e in range(count)]


def cg(g: Graph, values, b, x=None, values32=None, opts: ens_cg_opts | None = None, workspace=None, stream=None):
    """Ensemble Jacobi-CG (or FP32-in-FP64 refinement when opts.mixed).
    Returns (x, stats, status)."""
    s = values.shape[1]
    if opts is None:
        opts = cg_opts()
    if x is None:
        x = torch.zeros_like(b)
    nbytes = cg_workspace_bytes(g, s, opts)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    stats = (ens_cg_stat * s)()
    gc = g.c()
    st = _check(lib().ens_cg(ctypes.byref(gc), s, _ptr(values), _ptr(values32), _ptr(b), _ptr(x),
                             ctypes.byref(opts), _ptr(workspace), workspace.numel(), stats, _stream(stream)),
                "ens_cg", allow=(ENS_OK, ENS_W_NOT_CONVERGED))
    return x, _stats_list(stats, s), st


CG_NOALLOC_SCRATCH_BYTES = 256 << 20


def cg_noalloc(g: Graph, values, b, x, values32=None, opts: ens_cg_opts | None = None, stream=None):
    """ens_cg on the library's own scratch array (ens_cg_noalloc): nothing is
    allocated, x (in: x0, out: the solution) must be given.  Returns (x,
    stats, status)."""
    s = values.shape[1]
    if opts is None:
        opts = cg_opts()
    stats = (ens_cg_stat * s)()
    gc = g.c()
    st = _check(lib().ens_cg_noalloc(ctypes.byref(gc), s, _ptr(values), _ptr(values32), _ptr(b), _ptr(x),
                                     ctypes.byref(opts), stats, _stream(stream)),
                "ens_cg_noalloc", allow=(ENS_OK, ENS_W_NOT_CONVERGED))
    return x, _stats_list(stats, s), st


def scalar_cg(g: Graph, values_sm, b_sm, x_sm=None, opts: ens_cg_opts | None = None, lanes_per_row=0,
              workspace=None, stream=None):
    """s independent one-sample solves; sample-major values [s][nnz], b, x [s][n]."""
    s = values_sm.shape[0]
    if opts is None:
        opts = cg_opts()
    if x_sm is None:
        x_sm = torch.zeros_like(b_sm)
    nbytes = cg_workspace_bytes(g, 4, opts)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=b_sm.device)
    stats = (ens_cg_stat * s)()
    gc = g.c()
    st = _check(lib().ens_scalar_cg(ctypes.byref(gc), s, _ptr(values_sm), _ptr(b_sm), _ptr(x_sm),
                                    ctypes.byref(opts), lanes_per_row, _ptr(workspace), workspace.numel(), stats,
                                    _stream(stream)), "ens_scalar_cg", allow=(ENS_OK, ENS_W_NOT_CONVERGED))
    return x_sm, _stats_list(stats, s), st


class Multigrid:
    """Device hierarchy of the multigrid preconditioner for one ensemble."""

    def __init__(self, N: int, M: int, s: int, fp32: bool = False, L: float = 1.0, device="cuda", stream=None):
        nb = _SZ()
        _check(lib().ens_mg_bytes(N, M, s, int(fp32), ctypes.byref(nb)), "ens_mg_bytes")
        self.buffer = torch.empty(nb.value, dtype=torch.uint8, device=device)
        self.desc = ens_mg(N, M, s, int(fp32), self.buffer.data_ptr(), nb.value)
        self.L = L
        _check(lib().ens_mg_build(ctypes.byref(self.desc), L, _stream(stream)), "ens_mg_build")

    def __del__(self):
        # the library's record of this buffer goes before the memory does
        try:
            lib().ens_mg_release(ctypes.byref(self.desc))
        except Exception:
            pass

    def assemble_setup(self, g: Graph, kl, xi, sigma, values, rhs, values32=None, kappa0=1.0, f=1.0, stream=None,
                       galerkin=False):
        """Assemble the fine matrix into values (values32), rhs and set the
        hierarchy up in one call, the fine level's D^-1 and bound formed by
        the assembly; galerkin: coarse levels P^T A P of the level above
        (ens_mg_assemble_setup_galerkin) instead of their own assemblies."""
        prob = ens_problem(self.desc.M, self.L, kappa0, sigma, f)
        gc = g.c()
        self._values = (values, values32)
        fn = lib().ens_mg_assemble_setup_galerkin if galerkin else lib().ens_mg_assemble_setup
        _check(fn(ctypes.byref(self.desc), ctypes.byref(gc), _ptr(kl), ctypes.byref(prob), _ptr(xi), _ptr(values),
                  _ptr(values32), _ptr(rhs), _stream(stream)),
               "ens_mg_assemble_setup_galerkin" if galerkin else "ens_mg_assemble_setup")
        return self

    def level_values(self, level: int):
        """(N, FP64 values [nnz][s], FP32 values or None) of coarse level
        `level`, copied out of the hierarchy buffer."""
        Nl, v64, v32 = _I32(), _P(), _P()
        _check(lib().ens_mg_level_values(ctypes.byref(self.desc), level, ctypes.byref(Nl), ctypes.byref(v64),
                                         ctypes.byref(v32)), "ens_mg_level_values")
        nnz = (3 * Nl.value + 1) ** 3
        s = self.desc.s
        base = self.buffer.data_ptr()

        def view(ptr, dtype, width):
            off = ptr - base
            assert off % width == 0 and off + nnz * s * width <= self.buffer.numel()
            return self.buffer[off:off + nnz * s * width].view(dtype).view(nnz, s).clone()

        a = view(v64.value, torch.float64, 8)
        b = view(v32.value, torch.float32, 4) if v32.value else None
        return Nl.value, a, b

    def setup_galerkin(self, g: Graph, values, values32=None, stream=None):
        """Coarse levels as Galerkin products P^T A P from the FP64 fine
        matrix `values` (ens_mg_setup_galerkin)."""
        gc = g.c()
        self._values = (values, values32)
        _check(lib().ens_mg_setup_galerkin(ctypes.byref(self.desc), ctypes.byref(gc), _ptr(values), _ptr(values32),
                                           _stream(stream)), "ens_mg_setup_galerkin")
        return self

    def assemble_setup_adv(self, g: Graph, kl, xi, problem: ens_nl_problem, values, rhs, values32=None,
                           stream=None):
        """As assemble_setup, for the advection-diffusion operator D + alpha C
        of `problem` (its beta unused) on every level: a preconditioner for
        GMRES and Newton, which multigrid CG refuses."""
        if problem.M != self.desc.M or problem.L != self.L:
            raise ValueError("problem M / L differ from the hierarchy's")
        gc = g.c()
        self._values = (values, values32)
        _check(lib().ens_mg_assemble_setup_adv(ctypes.byref(self.desc), ctypes.byref(gc), _ptr(kl),
                                               ctypes.byref(problem), _ptr(xi), _ptr(values), _ptr(values32),
                                               _ptr(rhs), _stream(stream)), "ens_mg_assemble_setup_adv")
        return self

    def setup(self, g: Graph, values, xi, sigma, values32=None, L=None, kappa0=1.0, f=1.0, stream=None):
        if L is not None and L != self.L:
            raise ValueError("the hierarchy's KL tables were built for another correlation length")
        prob = ens_problem(self.desc.M, self.L, kappa0, sigma, f)
        gc = g.c()
        self._values = (values, values32)
        _check(lib().ens_mg_setup(ctypes.byref(self.desc), ctypes.byref(gc), _ptr(values), _ptr(values32),
                                  ctypes.byref(prob), _ptr(xi), _stream(stream)), "ens_mg_setup")
        return self


def cg_mg(g: Graph, values, b, mg: Multigrid, x=None, values32=None, opts: ens_cg_opts | None = None,
          workspace=None, stream=None):
    """Multigrid-preconditioned ensemble CG (opts.mixed: FP32 inner solves
    with an FP32 cycle inside the FP64 refinement).  Returns (x, stats,
    status)."""
    s = values.shape[1]
    if opts is None:
        opts = cg_opts()
    if x is None:
        x = torch.zeros_like(b)
    nbytes = cg_workspace_bytes(g, s, opts)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    stats = (ens_cg_stat * s)()
    gc = g.c()
    st = _check(lib().ens_cg_mg(ctypes.byref(gc), s, _ptr(values), _ptr(values32), _ptr(b), _ptr(x),
                                ctypes.byref(opts), ctypes.byref(mg.desc), _ptr(workspace), workspace.numel(), stats,
                                _stream(stream)),
                "ens_cg_mg", allow=(ENS_OK, ENS_W_NOT_CONVERGED))
    return x, _stats_list(stats, s), st


def scalar_cg_concurrent(g: Graph, values_sm, b_sm, x_sm=None, opts: ens_cg_opts | None = None, lanes_per_row=0,
                         streams=4, workspace=None, stream=None):
    """scalar_cg with up to `streams` one-sample solves in flight at once."""
    s = values_sm.shape[0]
    if opts is None:
        opts = cg_opts()
    if x_sm is None:
        x_sm = torch.zeros_like(b_sm)
    gc = g.c()
    nb = _SZ()
    _check(lib().ens_scalar_cg_concurrent_workspace_bytes(ctypes.byref(gc), streams, ctypes.byref(nb)),
           "ens_scalar_cg_concurrent_workspace_bytes")
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=b_sm.device)
    stats = (ens_cg_stat * s)()
    st = _check(lib().ens_scalar_cg_concurrent(ctypes.byref(gc), s, _ptr(values_sm), _ptr(b_sm), _ptr(x_sm),
                                               ctypes.byref(opts), lanes_per_row, streams, _ptr(workspace),
                                               workspace.numel(), stats, _stream(stream)),
                "ens_scalar_cg_concurrent", allow=(ENS_OK, ENS_W_NOT_CONVERGED))
    return x_sm, _stats_list(stats, s), st


def relayout(src: torch.Tensor, to_sample_major: bool, out=None, stream=None):
    """[rows][s] <-> [s][rows] (FP64)."""
    if to_sample_major:
        rows, s = src.shape
        if out is None:
            out = torch.empty((s, rows), dtype=src.dtype, device=src.device)
    else:
        s, rows = src.shape
        if out is None:
            out = torch.empty((rows, s), dtype=src.dtype, device=src.device)
    _check(lib().ens_relayout(_ptr(src), _ptr(out), rows, s, int(to_sample_major), _stream(stream)), "ens_relayout")
    return out


# ------------------------------------------------------------ measurement


def stream_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    nb = src.numel() * src.element_size()
    _check(lib().ens_stream_copy(_ptr(src), _ptr(dst), nb, _stream(stream)), "ens_stream_copy")


STREAM_READ_CHUNK_BYTES = 16384


def stream_read(src: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """Read every byte of src once (the read-only bandwidth ceiling); returns
    the XOR word of every STREAM_READ_CHUNK_BYTES piece."""
    nb = src.numel() * src.element_size()
    words = max(1, -(-nb // STREAM_READ_CHUNK_BYTES))
    if out is None:
        out = torch.empty(words, dtype=torch.int32, device=src.device)
    if out.numel() < words:
        raise ValueError(f"out must hold {words} words")
    _check(lib().ens_stream_read(_ptr(src), nb, _ptr(out), _stream(stream)), "ens_stream_read")
    return out


def stream_write(dst: torch.Tensor, value: int = 0, stream=None):
    """Write every byte of dst once (the write-only bandwidth ceiling):
    16-byte chunks (value, value ^ 1, value ^ 2, value ^ 3) as uint32."""
    nb = dst.numel() * dst.element_size()
    _check(lib().ens_stream_write(_ptr(dst), nb, value & 0xFFFFFFFF, _stream(stream)), "ens_stream_write")
    return dst


def stream_triad(a, b, c, q: float, stream=None):
    _check(lib().ens_stream_triad(_ptr(a), _ptr(b), _ptr(c), q, a.numel(), _stream(stream)), "ens_stream_triad")


def shutdown():
    """Release the library's per-device state (ens_shutdown); it is created
    again by the next call that needs it."""
    _check(lib().ens_shutdown(), "ens_shutdown")


def prof_enable(on: bool = True):
    _check(lib().ens_prof_enable(int(on)), "ens_prof_enable")


def prof_reset():
    _check(lib().ens_prof_reset(), "ens_prof_reset")


def prof_query(kernel_id: int):
    ms, n, by = _D(), _I64(), _D()
    _check(lib().ens_prof_query(kernel_id, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)), "ens_prof_query")
    return {"total_ms": ms.value, "launches": n.value, "bytes": by.value}


# ------------------------------------------------- learned initial guess

MLP_IN, MLP_HID, MLP_OUT = 10, 256, 32


def mlp_param_count() -> int:
    return int(lib().ens_mlp_param_count())


def mlp_init(seed: int, device="cuda") -> torch.Tensor:
    """Seeded FP32 parameters: every weight and bias of a layer uniform in
    +-1/sqrt(fan_in).  Layout W1 [256][10], b1 [256], W2 [256][256], b2 [256],
    W3 [32][256], b3 [32]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = []
    for rows, fan_in in ((MLP_HID, MLP_IN), (MLP_HID, MLP_HID), (MLP_OUT, MLP_HID)):
        lim = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, rows * fan_in))
        parts.append(rng.uniform(-lim, lim, rows))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == mlp_param_count()
    return torch.as_tensor(p, device=device)


def _mlp_ws(batch, device):
    b = _SZ()
    _check(lib().ens_mlp_workspace_bytes(batch, ctypes.byref(b)), "ens_mlp_workspace_bytes")
    return torch.empty(b.value, dtype=torch.uint8, device=device)


def mlp_forward(params: torch.Tensor, xi: torch.Tensor, workspace=None, stream=None):
    batch = xi.shape[0]
    out = torch.empty((batch, MLP_OUT), dtype=torch.float32, device=xi.device)
    ws = workspace if workspace is not None else _mlp_ws(batch, xi.device)
    _check(lib().ens_mlp_forward(_ptr(params), batch, _ptr(xi), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
           "ens_mlp_forward")
    return out


def mlp_grad(params, xi, target, workspace=None, stream=None):
    batch = xi.shape[0]
    out = torch.empty((batch, MLP_OUT), dtype=torch.float32, device=xi.device)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=xi.device)
    ws = workspace if workspace is not None else _mlp_ws(batch, xi.device)
    _check(lib().ens_mlp_grad(_ptr(params), batch, _ptr(xi), _ptr(target), _ptr(out), _ptr(grad), _ptr(loss),
                              _ptr(ws), ws.numel(), _stream(stream)), "ens_mlp_grad")
    return out, grad, loss


def mlp_train(params, adam_m, adam_v, step0, xi, target, batch, batch_idx, lr, loss=None, workspace=None,
              stream=None):
    steps = batch_idx.numel() // batch
    ws = workspace if workspace is not None else _mlp_ws(batch, xi.device)
    _check(lib().ens_mlp_train(_ptr(params), _ptr(adam_m), _ptr(adam_v), step0, _ptr(xi), _ptr(target),
                               xi.shape[0], batch, steps, _ptr(batch_idx), lr, _ptr(loss), _ptr(ws), ws.numel(),
                               _stream(stream)), "ens_mlp_train")
    return steps


def mlp_adam(params, grad, adam_m, adam_v, step, lr, stream=None):
    """One Adam step (step = t, 1-based) on FP32 device arrays, in place."""
    _check(lib().ens_mlp_adam(_ptr(params), _ptr(grad), _ptr(adam_m), _ptr(adam_v), params.numel(), step, lr,
                              _stream(stream)), "ens_mlp_adam")


def pod_collect(x, S, col0, stream=None):
    n, s = x.shape
    _check(lib().ens_pod_collect(_ptr(x), n, s, _ptr(S), S.shape[1], col0, _stream(stream)), "ens_pod_collect")


def pod_gram(S, stream=None):
    n, m = S.shape
    b = _SZ()
    _check(lib().ens_pod_gram_workspace_bytes(n, m, ctypes.byref(b)), "ens_pod_gram_workspace_bytes")
    ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=S.device)
    G = torch.empty((m, m), dtype=torch.float64, device=S.device)
    _check(lib().ens_pod_gram(_ptr(S), n, m, _ptr(G), _ptr(ws), ws.numel(), _stream(stream)), "ens_pod_gram")
    return G


def pod_eig(G, r, start, iters, stream=None):
    m, k = start.shape
    b = _SZ()
    _check(lib().ens_pod_eig_workspace_bytes(m, k, ctypes.byref(b)), "ens_pod_eig_workspace_bytes")
    ws = torch.empty(b.value, dtype=torch.uint8, device=G.device)
    V = torch.empty((m, r), dtype=torch.float64, device=G.device)
    lam = torch.empty(r, dtype=torch.float64, device=G.device)
    _check(lib().ens_pod_eig(_ptr(G), m, k, r, _ptr(start), iters, _ptr(V), _ptr(lam), _ptr(ws), ws.numel(),
                             _stream(stream)), "ens_pod_eig")
    return V, lam


def pod_basis(S, V, lam, stream=None):
    n, m = S.shape
    r = V.shape[1]
    Phi = torch.empty((n, r), dtype=torch.float64, device=S.device)
    _check(lib().ens_pod_basis(_ptr(S), n, m, _ptr(V), _ptr(lam), r, _ptr(Phi), _stream(stream)), "ens_pod_basis")
    return Phi


def pod_project(Phi, X, stream=None):
    n, r = Phi.shape
    s = X.shape[1]
    b = _SZ()
    _check(lib().ens_pod_project_workspace_bytes(n, r, s, ctypes.byref(b)), "ens_pod_project_workspace_bytes")
    ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=X.device)
    C = torch.empty((s, r), dtype=torch.float64, device=X.device)
    _check(lib().ens_pod_project(_ptr(Phi), _ptr(X), n, r, s, _ptr(C), _ptr(ws), ws.numel(), _stream(stream)),
           "ens_pod_project")
    return C


def pod_standardize(C, common=False, stream=None):
    """(mu, sd, T) of the coefficients C [m][r]: T = (C - mu) / sd with sd each
    coefficient's deviation, or with common the largest for all."""
    m, r = C.shape
    mu = torch.empty(r, dtype=torch.float64, device=C.device)
    sd = torch.empty(r, dtype=torch.float64, device=C.device)
    T = torch.empty((m, r), dtype=torch.float32, device=C.device)
    _check(lib().ens_pod_standardize(_ptr(C), m, r, int(common), _ptr(mu), _ptr(sd), _ptr(T), _stream(stream)),
           "ens_pod_standardize")
    return mu, sd, T


def pod_reconstruct(Phi, c, mu=None, sd=None, x0=None, stream=None):
    n, r = Phi.shape
    s = c.shape[0]
    if x0 is None:
        x0 = torch.empty((n, s), dtype=torch.float64, device=Phi.device)
    _check(lib().ens_pod_reconstruct(_ptr(Phi), n, r, _ptr(c), _ptr(mu), _ptr(sd), s, _ptr(x0), _stream(stream)),
           "ens_pod_reconstruct")
    return x0


# ------------------------------------------------------------------ batch


def batch_opts(rtol=1e-8, max_iter=10000, check_every=16, tile=4, use_graph=True) -> ens_batch_opts:
    return ens_batch_opts(rtol, max_iter, check_every, tile, int(use_graph))


def solve_batch(groups, s, opts: ens_batch_opts | None = None, workspace=None, stream=None,
                strict_workspace=False):
    """groups: list of (Graph, values [nnz][s], b [n][s], x [n][s]).  Returns
    (per-group stats lists, status, workspace).  A workspace smaller than
    required is replaced by a new one, or refused with strict_workspace."""
    if opts is None:
        opts = batch_opts()
    keep = []
    arr = (ens_group * len(groups))()
    stats = []
    for i, (g, v, b, x) in enumerate(groups):
        gc = g.c()
        st = (ens_cg_stat * s)()
        keep.append(gc)
        stats.append(st)
        arr[i] = ens_group(ctypes.pointer(gc), v.data_ptr(), b.data_ptr(), x.data_ptr(), st)
    nb = _SZ()
    _check(lib().ens_batch_workspace_bytes(arr, len(groups), s, ctypes.byref(opts), ctypes.byref(nb)),
           "ens_batch_workspace_bytes")
    if workspace is not None and workspace.numel() < nb.value and strict_workspace:
        raise EnsError(ENS_E_NOMEM, "solve_batch", f"workspace of {workspace.numel()} bytes, {nb.value} required")
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=groups[0][1].device)
    rc = _check(lib().ens_solve_batch(arr, len(groups), s, ctypes.byref(opts), _ptr(workspace), workspace.numel(),
                                      _stream(stream)), "ens_solve_batch", allow=(ENS_OK, ENS_W_NOT_CONVERGED))
    return [_stats_list(st, s) for st in stats], rc, workspace


def assemble_solve_batch(groups, inputs, s, M, sigma, opts: ens_batch_opts | None = None, workspace=None,
                         L=1.0, kappa0=1.0, f=1.0, stream=None, strict_workspace=False):
    """Assemble and solve a wave of groups in one call (ens_assemble_solve_batch).
    groups: list of (Graph, values [nnz][s], b [n][s], x [n][s]) -- values,
    b and x are written; inputs: list of (N, kl table, xi [s][M] device).
    Returns (per-group stats lists, status, workspace)."""
    if opts is None:
        opts = batch_opts()
    keep = []
    arr = (ens_group * len(groups))()
    inp = (ens_group_input * len(groups))()
    stats = []
    for i, ((g, v, b, x), (N, kl, xi)) in enumerate(zip(groups, inputs)):
        gc = g.c()
        st = (ens_cg_stat * s)()
        keep.append(gc)
        stats.append(st)
        arr[i] = ens_group(ctypes.pointer(gc), v.data_ptr(), b.data_ptr(), x.data_ptr(), st)
        inp[i] = ens_group_input(int(N), kl.data_ptr(), xi.data_ptr())
    prob = ens_problem(M, L, kappa0, sigma, f)
    nb = _SZ()
    _check(lib().ens_assemble_solve_batch_workspace_bytes(arr, inp, len(groups), s, ctypes.byref(prob),
                                                          ctypes.byref(opts), ctypes.byref(nb)),
           "ens_assemble_solve_batch_workspace_bytes")
    if workspace is not None and workspace.numel() < nb.value and strict_workspace:
        raise EnsError(ENS_E_NOMEM, "assemble_solve_batch",
                       f"workspace of {workspace.numel()} bytes, {nb.value} required")
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=groups[0][1].device)
    rc = _check(lib().ens_assemble_solve_batch(arr, inp, len(groups), s, ctypes.byref(prob), ctypes.byref(opts),
                                               _ptr(workspace), workspace.numel(), _stream(stream)),
                "ens_assemble_solve_batch", allow=(ENS_OK, ENS_W_NOT_CONVERGED))
    return [_stats_list(st, s) for st in stats], rc, workspace


def batch_autotune(meshes, M, sigma, xi_host, opts: ens_batch_opts | None = None, s_cand=(8, 16, 32),
                   tile_cand=(2, 4, 8), cache_path=None, want_scores=True, L=1.0, kappa0=1.0, f=1.0, stream=None):
    """Pick (s, tile) for ens_solve_batch by solving 32 samples per mesh with
    every candidate.  xi_host: [len(meshes)][32][M].  Returns (best_s,
    best_tile, {(s, tile): samples/s} or None when served from the cache)."""
    import numpy as np
    if opts is None:
        opts = batch_opts()
    m = np.ascontiguousarray(meshes, dtype=np.int32)
    xi = np.ascontiguousarray(xi_host, dtype=np.float64)
    if xi.shape != (len(m), 32, M):
        raise ValueError(f"xi_host must have shape ({len(m)}, 32, {M})")
    sc = np.ascontiguousarray(s_cand, dtype=np.int32)
    tc = np.ascontiguousarray(tile_cand, dtype=np.int32)
    scores = np.zeros(len(sc) * len(tc)) if want_scores else None
    bs, bt = _I32(), _I32()
    prob = ens_problem(M, L, kappa0, sigma, f)
    need = _SZ(0)
    _check(lib().ens_batch_autotune_workspace_bytes(m.ctypes.data, len(m), ctypes.byref(prob), sc.ctypes.data,
                                                    len(sc), tc.ctypes.data, len(tc), ctypes.byref(opts),
                                                    ctypes.byref(need)), "ens_batch_autotune_workspace_bytes")
    ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
    _check(lib().ens_batch_autotune(m.ctypes.data, len(m), ctypes.byref(prob), xi.ctypes.data, sc.ctypes.data,
                                    len(sc), tc.ctypes.data, len(tc), ctypes.byref(opts),
                                    None if cache_path is None else str(cache_path).encode(), ctypes.byref(bs),
                                    ctypes.byref(bt), None if scores is None else scores.ctypes.data,
                                    _ptr(ws), ws.numel(), _stream(stream)), "ens_batch_autotune")
    del ws
    table = None
    if scores is not None:
        table = {(int(a), int(b)): float(scores[i * len(tc) + j]) for i, a in enumerate(sc) for j, b in enumerate(tc)}
    return bs.value, bt.value, table
