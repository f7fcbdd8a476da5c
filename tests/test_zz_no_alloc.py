"""ens_cg_noalloc (the CG entry point that allocates nothing: its workspace is
the library's scratch array) against ens_cg with a caller workspace, through
the C ABI.  Bar: the same kernels in the same order on the same inputs, so
x and the per-sample statistics are bitwise equal.  Two calls in a row, the
second on a smaller problem (the scratch keeps the first call's contents),
in FP64 and in the FP32-in-FP64 refinement."""
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


def _system(E, N, s, M, sigma, seed, want32):
    g = E.graph_build(N)
    kl = E.kl_build(N, M)
    xt = torch.as_tensor(draw_xi(seed, s, M), device=DEV)
    vals, v32, rhs = E.assemble(g, kl, xt, M, sigma, want32=want32)
    return g, vals, v32, rhs


@pytest.mark.parametrize("mixed", [False, True])
def test_noalloc_cg_equals_cg_on_two_calls(E, mixed):
    cases = [(24, 16, 1900), (12, 8, 1901)]   # the second call is smaller
    for N, s, seed in cases:
        print(f"no-alloc CG N={N} s={s} mixed={mixed}", flush=True)
        g, vals, v32, rhs = _system(E, N, s, 10, 0.3, seed, mixed)
        opts = E.cg_opts(rtol=1e-8 if mixed else 1e-10, mixed=mixed, check_every=4)
        # a nonzero start exercises the initial residual
        x0 = torch.as_tensor(np.random.default_rng(seed).standard_normal((g.n, s)) * 1e-3, device=DEV)
        xa, sa, sta = E.cg(g, vals, rhs, x=x0.clone(), values32=v32, opts=opts)
        xb, sb, stb = E.cg_noalloc(g, vals, rhs, x0.clone(), values32=v32, opts=opts)
        torch.cuda.synchronize()
        assert sta == stb == E.ENS_OK
        assert torch.equal(xa, xb)
        assert sa == sb
        assert all(t["status"] == 0 for t in sb)


def test_noalloc_cg_refuses_a_problem_beyond_its_scratch(E):
    g = E.graph_build(64)
    b = torch.zeros((g.n, 32), dtype=torch.float64, device=DEV)
    vals = torch.zeros((16, 32), dtype=torch.float64, device=DEV)   # never read: refused first
    with pytest.raises(E.EnsError):
        E.cg_noalloc(g, vals, b, torch.zeros_like(b))
