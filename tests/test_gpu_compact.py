"""GPU parity of compaction (Sec. 3.7: a finished sample still costs its
share of every pass over the ensemble): once at most s/2 samples iterate,
they finish in an ensemble of s/2.  Each sample's solve is the uncompacted
one up to rounding: against the oracle at the GPU's iteration counts
(relative 1e-9), the oracle's own counts within +-1, the true residual at
the tolerance.  Without a pause (equal counts, or s = 4) nothing moves and
the result is bitwise the uncompacted one."""
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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _system(E, N, s, M, sigma, seed):
    xi = draw_xi(seed, s, M)
    g, kl = E.graph_build(N), E.kl_build(N, M)
    v, _, b = E.assemble(g, kl, torch.as_tensor(xi, device=DEV), M, sigma)
    return g, v, b, xi


@pytest.mark.parametrize("N,s,sigma", [(12, 16, 0.5), (10, 32, 0.5), (14, 8, 0.5)])
def test_compacted_solve_matches_oracle(E, orc, N, s, sigma):
    M, rtol = 10, 1e-10
    g, v, b, xi = _system(E, N, s, M, sigma, 6000 + N + s)
    # counts here spread over a few iterations only: poll after every one
    x0, st0, rc0 = E.cg(g, v, b, opts=E.cg_opts(rtol=rtol, check_every=1))
    x1, st1, rc1 = E.cg(g, v, b, opts=E.cg_opts(rtol=rtol, check_every=1, compact=True))
    assert rc0 == E.ENS_OK and rc1 == E.ENS_OK
    moved = [t["compacted"] for t in st1]
    assert 0 < sum(moved) <= s // 2, moved
    assert not any(t["compacted"] for t in st0)
    rp, ci = orc.graph(N)
    ov, ob = orc.assemble_ensemble(N, rp, ci, M, 1.0, 1.0, sigma, 1.0, xi)
    it1 = np.array([t["iters"] for t in st1], np.int32)
    xo, _, _, _ = orc.ens_pcg(rp, ci, ov, ob, fixed_iters=it1)
    _, itt, _, _ = orc.ens_pcg(rp, ci, ov, ob, rtol=rtol)
    true = orc.ens_true_residual(rp, ci, ov, ob, _np(x1))
    xg = _np(x1)
    for e in range(s):
        assert st1[e]["status"] == 0
        assert _rel(xg[:, e], xo[:, e]) <= 1e-9, (e, _rel(xg[:, e], xo[:, e]))
        assert abs(int(itt[e]) - int(it1[e])) <= 1, (e, itt[e], it1[e])
        assert abs(st0[e]["iters"] - st1[e]["iters"]) <= 1
        assert true[e] <= rtol * (1 + 1e-6)
        assert abs(st1[e]["rel_res"] - true[e]) <= 1e-6 * rtol + 1e-3 * true[e]
    # samples finished before the pause are untouched by it, bitwise
    for e in range(s):
        if not moved[e]:
            assert np.array_equal(xg[:, e], _np(x0)[:, e])


def test_no_pause_leaves_the_solve_bitwise_unchanged(E):
    # s = 4 never compacts; equal coefficients give equal counts, so no poll
    # finds between 1 and s/2 samples still iterating
    for N, s, sigma in ((10, 4, 0.5), (10, 16, 0.0)):
        g, v, b, _ = _system(E, N, s, 10, sigma, 6100 + s)
        x0, st0, _ = E.cg(g, v, b, opts=E.cg_opts(rtol=1e-10, check_every=2))
        x1, st1, _ = E.cg(g, v, b, opts=E.cg_opts(rtol=1e-10, check_every=2, compact=True))
        assert torch.equal(x0, x1)
        assert [t["iters"] for t in st0] == [t["iters"] for t in st1]
        assert not any(t["compacted"] for t in st1)


def test_compaction_refusals_and_workspace(E):
    g, v, b, _ = _system(E, 6, 16, 10, 0.3, 6200)
    with pytest.raises(E.EnsError, match="compaction"):
        E.cg(g, v, b, values32=v.to(torch.float32), opts=E.cg_opts(mixed=True, compact=True))
    with pytest.raises(E.EnsError, match="compaction"):
        E.cg(g, v, b, opts=E.cg_opts(coupled=True, compact=True))
    plain = E.cg_workspace_bytes(g, 16, E.cg_opts())
    comp = E.cg_workspace_bytes(g, 16, E.cg_opts(compact=True))
    assert comp - plain >= g.nnz * 8 * 8 + 5 * g.n * 8 * 8
    assert E.cg_workspace_bytes(g, 4, E.cg_opts(compact=True)) == E.cg_workspace_bytes(g, 4, E.cg_opts())
