"""Resident device pool for batched solves that exceed device memory.

A batch of sample groups (an ensemble of s samples on one mesh each) is
streamed through one preallocated device buffer in waves: a wave is the
longest run of consecutive groups whose buffers (matrix values, load vector,
solution) and solver workspace fit the pool; its groups are assembled into the
pool and solved by one ens_assemble_solve_batch call (the assemblies, the
solver's set-up and its first chunk of iterations one captured graph), then
the next wave reuses the same memory.  Graphs and KL tables are shared by all groups on one mesh and
stay resident outside the pool.

The wave planner is host logic only (no device calls).
"""
from __future__ import annotations

from dataclasses import dataclass

ALIGN = 256


def _r(b: int) -> int:
    return (b + ALIGN - 1) // ALIGN * ALIGN


def mesh_sizes(N: int) -> tuple[int, int]:
    """(nodes, stored entries) of the N^3 Q1 hexahedral mesh of the unit cube."""
    return (N + 1) ** 3, (3 * N + 1) ** 3


def group_buffer_bytes(N: int, s: int) -> int:
    """values [nnz][s], b and x [n][s], FP64, each 256-byte aligned."""
    n, nnz = mesh_sizes(N)
    return _r(8 * nnz * s) + 2 * _r(8 * n * s)


def group_workspace_bound(N: int, s: int) -> int:
    """Upper bound of one group's share of the ens_assemble_solve_batch
    workspace: four solver vectors [n][s], per-block partials, per-group
    tables and the assembly's workgroup table (one entry per 32 nodes)."""
    n, _ = mesh_sizes(N)
    return 4 * _r(8 * n * s) + 16 * 8 * n + 64 * 1024 + _r(4 * (n // 32 + 3 * (N + 1) ** 2))


@dataclass
class Wave:
    first: int          # index of the first group
    count: int          # groups in the wave
    buffer_bytes: int   # pool bytes taken by group buffers
    workspace_bound: int


def plan_waves(meshes, s: int, pool_bytes: int) -> list[Wave]:
    """Split groups (mesh size per group, in order) into consecutive waves that
    fit `pool_bytes`.  Raises ValueError when one group alone does not fit."""
    waves: list[Wave] = []
    i = 0
    meshes = [int(N) for N in meshes]
    while i < len(meshes):
        buf = ws = 0
        j = i
        while j < len(meshes):
            b = group_buffer_bytes(meshes[j], s)
            w = group_workspace_bound(meshes[j], s)
            if buf + b + ws + w > pool_bytes:
                break
            buf += b
            ws += w
            j += 1
        if j == i:
            need = group_buffer_bytes(meshes[i], s) + group_workspace_bound(meshes[i], s)
            raise ValueError(f"group {i} (N={meshes[i]}, s={s}) needs {need} bytes, more than the pool's "
                             f"{pool_bytes}")
        waves.append(Wave(i, j - i, buf, ws))
        i = j
    return waves


class BatchPool:
    """Runs the batched solve of many groups through one device buffer."""

    def __init__(self, ens, meshes, s: int, M: int, pool_bytes: int, L: float = 1.0, device="cuda"):
        import torch

        self.ens = ens
        self.meshes = [int(N) for N in meshes]
        self.s = s
        self.M = M
        self.L = L
        self.pool_bytes = int(pool_bytes)
        self.waves = plan_waves(self.meshes, s, self.pool_bytes)
        self.pool = torch.empty(self.pool_bytes, dtype=torch.uint8, device=device)
        self.graphs = {}
        for N in sorted(set(self.meshes)):
            self.graphs[N] = (ens.graph_build(N), ens.kl_build(N, M, L))

    def group_by_contrast(self, xi_groups, sigma: float, kappa0: float = 1.0):
        """Regroup the samples of the groups on each mesh by the contrast
        kmax / kmin of their coefficient over that mesh's Gauss points
        (Sec. 3.7: samples of similar parameter variation need similar
        iteration counts, and an ensemble runs as long as its slowest
        sample).  Returns (xi regrouped [groups][s][M] on the device,
        order [groups * s]: order[g * s + j] is the draw-order index of the
        sample now at position j of group g)."""
        import numpy as np
        import torch

        ens, s = self.ens, self.s
        G = len(self.meshes)
        flat = xi_groups.reshape(G * s, -1)
        order = np.arange(G * s, dtype=np.int64)
        meshes = np.asarray(self.meshes)
        for N in sorted(set(self.meshes)):
            gidx = np.flatnonzero(meshes == N)
            samples = (gidx[:, None] * s + np.arange(s)[None, :]).reshape(-1)
            _, kl = self.graphs[N]
            kmin, kmax = ens.kl_extrema(N, kl, flat[torch.as_tensor(samples, device=flat.device)].contiguous(),
                                        self.M, sigma, L=self.L, kappa0=kappa0)
            perm = ens.group_order((kmax / kmin).cpu().numpy())
            order[samples] = samples[perm]
        regrouped = flat[torch.as_tensor(order, device=flat.device)].reshape(xi_groups.shape).contiguous()
        return regrouped, order

    def _carve(self, off: int, nbytes: int, shape):
        import torch

        t = self.pool[off:off + nbytes].view(torch.float64)
        n = 1
        for d in shape:
            n *= d
        return t[:n].view(*shape), off + _r(nbytes)

    def run(self, xi_groups, sigma: float, opts, kappa0: float = 1.0, f: float = 1.0, on_wave=None):
        """xi_groups: device tensor [groups][s][M] of KL inputs.  Assembles and
        solves every group; returns the per-group stats lists and the worst
        status.  Solutions of a wave live in the pool until the next wave
        overwrites them; `on_wave(wave, groups, stats)` sees them first."""
        ens, s = self.ens, self.s
        all_stats = []
        worst = ens.ENS_OK
        for wv in self.waves:
            off = 0
            groups, inputs = [], []
            for gi in range(wv.first, wv.first + wv.count):
                N = self.meshes[gi]
                g, kl = self.graphs[N]
                n, nnz = mesh_sizes(N)
                vals, off = self._carve(off, 8 * nnz * s, (nnz, s))
                b, off = self._carve(off, 8 * n * s, (n, s))
                x, off = self._carve(off, 8 * n * s, (n, s))
                groups.append((g, vals, b, x))
                inputs.append((N, kl, xi_groups[gi]))
            # the wave's assemblies, the solver's set-up and its first chunk
            # of iterations run as one captured graph
            ws = self.pool[off:]
            stats, rc, used = ens.assemble_solve_batch(groups, inputs, s, self.M, sigma, opts, workspace=ws, L=self.L,
                                                       kappa0=kappa0, f=f, strict_workspace=True)
            if on_wave is not None:
                on_wave(wv, groups, stats)
            all_stats.extend(stats)
            if rc != ens.ENS_OK:
                worst = rc
        return all_stats, worst
