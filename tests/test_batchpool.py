"""Host logic of the batched-solve pool: wave planning (no device calls)."""
import pytest

from paper_1511_03703_amd import batchpool as bp
from workloads import batch_meshes


def test_mesh_sizes_match_q1_counts():
    assert bp.mesh_sizes(16) == (4913, 117649)
    assert bp.mesh_sizes(64) == (274625, 7189057)
    assert bp.mesh_sizes(128) == (2146689, 57066625)


@pytest.mark.parametrize("s", [8, 16, 32])
@pytest.mark.parametrize("pool_gb", [40, 96, 200])
def test_waves_cover_groups_in_order_within_budget(s, pool_gb):
    meshes = batch_meshes()
    pool = pool_gb << 30
    waves = bp.plan_waves(meshes, s, pool)
    assert waves[0].first == 0
    for a, b in zip(waves, waves[1:]):
        assert b.first == a.first + a.count
    assert waves[-1].first + waves[-1].count == len(meshes)
    for w in waves:
        assert w.count >= 1
        assert w.buffer_bytes + w.workspace_bound <= pool
        assert w.buffer_bytes == sum(bp.group_buffer_bytes(N, s) for N in meshes[w.first:w.first + w.count])
    # each wave is maximal: the next group would not have fit
    for a, b in zip(waves, waves[1:]):
        N = meshes[b.first]
        assert (a.buffer_bytes + a.workspace_bound + bp.group_buffer_bytes(N, s)
                + bp.group_workspace_bound(N, s)) > pool


def test_group_larger_than_pool_is_refused():
    with pytest.raises(ValueError):
        bp.plan_waves([96], 32, 1 << 30)
    assert bp.plan_waves([], 32, 1 << 30) == []


def test_batch_memory_exceeds_one_device_at_large_s():
    # the 256-group batch does not fit 288 GB at s = 32, so it must stream
    meshes = batch_meshes()
    total = sum(bp.group_buffer_bytes(N, 32) + bp.group_workspace_bound(N, 32) for N in meshes)
    assert total > 288e9
