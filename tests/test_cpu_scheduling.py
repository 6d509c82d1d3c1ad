"""Host-side scheduling logic of the batching and serving layers (no GPU):
the eigensolve schedule of a BatchPlan (`size_classes`), the serving
executor's HBM footprint and latency statistics, and the autotuned tile
table."""
import math
from types import SimpleNamespace

import numpy as np
import pytest


def _flatten(lanes):
    return [k for lane in lanes for g in lane for k in g]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_size_classes_partition_and_grouping(seed):
    from paper_2005_03426_amd.batch import size_classes
    rng = np.random.default_rng(seed)
    sizes = [int(x) for x in np.exp(rng.uniform(math.log(2), math.log(3000), 300)).astype(int)]
    lanes = size_classes(sizes, small_max=64, group_max=16, lanes=4)
    assert 1 <= len(lanes) <= 4
    flat = _flatten(lanes)
    assert sorted(flat) == list(range(len(sizes)))          # every problem exactly once
    groups = [g for lane in lanes for g in lane]
    small = [g for g in groups if all(sizes[k] <= 64 for k in g)]
    assert len(small) == 1 and sorted(small[0]) == [k for k, m in enumerate(sizes) if m <= 64]
    for g in groups:
        if g is small[0]:
            continue
        assert len(g) <= 16
        octs = {int(sizes[k] - 1).bit_length() for k in g}
        assert len(octs) == 1                               # one octave of the order per group
        assert [sizes[k] for k in g] == sorted((sizes[k] for k in g), reverse=True)


def test_size_classes_balances_the_largest_groups_over_lanes():
    from paper_2005_03426_amd.batch import size_classes
    sizes = [1900] * 8 + [40] * 10
    lanes = size_classes(sizes, group_max=2, lanes=4)
    big_per_lane = [sum(1 for g in lane for k in g if sizes[k] == 1900) for lane in lanes]
    assert len(lanes) == 4 and big_per_lane == [2, 2, 2, 2]


def test_footprint_covers_matrix_workspace_and_retry():
    from paper_2005_03426_amd import serve, eigh_workspace_bytes, MMF_C128, MMF_C64_REFINED
    prev = 0
    for M in (50, 400, 2000, 6000, 12000):
        D = 5
        f = serve.footprint_bytes(M, D, 32)
        assert f >= 16 * M * M + eigh_workspace_bytes(M, MMF_C128)
        assert f > prev
        prev = f
        # a mixed-precision request also covers its complex128 retry
        fr = serve.footprint_bytes(M, D, 32, MMF_C64_REFINED)
        assert fr >= 16 * M * M + max(eigh_workspace_bytes(M, MMF_C64_REFINED), eigh_workspace_bytes(M, MMF_C128))


def test_latency_stats():
    from paper_2005_03426_amd import serve
    done = [SimpleNamespace(arrival=0.1 * k, done=0.1 * k + 0.5 + 0.01 * k, latency=0.5 + 0.01 * k) for k in range(100)]
    st = serve.latency_stats(done)
    assert st["count"] == 100
    span = done[-1].done - done[0].arrival
    assert st["makespan_s"] == pytest.approx(span)
    assert st["solves_per_s"] == pytest.approx(100 / span)
    lat = np.array([d.latency for d in done])
    assert st["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert st["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)


def test_tune_table_entries_are_valid():
    from paper_2005_03426_amd import autotune
    tab = autotune.load_table()
    assert tab is not None and len(tab) == 8
    assert all(int(x) in (0, 64, 128, 256, 512) for x in tab)
