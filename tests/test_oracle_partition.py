"""The key-partitioned, multi-threaded oracle run (oracle/parallel.py) against
one plain run over the whole trace: the root splits into the subtrees of the
top-level values, so instances, nodes and root counts of disjoint partitions
together must equal the whole trace's (the additivity of root counts), for any
number of partitions, with excluded events and data predicates present."""
import numpy as np
import pytest

from oracle import parallel
from oracle.run import evaluate_workload, oracle_property
from paper_1411_2239_amd import workloads as W

from _util import prop_workload


def _same(a, b, n_levels):
    assert np.array_equal(a.root_verdict, b.root_verdict)
    assert np.array_equal(a.root_counts, b.root_counts)
    assert np.array_equal(a.inst_keys, b.inst_keys)
    assert np.array_equal(a.inst_verdict, b.inst_verdict)
    for m in range(1, n_levels):
        assert np.array_equal(a.level_keys[m], b.level_keys[m])
        assert np.array_equal(a.level_counts[m], b.level_counts[m])
        assert np.array_equal(a.level_verdict[m], b.level_verdict[m])


@pytest.mark.parametrize("n_levels,parts", [(1, 1), (1, 7), (2, 3), (3, 16), (2, 64)])
def test_partitioned_equals_whole(n_levels, parts):
    wl = prop_workload(30_000, n_levels, [50, 9, 5][:n_levels], seed=11 + n_levels, n_props=4)
    props = [oracle_property(s, wl.layout) for s in wl.props]
    whole = evaluate_workload(wl)
    split = parallel.evaluate_partitioned(wl.raw(), wl.layout, props, n_parts=parts, threads=4)
    _same(split, whole, n_levels)


def test_partitioned_user_requests_and_predicates():
    for wl in (W.gen_user_requests(200_000, 400, seed=5), W.gen_chunk_uploads(100_000, 300, n_preds=2, seed=6)):
        props = [oracle_property(s, wl.layout) for s in wl.props]
        _same(parallel.evaluate_partitioned(wl.raw(), wl.layout, props, n_parts=8, threads=8),
              evaluate_workload(wl), wl.layout.n_keys)


def test_partitioned_with_excluded_events():
    wl = W.gen_user_requests(50_000, 100, seed=9)
    rec = wl.records.copy()
    rec["type"][::7] = 999          # no cluster
    wl2 = W.Workload(wl.name, rec, wl.layout, wl.props)
    props = [oracle_property(s, wl.layout) for s in wl.props]
    _same(parallel.evaluate_partitioned(wl2.raw(), wl.layout, props, n_parts=5, threads=3),
          evaluate_workload(wl2), 2)


def test_empty_partitions():
    wl = prop_workload(100, 1, [2], seed=3, n_props=2)
    props = [oracle_property(s, wl.layout) for s in wl.props]
    _same(parallel.evaluate_partitioned(wl.raw(), wl.layout, props, n_parts=32, threads=4),
          evaluate_workload(wl), 1)
