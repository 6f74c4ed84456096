"""Pins of the oracle's verdict timeline: for every instance, the length of
its shortest prefix whose LTL4 verdict is T or F (0: the empty prefix), or
NEVER.  Closed forms: F a is first T at the first a, G a first F at the first
event without a, a valid body is T before any event; and the timeline agrees
with the final instance verdicts (T or F at the end iff some prefix was)."""
import numpy as np
import pytest

from oracle.cref import NEVER
from oracle.run import evaluate_workload

from _util import prop_workload


def _clusters(wl):
    """Events of every instance in trace order, instances in key order."""
    keys = np.stack([wl.records[f"k{m}"] for m in range(wl.layout.n_keys)], axis=1).astype(np.int64)
    order = np.lexsort(tuple(keys[:, m] for m in reversed(range(keys.shape[1]))))   # stable: trace order inside
    ks = keys[order]
    starts = np.flatnonzero(np.r_[True, np.any(ks[1:] != ks[:-1], axis=1)])
    ends = np.r_[starts[1:], len(order)]
    return [order[s:e] for s, e in zip(starts, ends)]


def _first(mask):
    idx = np.flatnonzero(mask)
    return int(idx[0]) + 1 if idx.size else NEVER


@pytest.mark.parametrize("formula,want", [
    ("F a", lambda ev_a: _first(ev_a)),
    ("G a", lambda ev_a: _first(~ev_a)),
])
def test_closed_forms(formula, want):
    wl = prop_workload(3_000, 1, [40], seed=7, n_props=1, formulas=[formula], quants=[[("E", ">=", 1)]])
    o = evaluate_workload(wl)
    has_a = (wl.records["type"] & 1).astype(bool)          # proposition a is type bit 0
    exp = np.array([want(has_a[c]) for c in _clusters(wl)], dtype=np.uint32)
    assert np.array_equal(o.inst_conc[0], exp)


def test_valid_body_is_conclusive_before_any_event():
    wl = prop_workload(2_000, 2, [5, 9], seed=8, n_props=1, formulas=["true"], quants=[[("E", ">=", 1)] * 2])
    o = evaluate_workload(wl)
    assert (o.inst_conc == 0).all()


def test_timeline_agrees_with_final_verdicts():
    wl = prop_workload(20_000, 2, [30, 40], seed=9, n_props=8)
    o = evaluate_workload(wl)
    lengths = np.array([len(c) for c in _clusters(wl)])
    for p in range(8):
        conclusive_end = np.isin(o.inst_verdict[p], (0, 5))
        assert np.array_equal(conclusive_end, o.inst_conc[p] != NEVER)
        fin = o.inst_conc[p][o.inst_conc[p] != NEVER]
        assert (fin <= lengths[o.inst_conc[p] != NEVER]).all()
