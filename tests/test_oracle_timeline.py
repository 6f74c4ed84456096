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


@pytest.mark.parametrize("formula,want", [
    ("F a", lambda a_so_far, not_a_so_far: np.where(a_so_far, 5, 2)),
    ("G a", lambda a_so_far, not_a_so_far: np.where(not_a_so_far, 0, 3)),
])
def test_event_verdicts_closed_forms(formula, want):
    # after each event: F a is T once an a was seen in the instance, else Fp;
    # G a is F once an event without a was seen, else Tp
    wl = prop_workload(3_000, 1, [40], seed=17, n_props=1, formulas=[formula], quants=[[("E", ">=", 1)]])
    o = evaluate_workload(wl)
    has_a = (wl.records["type"] & 1).astype(bool)
    exp = np.zeros(wl.n_events, dtype=np.uint8)
    for c in _clusters(wl):
        exp[c] = want(np.cumsum(has_a[c]) > 0, np.cumsum(~has_a[c]) > 0)
    assert np.array_equal(o.event_verdict[0], exp)


def test_event_verdicts_mark_excluded_events_and_end_in_the_instance_verdict():
    wl = prop_workload(5_000, 2, [10, 20], seed=18, n_props=3)
    rng = np.random.default_rng(18)
    t = wl.records["type"].copy()
    out = rng.random(wl.n_events) < 0.2
    t[out] = 300
    wl.records["type"] = t
    wl.layout.type_bytes = 2
    o = evaluate_workload(wl)
    assert (o.event_verdict[:, out] == 0xFF).all() and (o.event_verdict[:, ~out] <= 5).all()
    # the last event of every instance carries the instance's verdict
    keys = np.stack([wl.records["k0"], wl.records["k1"]], axis=1).astype(np.int64)
    keys[out] = -1
    inst = {tuple(k): i for i, k in enumerate(o.inst_keys.astype(np.int64))}
    last = {}
    for pos in range(wl.n_events):
        if not out[pos]:
            last[tuple(keys[pos])] = pos
    for k, pos in last.items():
        assert np.array_equal(o.event_verdict[:, pos], o.inst_verdict[:, inst[k]])
