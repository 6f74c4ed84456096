"""Pins of the oracle's parent-event reading (the proxy-cache case study of
Section 5: per-video events seen by every request of the video).

Reading: with parent events on, an event that carries the values of
x_0..x_{n-2} and none for x_{n-1} joins u^D of every instance D whose first
n-1 values are its own, at its trace position; it adds no value vector
(Eq. 5), so no instance and no node.

Pins, none of which re-types the merge the C oracle performs:
* clusters written out by hand for a small video/request trace, with the
  leaf verdict of each taken from the Def. 5 tableau on the hand-written word;
* replication: the same trace where every parent event is replaced by one
  full event per existing child of its parent, at the same position, gives
  the same instances, nodes and verdicts under the plain reading (which the
  other oracle tests pin);
* the Python restatement (the definition of u^D written out as a filter over
  the trace) agrees with the C oracle at 1-3 levels with excluded events;
* parent events under a parent with no instance change nothing.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import cref
from oracle.counting import evaluate
from oracle.ltl import BOT, BOT_P, TOP, TOP_C, ltl4, parse
from oracle.run import oracle_monitor

OPS = ("<", "<=", ">", ">=", "=")
NAMES = "abc"


def _props(specs, class_props):
    out = []
    for f, q in specs:
        m = oracle_monitor(f)
        out.append(cref.OracleProperty(np.array(m.class_table(class_props), dtype=np.uint32),
                                       np.array(m.label, dtype=np.uint8), m.q0, q))
    return out


def _run(rec, n_levels, cot, kp, specs, class_props, parent_events):
    return cref.evaluate_records(rec.view(np.uint8).reshape(-1), 4 * (2 + n_levels), 4, 4,
                                 [8 + 4 * m for m in range(n_levels)], [4] * n_levels, cot, kp,
                                 _props(specs, class_props), parent_events=parent_events)


# --- a video/request trace, clusters by hand ---------------------------------------
# types: 0 insert(v), 1 evict(v)  [parent events: carry only the video]
#        2 local request(v, r), 3 external request(v, r)
# propositions: a = insert, b = evict, c = external
CLASS_PROPS = [frozenset("a"), frozenset("b"), frozenset(), frozenset("c")]
LEAF = "F(a & (!b U c))"     # an external request while the video is cached


def _video_trace(rows):
    rec = np.zeros((len(rows), 4), dtype=np.uint32)
    for i, (t, v, r) in enumerate(rows):
        rec[i] = (i, t, v, r)
    cot = np.zeros(256, dtype=np.uint8)
    cot[:4] = [0, 1, 2, 3]
    kp = np.zeros(256, dtype=np.uint8)
    kp[:2] = 0b01
    kp[2:4] = 0b11
    return rec, cot, kp


def test_hand_written_clusters():
    rows = [(2, 1, 7),      # 0 local request r7 of v1 (before any insert)
            (0, 1, 0),      # 1 insert v1
            (3, 1, 8),      # 2 external r8 of v1: while cached
            (1, 1, 0),      # 3 evict v1
            (3, 1, 7),      # 4 external r7 of v1: not cached any more
            (0, 2, 0),      # 5 insert v2 (v2 has no request: no instance)
            (3, 3, 1),      # 6 external r1 of v3 (v3 never cached)
            (0, 1, 0),      # 7 insert v1 again
            (2, 1, 9)]      # 8 local r9 of v1
    rec, cot, kp = _video_trace(rows)
    spec = [(LEAF, [("A", ">=", Fraction(1)), ("E", "=", 0)])]
    res = _run(rec, 2, cot, kp, spec, CLASS_PROPS, True)
    P = CLASS_PROPS
    # u^D written out by hand: own events and v's inserts/evicts, in trace order
    slices = {(1, 7): [P[2], P[0], P[1], P[3], P[0]],
              (1, 8): [P[0], P[3], P[1], P[0]],
              (1, 9): [P[0], P[1], P[0], P[2]],
              (3, 1): [P[3]]}
    f = parse(LEAF)
    assert [tuple(k) for k in res.inst_keys] == sorted(slices)
    want = [ltl4(f, slices[d]) for d in sorted(slices)]
    assert list(res.inst_verdict[0]) == want
    # closed forms of the leaf on these words
    assert want == [BOT_P, TOP, BOT_P, BOT_P]
    # v1: one instance is T, so E=0 fails for good (Table 1, row =); v3: no T
    # child yet, but a new one may come: currently true
    assert [tuple(k) for k in res.level_keys[1]] == [(1,), (3,)]
    assert list(res.level_counts[1][0, 0]) == [0, 0, 2, 0, 0, 1]
    assert list(res.level_verdict[1][0]) == [BOT, TOP_C]
    assert res.root_verdict[0] == BOT
    # without the option the parent events join no cluster
    res0 = _run(rec, 2, cot, kp, spec, CLASS_PROPS, False)
    assert list(res0.inst_verdict[0]) == [ltl4(f, [P[2], P[3]]), ltl4(f, [P[3]]), ltl4(f, [P[2]]), ltl4(f, [P[3]])]
    assert list(res0.inst_verdict[0]) == [BOT_P] * 4
    # per-event verdicts: own events only; a parent event is in several clusters
    ev = res.event_verdict[0]
    assert ev[1] == 0xFF and ev[3] == 0xFF and ev[5] == 0xFF and ev[7] == 0xFF
    assert ev[2] == TOP and ev[8] == BOT_P


def test_one_level_events_without_a_key_join_every_cluster():
    # single quantifier over sockets; type 0 carries no key (a global event)
    cp = [frozenset("a"), frozenset("b")]
    rows = [(1, 5), (0, 0), (1, 6), (1, 5)]
    rec = np.zeros((4, 3), dtype=np.uint32)
    for i, (t, k) in enumerate(rows):
        rec[i] = (i, t, k)
    cot = np.zeros(256, dtype=np.uint8)
    cot[:2] = [0, 1]
    kp = np.zeros(256, dtype=np.uint8)
    kp[1] = 1
    spec = [("b U a", [("A", ">=", Fraction(1))])]
    res = _run(rec, 1, cot, kp, spec, cp, True)
    f = parse("b U a")
    assert [tuple(k) for k in res.inst_keys] == [(5,), (6,)]
    assert list(res.inst_verdict[0]) == [ltl4(f, [cp[1], cp[0], cp[1]]), ltl4(f, [cp[0], cp[1]])]
    assert list(res.inst_verdict[0]) == [TOP, TOP]
    res0 = _run(rec, 1, cot, kp, spec, cp, False)
    assert list(res0.inst_verdict[0]) == [ltl4(f, [cp[1], cp[1]]), ltl4(f, [cp[1]])]


# --- random traces ------------------------------------------------------------
def _random_case(seed):
    rng = np.random.default_rng(0xCA5E + seed)
    n_levels = 1 + seed % 3
    n = int(rng.integers(1, 70))
    rec = np.zeros((n, 2 + n_levels), dtype=np.uint32)
    typ = rng.integers(0, 8, size=n).astype(np.uint32)
    rec[:, 0] = np.arange(n)
    rec[:, 1] = typ
    rec[:, 2:] = rng.integers(0, 3, size=(n, n_levels))
    full = (1 << n_levels) - 1
    cot = np.zeros(256, dtype=np.uint8)
    cot[:8] = np.arange(8)
    kp = np.zeros(256, dtype=np.uint8)
    kp[:8] = full
    kp[5] = full >> 1                 # parent events
    kp[6] = full >> 1
    kp[7] = int(rng.integers(0, full + 1)) if n_levels > 1 else 0   # some other key set, often excluded
    class_props = [frozenset(NAMES[i] for i in range(3) if (c >> i) & 1) for c in range(8)]
    pool = ["G(a -> F b)", "a U b", "G(a -> X b)", "F(a & X F a)", "!X a", "G a | (b U c)", "F(a & (!b U c))"]
    specs = []
    for _ in range(2):
        f = pool[int(rng.integers(0, len(pool)))]
        q = []
        for _ in range(n_levels):
            kind = "A" if rng.random() < 0.5 else "E"
            op = OPS[int(rng.integers(0, 5))]
            const = Fraction(int(rng.integers(0, 4)), 3) if kind == "A" else int(rng.integers(0, 3))
            q.append((kind, op, const))
        specs.append((f, q))
    return n_levels, rec, typ, cot, kp, class_props, specs


def _compare(res, root, nodes, leaves, p, n_levels):
    assert res.root_verdict[p] == root
    assert list(res.root_counts[p]) == nodes[()][0]
    assert res.inst_keys.shape[0] == len(leaves)
    for i, d in enumerate(sorted(leaves)):
        assert tuple(res.inst_keys[i]) == d
        assert res.inst_verdict[p, i] == leaves[d]
    for m in range(1, n_levels):
        pres = sorted(k for k in nodes if len(k) == m)
        assert res.level_keys[m].shape[0] == len(pres)
        for j, pre in enumerate(pres):
            assert tuple(res.level_keys[m][j]) == pre
            assert list(res.level_counts[m][p, j]) == nodes[pre][0]
            assert res.level_verdict[m][p, j] == nodes[pre][1]


@pytest.mark.parametrize("seed", range(30))
def test_c_matches_python_definition(seed):
    n_levels, rec, typ, cot, kp, class_props, specs = _random_case(seed)
    res = _run(rec, n_levels, cot, kp, specs, class_props, True)
    full = (1 << n_levels) - 1
    events = []
    for i in range(rec.shape[0]):
        t = int(typ[i])
        k = int(kp[t])
        if k == full:
            key = tuple(int(x) for x in rec[i, 2:])
        elif k == full >> 1:
            key = tuple(int(x) for x in rec[i, 2:2 + n_levels - 1])
        else:
            key = None
        events.append((class_props[int(cot[t])], key))
    for p, (f, q) in enumerate(specs):
        ff = parse(f)
        root, nodes, leaves = evaluate(events, q, lambda w: ltl4(ff, w), parent_events=True)
        _compare(res, root, nodes, leaves, p, n_levels)


@pytest.mark.parametrize("seed", range(30))
def test_replication_gives_the_same_results(seed):
    """Replace each parent event by one full event per existing child of its
    parent (same letter, same place in the trace) and evaluate without parent
    events: every output agrees."""
    n_levels, rec, typ, cot, kp, class_props, specs = _random_case(seed)
    full = (1 << n_levels) - 1
    n = rec.shape[0]
    is_full = np.array([kp[int(t)] == full for t in typ])
    is_par = np.array([kp[int(t)] == full >> 1 for t in typ])
    children = {}
    for i in np.nonzero(is_full)[0]:
        d = tuple(int(x) for x in rec[i, 2:])
        children.setdefault(d[:-1], set()).add(d[-1])
    rows = []
    for i in range(n):
        if is_par[i]:
            pre = tuple(int(x) for x in rec[i, 2:2 + n_levels - 1])
            for c in sorted(children.get(pre, ())):
                r = rec[i].copy()
                r[1] = 8 + int(typ[i])          # a full-key copy with the same letter
                r[2 + n_levels - 1] = c
                rows.append(r)
        elif not is_full[i]:
            rows.append(rec[i].copy())          # excluded either way
        else:
            rows.append(rec[i].copy())
    rec2 = np.array(rows, dtype=np.uint32).reshape(-1, 2 + n_levels)
    rec2[:, 0] = np.arange(rec2.shape[0])
    cot2 = cot.copy()
    kp2 = kp.copy()
    for t in range(8):
        cot2[8 + t] = cot[t]
        kp2[8 + t] = full
    a = _run(rec, n_levels, cot, kp, specs, class_props, True)
    b = _run(rec2, n_levels, cot2, kp2, specs, class_props, False)
    assert np.array_equal(a.inst_keys, b.inst_keys)
    assert np.array_equal(a.inst_verdict, b.inst_verdict)
    for m in range(n_levels):
        assert np.array_equal(a.level_keys[m], b.level_keys[m])
        assert np.array_equal(a.level_counts[m], b.level_counts[m])
        assert np.array_equal(a.level_verdict[m], b.level_verdict[m])


def test_parent_events_without_instances_change_nothing():
    n_levels, rec, typ, cot, kp, class_props, specs = _random_case(4)
    full = (1 << n_levels) - 1
    # parent events under parents no full event has: prefix values 9
    extra = np.zeros((5, 2 + n_levels), dtype=np.uint32)
    extra[:, 1] = 5
    extra[:, 2:] = 9
    rec2 = np.concatenate([rec, extra, rec[:0]])
    rec2[:, 0] = np.arange(rec2.shape[0])
    assert kp[5] == full >> 1
    a = _run(rec, n_levels, cot, kp, specs, class_props, True)
    b = _run(rec2, n_levels, cot, kp, specs, class_props, True)
    assert np.array_equal(a.inst_verdict, b.inst_verdict)
    for m in range(n_levels):
        assert np.array_equal(a.level_counts[m], b.level_counts[m])


def test_propositional_leaf_with_exactly_zero():
    """The case study's literal shape A v: E=0 r: (cached & external), with
    both propositions on the request event itself: a leaf decided by the
    first event of its cluster (T or F), and E=0 false for good at the first
    T child (Table 1)."""
    cp = [frozenset(), frozenset("a"), frozenset("b"), frozenset("ab")]   # a = cached, b = external
    rows = [(3, 1, 1), (1, 1, 2), (2, 2, 3), (0, 2, 4), (1, 3, 5), (3, 3, 5)]
    rec = np.zeros((len(rows), 4), dtype=np.uint32)
    for i, (t, v, r) in enumerate(rows):
        rec[i] = (i, t, v, r)
    cot = np.zeros(256, dtype=np.uint8)
    cot[:4] = [0, 1, 2, 3]
    kp = np.zeros(256, dtype=np.uint8)
    kp[:4] = 0b11
    spec = [("a & b", [("A", ">=", Fraction(1)), ("E", "=", 0)])]
    res = _run(rec, 2, cot, kp, spec, cp, False)
    # (3,5): first event cached only, so F even though a later event has both
    assert list(res.inst_verdict[0]) == [TOP, BOT, BOT, BOT, BOT]
    assert list(res.level_verdict[1][0]) == [BOT, TOP_C, TOP_C]
    assert res.root_verdict[0] == BOT
    for w in itertools.product(cp, repeat=3):
        assert ltl4(parse("a & b"), list(w)) == (TOP if w[0] == cp[3] else BOT)
