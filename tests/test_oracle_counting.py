"""Pins of the oracle's counting semantics (oracle/counting.py, oracle/c)
against the paper's worked example, Table 1, the rule for the default A=1,
the informal readings of Section 2.3, and an enumeration of extensions."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import cref
from oracle.counting import evaluate, perm_sat, perm_viol, valuate, constraint
from oracle.ltl import BOT, BOT_C, BOT_P, TOP, TOP_C, TOP_P, ltl4, parse, props

HERE = os.path.dirname(os.path.abspath(__file__))
OPS = ["<", "<=", ">", ">=", "="]
PCT = [Fraction(0), Fraction(1, 3), Fraction(1, 2), Fraction(19, 20), Fraction(1)]
CNT = [0, 1, 2, 3]


def vec(**kw):
    v = [0] * 6
    names = {"F": BOT, "Fc": BOT_C, "Fp": BOT_P, "Tp": TOP_P, "Tc": TOP_C, "T": TOP}
    for k, n in kw.items():
        v[names[k]] = n
    return v


# --- worked example (golden fixture) -------------------------------------------
def test_worked_example():
    g = json.load(open(os.path.join(HERE, "golden", "worked_example.json")))
    f = parse(g["property"]["formula"])
    quants = [tuple(q) for q in g["property"]["quants"]]
    events = [(frozenset(e["props"]), (e["user"], e["rid"])) for e in g["trace"]]
    root, nodes, leaves = evaluate(events, quants, lambda w: ltl4(f, w))
    pr = g["printed"]
    assert len(leaves) == pr["value_vectors"]
    assert sum(nodes[()][0]) == pr["root_children"]
    assert nodes[("Adam",)][0][TOP] == pr["adam_true_children"]
    assert nodes[("Adam",)][1] == BOT                          # printed F
    assert nodes[("Jack",)][1] == TOP_C                        # printed T; see the fixture's reading
    assert root == BOT                                         # printed F
    assert nodes[()][0] == vec(F=1, Tc=1)


# --- Table 1 and the default A = 1 ---------------------------------------------
@pytest.mark.parametrize("l", [0, 1, 3, 5])
def test_table_one(l):
    for k in range(0, 9):
        v = vec(T=k, Fp=2)
        assert perm_sat("E", ">", l, v) == (k > l)
        assert perm_sat("E", ">=", l, v) == (k >= l)
        assert perm_viol("E", "=", l, v) == (k > l)
        assert perm_viol("E", "<", l, v) == (k >= l)
        assert perm_viol("E", "<=", l, v) == (k > l)
        for op in ("=", "<", "<="):
            assert not perm_sat("E", op, l, v)
        for op in (">", ">="):
            assert not perm_viol("E", op, l, v)


def test_default_forall_single_violation_is_permanent():
    for others in itertools.product(range(3), repeat=5):
        v = [1] + list(others)
        assert valuate("A", "=", 1, v) == BOT
        assert valuate("A", ">=", 1, v) == BOT


def test_default_forall_equals_at_least_one():
    # k <= N, so A=1 and A>=1 agree everywhere (reading A14)
    for v in itertools.product(range(3), repeat=6):
        assert valuate("A", "=", 1, list(v)) == valuate("A", ">=", 1, list(v))


# --- informal readings of Section 2.3 ------------------------------------------
def test_phi1_currently_true_and_false():
    # phi_1 = A>=50% f: opened(f) U close(f): closed files are permanently T
    assert valuate("A", ">=", Fraction(1, 2), vec(T=3, Fp=2)) == TOP_C
    assert valuate("A", ">=", Fraction(1, 2), vec(T=2, F=3)) == BOT_C


def test_phi2_never_currently_true():
    # phi_2 = A>=50% f: G(opened U close): leaves are only Tp / Fp (and at
    # least one file is in the trace)
    for tp in range(0, 8):
        for fp in range(0, 8):
            if tp + fp == 0:
                continue
            v = vec(Tp=tp, Fp=fp)
            r = valuate("A", ">=", Fraction(1, 2), v)
            assert r != TOP_C
            assert r == (TOP_P if 2 * tp >= tp + fp else BOT_P)


def test_no_children():
    # reading A11: the cascade with all counts zero
    assert valuate("A", ">=", Fraction(19, 20), [0] * 6) == TOP_C
    assert valuate("E", ">=", 500, [0] * 6) == BOT_C
    assert valuate("E", "<=", 3, [0] * 6) == TOP_C
    assert valuate("E", "=", 0, [0] * 6) == TOP_C


# --- closed forms of permanence against an enumeration of extensions -------------
def extensions(kind, const, v, extra):
    """All (k_sat, n) reachable from v by deciding the undecided children and
    adding up to `extra` new children (the extension model of reading A5)."""
    top, bot = v[TOP], v[BOT]
    undecided = sum(v) - top - bot
    for u_sat in range(undecided + 1):
        for m in range(extra + 1):
            for m_sat in range(m + 1):
                yield top + u_sat + m_sat, sum(v) + m


@pytest.mark.parametrize("kind,consts", [("A", PCT), ("E", CNT)])
def test_permanence_closed_forms_match_enumeration(kind, consts):
    extra = 60
    for const in consts:
        for op in OPS:
            for v in itertools.product(range(3), repeat=6):
                v = list(v)
                if sum(v) > 4:
                    continue
                ext = list(extensions(kind, const, v, extra))
                # permanently satisfied: every extension meets the constraint
                assert perm_sat(kind, op, const, v) == all(constraint(kind, op, const, k, n) for k, n in ext), \
                    (kind, op, const, v)
                # permanently violated: no extension meets it
                assert perm_viol(kind, op, const, v) == (not any(constraint(kind, op, const, k, n) for k, n in ext)), \
                    (kind, op, const, v)


# --- monotonicity over real trace extensions --------------------------------------
@pytest.mark.parametrize("quants", [
    [("A", "=", 1), ("E", "<=", 1)], [("E", ">=", 1), ("A", ">=", Fraction(1, 2))],
    [("E", "=", 1), ("E", ">", 0)], [("A", "<", Fraction(1, 2)), ("A", ">", 0)]])
def test_conclusive_root_verdicts_survive_extensions(quants):
    f = parse("a U b")
    letters = [frozenset(), frozenset("a"), frozenset("b")]
    keys = [(0, 0), (0, 1), (1, 0)]
    evs = [(lt, k) for lt in letters for k in keys]
    leaf = lambda w: ltl4(f, w)
    for n in range(1, 4):
        for trace in itertools.product(evs, repeat=n):
            r, _, _ = evaluate(list(trace), quants, leaf)
            if r in (TOP, BOT):
                for e in evs:
                    r2, _, _ = evaluate(list(trace) + [e], quants, leaf)
                    assert r2 == r, (trace, e, r, r2)


# --- the C restatement agrees with the Python oracle -------------------------------
def test_c_valuate_matches_python():
    for kind, consts in (("A", PCT), ("E", CNT + [7])):
        for const in consts:
            for op in OPS:
                for v in itertools.product(range(3), repeat=6):
                    assert cref.valuate(kind, op, const, list(v)) == valuate(kind, op, const, list(v))


def test_c_pipeline_matches_python():
    from oracle.run import oracle_monitor
    rng = np.random.default_rng(1234)
    formulas = ["G(a -> F b)", "a U b", "G(a -> X b)", "F(a & X F a)", "!X a", "G a | (b U c)"]
    for trial in range(12):
        n_levels = int(rng.integers(1, 4))
        n = int(rng.integers(1, 60))
        keys = rng.integers(0, 3, size=(n, n_levels))
        typ = rng.integers(0, 8, size=n)
        rec = np.zeros((n, 4 + n_levels), dtype=np.uint32)
        rec[:, 1] = typ
        rec[:, 4:] = keys
        class_props = [frozenset("abc"[i] for i in range(3) if (c >> i) & 1) for c in range(8)]
        specs = []
        for p in range(2):
            f = formulas[int(rng.integers(0, len(formulas)))]
            q = []
            for _ in range(n_levels):
                kind = "A" if rng.random() < 0.5 else "E"
                op = OPS[int(rng.integers(0, 5))]
                const = Fraction(int(rng.integers(0, 4)), 3) if kind == "A" else int(rng.integers(0, 3))
                q.append((kind, op, const))
            specs.append((f, q))
        props = []
        for f, q in specs:
            m = oracle_monitor(f)
            props.append(cref.OracleProperty(np.array(m.class_table(class_props), dtype=np.uint32),
                                             np.array(m.label, dtype=np.uint8), m.q0, q))
        cot = np.zeros(256, dtype=np.uint8)
        cot[:8] = np.arange(8)
        kp = np.zeros(256, dtype=np.uint8)
        kp[:8] = (1 << n_levels) - 1
        res = cref.evaluate_records(rec.view(np.uint8).reshape(-1), 4 * (4 + n_levels), 4, 4,
                                    [16 + 4 * m for m in range(n_levels)], [4] * n_levels, cot, kp, props)
        for p, (f, q) in enumerate(specs):
            ff = parse(f)
            events = [(class_props[int(typ[i])], tuple(int(x) for x in keys[i])) for i in range(n)]
            root, nodes, leaves = evaluate(events, q, lambda w: ltl4(ff, w))
            assert res.root_verdict[p] == root
            assert list(res.root_counts[p]) == nodes[()][0]
            for i, d in enumerate(sorted(leaves)):
                assert tuple(res.inst_keys[i]) == d
                assert res.inst_verdict[p, i] == leaves[d]
            for m in range(1, n_levels):
                for j, pre in enumerate(sorted(k for k in nodes if len(k) == m)):
                    assert tuple(res.level_keys[m][j]) == pre
                    assert list(res.level_counts[m][p, j]) == nodes[pre][0]
                    assert res.level_verdict[m][p, j] == nodes[pre][1]


def _pred_true(op, x, v):
    return [x < v, x <= v, x > v, x >= v, x == v, x != v][op]


@pytest.mark.parametrize("seed", range(40))
def test_c_pipeline_matches_python_levels_exclusions_predicates(seed):
    """The C restatement against the Python oracle with 1-4 quantifier levels,
    events that join no cluster (a type >= 256, or a type that lacks some
    level's key), and 0-2 data predicates that add letter bits.  The Python
    side takes each event's letter and key vector directly from the record
    fields, with the exclusion rule and the comparisons written out here."""
    from oracle.run import oracle_monitor
    rng = np.random.default_rng(0xC0DE + seed)
    n_levels = 1 + seed % 4
    n = int(rng.integers(1, 90))
    n_preds = int(rng.integers(0, 3))
    # record: ts, type, data, k0..k{n-1}
    rec = np.zeros((n, 3 + n_levels), dtype=np.uint32)
    typ = rng.integers(0, 6, size=n).astype(np.uint32)
    big = rng.random(n) < 0.1
    typ[big] = rng.choice([256, 300, 1 << 20, 0xFFFFFFFF], size=int(big.sum()))
    rec[:, 1] = typ
    rec[:, 2] = rng.integers(0, 10, size=n)
    rec[:, 3:] = rng.integers(0, 3, size=(n, n_levels))
    # types 0..3 carry propositions a, b by their bits; types 4, 5 reuse letters
    cot = np.zeros(256, dtype=np.uint8)
    cot[:6] = [0, 1, 2, 3, 1, 0]
    full = (1 << n_levels) - 1
    kp = np.zeros(256, dtype=np.uint8)
    kp[:6] = full
    kp[4] = full & ~(1 << int(rng.integers(0, n_levels)))   # type 4 lacks one level's key
    kp[5] = int(rng.integers(0, full + 1))                     # type 5: a random key set
    pred_shift = 2
    preds = [(8, 4, int(rng.integers(0, 6)), int(rng.integers(0, 10))) for _ in range(n_preds)]
    names = ["a", "b", "c", "d"]
    n_cls = 1 << (2 + n_preds)
    class_props = [frozenset(names[i] for i in range(4) if (c >> i) & 1) for c in range(n_cls)]
    pool = ["G(a -> F b)", "a U b", "G(a -> X b)", "F(a & X F a)", "!X a", "G a | (b U c)", "F c & G(b -> F a)",
            "G(c -> X d)", "(a U c) | G d"]
    allowed = set(names[:2 + n_preds])
    pool = [f for f in pool if set(props(parse(f))) <= allowed]
    specs = []
    for p in range(3):
        f = pool[int(rng.integers(0, len(pool)))]
        q = []
        for _ in range(n_levels):
            kind = "A" if rng.random() < 0.5 else "E"
            op = OPS[int(rng.integers(0, 5))]
            const = Fraction(int(rng.integers(0, 4)), 3) if kind == "A" else int(rng.integers(0, 3))
            q.append((kind, op, const))
        specs.append((f, q))
    oprops = []
    for f, q in specs:
        m = oracle_monitor(f)
        oprops.append(cref.OracleProperty(np.array(m.class_table(class_props), dtype=np.uint32),
                                          np.array(m.label, dtype=np.uint8), m.q0, q))
    res = cref.evaluate_records(rec.view(np.uint8).reshape(-1), 4 * (3 + n_levels), 4, 4,
                                [12 + 4 * m for m in range(n_levels)], [4] * n_levels, cot, kp, oprops,
                                preds=preds, pred_shift=pred_shift)
    events = []
    for i in range(n):
        t = int(typ[i])
        key = None
        if t < 256 and all((int(kp[t]) >> m) & 1 for m in range(n_levels)):
            key = tuple(int(x) for x in rec[i, 3:])
        cls = int(cot[t]) if t < 256 else 0
        for qi, (_, _, op, v) in enumerate(preds):
            if _pred_true(op, int(rec[i, 2]), v):
                cls += 1 << (pred_shift + qi)
        events.append((class_props[cls], key))
    for p, (f, q) in enumerate(specs):
        ff = parse(f)
        root, nodes, leaves = evaluate(events, q, lambda w: ltl4(ff, w))
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
