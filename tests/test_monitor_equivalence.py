"""Exact checks of the two monitor constructions used for every workload body.

* The product's compiler (formula progression with BDD residuals, then Moore
  minimisation) and the oracle's monitor (the reachable atom sets of a
  Lichtenstein-Pnueli tableau) are built by different techniques.  A
  breadth-first walk over their product automaton visits every pair of states
  that one word reaches in both machines; equal labels on every reachable pair
  means equal LTL4 verdicts (Def. 5/6) on every word of every length.

* The oracle's monitor against Def. 5 itself, on every word up to length 8
  over two propositions (7 over three): the LTL4 verdict of a word is T when no
  extension violates the formula, F when none satisfies it, else Tp or Fp by
  the FLTL value of the word (Def. 4).  The FLTL value is computed here for
  all words of one length at once by the backward recursion of the until
  (phi U psi holds at i iff psi holds at i, or phi holds at i and the until
  holds at i+1 < n), which differs from the oracle's direct "some k, all l < k"
  form and is checked against it on a sample.  The extension questions are
  the tableau's reachable atom sets, advanced one letter at a time.
"""
from __future__ import annotations

import itertools
import os
from collections import deque

import numpy as np
import pytest

from oracle.ltl import BOT, BOT_P, TOP, TOP_P, OracleMonitor, fltl, parse, props, tableau
from paper_1411_2239_amd import workloads as W
from paper_1411_2239_amd.monitor import compile_letters, compile_monitor

from _util import FORMULA_POOL, random_formula


def workload_bodies():
    specs = (W.socket_properties() + W.user_request_properties() + W.chunk_upload_properties(3)
             + W.timeline_properties() + list(W.LARGE_PROPERTIES) + W.batch_properties(16))
    seen = []
    for s in specs:
        if s.formula not in seen:
            seen.append(s.formula)
    return seen


BODIES = workload_bodies()


# --- product automaton ----------------------------------------------------------------
def _product_mismatch(d1, l1, q1, d2, l2, q2, n_letters):
    """Breadth-first walk over the pairs reachable from (q1, q2); returns a word
    on which the labels differ, or None."""
    start = (q1, q2)
    prev = {start: None}
    todo = deque([start])
    while todo:
        s = todo.popleft()
        a, b = s
        if l1[a] != l2[b]:
            word = []
            while prev[s] is not None:
                s, c = prev[s]
                word.append(c)
            return word[::-1]
        for c in range(n_letters):
            t = (d1[a][c], d2[b][c])
            if t not in prev:
                prev[t] = (s, c)
                todo.append(t)
    return None


def _letters_product(text):
    nd, nl, q0, letters = compile_letters(text)
    om = OracleMonitor(parse(text))
    # the oracle's table over the compiler's letter order
    col = [om.letter_index(lt) for lt in letters]
    od = [[row[j] for j in col] for row in om.delta]
    return _product_mismatch(nd, nl, q0, od, om.label, om.q0, len(letters)), letters


@pytest.mark.parametrize("text", BODIES)
def test_workload_bodies_compiled_equals_oracle_monitor(text):
    bad, letters = _letters_product(text)
    assert bad is None, (text, [sorted(letters[c]) for c in bad])


@pytest.mark.parametrize("text", FORMULA_POOL)
def test_pool_compiled_equals_oracle_monitor(text):
    bad, letters = _letters_product(text)
    assert bad is None, (text, [sorted(letters[c]) for c in bad])


def test_random_formulas_compiled_equals_oracle_monitor():
    rng = np.random.default_rng(0x1411)
    for _ in range(60):
        text = random_formula(rng, depth=4)
        bad, letters = _letters_product(text)
        assert bad is None, (text, [sorted(letters[c]) for c in bad])


@pytest.mark.parametrize("maker", [W.socket_layout, W.user_request_layout, lambda: W.chunk_upload_layout(3),
                                   lambda: W.prop_layout(3)])
def test_class_tables_equal(maker):
    """The class-indexed tables the library is given (compiled and minimised
    over the layout's event classes) against the oracle's table expanded to the
    same classes."""
    lay = maker()
    classes = [set(c) for c in lay.class_props]
    used = set().union(*classes)
    for text in BODIES:
        if not set(props(parse(text))) <= used:
            continue
        m = compile_monitor(text, classes)
        om = OracleMonitor(parse(text))
        od = om.class_table([frozenset(c) for c in classes])
        bad = _product_mismatch(m.delta.tolist(), m.label.tolist(), m.q0, od, om.label, om.q0, len(classes))
        assert bad is None, (text, bad)


@pytest.mark.parametrize("text,states", [("G(a -> X b)", 3), ("G((X(X(c))) U (G(G(b))))", 8),
                                         ("(!(G(a) | c)) U (X(X(b)))", 16)])
def test_large_trace_monitor_sizes(text, states):
    m = compile_monitor(text, [{p for i, p in enumerate("abc") if (c >> i) & 1} for c in range(8)])
    assert m.n_states == states


# --- the oracle's monitor against Def. 5 on every short word ---------------------------------
def _fltl_all(f, words, letters):
    """[w |=F f] (Def. 4) for every row w of `words` (letter indices, all of one length)."""
    n, L = words.shape
    memo = {}

    def val(g):
        if g in memo:
            return memo[g]
        op = g[0]
        if op == "true":
            r = np.ones((n, L), dtype=bool)
        elif op == "ap":
            has = np.array([g[1] in lt for lt in letters], dtype=bool)
            r = has[words]
        elif op == "not":
            r = ~val(g[1])
        elif op == "and":
            r = val(g[1]) & val(g[2])
        elif op == "X":
            r = np.zeros((n, L), dtype=bool)
            r[:, :-1] = val(g[1])[:, 1:]
        elif op == "U":
            a, b = val(g[1]), val(g[2])
            r = np.empty((n, L), dtype=bool)
            r[:, L - 1] = b[:, L - 1]
            for i in range(L - 2, -1, -1):
                r[:, i] = b[:, i] | (a[:, i] & r[:, i + 1])
        else:
            raise ValueError(op)
        memo[g] = r
        return r

    return val(f)[:, 0]


class _Extensions:
    """Def. 5's extension questions through the tableau: the atoms reachable
    at the last position with f true (resp. false) at position 0; an extension
    satisfying (violating) f exists iff one of them is 'good'."""

    def __init__(self, f, letters):
        self.t = tableau(f)
        self.f = f
        t = self.t
        self.lt = [frozenset(p for p in lt if p in t.aps) for lt in letters]
        self.sets = {}
        self.keys = []
        self.step_memo = {}
        self.first = np.array([[self._id(frozenset(j for j, a in enumerate(t.atoms)
                                                   if a[f] == pol and t.letter[j] == lt)) for lt in self.lt]
                               for pol in (True, False)], dtype=np.int64)

    def _id(self, s):
        i = self.sets.get(s)
        if i is None:
            i = len(self.keys)
            self.sets[s] = i
            self.keys.append(s)
        return i

    def step(self, ids, letter_idx):
        pairs = ids * len(self.lt) + letter_idx
        uniq, inv = np.unique(pairs, return_inverse=True)
        out = np.empty(len(uniq), dtype=np.int64)
        for k, p in enumerate(uniq):
            p = int(p)
            r = self.step_memo.get(p)
            if r is None:
                s, c = self.keys[p // len(self.lt)], self.lt[p % len(self.lt)]
                r = self._id(frozenset(w for v in s for w in self.t.succ[v] if self.t.letter[w] == c))
                self.step_memo[p] = r
            out[k] = r
        return out[inv]

    def good(self, ids):
        g = np.array([any(self.t.good[j] for j in s) for s in self.keys], dtype=bool)
        return g[ids]


def _all_words(k, L, chunk_first=None):
    w = np.array(list(itertools.product(range(k), repeat=L - (chunk_first is not None))), dtype=np.int64)
    if chunk_first is None:
        return w.reshape(-1, L)
    return np.concatenate([np.full((w.shape[0], 1), chunk_first), w.reshape(w.shape[0], -1)], axis=1)


def _check_definition(text, max_len):
    f = parse(text)
    om = OracleMonitor(f)
    letters = om.letters
    k = len(letters)
    ext = _Extensions(f, letters)
    od = np.array(om.delta, dtype=np.int64)
    lab = np.array(om.label, dtype=np.int64)
    checked = 0
    rng = np.random.default_rng(7)
    for L in range(1, max_len + 1):
        for first in (range(k) if L >= 7 else [None]):
            words = _all_words(k, L, first)
            # the monitor, one letter at a time (Def. 6)
            q = np.full(words.shape[0], om.q0, dtype=np.int64)
            for i in range(L):
                q = od[q, words[:, i]]
            got = lab[q]
            # Def. 5
            pos = ext.first[0][words[:, 0]]
            neg = ext.first[1][words[:, 0]]
            for i in range(1, L):
                pos = ext.step(pos, words[:, i])
                neg = ext.step(neg, words[:, i])
            can_sat, can_viol = ext.good(pos), ext.good(neg)
            fv = _fltl_all(f, words, letters)
            want = np.where(~can_viol, TOP, np.where(~can_sat, BOT, np.where(fv, TOP_P, BOT_P)))
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (text, [sorted(letters[c]) for c in words[bad[0]]], got[bad[0]], want[bad[0]])
            # the vectorised FLTL against the oracle's direct form, on a sample
            for j in rng.choice(words.shape[0], size=min(20, words.shape[0]), replace=False):
                assert fv[j] == fltl(f, [letters[c] for c in words[j]])
            checked += words.shape[0]
    return checked


def _max_len(text):
    n_props = len(props(parse(text)))
    if n_props <= 2:
        return 8
    return int(os.environ.get("LTL4C_WORDS3", "7"))


@pytest.mark.parametrize("text", BODIES)
def test_oracle_monitor_matches_definition_on_all_short_words(text):
    assert _check_definition(text, _max_len(text)) > 0


@pytest.mark.parametrize("text", ["G(a -> F b)", "G a | (b U c)", "X X X a", "(a U b) & (!a U c)",
                                  "G(a -> (b U c))", "F c & G(b -> F a)"])
def test_pool_oracle_monitor_matches_definition(text):
    assert _check_definition(text, _max_len(text)) > 0
