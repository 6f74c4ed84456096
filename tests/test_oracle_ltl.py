"""Pins of oracle/ltl.py against what the paper and the mathematics fix.

Each check is independent of the function it pins: closed forms derived by
hand, the standard semantics on ultimately periodic words, duality and the
permanence of T / F that Def. 5 implies."""
import itertools

import numpy as np
import pytest

from oracle.ltl import (BOT, BOT_P, TOP, TOP_P, OracleMonitor, fltl, ltl4, ltl_lasso, parse, tableau)

A, B, AB, E = frozenset("a"), frozenset("b"), frozenset("ab"), frozenset()
LETTERS2 = [E, A, B, AB]
LETTERS3 = [frozenset(s) for r in range(4) for s in itertools.combinations("abc", r)]


def words(letters, max_len):
    for n in range(1, max_len + 1):
        for w in itertools.product(letters, repeat=n):
            yield list(w)


# --- Def. 4 (FLTL) ---------------------------------------------------------
def test_fltl_closed_forms():
    Fa, Ga, Xa, nXa, aUb = map(parse, ["F a", "G a", "X a", "!X a", "a U b"])
    for w in words(LETTERS2, 6):
        has_a = ["a" in x for x in w]
        assert fltl(Fa, w) == any(has_a)
        assert fltl(Ga, w) == all(has_a)
        assert fltl(Xa, w) == (len(w) > 1 and has_a[1])          # strong next
        assert fltl(nXa, w) == (len(w) == 1 or not has_a[1])
        exp = any("b" in w[k] and all("a" in w[i] for i in range(k)) for k in range(len(w)))
        assert fltl(aUb, w) == exp


def test_fltl_strong_next_at_the_end():
    assert fltl(parse("X true"), [E]) is False
    assert fltl(parse("!X true"), [E]) is True
    assert fltl(parse("X true"), [E, E]) is True


# --- Def. 5 (LTL4) closed forms for the formulas the workloads use ---------
def test_ltl4_response_property():
    f = parse("G(a -> F b)")      # sockets / user requests: never conclusive
    for w in words(LETTERS2, 6):
        ok = all(any("b" in w[j] for j in range(i, len(w))) for i in range(len(w)) if "a" in w[i])
        assert ltl4(f, w) == (TOP_P if ok else BOT_P)


def test_ltl4_literal_reading_of_case_study_one():
    f = parse("(G a) -> (F b)")   # T once some event has b or lacks a
    for w in words(LETTERS2, 6):
        assert ltl4(f, w) == (TOP if any("b" in x or "a" not in x for x in w) else BOT_P)


def test_ltl4_next_property():
    f = parse("G(a -> X b)")
    for w in words(LETTERS2, 6):
        n = len(w)
        if any("a" in w[i] and "b" not in w[i + 1] for i in range(n - 1)):
            exp = BOT
        elif "a" in w[-1]:
            exp = BOT_P
        else:
            exp = TOP_P
        assert ltl4(f, w) == exp


@pytest.mark.parametrize("k", [1, 2, 3])
def test_ltl4_counting_chain(k):
    # phi_1 = F a, phi_k = F(a & X phi_{k-1}): T iff at least k events carry a
    text = "F a"
    for _ in range(k - 1):
        text = f"F(a & X({text}))"
    f = parse(text)
    for w in words([E, A], 7):
        assert ltl4(f, w) == (TOP if sum("a" in x for x in w) >= k else BOT_P)


def test_ltl4_state_formula_decides_at_first_event():
    f = parse("a & b")
    for w in words(LETTERS2, 4):
        assert ltl4(f, w) == (TOP if "a" in w[0] and "b" in w[0] else BOT)


# --- invariants ----------------------------------------------------------------
DUAL = {TOP: BOT, BOT: TOP, TOP_P: BOT_P, BOT_P: TOP_P}
FORMULAS = ["G(a -> F b)", "G a | (b U c)", "a U (b U c)", "X X a", "G F a", "F G a", "G(a -> X X b)",
            "(a U b) & (!a U c)", "F(a & X F a)", "!X a", "X !a", "G(a -> (b U c))"]


@pytest.mark.parametrize("text", FORMULAS)
def test_duality(text):
    f, nf = parse(text), parse(f"!({text})")
    for w in words(LETTERS3, 3):
        assert ltl4(nf, w) == DUAL[ltl4(f, w)]


@pytest.mark.parametrize("text", FORMULAS)
def test_conclusive_verdicts_are_permanent(text):
    f = parse(text)
    for w in words(LETTERS3, 3):
        v = ltl4(f, w)
        if v in (TOP, BOT):
            for x in LETTERS3:
                assert ltl4(f, w + [x]) == v


def _lassos(letters, max_len):
    for n in range(1, max_len + 1):
        for split in range(n):
            for seq in itertools.product(letters, repeat=n):
                yield list(seq[:split]), list(seq[split:])


@pytest.mark.parametrize("text", ["G(a -> F b)", "G a | (b U c)", "X X a", "G F a", "F G a",
                                  "(a U b) & (!a U c)", "G(a -> X b)"])
def test_tableau_answers_have_lasso_witnesses(text):
    """Whenever Def. 5 says an extension exists (for f or for !f), a short
    ultimately periodic extension exists, checked by the lasso semantics."""
    f = parse(text)
    letters = LETTERS3 if "c" in text else LETTERS2
    cands = list(_lassos(letters, 3))
    for w in words(letters, 2):
        v = ltl4(f, w)
        sat_ext = any(ltl_lasso(f, w + x, y) for x, y in cands)
        viol_ext = any(not ltl_lasso(f, w + x, y) for x, y in cands)
        assert sat_ext == (v != BOT)
        assert viol_ext == (v != TOP)


def test_unsatisfiable_and_valid():
    assert not tableau(parse("G a & F !a")).satisfiable()
    assert tableau(parse("G a | F !a")).valid()
    assert tableau(parse("G F a")).satisfiable() and not tableau(parse("G F a")).valid()


# --- Def. 6: the oracle's monitor reproduces Def. 5 word by word -------------
@pytest.mark.parametrize("text", FORMULAS + ["G(a -> F b)"])
def test_oracle_monitor_matches_definition(text):
    f = parse(text)
    m = OracleMonitor(f)
    letters = LETTERS3 if "c" in text else LETTERS2
    for w in words(letters, 4 if "c" in text else 6):
        assert m.run(w) == ltl4(f, w)


def test_figure_one_formula_trap_states():
    # Fig. 1's formula: its monitor has absorbing T and F states (Section 2.2.3)
    m = OracleMonitor(parse("G a | (b U c)"))
    for q, lab in enumerate(m.label):
        if lab in (TOP, BOT):
            for q2 in m.delta[q]:
                assert m.label[q2] == lab
    assert TOP in m.label and BOT in m.label
