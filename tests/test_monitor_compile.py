"""The product's monitor compiler against the oracle: the compiled table must
give the oracle's LTL4 verdict (Def. 5) on every word, and be minimal."""
import itertools

import numpy as np
import pytest

from oracle.ltl import ltl4, parse
from paper_1411_2239_amd.monitor import compile_letters, compile_monitor

from _util import FORMULA_POOL, random_formula


def _check_letters(text, max_len):
    nd, nl, q0, letters = compile_letters(text)
    f = parse(text)
    for n in range(1, max_len + 1):
        for w in itertools.product(range(len(letters)), repeat=n):
            q = q0
            for c in w:
                q = nd[q][c]
            assert nl[q] == ltl4(f, [letters[c] for c in w]), (text, w)
    return nd, nl


def _minimal(nd, nl):
    # no two states have the same label and the same successor blocks after refinement
    n, k = len(nd), len(nd[0])
    block = list(nl)
    while True:
        sig = [(block[q],) + tuple(block[nd[q][c]] for c in range(k)) for q in range(n)]
        ids = {}
        nb = [ids.setdefault(s, len(ids)) for s in sig]
        if len(set(nb)) == len(set(block)):
            return len(set(nb)) == n
        block = nb


@pytest.mark.parametrize("text", FORMULA_POOL)
def test_pool_formulas_match_oracle(text):
    nd, nl = _check_letters(text, 5 if "c" not in text else 3)
    assert _minimal(nd, nl)


def test_random_formulas_match_oracle():
    rng = np.random.default_rng(2239)
    for _ in range(40):
        text = random_formula(rng, depth=3)
        nd, nl = _check_letters(text, 3)
        assert _minimal(nd, nl), text


@pytest.mark.parametrize("text,states", [("G(a -> F b)", 2), ("(G a) -> (F b)", 2), ("G(a -> X b)", 3),
                                         ("F(a & X F a)", 3), ("F(a & X(F(a & X F a)))", 4)])
def test_expected_sizes(text, states):
    nd, _, _, _ = compile_letters(text)
    assert len(nd) == states


def test_class_expansion_and_minimisation():
    # sockets: 4 event types, two of which carry no proposition
    classes = [set(), {"receive"}, {"respond"}, set()]
    m = compile_monitor("G(receive -> F respond)", classes)
    assert m.n_classes == 4 and m.n_states == 2
    f = parse("G(receive -> F respond)")
    for n in range(1, 6):
        for w in itertools.product(range(4), repeat=n):
            assert m.run(w) == ltl4(f, [frozenset(classes[c]) for c in w])


def test_too_many_states_rejected():
    text = "X " * 16 + "a"          # must remember 16 positions: more than 16 states
    with pytest.raises(ValueError):
        compile_monitor(text, [set(), {"a"}])


def test_sixteen_states_accepted():
    text = "X " * 13 + "a"
    m = compile_monitor(text, [set(), {"a"}])
    assert m.n_states <= 16
