"""Pins of the oracle's data predicates (propositions computed from a record
field, Section 5's cloud-storage case study) against its plain type letters,
which the other oracle tests pin: a predicate that always holds must act as a
fixed shift of every letter, a predicate on the type field must reproduce the
proposition the type table gives, and each comparison must split a range of
field values where the comparison with a constant does."""
import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import workloads as W


def _base(n=20_000, users=200, seed=3):
    return W.gen_chunk_uploads(n, users, n_preds=1, seed=seed)


def _same(a, b):
    assert np.array_equal(a.root_verdict, b.root_verdict)
    assert np.array_equal(a.root_counts, b.root_counts)
    assert np.array_equal(a.inst_keys, b.inst_keys)
    assert np.array_equal(a.inst_verdict, b.inst_verdict)


def test_always_true_predicate_is_a_letter_shift():
    wl = _base()
    lay = wl.layout
    # avg_chunk >= 0 holds for every record: every event takes the letter
    # of its type plus 2, the same as a type table shifted by 2
    lay.preds = [(12, 4, 3, 0)]
    with_pred = evaluate_workload(wl)
    lay.preds = []
    lay.class_of_type = lay.class_of_type.copy()
    lay.class_of_type[:2] += 2
    shifted = evaluate_workload(wl)
    _same(with_pred, shifted)


def test_predicate_on_the_type_field_reproduces_the_type_letter():
    wl = _base(seed=4)
    lay = wl.layout
    plain = evaluate_workload(wl)
    # 'upload' read off the type field by a predicate (type == 0), the type
    # table folding both types into one letter
    lay.preds = [(4, 4, 4, 0), (12, 4, 0, W.CHUNK_MAX)]
    lay.class_of_type = np.zeros(256, dtype=np.uint8)
    lay.pred_shift = 0
    lay.class_props = [{n for n, bit in (("upload", 1), ("small", 2)) if c & bit} for c in range(4)]
    _same(evaluate_workload(wl), plain)


@pytest.mark.parametrize("op,holds", [(0, lambda x: x < 5), (1, lambda x: x <= 5), (2, lambda x: x > 5),
                                      (3, lambda x: x >= 5), (4, lambda x: x == 5), (5, lambda x: x != 5)])
def test_each_comparison_splits_the_values(op, holds):
    # one event per user, field values 0..9: 'F small' is T (5) exactly where
    # the predicate holds; where it fails the one-event word leaves F
    # unsettled, Bp (2)
    n = 10
    rec = np.zeros(n, dtype=W.REC16)
    rec["k0"] = np.arange(n, dtype=np.uint32)
    rec["k1"] = np.arange(n, dtype=np.uint32)
    lay = W.chunk_upload_layout(1, 4)
    lay.preds = [(12, 4, op, 5)]
    wl = W.Workload("cmp", rec, lay, [W.PropertySpec("F small", [("E", ">=", 1)], "cmp")])
    o = evaluate_workload(wl)
    want = np.array([5 if holds(x) else 2 for x in range(n)], dtype=np.uint8)
    assert np.array_equal(o.inst_verdict[0], want)
