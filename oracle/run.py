"""Oracle evaluation of a workload (TEST INFRASTRUCTURE ONLY).

Builds the oracle's own monitor for every property formula (oracle.ltl, from
the formula text, independent of the product's compiler), expands it to the
layout's event classes, and runs the plain C evaluator.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import cref
from .ltl import OracleMonitor, parse

_MONITORS = {}


def oracle_monitor(formula):
    m = _MONITORS.get(formula)
    if m is None:
        m = OracleMonitor(parse(formula))
        _MONITORS[formula] = m
    return m


def quants_of(spec):
    out = []
    for kind, op, const in spec.quants:
        out.append((kind, op, Fraction(str(const)) if kind == "A" else int(const)))
    return out


def oracle_property(spec, layout):
    m = oracle_monitor(spec.formula)
    table = np.array(m.class_table([frozenset(c) for c in layout.class_props]), dtype=np.uint32)
    return cref.OracleProperty(table, np.array(m.label, dtype=np.uint8), m.q0, quants_of(spec))


def evaluate_workload(wl, specs=None, records=None):
    """Run the C oracle on a workload (optionally a subset of its records)."""
    lay = wl.layout
    specs = specs if specs is not None else wl.props
    recs = wl.raw() if records is None else np.ascontiguousarray(records).view(np.uint8).reshape(-1)
    return cref.evaluate_records(recs, lay.record_bytes, lay.type_offset, lay.type_bytes,
                                 lay.key_offsets, lay.key_bytes, lay.class_of_type, lay.key_present,
                                 [oracle_property(s, lay) for s in specs],
                                 preds=lay.preds, pred_shift=lay.pred_shift,
                                 parent_events=getattr(lay, "parent_events", False))
