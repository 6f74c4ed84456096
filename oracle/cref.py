"""ctypes wrapper and build step for the plain C oracle (oracle/c/ltl4c_oracle.c).

TEST INFRASTRUCTURE ONLY (see the header of oracle/ltl.py).  The product
library never loads this.

`build()` compiles the C file with gcc into oracle/c/libltl4c_oracle.so.
`evaluate_records()` runs it on a numpy record array and returns plain numpy
arrays: per-instance keys and verdicts, per-level node keys, counts and
verdicts, all in lexicographic order of the value vectors.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "ltl4c_oracle.c")
LIB = os.path.join(HERE, "c", "libltl4c_oracle.so")

KIND = {"A": 0, "E": 1}
NEVER = 0xFFFFFFFF   # inst_conc: no prefix of the instance has a T or F verdict
OPCODE = {"<": 0, "<=": 1, ">": 2, ">=": 3, "=": 4}


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", LIB, SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


class _Layout(C.Structure):
    _fields_ = [("record_bytes", C.c_uint32), ("type_offset", C.c_uint32), ("type_bytes", C.c_uint32),
                ("n_keys", C.c_uint32), ("key_offset", C.c_uint32 * 4), ("key_bytes", C.c_uint32 * 4),
                ("class_of_type", C.POINTER(C.c_uint8)), ("key_present", C.POINTER(C.c_uint8)),
                ("n_preds", C.c_uint32), ("pred_shift", C.c_uint32),
                ("pred_offset", C.c_uint32 * 3), ("pred_bytes", C.c_uint32 * 3),
                ("pred_op", C.c_uint32 * 3), ("pred_value", C.c_uint32 * 3),
                ("parent_events", C.c_uint32)]


class _Prop(C.Structure):
    _fields_ = [("n_states", C.c_uint32), ("n_classes", C.c_uint32), ("q0", C.c_uint32), ("pad", C.c_uint32),
                ("delta", C.POINTER(C.c_uint32)), ("label", C.POINTER(C.c_uint8)),
                ("kind", C.c_uint8 * 4), ("op", C.c_uint8 * 4),
                ("num", C.c_uint64 * 4), ("den", C.c_uint64 * 4)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB)
        lib.ora_eval.restype = C.c_void_p
        lib.ora_eval.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(_Layout), C.POINTER(_Prop), C.c_int]
        lib.ora_free.argtypes = [C.c_void_p]
        lib.ora_n_inst.restype = C.c_uint64
        lib.ora_n_inst.argtypes = [C.c_void_p]
        lib.ora_level_nodes.restype = C.c_uint64
        lib.ora_level_nodes.argtypes = [C.c_void_p, C.c_int]
        for name, ty in (("ora_inst_keys", C.c_uint32), ("ora_inst_verdict", C.c_uint8), ("ora_inst_conc", C.c_uint32),
                         ("ora_event_verdict", C.c_uint8)):
            getattr(lib, name).restype = C.POINTER(ty)
            getattr(lib, name).argtypes = [C.c_void_p]
        for name, ty in (("ora_level_keys", C.c_uint32), ("ora_level_counts", C.c_uint64),
                         ("ora_level_verdict", C.c_uint8)):
            getattr(lib, name).restype = C.POINTER(ty)
            getattr(lib, name).argtypes = [C.c_void_p, C.c_int]
        lib.ora_valuate.restype = C.c_uint8
        lib.ora_valuate.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_uint64, C.POINTER(C.c_uint64)]
        _lib = lib
    return _lib


def valuate(kind, op, const, v):
    """The C restatement of Def. 7, for cross-checking against oracle.counting."""
    fr = Fraction(const)
    arr = (C.c_uint64 * 6)(*v)
    return _load().ora_valuate(KIND[kind], OPCODE[op], fr.numerator, fr.denominator, arr)


@dataclass
class OracleProperty:
    """One property for the C oracle: a monitor table over event classes and
    the quantifier string Q_0..Q_{n-1} as (kind, op, const) triples."""
    delta: np.ndarray        # [n_states, n_classes] state indices
    label: np.ndarray        # [n_states] verdict codes
    q0: int
    quants: list


@dataclass
class OracleResult:
    inst_keys: np.ndarray        # [n_inst, n_levels] uint32
    inst_verdict: np.ndarray     # [n_props, n_inst] uint8
    level_keys: list             # level m: [nodes, m] uint32
    level_counts: list           # level m: [n_props, nodes, 6] uint64
    level_verdict: list          # level m: [n_props, nodes] uint8
    inst_conc: np.ndarray = None # [n_props, n_inst] uint32: prefix length at the first T/F verdict, or NEVER
    event_verdict: np.ndarray = None  # [n_props, n_events] uint8, trace order; 0xFF: the event joins no cluster

    @property
    def root_verdict(self):
        return self.level_verdict[0][:, 0]

    @property
    def root_counts(self):
        return self.level_counts[0][:, 0, :]


def evaluate_records(records, record_bytes, type_offset, type_bytes, key_offsets, key_bytes,
                     class_of_type, key_present, props, preds=(), pred_shift=0, parent_events=False):
    """Run the C oracle.  `records` is a uint8 buffer of n * record_bytes bytes.
    preds: data predicates (offset, bytes, op, value), op 0..5 = < <= > >= == !=.
    parent_events: an event whose type carries every key but the innermost
    joins the cluster of every instance under its parent (see the C file)."""
    lib = _load()
    buf = np.ascontiguousarray(records).view(np.uint8).reshape(-1)
    n = buf.size // record_bytes
    cot = np.ascontiguousarray(class_of_type, dtype=np.uint8)
    kp = np.ascontiguousarray(key_present, dtype=np.uint8)
    assert cot.size == 256 and kp.size == 256
    nk = len(key_offsets)
    lay = _Layout(record_bytes, type_offset, type_bytes, nk,
                  (C.c_uint32 * 4)(*list(key_offsets) + [0] * (4 - nk)),
                  (C.c_uint32 * 4)(*list(key_bytes) + [0] * (4 - nk)),
                  cot.ctypes.data_as(C.POINTER(C.c_uint8)), kp.ctypes.data_as(C.POINTER(C.c_uint8)))
    if len(preds) > 3:
        raise ValueError("at most 3 data predicates")
    lay.parent_events = 1 if parent_events else 0
    lay.n_preds = len(preds)
    lay.pred_shift = pred_shift
    for q, (off, nb, op, val) in enumerate(preds):
        lay.pred_offset[q], lay.pred_bytes[q], lay.pred_op[q], lay.pred_value[q] = off, nb, op, val
    keep = []
    arr = (_Prop * len(props))()
    for i, p in enumerate(props):
        d = np.ascontiguousarray(p.delta, dtype=np.uint32)
        lab = np.ascontiguousarray(p.label, dtype=np.uint8)
        keep += [d, lab]
        if len(p.quants) != nk:
            raise ValueError("each property needs one quantifier per key level")
        kinds, ops, nums, dens = [0] * 4, [0] * 4, [0] * 4, [1] * 4
        for m, (kind, op, const) in enumerate(p.quants):
            fr = Fraction(const)
            kinds[m], ops[m], nums[m], dens[m] = KIND[kind], OPCODE[op], fr.numerator, fr.denominator
        arr[i] = _Prop(d.shape[0], d.shape[1], p.q0, 0,
                       d.ctypes.data_as(C.POINTER(C.c_uint32)), lab.ctypes.data_as(C.POINTER(C.c_uint8)),
                       (C.c_uint8 * 4)(*kinds), (C.c_uint8 * 4)(*ops),
                       (C.c_uint64 * 4)(*nums), (C.c_uint64 * 4)(*dens))
    res = lib.ora_eval(buf.ctypes.data, n, C.byref(lay), arr, len(props))
    if not res:
        raise RuntimeError("oracle evaluation failed")
    try:
        ni = lib.ora_n_inst(res)
        P = len(props)
        ik = np.ctypeslib.as_array(lib.ora_inst_keys(res), shape=(max(ni, 1) * nk,))[:ni * nk].reshape(ni, nk).copy()
        iv = np.ctypeslib.as_array(lib.ora_inst_verdict(res), shape=(max(P * ni, 1),))[:P * ni].reshape(P, ni).copy()
        ic = np.ctypeslib.as_array(lib.ora_inst_conc(res), shape=(max(P * ni, 1),))[:P * ni].reshape(P, ni).copy()
        evv = np.ctypeslib.as_array(lib.ora_event_verdict(res), shape=(max(P * n, 1),))[:P * n].reshape(P, n).copy()
        lk, lc, lv = [], [], []
        for m in range(nk):
            nodes = lib.ora_level_nodes(res, m)
            keys = np.ctypeslib.as_array(lib.ora_level_keys(res, m), shape=(max(nodes * m, 1),))
            lk.append(keys[:nodes * m].reshape(nodes, m).copy())
            cnt = np.ctypeslib.as_array(lib.ora_level_counts(res, m), shape=(P * nodes * 6,))
            lc.append(cnt.reshape(P, nodes, 6).copy())
            ver = np.ctypeslib.as_array(lib.ora_level_verdict(res, m), shape=(P * nodes,))
            lv.append(ver.reshape(P, nodes).copy())
        return OracleResult(ik, iv, lk, lc, lv, ic, evv)
    finally:
        lib.ora_free(res)
