"""ctypes binding of the C ABI in include/ltl4c.h.

Argument marshalling only: every step of the monitoring path runs in the HIP
kernels of libltl4c.so.  Device memory and streams come from PyTorch (ROCm):
records, the workspace and the outputs are torch tensors on the context's
device, and work is enqueued on torch's current stream.

If the library has not been built, `load()` raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libltl4c.so")
# kernel schedules tuned on the GPU by bench.py --tune (ltl4c_schedule_save); a
# context loads them unless use_tuned=False, and they apply only on the
# architecture they were tuned on
SCHEDULES_PATH = os.path.join(HERE, "schedules.json")

OK, EINVAL, ENOMEM, ECAPACITY, EDEVICE, EADMIT, ESEQ, EUNSUPPORTED, ERANGE = 0, -1, -2, -3, -4, -5, -6, -7, -8
BOT, BOT_C, BOT_P, TOP_P, TOP_C, TOP = range(6)
OPT_SORT_TILE = 0
OPT_SCAN_TILE = 1
VERDICT_NAMES = ["F", "Fc", "Fp", "Tp", "Tc", "T"]
NEVER = 0xFFFFFFFF   # timeline: the instance never became conclusive
NO_INSTANCE = 0xFF   # event verdicts: the event joins no cluster
KIND = {"A": 0, "E": 1}
OP = {"<": 0, "<=": 1, ">": 2, ">=": 3, "=": 4}


class LTL4CError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class Layout(C.Structure):
    _fields_ = [("record_bytes", C.c_uint32), ("type_offset", C.c_uint32), ("type_bytes", C.c_uint32),
                ("n_keys", C.c_uint32), ("key_offset", C.c_uint32 * 4), ("key_bytes", C.c_uint32 * 4),
                ("key_bits", C.c_uint32 * 4), ("n_classes", C.c_uint32),
                ("class_of_type", C.c_uint8 * 256), ("key_present", C.c_uint8 * 256),
                ("n_preds", C.c_uint32), ("pred_shift", C.c_uint32), ("pred", C.c_uint32 * 12),
                ("parent_events", C.c_uint32)]


class MonitorDesc(C.Structure):
    _fields_ = [("n_states", C.c_uint32), ("n_classes", C.c_uint32), ("q0", C.c_uint32),
                ("delta", C.POINTER(C.c_uint8)), ("label", C.POINTER(C.c_uint8))]


class Quant(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("op", C.c_uint32), ("num", C.c_uint32), ("den", C.c_uint32)]


class PropertyDesc(C.Structure):
    _fields_ = [("monitor", C.c_int32), ("n_levels", C.c_uint32), ("q", Quant * 4)]


class Tuned(C.Structure):
    _fields_ = [("sort_tile", C.c_int32), ("scan_tile", C.c_int32), ("tuned_us", C.c_double),
                ("default_us", C.c_double), ("candidates", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("root_verdict", C.c_void_p), ("root_counts", C.c_void_p), ("sizes", C.c_void_p),
                ("capacity", C.c_uint64), ("inst_keys", C.c_void_p), ("inst_verdict", C.c_void_p),
                ("node_keys", C.c_void_p * 4), ("node_counts", C.c_void_p * 4), ("node_verdict", C.c_void_p * 4),
                ("inst_conclusive", C.c_void_p), ("event_verdict", C.c_void_p),
                ("inst_key_values", C.c_void_p), ("node_key_values", C.c_void_p * 4)]


_lib = None

# (name, restype, argtypes) for every function of include/ltl4c.h
SIGNATURES = [
    ("ltl4c_create", C.c_int32, [C.POINTER(C.c_void_p), C.c_int32]),
    ("ltl4c_destroy", C.c_int32, [C.c_void_p]),
    ("ltl4c_set_stream", C.c_int32, [C.c_void_p, C.c_void_p]),
    ("ltl4c_last_error", C.c_char_p, []),
    ("ltl4c_status_str", C.c_char_p, [C.c_int32]),
    ("ltl4c_set_layout", C.c_int32, [C.c_void_p, C.POINTER(Layout)]),
    ("ltl4c_add_monitor", C.c_int32, [C.c_void_p, C.POINTER(MonitorDesc), C.POINTER(C.c_int32)]),
    ("ltl4c_add_property", C.c_int32, [C.c_void_p, C.POINTER(PropertyDesc), C.POINTER(C.c_int32)]),
    ("ltl4c_workspace_bytes", C.c_int32,
     [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_uint64)]),
    ("ltl4c_eval", C.c_int32,
     [C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.c_int32, C.c_void_p, C.c_uint64,
      C.POINTER(Result)]),
    ("ltl4c_eval_noalloc", C.c_int32,
     [C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.c_int32, C.POINTER(Result)]),
    ("ltl4c_batch_workspace_bytes", C.c_int32, [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                                C.POINTER(C.c_uint64)]),
    ("ltl4c_eval_batch", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64), C.c_int32,
                                     C.POINTER(C.c_int32), C.c_int32, C.c_void_p, C.c_uint64, C.c_void_p,
                                     C.c_void_p]),
    ("ltl4c_wait", C.c_int32, [C.c_void_p]),
    ("ltl4c_set_memory_budget", C.c_int32, [C.c_void_p, C.c_uint64]),
    ("ltl4c_group_bytes", C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.c_uint32, C.c_uint32,
                                      C.c_uint64, C.POINTER(C.c_uint64)]),
    ("ltl4c_group_open", C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.c_uint32, C.c_uint32,
                                     C.c_uint64, C.POINTER(C.c_int32)]),
    ("ltl4c_group_close", C.c_int32, [C.c_void_p, C.c_int32]),
    ("ltl4c_group_push", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_uint64),
                                     C.POINTER(C.c_uint32), C.c_int32]),
    ("ltl4c_group_push_chunks", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_uint64),
                                            C.POINTER(C.c_uint32), C.c_int32]),
    ("ltl4c_group_read", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("ltl4c_group_read_nodes", C.c_int32, [C.c_void_p, C.c_int32, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_uint64, C.c_void_p]),
    ("ltl4c_group_open_pool", C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.c_uint32, C.c_uint64,
                                          C.c_uint64, C.POINTER(C.c_int32)]),
    ("ltl4c_stream_open", C.c_int32, [C.c_void_p, C.c_int32, C.c_uint32, C.c_uint32, C.c_uint64]),
    ("ltl4c_stream_close", C.c_int32, [C.c_void_p, C.c_int32, C.c_uint32]),
    ("ltl4c_stream_poll", C.c_int32, [C.c_void_p, C.c_int32, C.c_uint32, C.POINTER(C.c_uint64),
                                      C.POINTER(C.c_uint64)]),
    ("ltl4c_group_stalled", C.c_int32, [C.c_void_p, C.c_int32, C.c_uint64, C.POINTER(C.c_uint32), C.c_uint32,
                                        C.POINTER(C.c_uint32)]),
    ("ltl4c_group_push_seq", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_uint64),
                                         C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.c_int32, C.c_int32]),
    ("ltl4c_group_snapshot", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_uint64)]),
    ("ltl4c_group_restore", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_uint64]),
    ("ltl4c_set_option", C.c_int32, [C.c_void_p, C.c_int32, C.c_int64]),
    ("ltl4c_tune_workspace_bytes", C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64), C.c_int32,
                                               C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_uint64)]),
    ("ltl4c_tune", C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_uint64), C.c_int32,
                               C.POINTER(C.c_int32), C.c_int32, C.c_void_p, C.c_uint64, C.c_int32, C.c_void_p]),
    ("ltl4c_schedule_save", C.c_int32, [C.c_void_p, C.c_char_p]),
    ("ltl4c_schedule_load", C.c_int32, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int32)]),
    ("ltl4c_schedule_clear", C.c_int32, [C.c_void_p]),
    ("ltl4c_graph_eval", C.c_int32, [C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.c_int32,
                                     C.c_void_p, C.c_uint64, C.POINTER(Result), C.POINTER(C.c_int32)]),
    ("ltl4c_graph_eval_batch", C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64), C.c_int32,
                                           C.POINTER(C.c_int32), C.c_int32, C.c_void_p, C.c_uint64, C.c_void_p,
                                           C.c_void_p, C.POINTER(C.c_int32)]),
    ("ltl4c_graph_group_push", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_uint64),
                                           C.POINTER(C.c_uint32), C.c_int32, C.POINTER(C.c_int32)]),
    ("ltl4c_graph_launch", C.c_int32, [C.c_void_p, C.c_int32]),
    ("ltl4c_graph_destroy", C.c_int32, [C.c_void_p, C.c_int32]),
    ("ltl4c_profile_enable", C.c_int32, [C.c_void_p, C.c_int32]),
    ("ltl4c_profile_get", C.c_int32,
     [C.c_void_p, C.c_int32, C.c_char_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    ("ltl4c_profile_reset", C.c_int32, [C.c_void_p]),
]


def load(path=LIB_PATH):
    """Open libltl4c.so; raises if it has not been built.

    torch is imported first so that the library binds to the HIP runtime torch
    already loaded: one process must not hold two HIP runtimes."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401

        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback path)")
        lib = C.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status, where):
    if status != OK:
        lib = load()
        raise LTL4CError(status, where, lib.ltl4c_last_error().decode())


def quant_desc(kind, op, const):
    """('A', '>=', '19/20') or ('E', '<=', 3) -> Quant."""
    if kind == "A":
        fr = Fraction(str(const))
        if not (0 <= fr <= 1):
            raise ValueError("percentage constant must be in [0, 1]")
        if fr.denominator >= 1 << 32:
            # the ABI holds num/den in 32-bit fields; the exact constant must fit
            raise ValueError(f"percentage constant {const!r} needs a denominator below 2^32")
        return Quant(KIND[kind], OP[op], fr.numerator, fr.denominator)
    if kind != "E":
        raise ValueError(f"unknown quantifier kind {kind!r}")
    fr = Fraction(str(const))
    if fr.denominator != 1 or not (0 <= fr < 1 << 32):
        raise ValueError(f"instance-count constant {const!r} must be an integer in [0, 2^32)")
    return Quant(KIND[kind], OP[op], int(fr), 1)


def layout_desc(layout):
    """workloads.Layout -> ctypes Layout."""
    d = Layout()
    d.record_bytes = layout.record_bytes
    d.type_offset = layout.type_offset
    d.type_bytes = layout.type_bytes
    d.n_keys = layout.n_keys
    for m in range(layout.n_keys):
        d.key_offset[m] = layout.key_offsets[m]
        d.key_bytes[m] = layout.key_bytes[m]
        d.key_bits[m] = layout.key_bits[m]
    d.n_classes = layout.n_classes
    C.memmove(d.class_of_type, np.ascontiguousarray(layout.class_of_type, dtype=np.uint8).ctypes.data, 256)
    C.memmove(d.key_present, np.ascontiguousarray(layout.key_present, dtype=np.uint8).ctypes.data, 256)
    preds = getattr(layout, "preds", [])
    d.n_preds = len(preds)
    d.pred_shift = getattr(layout, "pred_shift", 0)
    for q, (off, nb, op, val) in enumerate(preds[:3]):
        d.pred[4 * q:4 * q + 4] = [off, nb, op, val]
    d.parent_events = 1 if getattr(layout, "parent_events", False) else 0
    return d


@dataclass
class EvalResult:
    """Device tensors of one evaluation (valid after Context.wait())."""
    root_verdict: object
    root_counts: object
    sizes: object
    inst_keys: object = None
    inst_verdict: object = None
    node_keys: list = None
    node_counts: list = None
    node_verdict: list = None
    inst_conclusive: object = None   # [n_props * capacity] int32 (NEVER = -1): verdict timeline
    event_verdict: object = None     # [n_props * n_events] uint8, trace order (NO_INSTANCE = 255)
    inst_key_values: object = None   # [capacity * n_levels] int32: the values of each instance's vector
    node_key_values: list = None     # level m: [capacity * m] int32


class Context:
    """One ltl4c context on a HIP device, driven from torch tensors."""

    def __init__(self, device=0, use_tuned=True):
        """use_tuned: load the committed schedule table (SCHEDULES_PATH),
        which applies only on the architecture it was tuned on."""
        import torch
        self.torch = torch
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        _check(self.lib.ltl4c_create(C.byref(h), device), "ltl4c_create")
        self.h = h
        self.n_levels = None
        self._workspace = None
        self.schedules_loaded = 0
        if use_tuned and os.path.exists(SCHEDULES_PATH):
            self.schedules_loaded = self.load_schedules(SCHEDULES_PATH)

    def close(self):
        if self.h:
            self.lib.ltl4c_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self):
        s = self.torch.cuda.current_stream(self.device).cuda_stream
        _check(self.lib.ltl4c_set_stream(self.h, C.c_void_p(s)), "ltl4c_set_stream")

    def set_layout(self, layout):
        self.n_levels = layout.n_keys
        self.key_bits = list(layout.key_bits)
        self.record_bytes = layout.record_bytes
        self.n_classes = layout.n_classes
        self.class_props = layout.class_props
        _check(self.lib.ltl4c_set_layout(self.h, C.byref(layout_desc(layout))), "ltl4c_set_layout")

    def add_monitor(self, mon):
        delta = np.ascontiguousarray(mon.delta, dtype=np.uint8)
        label = np.ascontiguousarray(mon.label, dtype=np.uint8)
        d = MonitorDesc(delta.shape[0], delta.shape[1], int(mon.q0),
                        delta.ctypes.data_as(C.POINTER(C.c_uint8)), label.ctypes.data_as(C.POINTER(C.c_uint8)))
        i = C.c_int32()
        _check(self.lib.ltl4c_add_monitor(self.h, C.byref(d), C.byref(i)), "ltl4c_add_monitor")
        return i.value

    def add_property(self, monitor_id, quants):
        p = PropertyDesc()
        p.monitor = monitor_id
        p.n_levels = len(quants)
        for m, (kind, op, const) in enumerate(quants):
            p.q[m] = quant_desc(kind, op, const)
        i = C.c_int32()
        _check(self.lib.ltl4c_add_property(self.h, C.byref(p), C.byref(i)), "ltl4c_add_property")
        return i.value

    def add_spec(self, spec):
        """Compile a workloads.PropertySpec for the current layout and register it."""
        from .monitor import compile_monitor
        mon = compile_monitor(spec.formula, self.class_props)
        return self.add_property(self.add_monitor(mon), spec.quants)

    def workspace_bytes(self, n_events, props):
        arr = (C.c_int32 * len(props))(*props)
        b = C.c_uint64()
        _check(self.lib.ltl4c_workspace_bytes(self.h, n_events, arr, len(props), C.byref(b)),
               "ltl4c_workspace_bytes")
        return b.value

    def workspace(self, n_events, props):
        need = self.workspace_bytes(n_events, props)
        ws = self._workspace
        if ws is None or ws.numel() < need:
            ws = self.torch.empty(max(need, 256), dtype=self.torch.uint8, device=f"cuda:{self.device}")
            self._workspace = ws
        return ws

    def alloc_result(self, n_props, capacity=0, instances=False, nodes=False, timeline=False, n_events=0,
                     key_values=False):
        """timeline: per-instance first conclusive prefix; n_events > 0: the
        verdict after every event (in trace order) for that many events;
        key_values: the key values of every instance and node (with
        instances / nodes)."""
        t, dev = self.torch, f"cuda:{self.device}"
        L = self.n_levels
        r = EvalResult(t.empty(n_props, dtype=t.uint8, device=dev),
                       t.empty(n_props * 6, dtype=t.int64, device=dev),
                       t.empty(1 + L, dtype=t.int64, device=dev))
        if instances:
            r.inst_keys = t.empty(capacity, dtype=t.int64, device=dev)
            r.inst_verdict = t.empty(n_props * capacity, dtype=t.uint8, device=dev)
        if timeline:
            r.inst_conclusive = t.empty(n_props * capacity, dtype=t.int32, device=dev)
        if n_events:
            r.event_verdict = t.empty(n_props * n_events, dtype=t.uint8, device=dev)
        if nodes:
            r.node_keys = [None] + [t.empty(capacity, dtype=t.int64, device=dev) for _ in range(1, L)]
            r.node_counts = [None] + [t.empty(n_props * capacity * 6, dtype=t.int32, device=dev)
                                      for _ in range(1, L)]
            r.node_verdict = [None] + [t.empty(n_props * capacity, dtype=t.uint8, device=dev)
                                       for _ in range(1, L)]
        if key_values and instances:
            r.inst_key_values = t.empty(capacity * L, dtype=t.int32, device=dev)
        if key_values and nodes:
            r.node_key_values = [None] + [t.empty(capacity * m, dtype=t.int32, device=dev) for m in range(1, L)]
        r.capacity = capacity
        r.key_bits = list(self.key_bits)
        return r

    def eval_into(self, records, n_events, props, result, workspace):
        """Enqueue one evaluation; `records` is a device tensor of n_events records."""
        self._bind_stream()
        res = self._result_desc(result)
        arr = (C.c_int32 * len(props))(*props)
        _check(self.lib.ltl4c_eval(self.h, C.c_void_p(records.data_ptr() if n_events else 0), n_events, arr,
                                   len(props), C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                   C.byref(res)), "ltl4c_eval")

    def _result_desc(self, result):
        res = Result()
        res.root_verdict = result.root_verdict.data_ptr()
        res.root_counts = result.root_counts.data_ptr()
        res.sizes = result.sizes.data_ptr()
        res.capacity = getattr(result, "capacity", 0)
        if result.inst_verdict is not None:
            res.inst_keys = result.inst_keys.data_ptr()
            res.inst_verdict = result.inst_verdict.data_ptr()
        if getattr(result, "inst_conclusive", None) is not None:
            res.inst_conclusive = result.inst_conclusive.data_ptr()
        if getattr(result, "event_verdict", None) is not None:
            res.event_verdict = result.event_verdict.data_ptr()
        if result.node_counts is not None:
            for m in range(1, self.n_levels):
                res.node_keys[m] = result.node_keys[m].data_ptr()
                res.node_counts[m] = result.node_counts[m].data_ptr()
                res.node_verdict[m] = result.node_verdict[m].data_ptr()
        if getattr(result, "inst_key_values", None) is not None:
            res.inst_key_values = result.inst_key_values.data_ptr()
        if getattr(result, "node_key_values", None) is not None:
            for m in range(1, self.n_levels):
                res.node_key_values[m] = result.node_key_values[m].data_ptr()
        return res

    def eval_noalloc_into(self, records, n_events, props, result):
        """Enqueue one evaluation in the library's own scratch memory (no
        workspace, no allocation by the library)."""
        self._bind_stream()
        res = self._result_desc(result)
        arr = (C.c_int32 * len(props))(*props)
        _check(self.lib.ltl4c_eval_noalloc(self.h, C.c_void_p(records.data_ptr() if n_events else 0), n_events, arr,
                                           len(props), C.byref(res)), "ltl4c_eval_noalloc")

    def eval(self, records, props, instances=False, nodes=False, capacity=None, timeline=False, events=False,
             key_values=False):
        """Evaluate and wait; returns an EvalResult of device tensors."""
        n = records.numel() // self.record_bytes
        if capacity is None:
            capacity = max(n, 1)
        r = self.alloc_result(len(props), capacity, instances, nodes, timeline, n if events else 0, key_values)
        self.eval_into(records, n, props, r, self.workspace(n, props))
        self.wait()
        return r

    def wait(self):
        _check(self.lib.ltl4c_wait(self.h), "ltl4c_wait")

    def set_option(self, option, value):
        _check(self.lib.ltl4c_set_option(self.h, option, value), "ltl4c_set_option")
        self._workspace = None

    def batch_workspace(self, n_events, n_traces, props):
        arr = (C.c_int32 * len(props))(*props)
        b = C.c_uint64()
        _check(self.lib.ltl4c_batch_workspace_bytes(self.h, n_events, n_traces, arr, len(props), C.byref(b)),
               "ltl4c_batch_workspace_bytes")
        need = max(b.value, 256)
        ws = self._workspace
        if ws is None or ws.numel() < need:
            ws = self.torch.empty(need, dtype=self.torch.uint8, device=f"cuda:{self.device}")
            self._workspace = ws
        return ws

    def eval_batch_into(self, records, offsets, props, verdict, counts, workspace):
        """Enqueue a batch: trace t = records [offsets[t], offsets[t+1])."""
        self._bind_stream()
        nt = len(offsets) - 1
        off = (C.c_uint64 * (nt + 1))(*[int(x) for x in offsets])
        arr = (C.c_int32 * len(props))(*props)
        _check(self.lib.ltl4c_eval_batch(self.h, C.c_void_p(records.data_ptr() if int(offsets[-1]) else 0), off, nt,
                                         arr, len(props), C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                         C.c_void_p(verdict.data_ptr()), C.c_void_p(counts.data_ptr())),
               "ltl4c_eval_batch")

    def eval_batch(self, records, offsets, props):
        """Evaluate and wait: (verdict [T, P], counts [T, P, 6]) as numpy."""
        t, dev = self.torch, f"cuda:{self.device}"
        nt = len(offsets) - 1
        v = t.empty(nt * len(props), dtype=t.uint8, device=dev)
        c = t.empty(nt * len(props) * 6, dtype=t.int64, device=dev)
        self.eval_batch_into(records, offsets, props, v, c, self.batch_workspace(int(offsets[-1]), nt, props))
        self.wait()
        return v.cpu().numpy().reshape(nt, len(props)), c.cpu().numpy().reshape(nt, len(props), 6)

    # ---- autotuned schedules -------------------------------------------------
    def tune(self, records, props, n_events=None, offsets=None, reps=5):
        """Time the kernel schedules on these records (one trace of n_events,
        or a batch given by offsets) and keep the fastest for this shape
        class.  Returns {sort_tile, scan_tile, tuned_us, default_us, candidates}."""
        self._bind_stream()
        arr = (C.c_int32 * len(props))(*props)
        if offsets is not None:
            nt = len(offsets) - 1
            off = (C.c_uint64 * (nt + 1))(*[int(x) for x in offsets])
            n = int(offsets[-1])
        else:
            nt, off, n = 0, None, int(n_events)
        b = C.c_uint64()
        _check(self.lib.ltl4c_tune_workspace_bytes(self.h, n, off, nt, arr, len(props), C.byref(b)),
               "ltl4c_tune_workspace_bytes")
        self._workspace = None
        ws = self.torch.empty(max(b.value, 256), dtype=self.torch.uint8, device=f"cuda:{self.device}")
        t = Tuned()
        _check(self.lib.ltl4c_tune(self.h, C.c_void_p(records.data_ptr() if n else 0), n, off, nt, arr, len(props),
                                   C.c_void_p(ws.data_ptr()), ws.numel(), reps, C.byref(t)), "ltl4c_tune")
        del ws
        return {"sort_tile": t.sort_tile, "scan_tile": t.scan_tile, "tuned_us": t.tuned_us,
                "default_us": t.default_us, "candidates": t.candidates}

    def save_schedules(self, path):
        _check(self.lib.ltl4c_schedule_save(self.h, os.fsencode(path)), "ltl4c_schedule_save")

    def load_schedules(self, path):
        n = C.c_int32()
        _check(self.lib.ltl4c_schedule_load(self.h, os.fsencode(path), C.byref(n)), "ltl4c_schedule_load")
        self._workspace = None
        return n.value

    def clear_schedules(self):
        _check(self.lib.ltl4c_schedule_clear(self.h), "ltl4c_schedule_clear")
        self._workspace = None

    # ---- graphs ----------------------------------------------------------------
    def graph_eval(self, records, n_events, props, result, workspace):
        """Capture one evaluation (same arguments as eval_into) into a graph; returns its id."""
        self._bind_stream()
        res = self._result_desc(result)
        arr = (C.c_int32 * len(props))(*props)
        g = C.c_int32()
        _check(self.lib.ltl4c_graph_eval(self.h, C.c_void_p(records.data_ptr() if n_events else 0), n_events, arr,
                                         len(props), C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                         C.byref(res), C.byref(g)), "ltl4c_graph_eval")
        return g.value

    def graph_eval_batch(self, records, offsets, props, verdict, counts, workspace):
        """Capture one batch evaluation (same arguments as eval_batch_into); returns its id."""
        self._bind_stream()
        nt = len(offsets) - 1
        off = (C.c_uint64 * (nt + 1))(*[int(x) for x in offsets])
        arr = (C.c_int32 * len(props))(*props)
        g = C.c_int32()
        _check(self.lib.ltl4c_graph_eval_batch(self.h, C.c_void_p(records.data_ptr() if int(offsets[-1]) else 0),
                                               off, nt, arr, len(props), C.c_void_p(workspace.data_ptr()),
                                               workspace.numel(), C.c_void_p(verdict.data_ptr()),
                                               C.c_void_p(counts.data_ptr()), C.byref(g)), "ltl4c_graph_eval_batch")
        return g.value

    def graph_launch(self, graph):
        self._bind_stream()
        _check(self.lib.ltl4c_graph_launch(self.h, graph), "ltl4c_graph_launch")

    def graph_destroy(self, graph):
        self._bind_stream()
        _check(self.lib.ltl4c_graph_destroy(self.h, graph), "ltl4c_graph_destroy")

    def set_memory_budget(self, nbytes):
        _check(self.lib.ltl4c_set_memory_budget(self.h, nbytes), "ltl4c_set_memory_budget")

    def group_bytes(self, props, max_streams, max_bindings, max_batch):
        arr = (C.c_int32 * len(props))(*props)
        b = C.c_uint64()
        _check(self.lib.ltl4c_group_bytes(self.h, arr, len(props), max_streams, max_bindings, max_batch,
                                          C.byref(b)), "ltl4c_group_bytes")
        return b.value

    def profile(self, on=True):
        _check(self.lib.ltl4c_profile_enable(self.h, 1 if on else 0), "ltl4c_profile_enable")

    def profile_reset(self):
        _check(self.lib.ltl4c_profile_reset(self.h), "ltl4c_profile_reset")

    def profile_read(self):
        """{kernel name: (total ms, launches)} since the last reset."""
        out, i = {}, 0
        buf = C.create_string_buffer(64)
        while True:
            ms, cnt = C.c_double(), C.c_uint64()
            s = self.lib.ltl4c_profile_get(self.h, i, buf, 64, C.byref(ms), C.byref(cnt))
            if s != OK:
                break
            out[buf.value.decode()] = (ms.value, cnt.value)
            i += 1
        return out


class StreamGroup:
    """Online monitoring of many streams with device-resident state.

    pool_bindings=None: every stream is admitted at once with max_bindings
    (ltl4c_group_open).  Otherwise the group is a pool of that many binding
    slots and streams are admitted one by one with open_stream()."""

    def __init__(self, ctx, props, max_streams, max_bindings, max_batch, pool_bindings=None):
        self.ctx, self.lib, self.props = ctx, ctx.lib, list(props)
        self.max_streams = max_streams
        arr = (C.c_int32 * len(props))(*props)
        g = C.c_int32()
        if pool_bindings is None:
            _check(self.lib.ltl4c_group_open(ctx.h, arr, len(props), max_streams, max_bindings, max_batch,
                                             C.byref(g)), "ltl4c_group_open")
        else:
            _check(self.lib.ltl4c_group_open_pool(ctx.h, arr, len(props), max_streams, pool_bindings, max_batch,
                                                  C.byref(g)), "ltl4c_group_open_pool")
        self.id = g.value
        t, dev = ctx.torch, f"cuda:{ctx.device}"
        self.verdict = t.empty(max_streams * len(props), dtype=t.uint8, device=dev)
        self.counts = t.empty(max_streams * len(props) * 6, dtype=t.int64, device=dev)
        self.bindings = t.empty(max_streams, dtype=t.int64, device=dev)

    def push(self, records, offsets, streams):
        """Enqueue chunks: records is a device tensor; offsets (len n+1) and
        streams (len n) are host sequences."""
        self.ctx._bind_stream()
        n = len(streams)
        off = (C.c_uint64 * (n + 1))(*[int(x) for x in offsets])
        st = (C.c_uint32 * n)(*[int(x) for x in streams])
        _check(self.lib.ltl4c_group_push(self.ctx.h, self.id, C.c_void_p(records.data_ptr()), off, st, n),
               "ltl4c_group_push")

    def push_chunks(self, ptrs, sizes, streams):
        """Enqueue chunks held in separate device buffers (addresses in ptrs)."""
        self.ctx._bind_stream()
        n = len(streams)
        p = (C.c_void_p * n)(*[int(x) for x in ptrs])
        sz = (C.c_uint64 * n)(*[int(x) for x in sizes])
        st = (C.c_uint32 * n)(*[int(x) for x in streams])
        _check(self.lib.ltl4c_group_push_chunks(self.ctx.h, self.id, p, sz, st, n), "ltl4c_group_push_chunks")

    def push_seq(self, ptrs, sizes, streams, seqs, on_device=True):
        """Enqueue chunks with sequence numbers; ptrs are device addresses, or
        pinned host addresses when on_device is False."""
        self.ctx._bind_stream()
        n = len(streams)
        p = (C.c_void_p * n)(*[int(x) for x in ptrs])
        sz = (C.c_uint64 * n)(*[int(x) for x in sizes])
        st = (C.c_uint32 * n)(*[int(x) for x in streams])
        sq = (C.c_uint64 * n)(*[int(x) for x in seqs])
        _check(self.lib.ltl4c_group_push_seq(self.ctx.h, self.id, p, sz, st, sq, n, 1 if on_device else 0),
               "ltl4c_group_push_seq")

    def capture_push(self, ptrs, sizes, streams):
        """Capture a push of device chunks (as push_chunks) into a graph of the
        context; every ctx.graph_launch(id) then pushes the chunks' current
        contents.  Returns the graph id."""
        self.ctx._bind_stream()
        n = len(streams)
        p = (C.c_void_p * n)(*[int(x) for x in ptrs])
        sz = (C.c_uint64 * n)(*[int(x) for x in sizes])
        st = (C.c_uint32 * n)(*[int(x) for x in streams])
        g = C.c_int32()
        _check(self.lib.ltl4c_graph_group_push(self.ctx.h, self.id, p, sz, st, n, C.byref(g)),
               "ltl4c_graph_group_push")
        return g.value

    def open_stream(self, stream, max_bindings, first_seq=0):
        self.ctx._bind_stream()
        _check(self.lib.ltl4c_stream_open(self.ctx.h, self.id, stream, max_bindings, first_seq), "ltl4c_stream_open")

    def close_stream(self, stream):
        self.ctx._bind_stream()
        _check(self.lib.ltl4c_stream_close(self.ctx.h, self.id, stream), "ltl4c_stream_close")

    def poll(self, stream):
        """(next sequence number expected, chunks applied on the device)."""
        a, b = C.c_uint64(), C.c_uint64()
        _check(self.lib.ltl4c_stream_poll(self.ctx.h, self.id, stream, C.byref(a), C.byref(b)), "ltl4c_stream_poll")
        return a.value, b.value

    def stalled(self, idle_s):
        out = (C.c_uint32 * self.max_streams)()
        n = C.c_uint32()
        _check(self.lib.ltl4c_group_stalled(self.ctx.h, self.id, int(idle_s * 1e9), out, self.max_streams,
                                            C.byref(n)), "ltl4c_group_stalled")
        return list(out[:n.value])

    def read_nodes(self, level, capacity):
        """(keys [n], counts [P, n, 6], verdict [P, n]) of the level's nodes, sorted by key."""
        t, dev = self.ctx.torch, f"cuda:{self.ctx.device}"
        P = len(self.props)
        keys = t.empty(capacity, dtype=t.int64, device=dev)
        counts = t.empty(P * capacity * 6, dtype=t.int32, device=dev)
        verdict = t.empty(P * capacity, dtype=t.uint8, device=dev)
        n = t.zeros(1, dtype=t.int64, device=dev)
        self.ctx._bind_stream()
        _check(self.lib.ltl4c_group_read_nodes(self.ctx.h, self.id, level, C.c_void_p(keys.data_ptr()),
                                               C.c_void_p(counts.data_ptr()), C.c_void_p(verdict.data_ptr()),
                                               capacity, C.c_void_p(n.data_ptr())), "ltl4c_group_read_nodes")
        self.ctx.wait()
        k = int(n.item())
        kk = keys[:k].cpu().numpy().view(np.uint64)
        o = np.argsort(kk, kind="stable")
        c = counts.view(P, capacity, 6)[:, :k].cpu().numpy()[:, o]
        v = verdict.view(P, capacity)[:, :k].cpu().numpy()[:, o]
        return kk[o], c, v

    def read(self):
        """(verdict [S, P], counts [S, P, 6], bindings [S]) as numpy, after a wait."""
        self.ctx._bind_stream()
        _check(self.lib.ltl4c_group_read(self.ctx.h, self.id, C.c_void_p(self.verdict.data_ptr()),
                                         C.c_void_p(self.counts.data_ptr()), C.c_void_p(self.bindings.data_ptr())),
               "ltl4c_group_read")
        self.ctx.wait()
        P = len(self.props)
        return (self.verdict.cpu().numpy().reshape(self.max_streams, P),
                self.counts.cpu().numpy().reshape(self.max_streams, P, 6),
                self.bindings.cpu().numpy())

    def snapshot(self):
        n = C.c_uint64()
        _check(self.lib.ltl4c_group_snapshot(self.ctx.h, self.id, None, C.byref(n)), "ltl4c_group_snapshot")
        buf = np.empty(n.value, dtype=np.uint8)
        _check(self.lib.ltl4c_group_snapshot(self.ctx.h, self.id, C.c_void_p(buf.ctypes.data), C.byref(n)),
               "ltl4c_group_snapshot")
        return buf

    def restore(self, buf):
        _check(self.lib.ltl4c_group_restore(self.ctx.h, self.id, C.c_void_p(buf.ctypes.data), buf.size),
               "ltl4c_group_restore")

    def close(self):
        if self.id is not None:
            self.lib.ltl4c_group_close(self.ctx.h, self.id)
            self.id = None


def open_workload(wl, device=0):
    """Context with the workload's layout and properties registered.

    Returns (ctx, prop_ids, device records tensor)."""
    import torch
    ctx = Context(device)
    ctx.set_layout(wl.layout)
    ids = [ctx.add_spec(p) for p in wl.props]
    rec = torch.from_numpy(np.ascontiguousarray(wl.raw())).to(f"cuda:{device}")
    return ctx, ids, rec
