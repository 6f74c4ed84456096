"""The plain C oracle run over disjoint key partitions, on several host threads
(TEST INFRASTRUCTURE ONLY; see the header of oracle/ltl.py).

Section 2.4's quantifier tree splits at the root: the subtree of a top-level
value d0 (every instance whose vector starts with d0, and every node below it)
depends only on the events that carry d0.  So the trace can be cut by the
value of key 0 into disjoint partitions, each evaluated on its own by the
unchanged single-threaded C oracle; the instances and nodes of all partitions
together are those of the whole trace, and the root's child-verdict counts
(Def. 8) are the sums of the partitions' root counts.  The root verdict is then
Def. 7 on the summed counts (oracle/counting.valuate).  This is also the
paper's parallel CPU variant (one worker per partition of the bindings).

ctypes releases the interpreter lock during the C call, so the partitions run
concurrently on a thread pool.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import cref
from .counting import valuate


def host_threads(cap=16):
    """Threads to use: the CPUs this process may run on, at most `cap`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _field(rec2d, off, nbytes):
    if nbytes == 4 and off % 4 == 0 and rec2d.shape[1] % 4 == 0:
        return rec2d.view(np.uint32)[:, off // 4].astype(np.uint64)
    v = np.zeros(rec2d.shape[0], dtype=np.uint64)
    for b in range(nbytes):
        v |= rec2d[:, off + b].astype(np.uint64) << np.uint64(8 * b)
    return v


def partition_ids(records_u8, layout, n_parts):
    """Partition of every record: a multiplicative hash of its key-0 field."""
    rb = layout.record_bytes
    rec2d = records_u8.reshape(-1, rb)
    k0 = _field(rec2d, layout.key_offsets[0], layout.key_bytes[0])
    h = (k0 * np.uint64(0x9E3779B97F4A7C15)) >> np.uint64(40)
    return (h % np.uint64(n_parts)).astype(np.uint8 if n_parts <= 256 else np.int64)


def _merge_levels(parts, n_props, n_levels):
    """Concatenate the partitions' instances and nodes and put them back in
    lexicographic order of their value vectors."""
    def order(keys):
        if keys.shape[0] == 0:
            return np.zeros(0, dtype=np.int64)
        return np.lexsort(keys.T[::-1])

    ik = np.concatenate([p.inst_keys for p in parts], axis=0)
    iv = np.concatenate([p.inst_verdict for p in parts], axis=1)
    o = order(ik)
    out = {"inst_keys": ik[o], "inst_verdict": iv[:, o]}
    lk, lc, lv = [None] * n_levels, [None] * n_levels, [None] * n_levels
    for m in range(1, n_levels):
        k = np.concatenate([p.level_keys[m] for p in parts], axis=0)
        c = np.concatenate([p.level_counts[m] for p in parts], axis=1)
        v = np.concatenate([p.level_verdict[m] for p in parts], axis=1)
        o = order(k)
        lk[m], lc[m], lv[m] = k[o], c[:, o], v[:, o]
    out.update(level_keys=lk, level_counts=lc, level_verdict=lv)
    return out


def evaluate_partitioned(records_u8, layout, props, n_parts=None, threads=None, parts_idx=None):
    """The C oracle over key-0 partitions.  `props` are cref.OracleProperty.
    Returns a cref.OracleResult (without the per-event timeline outputs)."""
    threads = threads or host_threads()
    n_parts = n_parts or threads
    recs = np.ascontiguousarray(records_u8).view(np.uint8).reshape(-1)
    rb = layout.record_bytes
    rec2d = recs.reshape(-1, rb)
    pid = partition_ids(recs, layout, n_parts) if parts_idx is None else parts_idx
    # a stable grouping keeps trace order inside every partition
    order = np.argsort(pid, kind="stable")
    bounds = np.concatenate([[0], np.cumsum(np.bincount(pid, minlength=n_parts))])

    def run(p):
        rows = order[bounds[p]:bounds[p + 1]]
        sub = np.ascontiguousarray(rec2d[rows]).reshape(-1)
        return cref.evaluate_records(sub, rb, layout.type_offset, layout.type_bytes, layout.key_offsets,
                                     layout.key_bytes, layout.class_of_type, layout.key_present, props,
                                     preds=getattr(layout, "preds", ()), pred_shift=getattr(layout, "pred_shift", 0))

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(run, range(n_parts)))
    return merge_partitions(parts, props, layout.n_keys)


def merge_partitions(parts, props, n_levels):
    P = len(props)
    merged = _merge_levels(parts, P, n_levels)
    root_counts = np.zeros((P, 1, 6), dtype=np.uint64)
    for p in parts:
        root_counts += p.level_counts[0]
    root_verdict = np.zeros((P, 1), dtype=np.uint8)
    for i, pr in enumerate(props):
        kind, op, const = pr.quants[0]
        root_verdict[i, 0] = valuate(kind, op, const, [int(x) for x in root_counts[i, 0]])
    lk, lc, lv = merged["level_keys"], merged["level_counts"], merged["level_verdict"]
    lk[0] = np.zeros((1, 0), dtype=np.uint32)
    lc[0] = root_counts
    lv[0] = root_verdict
    return cref.OracleResult(merged["inst_keys"], merged["inst_verdict"], lk, lc, lv)


def evaluate_many(jobs, threads=None):
    """Independent oracle evaluations on a thread pool: jobs is a list of
    zero-argument callables (each calling cref.evaluate_records)."""
    threads = threads or host_threads()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda j: j(), jobs))
