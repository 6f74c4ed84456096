"""Batches of independent traces against the oracle: every trace's root
verdict and counts equal the oracle's on that trace alone."""
import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import lib
from paper_1411_2239_amd import workloads as W

pytestmark = pytest.mark.gpu


def _check_batch(n_traces, min_len, max_len, n_props, seed, sample=None):
    import torch
    wl, offsets = W.gen_batch(n_traces, min_len, max_len, seed=seed, n_props=n_props)
    print(f"[case] batch traces={n_traces} events={wl.n_events} props={n_props}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    v, c = ctx.eval_batch(rec, offsets, ids)
    traces = range(n_traces) if sample is None else np.random.default_rng(seed).choice(n_traces, sample, replace=False)
    for t in traces:
        o = evaluate_workload(wl, records=wl.records[offsets[t]:offsets[t + 1]])
        assert np.array_equal(v[t], o.root_verdict), (t, v[t], o.root_verdict)
        assert np.array_equal(c[t], o.root_counts.astype(np.int64)), t
    ctx.close()
    return v, c


def test_batch_small_all_traces():
    _check_batch(40, 10, 5000, 16, seed=1)


def test_batch_with_empty_and_tiny_traces():
    import torch
    wl, offsets = W.gen_batch(12, 1, 40, seed=2, n_props=4)
    # make traces 3 and 7 empty
    lens = np.diff(offsets)
    lens[3] = 0
    lens[7] = 0
    keep = np.concatenate([np.arange(offsets[t], offsets[t] + lens[t]) for t in range(12)]).astype(np.int64)
    wl.records = wl.records[keep]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    ctx, ids, rec = lib.open_workload(wl)
    v, c = ctx.eval_batch(rec, offsets, ids)
    for t in range(12):
        o = evaluate_workload(wl, records=wl.records[offsets[t]:offsets[t + 1]])
        assert np.array_equal(v[t], o.root_verdict) and np.array_equal(c[t], o.root_counts.astype(np.int64))
    ctx.close()


def test_batch_equals_per_trace_eval():
    import torch
    wl, offsets = W.gen_batch(16, 100, 20000, seed=3, n_props=6)
    ctx, ids, rec = lib.open_workload(wl)
    v, c = ctx.eval_batch(rec, offsets, ids)
    rb = wl.layout.record_bytes
    for t in range(16):
        sub = rec[offsets[t] * rb:offsets[t + 1] * rb]
        r = ctx.eval(sub, ids)
        assert np.array_equal(v[t], r.root_verdict.cpu().numpy())
        assert np.array_equal(c[t], r.root_counts.cpu().numpy().reshape(-1, 6))
    ctx.close()


def test_batch_4096_traces_sampled():
    _check_batch(4096, 100, 20000, 16, seed=4, sample=24)


def test_batch_4096_traces_full_size_every_trace():
    """The benchmark's batch: 4096 traces of 1k-1M events (log-uniform),
    16 properties; every trace's 16 root verdicts and count vectors against
    the C oracle on that trace alone (traces spread over the host's cores)."""
    import torch
    from oracle import cref, parallel
    from oracle.run import oracle_property
    wl, offsets = W.gen_batch(4096)
    print(f"[case] batch full size: 4096 traces, {wl.n_events} events, 16 properties", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    v, c = ctx.eval_batch(rec, offsets, ids)
    del rec
    ctx.close()
    torch.cuda.empty_cache()
    lay = wl.layout
    props = [oracle_property(s, lay) for s in wl.props]
    raw = wl.raw()
    rb = lay.record_bytes

    def job(t):
        a, b = int(offsets[t]), int(offsets[t + 1])
        return lambda: cref.evaluate_records(raw[a * rb:b * rb], rb, lay.type_offset, lay.type_bytes,
                                             lay.key_offsets, lay.key_bytes, lay.class_of_type, lay.key_present,
                                             props)
    # longest traces first keeps the pool busy to the end
    order = np.argsort(-np.diff(offsets))
    res = parallel.evaluate_many([job(int(t)) for t in order])
    for t, o in zip(order, res):
        assert np.array_equal(v[t], o.root_verdict), (t, v[t], o.root_verdict)
        assert np.array_equal(c[t], o.root_counts.astype(np.int64)), t
