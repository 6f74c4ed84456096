"""Online monitoring (stream groups) against the oracle.

After every push the truth value of each stream must equal the offline
oracle's verdict on that stream's concatenated prefix: online and offline
evaluation agree (Section 4, online mode), whatever the chunking."""
import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import lib
from paper_1411_2239_amd import workloads as W

from _util import prop_workload

pytestmark = pytest.mark.gpu


def _stream_traces(kind, n_streams, n_events, seed):
    out = []
    for s in range(n_streams):
        if kind == "users":
            out.append(W.gen_user_requests(n_events=n_events, n_users=40, seed=seed + s))
        elif kind == "sockets":
            out.append(W.gen_sockets(n_events=n_events, n_sockets=30, seed=seed + s))
        elif kind == "chunks":
            out.append(W.gen_chunk_uploads(n_events, 50, n_preds=2, seed=seed + s))
        else:
            out.append(prop_workload(n_events, 3, [3, 4, 5], seed=seed + s, n_props=2,
                                     formulas=["G(a -> F b)", "a U (b U c)"],
                                     quants=[[("A", ">=", "1/2"), ("E", "<=", 2), ("A", "=", 1)],
                                             [("E", ">", 1), ("A", "<", "3/4"), ("E", ">=", 1)]]))
    # every stream shares the layout and properties of stream 0
    for wl in out[1:]:
        wl.layout, wl.props = out[0].layout, out[0].props
    return out


def _check_group(kind, n_streams=5, n_events=3000, pushes=6, seed=100, snapshot_at=None):
    import torch
    traces = _stream_traces(kind, n_streams, n_events, seed)
    print(f"[case] serving {kind} streams={n_streams} events/stream={n_events}", flush=True)
    ctx, ids, _ = lib.open_workload(traces[0])
    rb = traces[0].layout.record_bytes
    grp = lib.StreamGroup(ctx, ids, max_streams=n_streams + 3, max_bindings=4096, max_batch=n_events * n_streams)
    rng = np.random.default_rng(seed)
    pos = [0] * n_streams
    snap = None
    history = []
    for k in range(pushes):
        chunks = []
        for _ in range(int(rng.integers(1, 2 * n_streams + 1))):
            s = int(rng.integers(0, n_streams))
            size = int(rng.integers(0, n_events // 3 + 1))
            size = min(size, n_events - pos[s])
            chunks.append((s, pos[s], pos[s] + size))
            pos[s] += size
        raw = np.concatenate([traces[s].raw()[a * rb:b * rb] for s, a, b in chunks] + [np.zeros(0, np.uint8)])
        offsets = np.concatenate([[0], np.cumsum([b - a for _, a, b in chunks])])
        if offsets[-1] > 0:
            dev = torch.from_numpy(raw).to("cuda:0")
            grp.push(dev, offsets, [s for s, _, _ in chunks])
        verdict, counts, bindings = grp.read()
        for s in range(n_streams):
            o = evaluate_workload(traces[s], records=traces[s].records[:pos[s]])
            assert np.array_equal(verdict[s], o.root_verdict), (k, s, verdict[s], o.root_verdict)
            assert np.array_equal(counts[s], o.root_counts.astype(np.int64)), (k, s)
            assert bindings[s] == o.inst_keys.shape[0], (k, s, bindings[s], o.inst_keys.shape)
        for s in range(n_streams, n_streams + 3):   # never-fed streams: empty trees
            o = evaluate_workload(traces[0], records=traces[0].records[:0])
            assert np.array_equal(verdict[s], o.root_verdict) and bindings[s] == 0
        history.append((verdict.copy(), counts.copy()))
        if snapshot_at == k:
            snap = (grp.snapshot(), list(pos), k)
    grp.close()
    ctx.close()
    return traces, snap, history


def test_serving_users_two_levels():
    _check_group("users")


def test_serving_sockets_one_level():
    _check_group("sockets", n_streams=4, n_events=4000)


def test_serving_data_predicates():
    # letters that depend on record data (two predicates) in the online mode
    _check_group("chunks", n_streams=4, n_events=3000)


def test_serving_three_levels_two_properties():
    _check_group("props", n_streams=3, n_events=2500)


def test_serving_single_big_push_equals_offline():
    import torch
    wl = W.gen_user_requests(n_events=200_000, n_users=200, seed=5)
    ctx, ids, rec = lib.open_workload(wl)
    grp = lib.StreamGroup(ctx, ids, max_streams=1, max_bindings=1 << 17, max_batch=wl.n_events)
    grp.push(rec, [0, wl.n_events], [0])
    v, c, b = grp.read()
    o = evaluate_workload(wl)
    assert np.array_equal(v[0], o.root_verdict) and np.array_equal(c[0], o.root_counts.astype(np.int64))
    assert b[0] == o.inst_keys.shape[0]
    grp.close()
    ctx.close()


def test_snapshot_restore_resumes_identically():
    import torch
    traces = _stream_traces("users", 3, 3000, 77)
    ctx, ids, _ = lib.open_workload(traces[0])
    rb = traces[0].layout.record_bytes
    grp = lib.StreamGroup(ctx, ids, max_streams=3, max_bindings=4096, max_batch=9000)

    def push_range(s, a, b):
        dev = torch.from_numpy(np.ascontiguousarray(traces[s].raw()[a * rb:b * rb])).to("cuda:0")
        grp.push(dev, [0, b - a], [s])

    for s in range(3):
        push_range(s, 0, 1000)
    snap = grp.snapshot()
    for s in range(3):
        push_range(s, 1000, 3000)
    full = grp.read()
    grp.restore(snap)
    for s in range(3):
        push_range(s, 1000, 2000)
        push_range(s, 2000, 3000)
    again = grp.read()
    for x, y in zip(full, again):
        assert np.array_equal(x, y)
    grp.close()
    ctx.close()


def test_admission_by_memory_budget():
    wl = W.gen_sockets(n_events=100, n_sockets=10)
    ctx, ids, _ = lib.open_workload(wl)
    need = ctx.group_bytes(ids, 8, 1000, 10_000)
    ctx.set_memory_budget(need - 1)
    with pytest.raises(lib.LTL4CError) as e:
        lib.StreamGroup(ctx, ids, 8, 1000, 10_000)
    assert e.value.status == lib.EADMIT
    ctx.set_memory_budget(need)
    g = lib.StreamGroup(ctx, ids, 8, 1000, 10_000)
    with pytest.raises(lib.LTL4CError) as e2:     # nothing left for a second group
        lib.StreamGroup(ctx, ids, 8, 1000, 10_000)
    assert e2.value.status == lib.EADMIT
    g.close()
    lib.StreamGroup(ctx, ids, 8, 1000, 10_000).close()   # room again after close
    ctx.close()


def test_binding_capacity_is_reported():
    import torch
    wl = W.gen_sockets(n_events=2000, n_sockets=500, seed=3)
    ctx, ids, rec = lib.open_workload(wl)
    grp = lib.StreamGroup(ctx, ids, max_streams=1, max_bindings=100, max_batch=2000)
    grp.push(rec, [0, 2000], [0])
    with pytest.raises(lib.LTL4CError) as e:
        grp.read()
    assert e.value.status == lib.ECAPACITY
    grp.close()
    ctx.close()


def test_push_chunks_from_separate_buffers():
    import torch
    traces = _stream_traces("users", 4, 3000, 300)
    ctx, ids, _ = lib.open_workload(traces[0])
    rb = traces[0].layout.record_bytes
    grp = lib.StreamGroup(ctx, ids, max_streams=4, max_bindings=4096, max_batch=12000)
    dev = [torch.from_numpy(np.ascontiguousarray(t.raw())).to("cuda:0") for t in traces]
    rng = np.random.default_rng(1)
    pos = [0] * 4
    for k in range(5):
        ptrs, sizes, streams = [], [], []
        for _ in range(6):
            s = int(rng.integers(0, 4))
            size = min(int(rng.integers(1, 900)), 3000 - pos[s])
            ptrs.append(dev[s].data_ptr() + pos[s] * rb)
            sizes.append(size)
            streams.append(s)
            pos[s] += size
        grp.push_chunks(ptrs, sizes, streams)
        verdict, counts, bindings = grp.read()
        for s in range(4):
            o = evaluate_workload(traces[s], records=traces[s].records[:pos[s]])
            assert np.array_equal(verdict[s], o.root_verdict) and np.array_equal(counts[s], o.root_counts.astype(np.int64))
            assert bindings[s] == o.inst_keys.shape[0]
    grp.close()
    ctx.close()
