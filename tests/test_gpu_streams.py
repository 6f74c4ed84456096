"""Streams of a group (online mode, Section 4): admission of single streams
from a pool of binding slots, per-stream chunk sequence numbers, pushes from
pinned host memory, stream close and reopen, completion polling, stalled
streams, and the quantifier nodes read back from the device.  After every
accepted push, each stream's verdict, counts and binding count equal the
oracle's offline result on the stream's chunks so far."""
import time

import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import lib
from paper_1411_2239_amd import workloads as W

pytestmark = pytest.mark.gpu


def _traces(n_streams, n_events, seed, users=40):
    out = [W.gen_user_requests(n_events=n_events, n_users=users, seed=seed + s) for s in range(n_streams)]
    for wl in out[1:]:
        wl.layout, wl.props = out[0].layout, out[0].props
    return out


def _check(grp, traces, fed, streams=None):
    """fed[s]: records of stream s pushed so far (a numpy structured array)."""
    verdict, counts, bindings = grp.read()
    for s in (range(len(traces)) if streams is None else streams):
        o = evaluate_workload(traces[s], records=fed[s])
        assert np.array_equal(verdict[s], o.root_verdict), (s, verdict[s], o.root_verdict)
        assert np.array_equal(counts[s], o.root_counts.astype(np.int64)), s
        assert bindings[s] == o.inst_keys.shape[0], (s, bindings[s], o.inst_keys.shape)


def test_sequence_numbers_reject_gaps_and_duplicates():
    import torch
    print("[case] streams: sequence numbers", flush=True)
    traces = _traces(3, 3000, 500)
    ctx, ids, _ = lib.open_workload(traces[0])
    rb = traces[0].layout.record_bytes
    dev = [torch.from_numpy(np.ascontiguousarray(t.raw())).to("cuda:0") for t in traces]
    grp = lib.StreamGroup(ctx, ids, 3, 4096, 9000, pool_bindings=3 * 4096)
    for s in range(3):
        grp.open_stream(s, 4096, first_seq=10 * s)
    pos = [0, 0, 0]
    seq = [0, 10, 20]

    def chunk(s, n):
        p = dev[s].data_ptr() + pos[s] * rb
        return p, n

    # two chunks of stream 1 and one of stream 0 in one push
    p0, _ = chunk(0, 500)
    p1 = dev[1].data_ptr()
    grp.push_seq([p0, p1, p1 + 400 * rb], [500, 400, 300], [0, 1, 1], [0, 10, 11])
    pos = [500, 700, 0]
    seq = [1, 12, 20]
    _check(grp, traces, [traces[s].records[:pos[s]] for s in range(3)])
    # a duplicate (stream 1 repeats 11) and a gap (stream 2 skips 20) are refused whole
    for bad in ([[0, 1], [1, 11]], [[2, 21]], [[0, 1], [2, 20], [2, 22]]):
        ptrs = [dev[s].data_ptr() + pos[s] * rb for s, _ in bad]
        with pytest.raises(lib.LTL4CError) as e:
            grp.push_seq(ptrs, [100] * len(bad), [s for s, _ in bad], [q for _, q in bad])
        assert e.value.status == lib.ESEQ
    _check(grp, traces, [traces[s].records[:pos[s]] for s in range(3)])
    assert grp.poll(1) == (12, 12)
    # the accepted continuation
    grp.push_seq([dev[2].data_ptr(), dev[1].data_ptr() + pos[1] * rb], [800, 250], [2, 1], [20, 12])
    pos = [500, 950, 800]
    _check(grp, traces, [traces[s].records[:pos[s]] for s in range(3)])
    assert grp.poll(2) == (21, 21) and grp.poll(0) == (1, 1)
    grp.close()
    ctx.close()


def test_pool_admission_close_and_reopen():
    import torch
    print("[case] streams: admission from a binding pool", flush=True)
    traces = _traces(3, 4000, 600)
    ctx, ids, _ = lib.open_workload(traces[0])
    rb = traces[0].layout.record_bytes
    dev = [torch.from_numpy(np.ascontiguousarray(t.raw())).to("cuda:0") for t in traces]
    grp = lib.StreamGroup(ctx, ids, 4, 0, 12000, pool_bindings=10_000)
    grp.open_stream(0, 6000)
    with pytest.raises(lib.LTL4CError) as e:
        grp.open_stream(1, 5000)                 # 6000 + 5000 > 10000
    assert e.value.status == lib.EADMIT
    with pytest.raises(lib.LTL4CError) as e:
        grp.open_stream(0, 10)                   # already open
    assert e.value.status == lib.ESEQ
    grp.open_stream(1, 4000)
    with pytest.raises(lib.LTL4CError) as e:     # stream 2 is not admitted
        grp.push_chunks([dev[2].data_ptr()], [100], [2])
    assert e.value.status == lib.ESEQ
    grp.push_chunks([dev[0].data_ptr(), dev[1].data_ptr()], [3000, 2000], [0, 1])
    _check(grp, traces, [traces[0].records[:3000], traces[1].records[:2000]], streams=[0, 1])
    # closing stream 0 frees its slots and its reservation
    grp.close_stream(0)
    with pytest.raises(lib.LTL4CError) as e:
        grp.push_chunks([dev[0].data_ptr()], [10], [0])
    assert e.value.status == lib.ESEQ
    grp.open_stream(2, 6000)
    grp.push_chunks([dev[2].data_ptr(), dev[1].data_ptr() + 2000 * rb], [2500, 2000], [2, 1])
    v, c, b = grp.read()
    empty = evaluate_workload(traces[0], records=traces[0].records[:0])
    assert b[0] == 0 and np.array_equal(v[0], empty.root_verdict)
    assert np.array_equal(c[0], empty.root_counts.astype(np.int64))
    _check(grp, traces, [None, traces[1].records[:4000], traces[2].records[:2500]], streams=[1, 2])
    # stream 0 again, from scratch: it reuses the dead slots of its first life
    grp.close_stream(2)
    grp.open_stream(0, 6000)
    grp.push_chunks([dev[0].data_ptr() + 500 * rb], [3500], [0])
    _check(grp, traces, [traces[0].records[500:4000], traces[1].records[:4000]], streams=[0, 1])
    grp.close()
    ctx.close()


def test_per_stream_binding_limit():
    import torch
    print("[case] streams: per-stream binding limit", flush=True)
    wl = W.gen_sockets(n_events=2000, n_sockets=500, seed=3)
    ctx, ids, rec = lib.open_workload(wl)
    grp = lib.StreamGroup(ctx, ids, 2, 0, 2000, pool_bindings=4000)
    grp.open_stream(0, 100)
    grp.open_stream(1, 3000)
    grp.push(rec, [0, 2000], [1])
    grp.read()                                    # stream 1 has room
    grp.push(rec, [0, 2000], [0])
    with pytest.raises(lib.LTL4CError) as e:
        grp.read()
    assert e.value.status == lib.ECAPACITY
    grp.close()
    ctx.close()


def test_pinned_host_pushes_match_offline():
    import torch
    print("[case] streams: pinned host pushes", flush=True)
    traces = _traces(4, 6000, 700)
    ctx, ids, _ = lib.open_workload(traces[0])
    rb = traces[0].layout.record_bytes
    host = [torch.from_numpy(np.ascontiguousarray(t.raw())).pin_memory() for t in traces]
    dev = [h.to("cuda:0") for h in host]
    grp = lib.StreamGroup(ctx, ids, 4, 8192, 16000, pool_bindings=4 * 8192)
    for s in range(4):
        grp.open_stream(s, 8192)
    rng = np.random.default_rng(5)
    pos, seq = [0] * 4, [0] * 4
    for k in range(10):
        ptrs, sizes, streams, seqs = [], [], [], []
        on_device = k % 3 == 2                    # host and device pushes interleave
        for _ in range(int(rng.integers(1, 7))):
            s = int(rng.integers(0, 4))
            size = min(int(rng.integers(0, 1200)), 6000 - pos[s])
            base = (dev if on_device else host)[s].data_ptr()
            ptrs.append(base + pos[s] * rb)
            sizes.append(size)
            streams.append(s)
            seqs.append(seq[s])
            pos[s] += size
            seq[s] += 1
        grp.push_seq(ptrs, sizes, streams, seqs, on_device=on_device)
        if k % 2 == 1:
            _check(grp, traces, [traces[s].records[:pos[s]] for s in range(4)])
    _check(grp, traces, [traces[s].records[:pos[s]] for s in range(4)])
    for s in range(4):
        assert grp.poll(s) == (seq[s], seq[s])
    # pageable host memory is refused
    pageable = np.ascontiguousarray(traces[0].raw()[:rb * 10])
    with pytest.raises(lib.LTL4CError) as e:
        grp.push_seq([pageable.ctypes.data], [10], [0], [seq[0]], on_device=False)
    assert e.value.status == lib.EINVAL
    grp.close()
    ctx.close()


def test_stalled_streams():
    import torch
    print("[case] streams: stalled detection", flush=True)
    traces = _traces(3, 500, 800)
    ctx, ids, _ = lib.open_workload(traces[0])
    dev = torch.from_numpy(np.ascontiguousarray(traces[0].raw())).to("cuda:0")
    grp = lib.StreamGroup(ctx, ids, 3, 1000, 500, pool_bindings=3000)
    grp.open_stream(0, 1000)
    grp.open_stream(2, 1000)
    time.sleep(0.3)
    grp.push_chunks([dev.data_ptr()], [500], [2])
    assert grp.stalled(0.2) == [0]               # stream 1 is not open, stream 2 just pushed
    assert sorted(grp.stalled(0.0)) == [0, 2]
    grp.close()
    ctx.close()


def test_level_one_nodes_match_oracle():
    import torch
    print("[case] streams: level-1 node counts", flush=True)
    traces = _traces(3, 5000, 900, users=60)
    ctx, ids, _ = lib.open_workload(traces[0])
    lay = traces[0].layout
    grp = lib.StreamGroup(ctx, ids, 3, 8192, 15000)
    dev = [torch.from_numpy(np.ascontiguousarray(t.raw())).to("cuda:0") for t in traces]
    grp.push_chunks([d.data_ptr() for d in dev], [5000, 3000, 4000], [0, 1, 2])
    keys, counts, verdict = grp.read_nodes(1, 1024)
    stream_bits = 2                               # ceil(log2 3)
    u_bits = lay.key_bits[0]
    stream_of = keys >> np.uint64(u_bits)
    user_of = keys & np.uint64((1 << u_bits) - 1)
    assert int(stream_of.max()) < 1 << stream_bits
    for s, n in zip(range(3), (5000, 3000, 4000)):
        o = evaluate_workload(traces[s], records=traces[s].records[:n])
        sel = stream_of == s
        assert np.array_equal(user_of[sel], o.level_keys[1][:, 0].astype(np.uint64))
        assert np.array_equal(counts[:, sel].astype(np.int64), o.level_counts[1].astype(np.int64))
        assert np.array_equal(verdict[:, sel], o.level_verdict[1])
    grp.close()
    ctx.close()
