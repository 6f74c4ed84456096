"""Online monitoring at the benchmark's scale: 64 streams, pools of 100,000
(user, req) bindings per stream, the benchmark's schedule of chunks of
4k-256k events pushed as they arrive.  After the schedule, every stream's root
verdict, root counts, binding count and level-1 (user) nodes equal the
oracle's offline result on that stream's concatenated chunks; once with the
chunks already in device memory and once pushed from pinned host memory with
sequence numbers."""
import numpy as np
import pytest

from oracle import cref, parallel
from oracle.run import oracle_property
from paper_1411_2239_amd import lib
from paper_1411_2239_amd import workloads as W

pytestmark = pytest.mark.gpu

N_STREAMS = 64
POOL_EVENTS = 1_000_000
N_CHUNKS = 1500
MAX_BATCH = 1 << 24


def _schedule():
    arr, streams, sizes = W.serving_schedule(N_CHUNKS, N_STREAMS)
    pos = [0] * N_STREAMS
    starts = []
    for st, sz in zip(streams, sizes):
        if pos[st] + sz > POOL_EVENTS:
            pos[st] = 0
        starts.append(pos[st])
        pos[st] += int(sz)
    return streams.astype(np.int64), sizes.astype(np.int64), np.array(starts, dtype=np.int64)


def _pushes(sizes):
    """The capacity run's pushes: as many arrived chunks as fit one push."""
    out, i = [], 0
    while i < len(sizes):
        j, tot = i, 0
        while j < len(sizes) and j - i < 4096 and tot + sizes[j] <= MAX_BATCH:
            tot += int(sizes[j])
            j += 1
        out.append((i, j))
        i = j
    return out


def test_serving_64_streams_full_scale():
    import torch
    print("[case] serving full scale: generating 64 stream pools", flush=True)
    lay = W.serving_layout(N_STREAMS)
    spec = W.user_request_properties()[0]
    pools = [W.gen_serving_pool(s, POOL_EVENTS) for s in range(N_STREAMS)]
    streams, sizes, starts = _schedule()
    ctx = lib.Context(0)
    ctx.set_layout(lay)
    pid = ctx.add_spec(spec)
    rb = lay.record_bytes
    dev = [torch.from_numpy(p.view(np.uint8)).to("cuda:0") for p in pools]
    host = [torch.from_numpy(p.view(np.uint8)).pin_memory() for p in pools]
    results = {}
    for mode in ("device", "pinned_host"):
        print(f"[case] serving full scale: {N_CHUNKS} chunks, {int(sizes.sum())} events, {mode}", flush=True)
        grp = lib.StreamGroup(ctx, [pid], N_STREAMS, 100_000, MAX_BATCH, pool_bindings=N_STREAMS * 100_000)
        for s in range(N_STREAMS):
            grp.open_stream(s, 100_000)
        seq = [0] * N_STREAMS
        for i, j in _pushes(sizes):
            base = dev if mode == "device" else host
            ptrs = [base[int(streams[k])].data_ptr() + int(starts[k]) * rb for k in range(i, j)]
            seqs = []
            for k in range(i, j):
                seqs.append(seq[int(streams[k])])
                seq[int(streams[k])] += 1
            grp.push_seq(ptrs, sizes[i:j], streams[i:j], seqs, on_device=(mode == "device"))
        v, c, b = grp.read()
        nk, nc, nv = grp.read_nodes(1, N_STREAMS * 1000)
        for s in range(N_STREAMS):
            assert grp.poll(s) == (seq[s], seq[s])
        results[mode] = (v, c, b, nk, nc, nv)
        grp.close()
    ctx.close()
    # the oracle on every stream's concatenated chunks
    props = [oracle_property(spec, lay)]

    def job(s):
        ks = np.nonzero(streams == s)[0]
        recs = np.concatenate([pools[s][starts[k]:starts[k] + sizes[k]] for k in ks] + [pools[s][:0]])
        raw = recs.view(np.uint8).reshape(-1)
        return lambda: cref.evaluate_records(raw, rb, lay.type_offset, lay.type_bytes, lay.key_offsets,
                                             lay.key_bytes, lay.class_of_type, lay.key_present, props)
    print("[case] serving full scale: oracle on 64 streams", flush=True)
    oracle = parallel.evaluate_many([job(s) for s in range(N_STREAMS)])
    u_bits = lay.key_bits[0]
    for mode, (v, c, b, nk, nc, nv) in results.items():
        stream_of = nk >> np.uint64(u_bits)
        user_of = nk & np.uint64((1 << u_bits) - 1)
        for s, o in enumerate(oracle):
            assert np.array_equal(v[s], o.root_verdict), (mode, s)
            assert np.array_equal(c[s], o.root_counts.astype(np.int64)), (mode, s)
            assert b[s] == o.inst_keys.shape[0], (mode, s, b[s], o.inst_keys.shape[0])
            sel = stream_of == s
            assert np.array_equal(user_of[sel], o.level_keys[1][:, 0].astype(np.uint64)), (mode, s)
            assert np.array_equal(nc[:, sel].astype(np.int64), o.level_counts[1].astype(np.int64)), (mode, s)
            assert np.array_equal(nv[:, sel], o.level_verdict[1]), (mode, s)
