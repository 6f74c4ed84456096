"""Composite keys wider than the 64-bit sort word (four levels of 32-bit
values, or two levels of random 32-bit ids): the library ranks every
level's values first.  Every root, count, instance and node against the
oracle (which works on the raw values), with the instance and node key
values compared element by element; and the calls that cannot wait for the
ranking refuse such layouts."""
import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import workloads as W

from _util import compare_full, prop_workload

pytestmark = pytest.mark.gpu


def widen(wl, seed):
    """Map each level's key values injectively onto random 32-bit values and
    declare 32-bit keys."""
    rng = np.random.Generator(np.random.PCG64(seed))
    for m in range(wl.layout.n_keys):
        col = wl.records[f"k{m}"]
        table = W.distinct_u32(rng, int(col.max()) + 1)
        wl.records[f"k{m}"] = table[col]
    wl.layout.key_bits = [32] * wl.layout.n_keys
    return wl


def check(wl, nodes=True):
    import torch
    from paper_1411_2239_amd import lib
    L = wl.layout.n_keys
    print(f"[case] {wl.name} n={wl.n_events} levels={L} bits={wl.layout.key_bits}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    r = ctx.eval(rec, ids, instances=True, nodes=nodes, key_values=True)
    torch.cuda.synchronize()
    ctx.close()
    o = evaluate_workload(wl)
    if sum(wl.layout.key_bits) > 40:
        r.key_bits = None            # packed keys are packed ranks: compared through their values below
    compare_full(r, o, len(ids), L)
    n_inst = int(r.sizes[0].item())
    kv = r.inst_key_values.cpu().numpy().view(np.uint32).reshape(-1, L)[:n_inst]
    assert np.array_equal(kv, o.inst_keys)
    if nodes:
        for m in range(1, L):
            nm = int(r.sizes[m].item())
            nv = r.node_key_values[m].cpu().numpy().view(np.uint32).reshape(-1, m)[:nm]
            assert np.array_equal(nv, o.level_keys[m]), m
    return r, o


@pytest.mark.parametrize("n,levels,keys", [(1, 2, [2, 2]), (4097, 2, [50, 70]), (200_000, 3, [40, 30, 20]),
                                           (300_000, 4, [10, 8, 6, 40])])
def test_wide_parity(n, levels, keys):
    check(widen(prop_workload(n, levels, keys, seed=n + levels, n_props=4), seed=levels))


def test_narrow_layout_key_values():
    # no ranking: the values are the packed fields themselves
    check(prop_workload(50_000, 3, [7, 9, 11], seed=5, n_props=2))


def test_wide_user_requests_full_size():
    """Config 2's trace with its users and requests renamed to random 32-bit
    ids (a 64-bit composite key)."""
    wl = W.gen_user_requests()
    widen(wl, seed=12)
    check(wl)


def test_wide_ids_with_parent_events_full_size():
    """The proxy trace with random 32-bit video and request ids and parent
    events: ranking, then the kind bit and the trace index in the word."""
    check(W.gen_proxy_cache(10_000_000, wide_ids=True))


def test_calls_that_cannot_rank_refuse():
    import torch
    from paper_1411_2239_amd import lib
    wl = widen(prop_workload(5000, 2, [9, 9], seed=3, n_props=1), seed=4)
    ctx, ids, rec = lib.open_workload(wl)
    n = wl.n_events
    r = ctx.alloc_result(len(ids), n, instances=True)
    with pytest.raises(lib.LTL4CError) as e:
        ctx.eval_noalloc_into(rec, n, ids, r)
    assert e.value.status == lib.EUNSUPPORTED
    with pytest.raises(lib.LTL4CError) as e:
        ctx.graph_eval(rec, n, ids, r, ctx.workspace(n, ids))
    assert e.value.status == lib.EUNSUPPORTED
    with pytest.raises(lib.LTL4CError) as e:
        ctx.eval_batch(rec, np.array([0, 2500, 5000], dtype=np.uint64), ids)
    assert e.value.status == lib.EUNSUPPORTED
    ctx.close()


def test_too_wide_even_ranked():
    """Four levels of 32-bit keys with 2^16 distinct values each: 64 bits of
    ranks do not fit either."""
    import torch
    from paper_1411_2239_amd import lib
    n = 1 << 16
    wl = prop_workload(n, 4, [2, 2, 2, 2], seed=9, n_props=1)
    rng = np.random.Generator(np.random.PCG64(10))
    for m in range(4):
        wl.records[f"k{m}"] = W.distinct_u32(rng, n)
    wl.layout.key_bits = [32] * 4
    ctx, ids, rec = lib.open_workload(wl)
    with pytest.raises(lib.LTL4CError) as e:
        ctx.eval(rec, ids)
    assert e.value.status == lib.EUNSUPPORTED
    ctx.close()
