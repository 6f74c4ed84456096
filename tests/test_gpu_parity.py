"""Parity of the HIP path (through the C ABI) with the oracle: every root
verdict, root count, instance verdict, node count and node verdict must be
equal, element by element.  Integer work: bit-exact is the bar."""
import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import workloads as W

from _util import compare_full, pack_keys, prop_workload

pytestmark = pytest.mark.gpu


def _run(wl, instances=True, nodes=True):
    import torch
    from paper_1411_2239_amd import lib
    print(f"[case] {wl.name} n={wl.n_events} props={len(wl.props)} levels={wl.layout.n_keys}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    r = ctx.eval(rec, ids, instances=instances, nodes=nodes)
    torch.cuda.synchronize()
    ctx.close()
    return r, len(ids)


def _check(wl, **kw):
    r, P = _run(wl, **kw)
    o = evaluate_workload(wl)
    compare_full(r, o, P, wl.layout.n_keys)
    if r.inst_keys is not None:
        n_inst = int(r.sizes[0].item())
        keys = r.inst_keys.cpu().numpy()[:n_inst].astype(np.uint64)
        assert np.array_equal(keys, pack_keys(o.inst_keys, wl.layout.key_bits))
    return r, o


def test_sockets_full_size():
    _check(W.gen_sockets())


def test_users_small():
    _check(W.gen_user_requests(n_events=300_000, n_users=500, seed=11))


def test_users_full_size():
    _check(W.gen_user_requests())


@pytest.mark.parametrize("n", [1, 2, 63, 4095, 4096, 4097, 8191, 12289])
def test_ragged_sizes(n):
    _check(prop_workload(n, 1, [37], seed=n, n_props=4))


def test_empty_trace():
    import torch
    from paper_1411_2239_amd import lib
    wl = prop_workload(1, 2, [3, 3], seed=5, n_props=2)
    ctx, ids, rec = lib.open_workload(wl)
    r = ctx.alloc_result(len(ids), 1, instances=True, nodes=True)
    ctx.eval_into(rec, 0, ids, r, ctx.workspace(0, ids))
    ctx.wait()
    o = evaluate_workload(wl, records=wl.records[:0])
    compare_full(r, o, len(ids), 2)
    ctx.close()


def test_one_cluster_spanning_many_tiles():
    # every event carries the same binding: one instance over 25 scan tiles
    _check(prop_workload(100_000, 1, [1], seed=3, n_props=8))


def test_every_event_its_own_instance():
    wl = prop_workload(20_000, 1, [1 << 30], seed=4, n_props=3, key_bits=[30])
    wl.records["k0"] = np.random.default_rng(4).permutation(1 << 20)[:20_000].astype(np.uint32)
    _check(wl)


def test_sixteen_properties():
    _check(prop_workload(60_000, 1, [500], seed=21, n_props=16))


@pytest.mark.parametrize("levels,keys", [(2, [40, 50]), (3, [5, 7, 9]), (4, [3, 4, 5, 6])])
def test_nested_quantifiers(levels, keys):
    _check(prop_workload(80_000, levels, keys, seed=100 + levels, n_props=5))


@pytest.mark.parametrize("instances", [True, False])
@pytest.mark.parametrize("case", ["users", "two", "three", "four", "two_wide"])
def test_without_node_outputs(case, instances):
    # root results (and instance verdicts when asked) with the node counts
    # kept in the workspace only
    if case == "users":
        wl = W.gen_user_requests(n_events=400_000, n_users=800, seed=51)
    elif case == "two":
        wl = prop_workload(120_000, 2, [40, 50], seed=52, n_props=3)
    elif case == "three":
        wl = prop_workload(120_000, 3, [5, 7, 9], seed=53, n_props=4)
    elif case == "four":
        wl = prop_workload(120_000, 4, [3, 4, 5, 6], seed=54, n_props=2)
    else:
        # parents spread far beyond the LDS window of a tile
        wl = prop_workload(150_000, 2, [20_000, 3], seed=55, n_props=1)
    r, P = _run(wl, instances=instances, nodes=False)
    compare_full(r, evaluate_workload(wl), P, wl.layout.n_keys)


@pytest.mark.parametrize("n_outer", [900, 30_000])
def test_root_level_counting(n_outer):
    # few or many level-1 nodes under the root, whose count ends with Def. 7
    # in the last block to finish
    _check(prop_workload(200_000, 2, [n_outer, 7], seed=17, n_props=3))


def test_wide_keys():
    # 3 x 19-bit keys: a 57-bit binding key, 7 radix passes of 9-bit digits
    wl = prop_workload(50_000, 3, [1 << 19, 1 << 19, 1 << 19], seed=8, n_props=2, key_bits=[19, 19, 19])
    rng = np.random.default_rng(8)
    for m in range(3):
        wl.records[f"k{m}"] = rng.integers(0, 3 if m < 2 else 1 << 19, size=50_000).astype(np.uint32)
    _check(wl)


def test_excluded_events():
    # 2-byte types: types >= 256 and types without the level-1 key join no cluster
    wl = prop_workload(40_000, 2, [20, 30], seed=9, n_props=3)
    rng = np.random.default_rng(9)
    t = wl.records["type"].copy()
    t[rng.random(40_000) < 0.1] = 300
    t[rng.random(40_000) < 0.1] = 9
    wl.records["type"] = t
    wl.layout.type_bytes = 2
    wl.layout.key_present[9] = 0b01
    wl.layout.class_of_type[9] = 0
    _check(wl)


def _excluded_workload(n, seed, p_out):
    # 27 key bits: three 9-bit or four 8-bit radix passes
    wl = prop_workload(n, 2, [20, 30], seed=seed, n_props=3, key_bits=[14, 13])
    rng = np.random.default_rng(seed)
    t = wl.records["type"].copy()
    t[rng.random(n) < p_out] = 300
    wl.records["type"] = t
    wl.layout.type_bytes = 2
    return wl


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6])
def test_excluded_events_sort_variants(variant):
    # the first radix pass drops excluded events (8- and 9-bit digit kernels);
    # the later passes and the scan read the kept count on the device
    import torch
    from paper_1411_2239_amd import lib
    wl = _excluded_workload(150_000, 60 + variant, 0.3)
    print(f"[case] excluded events, sort variant {variant}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    ctx.set_option(lib.OPT_SORT_TILE, variant)
    r = ctx.eval(rec, ids, instances=True, nodes=True)
    torch.cuda.synchronize()
    ctx.close()
    compare_full(r, evaluate_workload(wl), len(ids), 2)


@pytest.mark.parametrize("p_out", [1.0, 0.9999])
def test_all_or_nearly_all_events_excluded(p_out):
    # nothing (or a handful of events) survives the first radix pass
    _check(_excluded_workload(30_000, 71, p_out))


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6])
def test_sort_tile_variants(variant):
    import torch
    from paper_1411_2239_amd import lib
    wl = W.gen_user_requests(n_events=400_000, n_users=700, seed=31 + variant)
    print(f"[case] sort variant {variant}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    ctx.set_option(lib.OPT_SORT_TILE, variant)
    r = ctx.eval(rec, ids, instances=True, nodes=True)
    torch.cuda.synchronize()
    ctx.close()
    compare_full(r, evaluate_workload(wl), len(ids), 2)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("case", ["users", "one_cluster", "wide"])
def test_scan_tile_variants(variant, case):
    import torch
    from paper_1411_2239_amd import lib
    if case == "users":
        wl = W.gen_user_requests(n_events=500_000, n_users=900, seed=41)
    elif case == "one_cluster":
        wl = prop_workload(70_000, 1, [1], seed=42, n_props=3)
    else:
        wl = prop_workload(90_000, 2, [30, 40], seed=43, n_props=11)
    print(f"[case] scan variant {variant} {case}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    ctx.set_option(lib.OPT_SCAN_TILE, variant)
    r = ctx.eval(rec, ids, instances=True, nodes=True)
    torch.cuda.synchronize()
    ctx.close()
    compare_full(r, evaluate_workload(wl), len(ids), wl.layout.n_keys)


def test_repeated_evaluations_share_one_workspace():
    """Evaluations that reuse one workspace must not see each other's look-back
    words: alternate traces with equal keys and different event types on one
    context and check every result against the oracle."""
    import torch
    from paper_1411_2239_amd import lib
    a = W.gen_user_requests(n_events=400_000, n_users=500, seed=11)
    rng = np.random.default_rng(5)
    b_rec = a.records.copy()
    b_rec["type"] = rng.permutation(b_rec["type"])
    c_rec = a.records[: 150_001].copy()
    ctx, ids, _ = lib.open_workload(a)
    rb = a.layout.record_bytes
    for name, recs in (("a", a.records), ("b", b_rec), ("a", a.records), ("c", c_rec), ("b", b_rec)):
        print(f"[case] repeated evaluation {name} n={recs.shape[0]}", flush=True)
        dev = torch.from_numpy(recs.view(np.uint8).reshape(-1).copy()).to("cuda:0")
        r = ctx.eval(dev, ids, instances=True, nodes=True)
        torch.cuda.synchronize()
        o = evaluate_workload(a, records=recs)
        compare_full(r, o, len(ids), a.layout.n_keys)
        assert dev.numel() == recs.shape[0] * rb
    ctx.close()


def test_many_tiles_wide_monitors_spread_spine():
    """Four properties of 9-10 states (maps of four dwords) over 9M events:
    2,198 scan tiles, more than two passes of one spine block for records of
    this width, so the spine runs spread over blocks (chunk compositions, their
    scan, the tile prefixes)."""
    big = [W.BATCH_FORMULAS[i] for i in (6, 8, 9, 12)]
    _check(prop_workload(9_000_000, 2, [300, 4000], seed=91, n_props=4, formulas=big), instances=True, nodes=True)
