"""Parent events on the device (the proxy-cache case study of Section 5):
an event carrying every key but the innermost joins the cluster of every
instance under its parent.  Every root, count, instance verdict and node of
the HIP path against the oracle, element by element, at 1-3 levels, ragged
sizes, monitors up to 16 states, parents with thousands of parent events,
and the 10M-event proxy trace; the calls that do not take parent events
refuse them."""
import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import workloads as W

from _util import compare_full, pack_keys, prop_workload

pytestmark = pytest.mark.gpu

BIG = ["F(a & X(F(a & X F a)))", "G(a -> X X b)", "(a U b) & (!a U c)", "G(!a | X(b | X c))"]


def parent_workload(n, n_levels, keys, seed, n_props=3, p_parent=0.2, p_other=0.05, formulas=None):
    """prop_workload's records, where a fraction p_parent of the events get a
    type (8..15) that carries every key but the innermost (the innermost key
    field keeps a random value, which must be ignored), and p_other a type
    (16..23) that carries only the innermost key (joins no cluster)."""
    wl = prop_workload(n, n_levels, keys, seed, n_props=n_props, formulas=formulas)
    rng = np.random.Generator(np.random.PCG64(seed + 99))
    u = rng.random(n)
    t = wl.records["type"].copy()
    t[u < p_parent] |= 8
    t[(u >= p_parent) & (u < p_parent + p_other)] |= 16
    wl.records["type"] = t
    full = (1 << n_levels) - 1
    lay = wl.layout
    lay.class_of_type[8:16] = np.arange(8)
    lay.class_of_type[16:24] = np.arange(8)
    lay.key_present[8:16] = full >> 1
    lay.key_present[16:24] = 1 << (n_levels - 1) if n_levels > 1 else 0
    if n_levels == 1:
        lay.key_present[16:24] = 0xFE        # no key 0: for one level these are parent events too
    lay.parent_events = True
    wl.name = f"parent-{seed}"
    return wl


def _check(wl):
    import torch
    from paper_1411_2239_amd import lib
    print(f"[case] {wl.name} n={wl.n_events} levels={wl.layout.n_keys} props={len(wl.props)}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    r = ctx.eval(rec, ids, instances=True, nodes=True)
    torch.cuda.synchronize()
    ctx.close()
    o = evaluate_workload(wl)
    compare_full(r, o, len(ids), wl.layout.n_keys, key_bits=wl.layout.key_bits)
    return r, o


@pytest.mark.parametrize("n,levels,keys", [(1, 2, [3, 3]), (2, 1, [5]), (4097, 1, [37]), (50_000, 2, [40, 30]),
                                           (200_000, 3, [20, 10, 30]), (12_289, 2, [3, 5000])])
def test_parity(n, levels, keys):
    _check(parent_workload(n, levels, keys, seed=n + levels, n_props=4))


@pytest.mark.parametrize("levels", [1, 2])
def test_parity_sixteen_state_monitors(levels):
    keys = [50] if levels == 1 else [30, 40]
    _check(parent_workload(120_000, levels, keys, seed=7 + levels, n_props=4, formulas=BIG))


def test_few_parents_many_parent_events():
    """Half the events are parent events of 4 parents: every gap query walks a
    segment tree of ~16 levels."""
    _check(parent_workload(300_000, 2, [4, 2000], seed=31, n_props=3, p_parent=0.5))


def test_one_level_events_without_keys():
    # for one level a parent event carries no key: it joins every instance
    _check(parent_workload(100_000, 1, [300], seed=41, n_props=3, p_parent=0.1))


def test_no_parent_events_equals_plain_evaluation():
    import torch
    from paper_1411_2239_amd import lib
    wl = parent_workload(80_000, 2, [30, 50], seed=51, n_props=3, p_parent=0.0, p_other=0.0)
    r, o = _check(wl)
    wl.layout.parent_events = False
    ctx, ids, rec = lib.open_workload(wl)
    r2 = ctx.eval(rec, ids, instances=True, nodes=True)
    torch.cuda.synchronize()
    ctx.close()
    compare_full(r2, o, len(ids), 2)


def test_only_parent_events():
    _check(parent_workload(5000, 2, [7, 7], seed=61, n_props=2, p_parent=1.0, p_other=0.0))


def test_proxy_cache_full_size():
    """The 10M-event proxy trace with parent events; and its requests that
    were fetched externally while cached are exactly those the case study's
    literal formula (cached & external on the request event) finds."""
    import torch
    from paper_1411_2239_amd import lib
    wl = W.gen_proxy_cache(10_000_000)
    r, o = _check(wl)
    lit = W.gen_proxy_cache(10_000_000, literal=True)
    r2, o2 = _check(lit)
    n_inst = int(r.sizes[0].item())
    t_temporal = r.inst_verdict.cpu().numpy().reshape(len(wl.props), -1)[0, :n_inst] == lib.TOP
    t_literal = r2.inst_verdict.cpu().numpy().reshape(1, -1)[0, :n_inst] == lib.TOP
    assert np.array_equal(t_temporal, t_literal) and t_temporal.sum() > 0


def test_calls_without_parent_events_refuse_them():
    import torch
    from paper_1411_2239_amd import lib
    wl = parent_workload(1000, 2, [5, 5], seed=71, n_props=1)
    ctx, ids, rec = lib.open_workload(wl)
    with pytest.raises(lib.LTL4CError) as e:
        ctx.eval(rec, ids, instances=True, events=True)
    assert e.value.status == lib.EUNSUPPORTED
    with pytest.raises(lib.LTL4CError) as e:
        ctx.eval_batch(rec, np.array([0, 500, 1000], dtype=np.uint64), ids)
    assert e.value.status == lib.EUNSUPPORTED
    ctx.close()


def test_declared_widths_without_room_for_the_index_are_ranked():
    """The kind bit and the trace index ride in the sort word: declared key
    widths that leave no room for them make the library rank the keys."""
    wl = parent_workload(30_000, 2, [5, 400], seed=81, n_props=2)
    wl.layout.key_bits = [28, 28]
    _check_values(wl)


def _check_values(wl):
    import torch
    from paper_1411_2239_amd import lib
    ctx, ids, rec = lib.open_workload(wl)
    r = ctx.eval(rec, ids, instances=True, nodes=True, key_values=True)
    torch.cuda.synchronize()
    ctx.close()
    o = evaluate_workload(wl)
    r.key_bits = None
    compare_full(r, o, len(ids), 2)
    n_inst = int(r.sizes[0].item())
    assert np.array_equal(r.inst_key_values.cpu().numpy().view(np.uint32).reshape(-1, 2)[:n_inst], o.inst_keys)


@pytest.mark.parametrize("scan_tile", [0, 3, 4, 5])
def test_parity_every_scan_tile(scan_tile):
    """The own events are numbered by the look-back scan (tiles 0-3) or the
    split map scan (4, 5) before the parent kernels recompute the verdicts."""
    import torch
    from paper_1411_2239_amd import lib
    wl = parent_workload(70_001, 2, [30, 200], seed=101 + scan_tile, n_props=3)
    print(f"[case] {wl.name} scan tile {scan_tile}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    ctx.set_option(lib.OPT_SCAN_TILE, scan_tile)
    r = ctx.eval(rec, ids, instances=True, nodes=True)
    torch.cuda.synchronize()
    ctx.close()
    compare_full(r, evaluate_workload(wl), len(ids), 2, key_bits=wl.layout.key_bits)
