"""Verdict timeline of every instance (the length of its first prefix with a
T or F verdict) through the C ABI, element by element against the oracle."""
import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import workloads as W

from _util import compare_full, prop_workload

pytestmark = pytest.mark.gpu


def _run(wl, **kw):
    import torch
    from paper_1411_2239_amd import lib
    print(f"[case] timeline {wl.name} n={wl.n_events} props={len(wl.props)} levels={wl.layout.n_keys}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    for k, v in kw.items():
        ctx.set_option(getattr(lib, k), v)
    r = ctx.eval(rec, ids, instances=True, timeline=True)
    torch.cuda.synchronize()
    ctx.close()
    o = evaluate_workload(wl)
    compare_full(r, o, len(ids), wl.layout.n_keys)
    n_inst = int(r.sizes[0].item())
    got = r.inst_conclusive.cpu().numpy().view(np.uint32).reshape(len(ids), -1)[:, :n_inst]
    assert np.array_equal(got, o.inst_conc)
    return got


@pytest.mark.parametrize("n,levels,keys", [(200_000, 1, [300]), (200_000, 2, [40, 50]), (4097, 3, [3, 4, 5]),
                                           (100_000, 1, [1])])
def test_timeline_parity(n, levels, keys):
    got = _run(prop_workload(n, levels, keys, seed=90 + levels, n_props=8))
    assert (got != 0xFFFFFFFF).any()


def test_timeline_many_property_groups():
    # 16 properties: several scan launches write their own rows
    _run(prop_workload(60_000, 1, [500], seed=93, n_props=16))


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_timeline_scan_tiles(variant):
    # look-back scan tiles (0-3) and the split map scan's down sweep (4, 5)
    _run(prop_workload(150_000, 2, [20, 30], seed=94, n_props=4), OPT_SCAN_TILE=variant)


@pytest.mark.parametrize("variant", [3, 4, 5])
def test_event_verdicts_scan_tiles(variant):
    _run_events(prop_workload(90_001, 2, [30, 40], seed=96, n_props=5), OPT_SCAN_TILE=variant)


def test_timeline_never_conclusive():
    # G(issue -> F done) has no conclusive finite prefix
    got = _run(W.gen_user_requests(n_events=200_000, n_users=400, seed=95))
    assert (got == 0xFFFFFFFF).all()


def _run_events(wl, **kw):
    import torch
    from paper_1411_2239_amd import lib
    print(f"[case] event verdicts {wl.name} n={wl.n_events} props={len(wl.props)} levels={wl.layout.n_keys} {kw}",
          flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    for k, v in kw.items():
        ctx.set_option(getattr(lib, k), v)
    r = ctx.eval(rec, ids, events=True, timeline=True, instances=True)
    torch.cuda.synchronize()
    ctx.close()
    o = evaluate_workload(wl)
    compare_full(r, o, len(ids), wl.layout.n_keys)
    got = r.event_verdict.cpu().numpy().reshape(len(ids), -1)
    assert np.array_equal(got, o.event_verdict)
    n_inst = int(r.sizes[0].item())
    conc = r.inst_conclusive.cpu().numpy().view(np.uint32).reshape(len(ids), -1)[:, :n_inst]
    assert np.array_equal(conc, o.inst_conc)


@pytest.mark.parametrize("n,levels,keys", [(200_000, 1, [300]), (150_000, 2, [40, 50]), (4097, 3, [3, 4, 5])])
def test_event_verdicts_parity(n, levels, keys):
    _run_events(prop_workload(n, levels, keys, seed=110 + levels, n_props=6))


@pytest.mark.parametrize("variant", [0, 1, 6])
def test_event_verdicts_sort_tiles_with_excluded_events(variant):
    # the trace index rides between class and key bits: every radix digit
    # width and tile shape, and events dropped by the first pass
    wl = prop_workload(120_000, 2, [20, 30], seed=115 + variant, n_props=3, key_bits=[14, 13])
    t = wl.records["type"].copy()
    t[np.random.default_rng(variant).random(wl.n_events) < 0.25] = 300
    wl.records["type"] = t
    wl.layout.type_bytes = 2
    _run_events(wl, OPT_SORT_TILE=variant)


def test_event_verdicts_many_properties():
    _run_events(prop_workload(60_000, 1, [500], seed=118, n_props=16))


def test_event_verdicts_need_room_for_the_trace_index():
    import torch
    from paper_1411_2239_amd import lib
    # a 57-bit binding key leaves no room for a 17-bit trace index
    wl = prop_workload(100_000, 3, [1 << 19] * 3, seed=119, n_props=1, key_bits=[19, 19, 19])
    ctx, ids, rec = lib.open_workload(wl)
    with pytest.raises(lib.LTL4CError) as e:
        ctx.eval(rec, ids, events=True)
    assert e.value.status == lib.EUNSUPPORTED
    ctx.close()


def test_event_verdicts_full_size():
    """The bench's verdict-timeline workload at full size (10M events, 100,000
    Zipf keys, three properties that become conclusive): every event's verdict
    and every instance's first conclusive prefix equal the oracle's."""
    _run_events(W.gen_prop_trace(10_000_000, 100_000, 1.1, seed=7, props=W.timeline_properties()))
