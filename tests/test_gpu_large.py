"""One long trace with three properties of 3-, 8- and 16-state monitors in
one pass.  Scaled down: full parity.  Full size (500M events): the oracle
checks every instance of a key partition (keys with value % 128 == 0) and
properties that hold at any size (counts sum to the number of instances)."""
import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import lib
from paper_1411_2239_amd import workloads as W

from _util import compare_full

pytestmark = pytest.mark.gpu


def test_large_trace_scaled_down_full_parity():
    import torch
    wl = W.gen_large_trace(3_000_000, 20_000, seed=11)
    print(f"[case] large scaled n={wl.n_events}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    r = ctx.eval(rec, ids, instances=True)
    compare_full(r, evaluate_workload(wl), len(ids), 1)
    ctx.close()


def test_large_trace_full_size_sampled():
    import torch
    print("[case] large full size 500M events", flush=True)
    wl, rec = W.gen_large_trace_device()
    n = rec.numel() // 16
    ctx = lib.Context(0)
    ctx.set_layout(wl.layout)
    ids = [ctx.add_spec(p) for p in wl.props]
    r = ctx.eval(rec, ids, instances=True)
    n_inst = int(r.sizes[0].item())
    keys = r.inst_keys[:n_inst].cpu().numpy().astype(np.uint64)
    iv = r.inst_verdict.view(len(ids), -1)[:, :n_inst].cpu().numpy()
    # properties that hold at any size
    rc = r.root_counts.cpu().numpy().reshape(len(ids), 6)
    assert (rc.sum(axis=1) == n_inst).all()
    for p in range(len(ids)):
        assert np.array_equal(np.bincount(iv[p], minlength=6), rc[p])
    assert np.all(np.diff(keys.astype(np.int64)) > 0)
    # a key partition, evaluated by the oracle on exactly its events
    rv = rec.view(torch.int32).view(-1, 4)
    sel = (rv[:, 2].to(torch.int64) & 0xFFFFFFFF) % 128 == 0
    part = rv[sel].cpu().numpy().view(np.uint8).reshape(-1)
    o = evaluate_workload(wl, records=part)
    mine = (keys % 128) == 0
    assert np.array_equal(keys[mine], o.inst_keys[:, 0].astype(np.uint64))
    assert np.array_equal(iv[:, mine], o.inst_verdict)
    ctx.close()
