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


def test_large_trace_full_size_every_instance():
    """500M events, 1M Zipf keys, three properties (3/8/16-state monitors):
    the root verdicts and counts and every instance's key and verdict against
    the C oracle run over key-0 partitions on the host's cores (the root
    counts of disjoint partitions add up)."""
    import torch
    from oracle import parallel
    from oracle.run import oracle_property
    print("[case] large full size 500M events", flush=True)
    wl, rec = W.gen_large_trace_device()
    ctx = lib.Context(0)
    ctx.set_layout(wl.layout)
    ids = [ctx.add_spec(p) for p in wl.props]
    r = ctx.eval(rec, ids, instances=True, capacity=1 << 21)
    n_inst = int(r.sizes[0].item())
    print(f"[case] large: {n_inst} instances on the device; copying the trace to the host", flush=True)
    host = rec.cpu().numpy()
    del rec
    torch.cuda.empty_cache()
    props = [oracle_property(s, wl.layout) for s in wl.props]
    o = parallel.evaluate_partitioned(host, wl.layout, props, n_parts=64)
    print(f"[case] large: oracle done ({o.inst_keys.shape[0]} instances)", flush=True)
    compare_full(r, o, len(ids), 1)
    ctx.close()
