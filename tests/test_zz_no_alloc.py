"""The no-allocation entry point (ltl4c_eval_noalloc) against ltl4c_eval with a
caller workspace: the same roots, counts, instance keys and verdicts, and
node keys, counts and verdicts, on two calls in a row (the second on a
smaller trace, so stale scratch contents of the first would show), for plain
and parent-event layouts, and the clear refusal of a trace too large for the
scratch."""
import numpy as np
import pytest

from paper_1411_2239_amd import lib
from paper_1411_2239_amd import workloads as W

from _util import prop_workload

pytestmark = pytest.mark.gpu


def _same(a, b, n_props, n_levels):
    import torch
    torch.cuda.synchronize()
    assert np.array_equal(a.root_verdict.cpu().numpy(), b.root_verdict.cpu().numpy())
    assert np.array_equal(a.root_counts.cpu().numpy(), b.root_counts.cpu().numpy())
    sa, sb = a.sizes.cpu().numpy(), b.sizes.cpu().numpy()
    assert np.array_equal(sa, sb)
    ni = int(sa[0])
    assert np.array_equal(a.inst_keys[:ni].cpu().numpy(), b.inst_keys[:ni].cpu().numpy())
    assert np.array_equal(a.inst_verdict.view(n_props, -1)[:, :ni].cpu().numpy(),
                          b.inst_verdict.view(n_props, -1)[:, :ni].cpu().numpy())
    for m in range(1, n_levels):
        nm = int(sa[m])
        assert np.array_equal(a.node_keys[m][:nm].cpu().numpy(), b.node_keys[m][:nm].cpu().numpy())
        assert np.array_equal(a.node_counts[m].view(n_props, -1, 6)[:, :nm].cpu().numpy(),
                              b.node_counts[m].view(n_props, -1, 6)[:, :nm].cpu().numpy())
        assert np.array_equal(a.node_verdict[m].view(n_props, -1)[:, :nm].cpu().numpy(),
                              b.node_verdict[m].view(n_props, -1)[:, :nm].cpu().numpy())


@pytest.mark.parametrize("kind", ["users", "props3", "parent"])
def test_noalloc_equals_workspace_eval_twice(kind):
    import torch
    if kind == "parent":
        # parent events: the segment tree, sample table and run maps live in
        # the scratch as well
        from test_gpu_parent_events import parent_workload
        big = parent_workload(200_000, 2, [40, 300], seed=25, n_props=3)
        small = parent_workload(5_003, 2, [5, 9], seed=26, n_props=3)
        small.layout = big.layout
        L = 2
    elif kind == "users":
        big = W.gen_user_requests(n_events=1_500_000, n_users=2000, seed=21)
        small = W.gen_user_requests(n_events=90_001, n_users=300, seed=22)
        L = 2
    else:
        big = prop_workload(1_000_000, 3, [40, 30, 20], seed=23, n_props=5)
        small = prop_workload(7_777, 3, [5, 4, 3], seed=24, n_props=5, formulas=[s.formula for s in big.props],
                              quants=[s.quants for s in big.props])
        small.layout = big.layout
        L = 3
    print(f"[case] noalloc {kind}: {big.n_events} then {small.n_events} events", flush=True)
    ctx, ids, rec_big = lib.open_workload(big)
    rec_small = torch.from_numpy(np.ascontiguousarray(small.raw())).to("cuda:0")
    for rec, wl in ((rec_big, big), (rec_small, small)):
        n = wl.n_events
        ref = ctx.alloc_result(len(ids), n, instances=True, nodes=True)
        ctx.eval_into(rec, n, ids, ref, ctx.workspace(n, ids))
        ctx.wait()
        got = ctx.alloc_result(len(ids), n, instances=True, nodes=True)
        ctx.eval_noalloc_into(rec, n, ids, got)
        ctx.wait()
        _same(got, ref, len(ids), L)
    ctx.close()


def test_noalloc_refuses_traces_beyond_its_scratch():
    import torch
    wl = W.gen_user_requests(n_events=1000, n_users=10, seed=3)
    ctx, ids, rec = lib.open_workload(wl)
    n_big = 8_000_000
    assert ctx.workspace_bytes(n_big, ids) > 64 << 20
    big = torch.zeros(n_big * 16, dtype=torch.uint8, device="cuda:0")
    got = ctx.alloc_result(len(ids))
    with pytest.raises(lib.LTL4CError) as e:
        ctx.eval_noalloc_into(big, n_big, ids, got)
    assert e.value.status == lib.ENOMEM and "scratch" in str(e.value)
    # the largest trace it takes, by the workspace query
    lo, hi = 1, n_big
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if ctx.workspace_bytes(mid, ids) <= (64 << 20) - 8192:
            lo = mid
        else:
            hi = mid - 1
    print(f"[case] noalloc: largest user/request trace that fits: {lo} events", flush=True)
    ctx.eval_noalloc_into(big, lo, ids, got)
    ctx.wait()
    ctx.close()
