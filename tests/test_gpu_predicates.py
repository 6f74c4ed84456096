"""Data predicates as class bits (the cloud-storage case study of Section 5:
every event carries the user's average chunk size, compared with a maximum)
through the C ABI, element by element against the oracle."""
import ctypes

import numpy as np
import pytest

from oracle.run import evaluate_workload
from paper_1411_2239_amd import workloads as W

from _util import compare_full

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_preds,n,users", [(1, 300_000, 2_000), (2, 300_000, 2_000), (2, 4097, 37)])
def test_predicate_classes_parity(n_preds, n, users):
    import torch
    from paper_1411_2239_amd import lib
    wl = W.gen_chunk_uploads(n, users, n_preds=n_preds, seed=80 + n_preds)
    print(f"[case] chunk uploads n={n} preds={n_preds}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    r = ctx.eval(rec, ids, instances=True)
    torch.cuda.synchronize()
    ctx.close()
    compare_full(r, evaluate_workload(wl), len(ids), 1)


def test_predicate_classes_full_size():
    import torch
    from paper_1411_2239_amd import lib
    wl = W.gen_chunk_uploads(n_preds=2)
    print(f"[case] chunk uploads full size n={wl.n_events}", flush=True)
    ctx, ids, rec = lib.open_workload(wl)
    r = ctx.eval(rec, ids, instances=True)
    torch.cuda.synchronize()
    ctx.close()
    compare_full(r, evaluate_workload(wl), len(ids), 1)


def test_predicate_layout_validation():
    from paper_1411_2239_amd import lib
    ctx = lib.Context(0)
    bad = [
        (dict(preds=[(12, 4, 0, 1)] * 4), lib.EUNSUPPORTED),      # more than 3 predicates
        (dict(preds=[(12, 4, 6, 1)]), lib.EINVAL),                 # unknown comparison
        (dict(preds=[(13, 4, 0, 1)]), lib.EINVAL),                 # misaligned field
        (dict(preds=[(12, 4, 0, 1)], pred_shift=3), lib.EINVAL),   # letter 1 + 8 >= 4 classes
    ]
    for change, status in bad:
        lay = W.chunk_upload_layout(1)
        for k, v in change.items():
            setattr(lay, k, v)
        with pytest.raises(lib.LTL4CError) as e:
            ctx.set_layout(lay)
        assert e.value.status == status, (change, e.value.status)
    ctx.set_layout(W.chunk_upload_layout(2))
    ctx.close()
