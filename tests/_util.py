"""Helpers shared by the test modules (not collected by pytest)."""
from __future__ import annotations

import numpy as np

from paper_1411_2239_amd import workloads as W

FORMULA_POOL = [
    "G(a -> F b)", "(G a) -> (F b)", "G(a -> X b)", "G a | (b U c)", "F(a & X F a)",
    "a U (b U c)", "G(a -> X X b)", "!X a", "X !a", "G F a", "F G a", "(a U b) & (!a U c)",
    "G(a -> (b U c))", "F(a & X(F(a & X F a)))", "X X X a", "G(!a | X(b | X c))", "a", "true", "false",
    "F c & G(b -> F a)", "(a -> X b) U c", "G(a & b -> X !c)",
]


def random_formula(rng, depth=3, props=("a", "b", "c")):
    if depth == 0 or rng.random() < 0.25:
        return rng.choice(list(props) + ["true"])
    op = rng.choice(["!", "X", "F", "G", "&", "|", "U", "->"])
    if op in ("!", "X", "F", "G"):
        return f"{op}({random_formula(rng, depth - 1, props)})"
    return f"({random_formula(rng, depth - 1, props)}) {op} ({random_formula(rng, depth - 1, props)})"


def random_quant(rng):
    kind = rng.choice(["A", "E"])
    op = rng.choice(["<", "<=", ">", ">=", "="])
    if kind == "A":
        den = int(rng.choice([1, 2, 3, 4, 10, 20, 100]))
        num = int(rng.integers(0, den + 1))
        return (kind, op, f"{num}/{den}")
    return (kind, op, int(rng.integers(0, 6)))


def prop_workload(n_events, n_levels, keys_per_level, seed, n_props=3, formulas=None, quants=None,
                  key_bits=None, p_props=(0.3, 0.5, 0.4), n_classes_bits=3):
    """Records with proposition-bit types and n_levels uniform keys."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dt = np.dtype([("ts", "<u4"), ("type", "<u4")] + [(f"k{m}", "<u4") for m in range(max(2, n_levels))])
    rec = np.zeros(n_events, dtype=dt)
    rec["ts"] = np.arange(n_events, dtype=np.uint32)
    typ = np.zeros(n_events, dtype=np.uint32)
    for i, p in enumerate(p_props):
        typ |= (rng.random(n_events) < p).astype(np.uint32) << i
    rec["type"] = typ
    for m in range(n_levels):
        rec[f"k{m}"] = rng.integers(0, keys_per_level[m], size=n_events, dtype=np.uint32)
    rb = dt.itemsize
    names = "abcd"[:len(p_props)]
    ncls = 1 << len(p_props)
    cot = np.zeros(256, dtype=np.uint8)
    kp = np.zeros(256, dtype=np.uint8)
    cot[:ncls] = np.arange(ncls)
    kp[:ncls] = (1 << n_levels) - 1
    kb = key_bits or [max(1, int(k - 1).bit_length()) for k in keys_per_level]
    lay = W.Layout(rb, 4, 4, [8 + 4 * m for m in range(n_levels)], [4] * n_levels, kb, cot, kp,
                   [{names[i] for i in range(len(p_props)) if (c >> i) & 1} for c in range(ncls)])
    if formulas is None:
        formulas = [FORMULA_POOL[int(i)] for i in rng.integers(0, len(FORMULA_POOL), size=n_props)]
    specs = []
    for i, f in enumerate(formulas):
        q = quants[i] if quants is not None else [random_quant(rng) for _ in range(n_levels)]
        specs.append(W.PropertySpec(f, q, f"p{i}"))
    return W.Workload(f"props-{seed}", rec, lay, specs)


def compare_full(r, o, n_props, n_levels, check_instances=True, check_nodes=True, key_bits=None):
    """Element-by-element equality of a GPU EvalResult and an oracle result."""
    rv = r.root_verdict.cpu().numpy()
    assert np.array_equal(rv, o.root_verdict), (rv, o.root_verdict)
    rc = r.root_counts.cpu().numpy().reshape(n_props, 6)
    assert np.array_equal(rc, o.root_counts.astype(np.int64)), (rc, o.root_counts)
    sizes = r.sizes.cpu().numpy()
    n_inst = int(sizes[0])
    assert n_inst == o.inst_keys.shape[0], (n_inst, o.inst_keys.shape)
    for m in range(1, n_levels):
        assert int(sizes[m]) == o.level_keys[m].shape[0], (m, sizes, o.level_keys[m].shape)
    if key_bits is None:
        key_bits = getattr(r, "key_bits", None)
    if check_instances and r.inst_verdict is not None:
        iv = r.inst_verdict.cpu().numpy().reshape(n_props, -1)[:, :n_inst]
        assert np.array_equal(iv, o.inst_verdict)
        if key_bits is not None:
            ik = r.inst_keys.cpu().numpy().view(np.uint64)[:n_inst]
            assert np.array_equal(ik, pack_keys(o.inst_keys, key_bits[:n_levels]))
    if check_nodes and r.node_counts is not None:
        for m in range(1, n_levels):
            nm = int(sizes[m])
            if key_bits is not None and r.node_keys is not None and r.node_keys[m] is not None:
                nk = r.node_keys[m].cpu().numpy().view(np.uint64)[:nm]
                assert np.array_equal(nk, pack_keys(o.level_keys[m], key_bits[:m])), m
            nc = r.node_counts[m].cpu().numpy().reshape(n_props, -1, 6)[:, :nm]
            assert np.array_equal(nc.astype(np.int64), o.level_counts[m].astype(np.int64)), m
            nv = r.node_verdict[m].cpu().numpy().reshape(n_props, -1)[:, :nm]
            assert np.array_equal(nv, o.level_verdict[m]), m


def pack_keys(keys, bits):
    """Pack rows of key values (level 0 most significant) the way inst_keys are reported."""
    out = np.zeros(keys.shape[0], dtype=np.uint64)
    for m, b in enumerate(bits):
        out = (out << np.uint64(b)) | keys[:, m].astype(np.uint64)
    return out
