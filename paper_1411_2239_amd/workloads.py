"""Seeded synthetic workloads for LTL4-C monitoring.

This module only draws inputs: record arrays, the record layout, the
event-type table and the property specifications (formula text plus the
quantifier string).  It holds none of the method's arithmetic and is the one
module that both the product path and the test oracle read.

The paper's own case-study traces (Apache runs, Dropbox and YouTube datasets)
are not available; these generators stand in for them with the shapes the
case studies describe: a socket-keyed request/response trace, a two-level
user/request trace with Zipf-skewed request counts, and long single traces
with Zipf-skewed cluster lengths.

Every generator uses numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Layout:
    """Where the event type and the key fields sit inside one record."""
    record_bytes: int
    type_offset: int
    type_bytes: int
    key_offsets: list
    key_bytes: list
    key_bits: list                  # declared width of every key value
    class_of_type: np.ndarray       # [256] uint8
    key_present: np.ndarray         # [256] uint8, bit m = the type carries key m
    class_props: list               # class -> set of propositions that hold
    type_names: dict = field(default_factory=dict)
    # data predicates (offset, bytes, op, value), op 0..5 = < <= > >= == !=;
    # an event's class is class_of_type[type] + (holding predicates' bits) << pred_shift
    preds: list = field(default_factory=list)
    pred_shift: int = 0
    # parent events: an event whose type carries every key but the innermost
    # joins the cluster of every instance under its parent
    parent_events: bool = False

    @property
    def n_keys(self):
        return len(self.key_offsets)

    @property
    def n_classes(self):
        return len(self.class_props)


@dataclass
class PropertySpec:
    """phi = Q_0 ... Q_{n-1} psi: quantifiers as (kind, op, const) with kind
    'A' (percentage) or 'E' (instance count); const is a fraction string for
    'A' and an integer for 'E'."""
    formula: str
    quants: list
    name: str = ""


@dataclass
class Workload:
    name: str
    records: np.ndarray            # structured array
    layout: Layout
    props: list                    # [PropertySpec]

    @property
    def n_events(self):
        return int(self.records.shape[0])

    def raw(self):
        return self.records.view(np.uint8).reshape(-1)


def _type_table(n_types, class_of, all_keys_mask):
    cot = np.zeros(256, dtype=np.uint8)
    kp = np.zeros(256, dtype=np.uint8)
    for t in range(n_types):
        cot[t] = class_of[t]
        kp[t] = all_keys_mask
    return cot, kp


REC12 = np.dtype([("ts", "<u4"), ("type", "<u2"), ("pad", "<u2"), ("key", "<u4")])
REC16 = np.dtype([("ts", "<u4"), ("type", "<u4"), ("k0", "<u4"), ("k1", "<u4")])


def socket_layout():
    cot, kp = _type_table(4, [0, 1, 2, 3], 0b1)
    return Layout(12, 4, 2, [8], [4], [10], cot, kp,
                  [set(), {"receive"}, {"respond"}, set()],
                  {0: "open", 1: "receive", 2: "respond", 3: "close"})


def socket_properties():
    # Case study 1: at least 95% of sockets answer every request.  The
    # formula is printed in two ways in the paper; both are monitored.
    return [PropertySpec("G(receive -> F respond)", [("A", ">=", "19/20")], "sockets-G(r->Fs)"),
            PropertySpec("(G receive) -> (F respond)", [("A", ">=", "19/20")], "sockets-(Gr)->(Fs)")]


def gen_sockets(n_events=100_000, n_sockets=1000, seed=0x14112239 + 1):
    """Single quantifier over sockets; 12-byte records."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rec = np.zeros(n_events, dtype=REC12)
    rec["ts"] = np.arange(n_events, dtype=np.uint32)
    rec["type"] = rng.choice(4, size=n_events, p=[0.1, 0.5, 0.35, 0.05]).astype(np.uint16)
    rec["key"] = rng.integers(0, n_sockets, size=n_events, dtype=np.uint32)
    lay = socket_layout()
    lay.key_bits = [max(1, int(n_sockets - 1).bit_length())]
    return Workload("sockets", rec, lay, socket_properties())


def user_request_layout(user_bits=14, req_bits=22):
    cot, kp = _type_table(4, [0, 1, 2, 3], 0b11)
    return Layout(16, 4, 4, [8, 12], [4, 4], [user_bits, req_bits], cot, kp,
                  [{"issue"}, set(), {"done"}, set()],
                  {0: "issue", 1: "progress", 2: "done", 3: "other"})


def user_request_properties():
    return [PropertySpec("G(issue -> F done)", [("E", ">=", 500), ("A", ">=", "9/10")],
                         "users-E>=500-A>=0.9")]


def gen_user_requests(n_events=10_000_000, n_users=10_000, zipf_s=1.2, p_done=0.95,
                      seed=0x14112239 + 2):
    """Two nested quantifiers (user, request); 16-byte records.

    Request counts per user follow Zipf(zipf_s) over user ranks.  A request
    emits an issue event, a geometric number (mean 1) of progress events and,
    with probability p_done, a done event.  Events get random start times and
    exponential gaps; the trace is their time order, topped up with type-3
    events on existing requests to exactly n_events.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    mean_events = 1.0 + 1.0 + p_done
    n_req = max(n_users, int(n_events / mean_events))
    ranks = np.arange(1, n_users + 1, dtype=np.float64)
    w = ranks ** (-zipf_s)
    per_user = np.maximum(1, np.round(n_req * w / w.sum())).astype(np.int64)
    n_req = int(per_user.sum())
    user_ids = rng.permutation(n_users).astype(np.uint32)
    req_user = np.repeat(user_ids, per_user)
    req_ids = rng.permutation(n_req).astype(np.uint32)
    n_prog = rng.geometric(0.5, size=n_req) - 1
    done = rng.random(n_req) < p_done
    per_req = 1 + n_prog + done.astype(np.int64)
    # drop whole requests from the end until the trace fits
    csum = np.cumsum(per_req)
    keep = int(np.searchsorted(csum, n_events, side="right"))
    req_user, req_ids, n_prog, done, per_req = (a[:keep] for a in (req_user, req_ids, n_prog, done, per_req))
    total = int(per_req.sum())
    start = rng.random(keep) * 1e6
    ev_req = np.repeat(np.arange(keep), per_req)
    first = np.concatenate([[0], np.cumsum(per_req)[:-1]])
    pos_in_req = np.arange(total) - np.repeat(first, per_req)
    gaps = rng.exponential(1.0, size=total)
    gaps[first] = 0.0
    # time = start + cumulative gap inside the request
    cg = np.cumsum(gaps)
    cg = cg - np.repeat(cg[first], per_req)
    t = start[ev_req] + cg
    etype = np.where(pos_in_req == 0, 0, 1).astype(np.uint32)
    last = first + per_req - 1
    etype[last[done]] = 2
    n_noise = n_events - total
    if n_noise > 0:
        nr = rng.integers(0, keep, size=n_noise)
        t = np.concatenate([t, rng.random(n_noise) * 1e6])
        ev_req = np.concatenate([ev_req, nr])
        etype = np.concatenate([etype, np.full(n_noise, 3, dtype=np.uint32)])
    order = np.argsort(t, kind="stable")
    rec = np.zeros(n_events, dtype=REC16)
    rec["ts"] = np.arange(n_events, dtype=np.uint32)
    rec["type"] = etype[order]
    rec["k0"] = req_user[ev_req[order]]
    rec["k1"] = req_ids[ev_req[order]]
    lay = user_request_layout(max(1, int(n_users - 1).bit_length()), max(1, int(n_req - 1).bit_length()))
    return Workload("users", rec, lay, user_request_properties())


CHUNK_MAX = 4 << 20          # largest upload chunk, bytes


def chunk_upload_layout(n_preds=1, user_bits=14):
    """Records {ts, type, user, avg_chunk}: type 0 = upload, 1 = other; the
    propositions 'small' (avg_chunk < CHUNK_MAX) and, with n_preds = 2,
    'active' (avg_chunk != 0) are data predicates on the record, class bits
    1 and 2 above the type's letter."""
    cot = np.zeros(256, dtype=np.uint8)
    cot[1] = 1
    kp = np.zeros(256, dtype=np.uint8)
    kp[0] = kp[1] = 1
    preds = [(12, 4, 0, CHUNK_MAX)]                  # avg_chunk < CHUNK_MAX
    names = ["small"]
    if n_preds >= 2:
        preds.append((12, 4, 5, 0))                  # avg_chunk != 0
        names.append("active")
    props = []
    for c in range(2 << len(preds)):
        ps = {"upload"} if (c & 1) == 0 else set()
        ps |= {names[q] for q in range(len(preds)) if (c >> (1 + q)) & 1}
        props.append(ps)
    return Layout(16, 4, 4, [8], [4], [user_bits], cot, kp, props, {0: "upload", 1: "other"},
                  preds=preds, pred_shift=1)


def chunk_upload_properties(n_preds=1):
    out = [PropertySpec("F small", [("A", "=", 1)], "users-A=1-F-small"),
           PropertySpec("G(upload -> F small)", [("A", ">=", "19/20")], "users-A>=0.95-G(upload->F small)")]
    if n_preds >= 2:
        out.append(PropertySpec("G(active -> small) | F(upload & small)", [("E", ">=", 10)], "users-E>=10-active"))
    return out


def gen_chunk_uploads(n_events=10_000_000, n_users=10_000, zipf_s=1.1, p_heavy=0.02, n_preds=1,
                      seed=0x14112239 + 6):
    """Cloud-storage fairness shape (Section 5, second case study): every
    event carries the user's current average chunk size.  Users act with
    Zipf(zipf_s) frequencies; a fraction p_heavy of them only ever uploads
    maximum-size chunks (average at CHUNK_MAX), the others report averages
    below it, sometimes exactly at it, sometimes 0 (no upload yet)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ranks = zipf_ranks(rng, n_events, n_users, zipf_s)
    user_of_rank = rng.permutation(n_users).astype(np.uint32)
    user = user_of_rank[ranks]
    heavy = rng.random(n_users) < p_heavy
    typ = (rng.random(n_events) < 0.4).astype(np.uint32)          # 0 = upload (60 %)
    avg = rng.integers(1, CHUNK_MAX, size=n_events, dtype=np.int64)
    u = rng.random(n_events)
    avg[u < 0.05] = CHUNK_MAX
    avg[(u >= 0.05) & (u < 0.08)] = 0
    avg[heavy[user]] = CHUNK_MAX
    rec = np.zeros(n_events, dtype=REC16)
    rec["ts"] = np.arange(n_events, dtype=np.uint32)
    rec["type"] = typ
    rec["k0"] = user
    rec["k1"] = avg.astype(np.uint32)
    lay = chunk_upload_layout(n_preds, max(1, int(n_users - 1).bit_length()))
    return Workload("chunks", rec, lay, chunk_upload_properties(n_preds))


def prop_layout(n_props=3, n_levels=1, key_bits=None):
    """16-byte records whose type field is a bit set of propositions a, b, c, ...

    Class = type; class c carries the propositions whose bit is set in c.
    """
    names = "abcd"[:n_props]
    n_cls = 1 << n_props
    cot, kp = _type_table(n_cls, list(range(n_cls)), (1 << n_levels) - 1)
    offs = [8, 12][:n_levels]
    kb = key_bits or [32] * n_levels
    return Layout(16, 4, 4, offs, [4] * n_levels, kb, cot, kp,
                  [{names[i] for i in range(n_props) if (c >> i) & 1} for c in range(n_cls)])


def zipf_ranks(rng, n, n_ranks, s, dtype=np.float64):
    """Draw n ranks in [0, n_ranks) with P(r) proportional to (r+1)^-s."""
    w = np.arange(1, n_ranks + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return np.minimum(np.searchsorted(cdf.astype(dtype), rng.random(n, dtype=dtype), side="right"), n_ranks - 1)


def timeline_properties():
    """Properties over the propositions a, b, c of gen_prop_trace whose
    instances do reach a conclusive verdict on finite prefixes."""
    return [PropertySpec("F(a & X b)", [("A", ">=", "1/2")], "A>=1/2 F(a & X b)"),
            PropertySpec("G(b | c)", [("E", ">=", 100)], "E>=100 G(b | c)"),
            PropertySpec("!c U a", [("A", ">", "1/4")], "A>1/4 (!c U a)")]


def gen_prop_trace(n_events, n_keys, zipf_s, p_props=(0.02, 0.9, 0.5), seed=0, key_space_bits=32,
                   props=None, name="proptrace"):
    """One long trace: proposition bits drawn independently, keys Zipf-skewed
    over n_keys ranks and mapped to distinct random values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ranks = zipf_ranks(rng, n_events, n_keys, zipf_s)
    if key_space_bits >= 32:
        vals = np.unique(rng.integers(0, 1 << 32, size=int(n_keys * 1.2) + 16, dtype=np.uint64))
        while vals.size < n_keys:
            vals = np.unique(np.concatenate([vals, rng.integers(0, 1 << 32, size=n_keys, dtype=np.uint64)]))
        key_of_rank = rng.permutation(vals)[:n_keys].astype(np.uint32)
    else:
        key_of_rank = rng.permutation(1 << key_space_bits)[:n_keys].astype(np.uint32)
    typ = np.zeros(n_events, dtype=np.uint32)
    for i, p in enumerate(p_props):
        typ |= (rng.random(n_events) < p).astype(np.uint32) << i
    rec = np.zeros(n_events, dtype=REC16)
    rec["ts"] = np.arange(n_events, dtype=np.uint32)
    rec["type"] = typ
    rec["k0"] = key_of_rank[ranks]
    lay = prop_layout(len(p_props), 1, [key_space_bits])
    return Workload(name, rec, lay, props or [])


# --- proxy cache (Section 5, third case study) ---------------------------------
# Event types of the proxy-cache trace.  A cache insertion or eviction names
# only the video; a request and its progress and completion events name the
# video and the request.  Every request event tells whether it was served from
# the cache, fetched from outside, or fetched from outside although the video
# was cached (the fault the case study looks for).
PROXY_TYPES = {0: "insert", 1: "evict", 2: "request from cache", 3: "request fetched externally",
               4: "request fetched externally while cached", 5: "progress", 6: "done"}


def proxy_cache_layout(parent_events=True, vid_bits=12, req_bits=22):
    """Two quantifier levels (video, request).  With parent_events the cache
    insertions and evictions of a video join the cluster of every request of
    the video."""
    cot = np.zeros(256, dtype=np.uint8)
    kp = np.zeros(256, dtype=np.uint8)
    cot[:7] = np.arange(7)
    kp[0:2] = 0b01
    kp[2:7] = 0b11
    class_props = [{"insert"}, {"evict"}, {"request", "cached"}, {"request", "external"},
                   {"request", "external", "cached"}, {"progress"}, {"done"}]
    return Layout(16, 4, 4, [8, 12], [4, 4], [vid_bits, req_bits], cot, kp, class_props, dict(PROXY_TYPES),
                  parent_events=parent_events)


def proxy_cache_properties():
    """With parent events: at least 99% of videos have no request fetched
    externally while the video was inserted and not yet evicted (the case
    study's E=0 over requests, with the cache state taken from the video's
    own events), and 95% of videos complete 90% of their requests."""
    return [PropertySpec("F(insert & (!evict U external))", [("A", ">=", "99/100"), ("E", "=", 0)],
                         "A>=0.99 v: E=0 r: F(insert & (!evict U external))"),
            PropertySpec("G(request -> F done)", [("A", ">=", "19/20"), ("A", ">=", "9/10")],
                         "A>=0.95 v: A>=0.9 r: G(request -> F done)")]


def proxy_cache_literal_properties():
    """The case study's formula as printed: the leaf is the proposition
    cached & external, read at the first event of the request's cluster (its
    request event, without parent events)."""
    return [PropertySpec("cached & external", [("A", ">=", "99/100"), ("E", "=", 0)],
                         "A>=0.99 v: E=0 r: cached & external")]


def distinct_u32(rng, k):
    """k distinct random 32-bit values, in random order."""
    vals = np.unique(rng.integers(0, 1 << 32, size=int(k * 1.1) + 16, dtype=np.uint64))
    while vals.size < k:
        vals = np.unique(np.concatenate([vals, rng.integers(0, 1 << 32, size=k, dtype=np.uint64)]))
    return rng.permutation(vals)[:k].astype(np.uint32)


def gen_proxy_cache(n_events=10_000_000, n_videos=4096, zipf_s=1.0, mean_changes=4.0, p_fault=0.002,
                    mean_progress=1.5, p_done=0.95, seed=0x14112239 + 6, parent_events=True, literal=False,
                    wide_ids=False):
    """A proxy trace: requests for videos with Zipf popularity; each video's
    cache state alternates at Poisson(mean_changes) random times (the first
    change inserts it); a request while cached is served from the cache, but
    with probability p_fault fetched externally; a request while not cached is
    fetched externally.  Each request has Geometric(mean_progress) progress
    events and, with probability p_done, a completion.  The trace is the
    first n_events events in time order.  Keys: videos a seeded permutation of
    0..n_videos-1, requests one of 0..R-1; with wide_ids, distinct random
    32-bit values for both (a 64-bit composite key)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per_req = 1.0 + mean_progress + p_done
    n_req = int(n_events / per_req * 1.05) + 16
    vid_rank = zipf_ranks(rng, n_req, n_videos, zipf_s)
    t_req = rng.random(n_req)
    # cache change points, per video in time order
    n_chg = rng.poisson(mean_changes, size=n_videos)
    chg_vid = np.repeat(np.arange(n_videos), n_chg)
    chg_t = rng.random(chg_vid.size)
    o = np.lexsort((chg_t, chg_vid))
    chg_vid, chg_t = chg_vid[o], chg_t[o]
    first = np.concatenate([[0], np.cumsum(n_chg)[:-1]])
    chg_k = np.arange(chg_vid.size) - first[chg_vid]          # 0-based change index in the video
    # the state at a request: the parity of the changes before it
    before = np.searchsorted(chg_vid.astype(np.float64) + chg_t, vid_rank.astype(np.float64) + t_req) - first[vid_rank]
    cached = (before & 1) == 1
    fault = rng.random(n_req) < p_fault
    req_type = np.where(cached, np.where(fault, 4, 2), 3).astype(np.uint32)
    n_prog = rng.geometric(1.0 / (1.0 + mean_progress), size=n_req) - 1
    done = rng.random(n_req) < p_done
    gap = 1e-6
    # events: requests, progress, completions, cache changes
    prog_req = np.repeat(np.arange(n_req), n_prog)
    prog_k = np.arange(prog_req.size) - np.repeat(np.cumsum(n_prog) - n_prog, n_prog)
    t = np.concatenate([t_req, t_req[prog_req] + gap * (1 + prog_k) * rng.random(prog_req.size),
                        t_req[done] + gap * (2 + n_prog[done]), chg_t])
    typ = np.concatenate([req_type, np.full(prog_req.size, 5, np.uint32), np.full(int(done.sum()), 6, np.uint32),
                          np.where(chg_k % 2 == 0, 0, 1).astype(np.uint32)])
    vid = np.concatenate([vid_rank, vid_rank[prog_req], vid_rank[done], chg_vid])
    req = np.concatenate([np.arange(n_req), prog_req, np.nonzero(done)[0], np.zeros(chg_vid.size, np.int64)])
    order = np.argsort(t, kind="stable")[:n_events]
    if order.size < n_events:
        raise ValueError("generated too few events")
    if wide_ids:
        vid_key = distinct_u32(rng, n_videos)
        req_key = distinct_u32(rng, n_req)
    else:
        vid_key = rng.permutation(n_videos).astype(np.uint32)
        req_key = rng.permutation(n_req).astype(np.uint32)
    rec = np.zeros(n_events, dtype=REC16)
    rec["ts"] = np.arange(n_events, dtype=np.uint32)
    rec["type"] = typ[order]
    rec["k0"] = vid_key[vid[order]]
    parent = typ[order] < 2
    rec["k1"] = np.where(parent, 0, req_key[req[order]])
    vb = 32 if wide_ids else max(1, int(n_videos - 1).bit_length())
    rb = 32 if wide_ids else max(1, int(n_req - 1).bit_length())
    lay = proxy_cache_layout(parent_events and not literal, vb, rb)
    props = proxy_cache_literal_properties() if literal else proxy_cache_properties()
    return Workload("proxy", rec, lay, props)


def serving_layout(n_streams=64, users=1000, bindings=100_000):
    cot, kp = _type_table(4, [0, 1, 2, 3], 0b11)
    return Layout(16, 4, 1, [8, 12], [4, 4],
                  [max(1, int(users - 1).bit_length()), max(1, int(bindings - 1).bit_length())], cot, kp,
                  [{"issue"}, set(), {"done"}, set()],
                  {0: "issue", 1: "progress", 2: "done", 3: "other"})


def gen_serving_pool(stream, events, users=1000, bindings=100_000, zipf_s=1.2, seed=0x14112239 + 5):
    """Event pool of one log stream: `bindings` (user, req) pairs whose users
    follow Zipf(zipf_s) shares over `users` users; every event picks a
    binding uniformly; types issue/progress/done/other with probabilities
    0.3/0.3/0.35/0.05.  16-byte records in stream order."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919 * stream))
    user_of = zipf_ranks(rng, bindings, users, zipf_s).astype(np.uint32)
    req_ids = rng.permutation(bindings).astype(np.uint32)
    b = rng.integers(0, bindings, size=events)
    rec = np.zeros(events, dtype=REC16)
    rec["ts"] = np.arange(events, dtype=np.uint32)
    rec["type"] = rng.choice(4, size=events, p=[0.3, 0.3, 0.35, 0.05]).astype(np.uint32)
    rec["k0"] = user_of[b]
    rec["k1"] = req_ids[b]
    return rec


def serving_schedule(n_chunks, n_streams=64, offered_events_per_s=2e9, min_chunk=4096, max_chunk=262_144,
                     seed=0x14112239 + 6):
    """Open-loop arrivals: chunk sizes log-uniform in [min_chunk, max_chunk],
    streams uniform, Poisson arrivals at the offered aggregate event rate.
    Returns (arrival seconds, stream, size) arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.floor(np.exp(rng.uniform(np.log(min_chunk), np.log(max_chunk), size=n_chunks))).astype(np.int64)
    mean = (max_chunk - min_chunk) / (np.log(max_chunk) - np.log(min_chunk))
    gaps = rng.exponential(mean / offered_events_per_s, size=n_chunks)
    return np.cumsum(gaps), rng.integers(0, n_streams, size=n_chunks), sizes


# Sixteen LTL bodies over {a, b, c} of nesting depth <= 4, drawn by a seeded
# random search so that their minimal monitors over the 8 event classes have
# 3 to 16 states (3, 4, 5, ..., 16, plus a second 3- and 5-state one).
BATCH_FORMULAS = [
    "G(a -> X b)",
    "a U (b U c)",
    "G(a -> X X b)",
    "X X X a",
    "(!(X(G(b)))) & ((G(X(c))) -> (c))",
    "G((X(X(c))) U (G(G(b))))",
    "(X(X(a))) -> ((X(!(a))) -> (((c) -> (a)) U (G(a))))",
    "((b) U (((a) U (a)) U (G(a)))) | ((F((c) | (b))) & ((true) & ((c) U (a))))",
    "(!(X(X(a)))) | (((G(a)) | (F(b))) U (X(G(a))))",
    "(((X(b)) & (F(a))) | (G((c) -> (b)))) | ((G(X(b))) | (X(G(a))))",
    "((X(X(c))) -> (G((true) -> (a)))) -> (G(c))",
    "((!(a)) U (X(!(b)))) U ((G((c) U (c))) | (((c) U (b)) -> (G(b))))",
    "(((!(a)) U ((a) & (c))) -> ((X(a)) & ((b) U (a)))) U (X(X(b)))",
    "(!(G(a) | c)) U (X(X(b)))",
    "F(a & X F a)",
    "G a | (b U c)",
]
BATCH_QUANTS = [("A", ">=", "9/10"), ("E", ">=", 10), ("A", "=", 1), ("E", "<=", 5),
                ("A", ">", "1/2"), ("E", "=", 3), ("A", "<", "1/4"), ("E", ">", 100)]


def batch_properties(n=16):
    return [PropertySpec(BATCH_FORMULAS[i], [BATCH_QUANTS[i % len(BATCH_QUANTS)]], f"batch{i}") for i in range(n)]


def gen_batch(n_traces=4096, min_len=1000, max_len=1_000_000, p_prop=0.3, zipf_s=1.1, seed=0x14112239 + 4,
              n_props=16):
    """Many independent traces: lengths log-uniform in [min_len, max_len];
    three proposition bits, each Bernoulli(p_prop); keys Zipf(zipf_s) over
    max(16, length // 256) ranks mapped to a permutation of 0..K-1.
    Returns (Workload of the concatenated records, offsets)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = np.floor(np.exp(rng.uniform(np.log(min_len), np.log(max_len), size=n_traces))).astype(np.int64)
    offsets = np.concatenate([[0], np.cumsum(lengths)])
    rec = np.zeros(int(offsets[-1]), dtype=REC16)
    kmax = 16
    for t in range(n_traces):
        L = int(lengths[t])
        a, b = int(offsets[t]), int(offsets[t + 1])
        K = max(16, L // 256)
        kmax = max(kmax, K)
        ranks = zipf_ranks(rng, L, K, zipf_s, dtype=np.float32)
        perm = rng.permutation(K).astype(np.uint32)
        bits = (rng.random((3, L), dtype=np.float32) < p_prop).astype(np.uint32)
        rec["type"][a:b] = bits[0] | (bits[1] << 1) | (bits[2] << 2)
        rec["k0"][a:b] = perm[ranks]
        rec["ts"][a:b] = np.arange(L, dtype=np.uint32)
    lay = prop_layout(3, 1, [max(1, int(kmax - 1).bit_length())])
    lay.type_bytes = 1          # the type values fit one byte: no exclusion bit in the sort key
    return Workload("batch", rec, lay, batch_properties(n_props)), offsets


# One long trace, three properties evaluated in one pass; the monitors have 3,
# 8 and 16 states (the last two bodies come from the same seeded search).
LARGE_PROPERTIES = [
    PropertySpec("G(a -> X b)", [("A", ">=", "99/100")], "large-3"),
    PropertySpec("G((X(X(c))) U (G(G(b))))", [("E", ">=", 100_000)], "large-8"),
    PropertySpec("(!(G(a) | c)) U (X(X(b)))", [("A", ">", "1/4")], "large-16"),
]


def gen_large_trace(n_events=500_000_000, n_keys=1_000_000, zipf_s=1.1, p_props=(0.02, 0.9, 0.5),
                    seed=0x14112239 + 3, block=1 << 24):
    """A single long trace of 16-byte records: proposition bits a, b, c drawn
    independently; keys Zipf(zipf_s) over n_keys ranks, each rank mapped to a
    distinct random 32-bit value.  Generated in blocks to bound memory."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = np.unique(rng.integers(0, 1 << 32, size=int(n_keys * 1.1) + 64, dtype=np.uint64))
    while vals.size < n_keys:
        vals = np.unique(np.concatenate([vals, rng.integers(0, 1 << 32, size=n_keys, dtype=np.uint64)]))
    key_of_rank = rng.permutation(vals)[:n_keys].astype(np.uint32)
    w = np.arange(1, n_keys + 1, dtype=np.float64) ** (-zipf_s)
    cdf = (np.cumsum(w) / w.sum()).astype(np.float32)
    rec = np.zeros(n_events, dtype=REC16)
    for a in range(0, n_events, block):
        b = min(n_events, a + block)
        L = b - a
        ranks = np.minimum(np.searchsorted(cdf, rng.random(L, dtype=np.float32), side="right"), n_keys - 1)
        t = np.zeros(L, dtype=np.uint32)
        for i, p in enumerate(p_props):
            t |= (rng.random(L, dtype=np.float32) < p).astype(np.uint32) << i
        rec["type"][a:b] = t
        rec["k0"][a:b] = key_of_rank[ranks]
        rec["ts"][a:b] = np.arange(a, b, dtype=np.uint64).astype(np.uint32)
    lay = prop_layout(3, 1, [32])
    lay.type_bytes = 1
    return Workload("large", rec, lay, list(LARGE_PROPERTIES))


def gen_large_trace_device(n_events=500_000_000, n_keys=1_000_000, zipf_s=1.1, p_props=(0.02, 0.9, 0.5),
                           seed=0x14112239 + 3, device="cuda:0", block=1 << 26):
    """The gen_large_trace workload drawn directly in device memory with
    torch's seeded generator (for sizes where host generation is slow).
    Returns (Workload with records=None, device uint8 tensor of the records)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    vals = torch.unique(torch.randint(0, 1 << 32, (int(n_keys * 1.1) + 64,), generator=g, device=device,
                                      dtype=torch.int64))
    while vals.numel() < n_keys:
        more = torch.randint(0, 1 << 32, (n_keys,), generator=g, device=device, dtype=torch.int64)
        vals = torch.unique(torch.cat([vals, more]))
    key_of_rank = vals[torch.randperm(vals.numel(), generator=g, device=device)[:n_keys]]
    w = torch.arange(1, n_keys + 1, dtype=torch.float64, device=device) ** (-zipf_s)
    cdf = torch.cumsum(w, 0) / w.sum()
    rec = torch.empty((n_events, 4), dtype=torch.int32, device=device)
    for a in range(0, n_events, block):
        b = min(n_events, a + block)
        L = b - a
        ranks = torch.clamp(torch.searchsorted(cdf, torch.rand(L, generator=g, device=device, dtype=torch.float64),
                                               right=True), max=n_keys - 1)
        t = torch.zeros(L, dtype=torch.int32, device=device)
        for i, p in enumerate(p_props):
            t |= (torch.rand(L, generator=g, device=device) < p).to(torch.int32) << i
        rec[a:b, 0] = torch.arange(a, b, device=device, dtype=torch.int64).to(torch.int32)
        rec[a:b, 1] = t
        rec[a:b, 2] = key_of_rank[ranks].to(torch.int64).to(torch.int32)
        rec[a:b, 3] = 0
    lay = prop_layout(3, 1, [32])
    lay.type_bytes = 1
    return Workload("large", None, lay, list(LARGE_PROPERTIES)), rec.view(torch.uint8).reshape(-1)
