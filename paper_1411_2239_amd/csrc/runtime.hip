// Host runtime of libltl4c: the C ABI of include/ltl4c.h.
//
// Validates descriptors, keeps per-context device copies of the monitor
// tables and quantifiers ("plans"), lays out the caller's workspace and
// enqueues the kernel sequence of one evaluation on the context's stream:
//   zero -> classify -> radix passes -> scan -> (zero, count) per level
//   -> finalize
// which is Algorithm 1 (SortTrace, SpawnMonitors/Distribute as one flat scan,
// ApplyQuantifiers level by level) without host round trips.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "ltl4c.h"

using namespace ltl4c;

namespace {

thread_local std::string g_last_error = "";

int32_t fail(int32_t code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(LTL4C_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

struct MonitorHost {
    uint32_t n_states, n_classes, q0;
    std::vector<uint8_t> delta, label;
};

struct Timed {
    const char* name;
    hipEvent_t start, stop;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

uint32_t bits_for(uint32_t n_values) {  // bits to hold values 0..n_values-1
    uint32_t b = 0;
    while ((1u << b) < n_values) ++b;
    return b;
}

}  // namespace

// Scratch memory of the no-allocation entry point (ltl4c_eval_noalloc): a
// file-scope device array, so that a call needs no allocation at all.  Each
// device holds its own copy from the time the library is loaded until the
// process ends.  Host code never passes `scratch` itself to a kernel (in host
// code the name is only a stand-in): it uses the address hipGetSymbolAddress
// returns for the current device, kept per device in g_scratch_ptr.
constexpr uint64_t kNoAllocScratchBytes = LTL4C_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
hipError_t scratch_address(int device, uint8_t** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<uint8_t*>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace

// One tuned kernel schedule (radix-pass tile, map-scan tile) of a shape class.
struct SchedEntry {
    int kind = 0;                      // 0: one trace (ltl4c_eval), 1: a batch of traces (ltl4c_eval_batch)
    uint32_t key_bits = 0;             // packed key bits (with the trace id of a batch)
    uint32_t n_props = 0;
    uint32_t big = 0;                  // 1 when some monitor has more than 8 states
    uint32_t levels = 0;               // quantifier levels (plus the trace level of a batch)
    uint32_t log2n = 0;                // floor(log2(events))
    int sort = 1, scan = 3;
    double us = 0.0, default_us = 0.0; // measured median of the chosen and of the default schedule
};

// A captured kernel sequence (hipGraph) and what its replay must also do on the host.
struct GraphHost {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* table_dev = nullptr;         // the graph's own chunk / trace table
    int32_t group = -1;                // a group push: the group and its chunks' streams
    std::vector<uint32_t> streams;
};

struct ltl4c_ctx {
    int device = 0;
    std::vector<SchedEntry> sched;     // tuned schedules (ltl4c_tune, ltl4c_schedule_load)
    bool pin_sort = false, pin_scan = false;   // set by ltl4c_set_option: tuned schedules do not override
    hipStream_t cap_stream = nullptr;  // private stream for graph capture
    std::vector<GraphHost*> graphs;
    uint8_t* scratch = nullptr;        // this device's copy of `scratch`
    bool no_timing = false;            // launches without profiling events (no-allocation calls)
    hipStream_t stream = nullptr;
    bool has_layout = false;
    ltl4c_layout layout{};
    std::vector<MonitorHost> monitors;
    std::vector<ltl4c_property> props;
    std::map<std::vector<int32_t>, Plan*> plans;
    uint32_t* err_dev = nullptr;
    int sort_variant = kDefaultSortVariant;
    int scan_variant = kDefaultScanVariant;
    uint64_t budget = ~0ull, used = 0;
    uint32_t* batch_chunk_dev = nullptr;      // trace table of ltl4c_eval_batch
    uint32_t* batch_chunk_host = nullptr;     // pinned staging for it
    hipEvent_t batch_ev = nullptr;
    std::vector<struct GroupHost*> groups;
    bool prof = false;
    std::vector<Timed> timed;
    std::vector<hipEvent_t> free_events;
    std::vector<std::pair<std::string, std::pair<double, uint64_t>>> prof_acc;
};

namespace {

// Derived quantities of a layout shared by the workspace query and eval.
struct Geometry {
    uint32_t cbits, key_bits_total, sort_bits, n_pass;
    uint32_t ibits;                         // trace index bits between class and key (per-event verdicts)
    uint32_t digit_bits;                    // radix digit width: 8, or 9 when that saves a pass
    bool compact;                           // the first radix pass drops excluded events
    uint32_t stream_bits;                   // stream / trace id above the keys
    uint32_t n_levels;                      // levels of the monitor tree (quantifier nodes 0..n_levels-1)
    bool excl;
    uint32_t prefix_bits[kMaxLevels];       // bits of the packed prefix that identifies a level-m node
    bool parent;                            // parent events: a kind bit above the keys (1 = parent event)
};

// stream_is_level: the id above the keys is a tree level of its own (batches
// of traces: one subtree per trace); otherwise it only separates streams.
// compact: excluded events are dropped by the first radix pass instead of
// being sorted behind the others on an extra key bit (the consumers then read
// the kept count on the device).  wide: the sort variant has a thread per
// bucket for 9-bit digits.
Geometry geometry(const ltl4c_layout& L, uint32_t stream_bits = 0, bool stream_is_level = false,
                  bool compact = false, bool wide = false) {
    Geometry g{};
    g.cbits = bits_for(L.n_classes);
    // parent events sort after all own events on a kind bit above the keys,
    // placed like a stream id that is not a tree level
    g.parent = L.parent_events != 0;
    g.stream_bits = stream_bits + (g.parent ? 1u : 0u);
    g.n_levels = L.n_keys + (stream_is_level ? 1u : 0u);
    uint32_t kb = g.stream_bits;
    const uint32_t shift = stream_is_level ? 1u : 0u;
    if (stream_is_level) g.prefix_bits[0] = 0;
    for (uint32_t m = 0; m < L.n_keys; ++m) {
        if (m + shift < kMaxLevels) g.prefix_bits[m + shift] = kb;
        kb += L.key_bits[m];
    }
    g.key_bits_total = kb;
    const uint32_t need = (1u << L.n_keys) - 1u;
    g.excl = L.type_bytes > 1 || g.parent;
    for (int t = 0; t < 256 && !g.excl; ++t)
        if ((L.key_present[t] & need) != need) g.excl = true;
    g.compact = compact && g.excl && kb > 0;
    g.sort_bits = kb + (g.excl && !g.compact ? 1u : 0u);
    const uint32_t p8 = (g.sort_bits + kRadixBits - 1) / kRadixBits;
    const uint32_t p9 = (g.sort_bits + kRadixBitsWide - 1) / kRadixBitsWide;
    g.digit_bits = wide && p9 < p8 && (p9 << kRadixBitsWide) <= (uint32_t)kHistWords ? kRadixBitsWide : kRadixBits;
    g.n_pass = (g.sort_bits + g.digit_bits - 1) / g.digit_bits;
    return g;
}

struct WsLayout {
    uint64_t total;
    uint64_t zero_off, zero_words;
    uint64_t hist_off, n_valid_off, sort_ticket_off, scan_ticket_off, root_counts_off, sizes32_off, sizes64_off;
    uint64_t sort_status_off, scan_status_off;
    uint64_t words_a_off, words_b_off, inst_verdict_off, inst_parent_off, inst_start_off;
    uint64_t node_start_off[kMaxLevels], counts_off[kMaxLevels];
    uint64_t cap_node[kMaxLevels];
    uint32_t tiles_sort, tiles_scan;
    uint64_t ms_desc_off, ms_agg_off, ms_prefix_off, ms_trec_off, ms_chunk_off;   // the split map scan
    uint32_t ms_tiles;
    // parent events
    uint64_t pe_tree_off, pe_trec_off, pe_samples_off, pe_tile_agg_off, pe_tile_prefix_off, pe_tile_heads_off, pe_tile_hprefix_off;
    uint64_t pe_tree_lvl[kPeMaxTreeLevels], pe_tree_cnt[kPeMaxTreeLevels];
    uint32_t pe_levels, pe_tiles;
};

// Properties share scan launches by monitor size: up to 8 whose monitors have
// at most 8 states (two-dword maps), up to 4 of larger ones (four dwords).
// The numbering (instances, nodes, parents, sizes) comes from a launch of at
// most 4 properties, which runs first.
struct ScanGroup {
    uint32_t cnt, states;
    uint8_t idx[kScanGroupProps];
    bool structure;
};

std::vector<ScanGroup> scan_groups(const std::vector<uint32_t>& states) {
    std::vector<uint32_t> small, big;
    for (uint32_t i = 0; i < states.size(); ++i) (states[i] <= 8 ? small : big).push_back(i);
    std::vector<ScanGroup> out;
    auto emit = [&](const std::vector<uint32_t>& v, uint32_t per) {
        for (size_t i = 0; i < v.size(); i += per) {
            ScanGroup gr{};
            gr.cnt = (uint32_t)std::min<size_t>(per, v.size() - i);
            for (uint32_t k = 0; k < gr.cnt; ++k) {
                gr.idx[k] = (uint8_t)v[i + k];
                gr.states = std::max(gr.states, states[v[i + k]]);
            }
            out.push_back(gr);
        }
    };
    emit(big, 4);
    emit(small, kScanGroupProps);
    if (out.empty()) return out;
    size_t sg = 0;
    while (sg < out.size() && out[sg].cnt > 4) ++sg;
    if (sg == out.size()) {                 // only groups of 8: split the first one
        ScanGroup rest = out[0];
        rest.cnt = out[0].cnt - 4;
        for (uint32_t k = 0; k < rest.cnt; ++k) rest.idx[k] = out[0].idx[4 + k];
        out[0].cnt = 4;
        out.insert(out.begin() + 1, rest);
        sg = 0;
    }
    std::swap(out[0], out[sg]);
    out[0].structure = true;
    return out;
}

std::vector<uint32_t> monitor_states(const ltl4c_ctx* ctx, const int32_t* props, int32_t n_props) {
    std::vector<uint32_t> st;
    for (int32_t i = 0; i < n_props; ++i) st.push_back(ctx->monitors[ctx->props[props[i]].monitor].n_states);
    return st;
}

WsLayout plan_workspace(const ltl4c_layout& L, const Geometry& g, uint64_t n, uint32_t P, uint32_t n_scan_groups,
                        int sort_variant, int scan_variant) {
    WsLayout w{};
    const uint64_t st = sort_tile(sort_variant);
    w.tiles_sort = (uint32_t)((n + st - 1) / st);
    const uint64_t sct = scan_tile(scan_variant);
    w.tiles_scan = (uint32_t)((n + sct - 1) / sct);
    // zero block, in 32-bit words
    uint64_t z = 0;
    w.hist_off = z;        z += (uint64_t)g.n_pass << g.digit_bits;
    w.n_valid_off = z;     z += 64;
    w.sort_ticket_off = z; z += 64;
    w.scan_ticket_off = z; z += 64;
    w.root_counts_off = z; z += kMaxProps * 6;
    w.sizes32_off = z;     z += 64;
    w.sizes64_off = z;     z += 64;                      // 32 x uint64
    w.sort_status_off = z; z += ((uint64_t)g.n_pass * w.tiles_sort) << g.digit_bits;
    z = (z + 63) & ~63ull;
    w.scan_status_off = z; z += (uint64_t)n_scan_groups * w.tiles_scan * (2 * kScanRows);   // 2 kinds x 32-bit words
    z = (z + 63) & ~63ull;
    w.zero_off = 0;
    w.zero_words = z;
    uint64_t off = align256(z * 4);
    // (room for one map-scan run of 32 words past the end: its loads are unconditional)
    w.words_a_off = off;   off = align256(off + n * 8 + 256);
    w.words_b_off = off;   off = align256(off + n * 8 + 256);
    w.inst_verdict_off = off; off = align256(off + (uint64_t)P * n);
    w.inst_parent_off = 0;
    if (g.n_levels >= 2) {
        w.inst_parent_off = off;
        off = align256(off + 4 * n);
    }
    w.inst_start_off = off; off = align256(off + 4 * n);   // verdict timeline, when asked for
    // split map scan: a descriptor byte per word, a record per tile and its prefix
    w.ms_tiles = (uint32_t)((n + kMsTileMin - 1) / kMsTileMin);
    w.ms_desc_off = off;   off = align256(off + n + 64);
    w.ms_agg_off = off;    off = align256(off + 4ull * kMsRec * std::max<uint32_t>(w.ms_tiles, 1));
    w.ms_prefix_off = off; off = align256(off + 4ull * kMsRec * std::max<uint32_t>(w.ms_tiles, 1));
    w.ms_trec_off = off;   off = align256(off + 4ull * kMsThreadRec * kMsThreads * std::max<uint32_t>(w.ms_tiles, 1));
    // spine chunks (at least kMsSpineThreads tiles each): compositions, then prefixes
    w.ms_chunk_off = off;  off = align256(off + 2 * 4ull * kMsRec * (w.ms_tiles / kMsSpineThreads + 1));
    (void)L;
    for (uint32_t m = 1; m < g.n_levels; ++m) {
        uint64_t cap = n;
        if (g.prefix_bits[m] < 40) cap = std::min<uint64_t>(cap, 1ull << g.prefix_bits[m]);
        w.cap_node[m] = cap;
        w.node_start_off[m] = off; off = align256(off + cap * 4);
        w.counts_off[m] = off;     off = align256(off + (uint64_t)P * cap * 6 * 4);
    }
    if (g.parent) {
        // the segment tree over the parent events (levels 1 .. ceil(log2 n),
        // per property), and the tile aggregates and prefixes
        w.pe_levels = 0;
        uint64_t nodes = 0;
        for (uint32_t lv = 1; lv < (uint32_t)kPeMaxTreeLevels && (1ull << (lv - 1)) < n; ++lv) {
            w.pe_tree_cnt[lv] = (n + (1ull << lv) - 1) >> lv;
            w.pe_tree_lvl[lv] = nodes;
            nodes += (uint64_t)P * w.pe_tree_cnt[lv];
            w.pe_levels = lv;
        }
        w.pe_tree_off = off; off = align256(off + 16 * std::max<uint64_t>(nodes, 1));
        w.pe_tiles = (uint32_t)((n + kPeTile - 1) / kPeTile);
        const uint64_t t = std::max<uint32_t>(w.pe_tiles, 1);
        w.pe_tile_agg_off = off;     off = align256(off + 16 * t * P);
        w.pe_tile_prefix_off = off;  off = align256(off + 16 * t * P);
        w.pe_trec_off = off;         off = align256(off + 16 * t * kPeThreads * P);
        w.pe_samples_off = off;      off = align256(off + 8 * kPeSamples);
        w.pe_tile_heads_off = off;   off = align256(off + 4 * t);
        w.pe_tile_hprefix_off = off; off = align256(off + 4 * t);
    }
    w.total = off;
    return w;
}

int32_t check_layout(const ltl4c_layout* L) {
    if (!L) return fail(LTL4C_EINVAL, "layout is NULL");
    if (L->record_bytes < 4 || L->record_bytes > 256 || L->record_bytes % 4)
        return fail(LTL4C_EINVAL, "record_bytes must be a multiple of 4 in [4, 256]");
    auto field_ok = [&](uint32_t off, uint32_t bytes) {
        return (bytes == 1 || bytes == 2 || bytes == 4) && off % bytes == 0 && off + bytes <= L->record_bytes;
    };
    if (!field_ok(L->type_offset, L->type_bytes)) return fail(LTL4C_EINVAL, "bad type field");
    if (L->n_keys < 1 || L->n_keys > kMaxLevels) return fail(LTL4C_EUNSUPPORTED, "n_keys must be 1..4");
    for (uint32_t m = 0; m < L->n_keys; ++m) {
        if (!field_ok(L->key_offset[m], L->key_bytes[m])) return fail(LTL4C_EINVAL, "bad key field");
        if (L->key_bits[m] < 1 || L->key_bits[m] > 8 * L->key_bytes[m])
            return fail(LTL4C_EINVAL, "key_bits must be in [1, 8*key_bytes]");
    }
    if (L->n_classes < 1 || L->n_classes > LTL4C_MAX_CLASSES)
        return fail(LTL4C_EUNSUPPORTED, "n_classes must be 1..16");
    if (L->n_preds > 3) return fail(LTL4C_EUNSUPPORTED, "n_preds must be 0..3");
    for (uint32_t i = 0; i < L->n_preds; ++i) {
        if (!field_ok(L->pred[i].offset, L->pred[i].bytes)) return fail(LTL4C_EINVAL, "bad predicate field");
        if (L->pred[i].op > LTL4C_CMP_NE) return fail(LTL4C_EINVAL, "unknown predicate comparison");
    }
    if (L->n_preds > 0 && L->pred_shift > 3) return fail(LTL4C_EINVAL, "pred_shift must be 0..3");
    // the largest class any event can take: type class plus every predicate bit
    const uint32_t pred_top = L->n_preds ? ((1u << L->n_preds) - 1u) << L->pred_shift : 0u;
    for (int t = 0; t < 256; ++t)
        if ((uint32_t)L->class_of_type[t] + pred_top >= L->n_classes)
            return fail(LTL4C_EINVAL, "class_of_type entry (plus predicate bits) >= n_classes");
    if (L->parent_events > 1) return fail(LTL4C_EINVAL, "parent_events must be 0 or 1");
    // keys wider than the sort word are ranked by ltl4c_eval (batches and
    // stream groups check the width themselves)
    return LTL4C_OK;
}

// The declared widths do not fit the 64-bit sort word: ltl4c_eval ranks the
// key values first (the trace index of parent events counts).
bool needs_ranks(const ltl4c_layout& L, uint64_t n) {
    const Geometry g = geometry(L);
    const uint32_t ib = g.parent ? std::max<uint32_t>(1, bits_for((uint32_t)std::max<uint64_t>(n, 1))) : 0u;
    return g.cbits + ib + g.key_bits_total + (g.excl ? 1 : 0) > 63;
}

// Widths of ranked keys, at most: n events have at most n distinct values.
ltl4c_layout rank_sized(const ltl4c_layout& L, uint64_t n) {
    ltl4c_layout r = L;
    const uint32_t b = std::max<uint32_t>(1, bits_for((uint32_t)std::max<uint64_t>(n, 1)));
    for (uint32_t m = 0; m < L.n_keys; ++m) r.key_bits[m] = std::min(L.key_bits[m], b);
    return r;
}

// The ranking area at the start of the workspace (the evaluation's own
// workspace follows it).  Offsets in bytes.
struct RankRegion {
    uint64_t zero_off, zero_words;        // histograms [4][256], tickets, look-back status [4][tiles][256]
    uint64_t hist_w, ticket_w, status_w;  // word offsets inside the zero block
    uint64_t distinct_off;                // [4] distinct values per level
    uint64_t tile_cnt_off, tile_off_off;
    uint64_t rank_off[kMaxLevels], uniq_off[kMaxLevels];
    uint32_t tiles_sort;
    uint64_t total;
};

RankRegion rank_region(const ltl4c_layout& L, uint64_t n, int sort_variant) {
    RankRegion r{};
    const uint64_t st = sort_tile(sort_variant);
    r.tiles_sort = (uint32_t)((n + st - 1) / st);
    r.hist_w = 0;
    r.ticket_w = 4 * 256;
    r.status_w = r.ticket_w + 64;
    r.zero_words = r.status_w + 4ull * r.tiles_sort * 256;
    uint64_t off = 0;
    r.zero_off = off;       off = align256(off + 4 * r.zero_words);
    r.distinct_off = off;   off = align256(off + 64);
    const uint64_t tiles = std::max<uint64_t>(1, (n + kRankTile - 1) / kRankTile);
    r.tile_cnt_off = off;   off = align256(off + 4 * tiles);
    r.tile_off_off = off;   off = align256(off + 4 * tiles);
    for (uint32_t m = 0; m < L.n_keys; ++m) {
        r.rank_off[m] = off; off = align256(off + 4 * std::max<uint64_t>(n, 1));
        r.uniq_off[m] = off; off = align256(off + 4 * std::max<uint64_t>(n, 1));
    }
    r.total = off;
    return r;
}

// shift = 1 places the quantifiers one level down (level 0 gets a dummy
// E>=0): used when a batch adds a per-trace level above the quantifiers.
PropDev make_prop(const MonitorHost& M, const ltl4c_property& p, uint32_t shift = 0) {
    PropDev d;
    std::memset(&d, 0, sizeof d);
    for (uint32_t q = 0; q < M.n_states; ++q) d.label[q] = M.label[q];
    for (uint32_t c = 0; c < 16; ++c)
        for (uint32_t q = 0; q < 16; ++q) {
            const uint32_t to = (c < M.n_classes && q < M.n_states) ? M.delta[q * M.n_classes + c] : q;
            d.bmap[c][q / 4] |= to << (8 * (q % 4));
        }
    for (uint32_t q = 0; q < M.n_states; ++q) d.blabel[q / 8] |= (uint32_t)(M.label[q] & 15) << (4 * (q % 8));
    d.q0 = M.q0;
    d.n_states = M.n_states;
    if (shift) {
        d.kind[0] = LTL4C_Q_COUNT;
        d.op[0] = LTL4C_GE;
        d.num[0] = 0;
        d.den[0] = 1;
    }
    for (uint32_t l = 0; l < p.n_levels && l + shift < (uint32_t)kMaxLevels; ++l) {
        d.kind[l + shift] = p.q[l].kind;
        d.op[l + shift] = p.q[l].op;
        d.num[l + shift] = p.q[l].num;
        d.den[l + shift] = p.q[l].kind == LTL4C_Q_PERCENT ? p.q[l].den : 1u;
    }
    return d;
}

int32_t get_plan(ltl4c_ctx* ctx, const int32_t* props, int32_t n_props, Plan** out, uint32_t shift = 0) {
    std::vector<int32_t> key(props, props + n_props);
    if (shift) key.insert(key.begin(), -1);
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) {
        *out = it->second;
        return LTL4C_OK;
    }
    Plan host;
    std::memset(&host, 0, sizeof host);
    for (int32_t i = 0; i < n_props; ++i) {
        const ltl4c_property& p = ctx->props[props[i]];
        host.prop[i] = make_prop(ctx->monitors[p.monitor], p, shift);
    }
    std::memcpy(host.class_of_type, ctx->layout.class_of_type, 256);
    std::memcpy(host.key_present, ctx->layout.key_present, 256);
    Plan* dev = nullptr;
    HIP_TRY(hipMalloc(&dev, sizeof(Plan)));
    hipError_t e = hipMemcpy(dev, &host, sizeof(Plan), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return fail(LTL4C_EDEVICE, std::string("plan upload: ") + hipGetErrorString(e));
    }
    ctx->plans[key] = dev;
    *out = dev;
    return LTL4C_OK;
}

void drop_plans(ltl4c_ctx* ctx) {
    for (auto& kv : ctx->plans) (void)hipFree(kv.second);
    ctx->plans.clear();
}

int32_t check_props(ltl4c_ctx* ctx, const int32_t* props, int32_t n_props) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    if (!ctx->has_layout) return fail(LTL4C_EINVAL, "no layout set");
    if (!props || n_props < 1 || n_props > kMaxProps) return fail(LTL4C_EINVAL, "n_props must be 1..16");
    for (int32_t i = 0; i < n_props; ++i)
        if (props[i] < 0 || props[i] >= (int32_t)ctx->props.size()) return fail(LTL4C_EINVAL, "unknown property id");
    return LTL4C_OK;
}

// Kernel launches with optional event timing.
hipEvent_t take_event(ltl4c_ctx* ctx) {
    if (!ctx->free_events.empty()) {
        hipEvent_t e = ctx->free_events.back();
        ctx->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <typename F>
int32_t launch(ltl4c_ctx* ctx, const char* name, F&& f) {
    hipEvent_t a = nullptr, b = nullptr;
    const bool timed = ctx->prof && !ctx->no_timing;
    if (timed) {
        a = take_event(ctx);
        b = take_event(ctx);
        if (a) (void)hipEventRecord(a, ctx->stream);
    }
    hipError_t e = f();
    if (timed && a && b) {
        (void)hipEventRecord(b, ctx->stream);
        ctx->timed.push_back({name, a, b});
    }
    if (e != hipSuccess) return fail(LTL4C_EDEVICE, std::string(name) + ": " + hipGetErrorString(e));
    return LTL4C_OK;
}

int32_t drain_profile(ltl4c_ctx* ctx) {
    if (ctx->timed.empty()) return LTL4C_OK;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (auto& t : ctx->timed) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t.start, t.stop);
        bool found = false;
        for (auto& acc : ctx->prof_acc) {
            if (acc.first == t.name) {
                acc.second.first += ms;
                acc.second.second += 1;
                found = true;
                break;
            }
        }
        if (!found) ctx->prof_acc.push_back({t.name, {ms, 1}});
        ctx->free_events.push_back(t.start);
        ctx->free_events.push_back(t.stop);
    }
    ctx->timed.clear();
    return LTL4C_OK;
}

// zero-block must already be cleared.  Enqueues classify and the radix
// passes; *sorted receives the buffer holding the sorted words.
int32_t enqueue_front(ltl4c_ctx* ctx, const ltl4c_layout& L, const Geometry& g, const WsLayout& w, uint8_t* ws,
                      const void* d_records, uint64_t n, const Plan* plan, const uint32_t* chunk_off,
                      const uint32_t* chunk_stream, const uint64_t* chunk_ptr, uint32_t n_chunks, bool vec_ok,
                      uint64_t** sorted, int sort_variant, const uint32_t* const* rank = nullptr) {
    const uint32_t NL = L.n_keys;
    uint32_t* z = reinterpret_cast<uint32_t*>(ws);
    uint32_t* hist = z + w.hist_off;
    uint32_t* sort_ticket = z + w.sort_ticket_off;
    uint32_t* sort_status = z + w.sort_status_off;
    uint64_t* words_a = reinterpret_cast<uint64_t*>(ws + w.words_a_off);
    uint64_t* words_b = reinterpret_cast<uint64_t*>(ws + w.words_b_off);
    const hipStream_t st = ctx->stream;
    int32_t s;
    ClassifyArgs ca{};
    ca.records = static_cast<const uint8_t*>(d_records);
    ca.n = n;
    ca.record_bytes = L.record_bytes;
    ca.type_dw = L.type_offset / 4;
    ca.type_shift = (L.type_offset % 4) * 8;
    ca.type_mask = L.type_bytes == 4 ? 0xFFFFFFFFu : ((1u << (8 * L.type_bytes)) - 1u);
    ca.n_keys = NL;
    for (uint32_t m = 0; m < NL; ++m) {
        ca.key_dw[m] = L.key_offset[m] / 4;
        ca.key_shift[m] = (L.key_offset[m] % 4) * 8;
        ca.key_mask[m] = L.key_bytes[m] == 4 ? 0xFFFFFFFFu : ((1u << (8 * L.key_bytes[m])) - 1u);
        ca.key_bits[m] = L.key_bits[m];
    }
    ca.need_mask = (1u << NL) - 1u;
    ca.n_preds = L.n_preds;
    ca.pred_class_shift = L.pred_shift;
    for (uint32_t q = 0; q < L.n_preds && q < 3; ++q) {
        ca.pred_dw[q] = L.pred[q].offset / 4;
        ca.pred_shift[q] = (L.pred[q].offset % 4) * 8;
        ca.pred_mask[q] = L.pred[q].bytes == 4 ? 0xFFFFFFFFu : ((1u << (8 * L.pred[q].bytes)) - 1u);
        ca.pred_op[q] = L.pred[q].op;
        ca.pred_val[q] = L.pred[q].value;
    }
    ca.check_type_range = L.type_bytes > 1;
    ca.cbits = g.cbits;
    ca.ibits = g.ibits;
    ca.excl_shift = g.cbits + g.ibits + g.key_bits_total;
    ca.n_pass = g.n_pass;
    ca.digit_bits = g.digit_bits;
    ca.n_valid = g.compact ? z + w.n_valid_off : nullptr;
    ca.sort_shift = g.cbits + g.ibits;
    ca.plan = plan;
    ca.words = words_a;
    ca.hist = hist;
    ca.err = ctx->err_dev;
    ca.chunk_off = chunk_off;
    ca.chunk_stream = chunk_stream;
    ca.chunk_ptr = chunk_ptr;
    ca.n_chunks = n_chunks;
    ca.vec_ok = vec_ok ? 1u : 0u;
    ca.stream_shift = g.key_bits_total - g.stream_bits;
    if (rank)
        for (uint32_t m = 0; m < NL; ++m) ca.rank[m] = rank[m];
    ca.parent_mask = g.parent ? ca.need_mask >> 1 : 0xFFFFFFFFu;
    ca.n_par = g.parent ? z + w.n_valid_off + 1 : nullptr;
    s = launch(ctx, "classify", [&] { return launch_classify(ca, st); });
    if (s) return s;
    uint64_t* in = words_a;
    uint64_t* outw = words_b;
    for (uint32_t p = 0; p < g.n_pass; ++p) {
        SortPassArgs sa{};
        sa.in = in;
        sa.out = outw;
        sa.n = (uint32_t)n;
        sa.shift = g.cbits + g.ibits + g.digit_bits * p;
        sa.nbits = std::min<uint32_t>(g.digit_bits, g.sort_bits - g.digit_bits * p);
        sa.hist = hist + ((uint64_t)p << g.digit_bits);
        sa.status = sort_status + (((uint64_t)p * w.tiles_sort) << g.digit_bits);
        sa.ticket = sort_ticket + p;
        sa.n_valid = ca.n_valid;
        sa.drop_excl = g.compact && p == 0 ? 1u : 0u;
        sa.excl_shift = ca.excl_shift;
        sa.err = ctx->err_dev;
        s = launch(ctx, "sort_pass", [&] { return launch_sort_pass(sa, sort_variant, g.digit_bits, st); });
        if (s) return s;
        std::swap(in, outw);
    }
    *sorted = in;
    return LTL4C_OK;
}

}  // namespace


// A stream group: the resident monitor tree of up to max_streams streams.
struct GroupHost {
    std::vector<int32_t> props;
    std::vector<ScanGroup> sgroups;    // scan launches over the virtual properties
    int sort_variant = 0, scan_variant = 0;   // schedules fixed when the group opens
    uint32_t P = 0, V = 0, S = 0, max_bindings = 0;
    uint64_t table_bindings = 0;       // bindings the hash table is sized for (load factor <= 1/2)
    uint64_t admitted = 0;             // bindings reserved by the open streams
    uint64_t max_batch = 0;
    // per stream (host side): admission, sequence numbers, last push
    std::vector<uint8_t> open;
    std::vector<uint32_t> smax;
    std::vector<uint64_t> next_seq, done_seq;
    std::vector<std::chrono::steady_clock::time_point> last_push;
    struct Pending {
        hipEvent_t ev;
        std::vector<std::pair<uint32_t, uint64_t>> seq_after;   // (stream, next sequence number)
    };
    std::deque<Pending> pending;       // pushes whose completion poll has not seen yet
    std::vector<hipEvent_t> spare_events;
    // pushes from host memory: double-buffered device staging filled on a copy stream
    hipStream_t copy_stream = nullptr;
    uint8_t* stage[2] = {nullptr, nullptr};
    hipEvent_t stage_free[2] = {nullptr, nullptr}, stage_ready[2] = {nullptr, nullptr};
    int stage_i = 0;
    uint64_t stage_bytes = 0;
    Geometry g{};
    ltl4c_layout lay_ws{};             // layout copy with one level for workspace sizing
    Plan* vplan = nullptr;             // one virtual property per (property, start state)
    Plan* rplan = nullptr;             // the real properties
    uint8_t* state = nullptr;
    uint64_t state_bytes = 0;
    uint8_t* ws = nullptr;
    uint64_t ws_bytes = 0;
    WsLayout w{};
    uint64_t seg_keys_off = 0;         // inside ws, after the eval workspace
    GroupState gs{};
    uint32_t* chunk_dev = nullptr;     // [kMaxChunks + 1 offsets][kMaxChunks streams]
    uint32_t* chunk_host = nullptr;    // pinned ring of kChunkRing tables
    hipEvent_t ring_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int ring_i = 0;
    uint64_t total_bytes = 0;
};

namespace {

constexpr int kChunkRing = 4;
constexpr uint64_t kChunkTableWords = 4 * kMaxChunks + 4;   // offsets, streams, pointers

uint64_t pow2_at_least(uint64_t x) {
    uint64_t p = 1024;
    while (p < x) p <<= 1;
    return p;
}

// Offsets of the resident state of a group; fills gs pointers when base != nullptr.
uint64_t group_state_layout(const GroupHost& G, uint32_t L, uint8_t* base, GroupState* gs) {
    const uint64_t bcap = pow2_at_least(2ull * G.table_bindings);
    const uint64_t ncap = bcap;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t o = off;
        off = align256(off + bytes);
        return base ? base + o : nullptr;
    };
    uint8_t* bslot = take(16 * bcap);
    uint8_t* bstate = take((uint64_t)(G.P > 4 ? G.P - 4 : 0) * bcap);
    uint8_t* sb = take(4ull * G.S);
    uint8_t* smx = take(4ull * G.S);
    uint8_t* nk[kMaxLevels] = {}, *nc[kMaxLevels] = {}, *nv[kMaxLevels] = {}, *np[kMaxLevels] = {},
             *nd[kMaxLevels] = {}, *nl[kMaxLevels] = {};
    for (uint32_t m = 1; m < L; ++m) {
        nk[m] = take(8 * ncap);
        nc[m] = take(24ull * G.P * ncap);
        nv[m] = take((uint64_t)G.P * ncap);
        np[m] = take(4 * ncap);
        nd[m] = take(4 * ncap);
        nl[m] = take(4 * ncap);
    }
    uint8_t* rc = take(24ull * G.S * G.P);
    uint8_t* rv = take((uint64_t)G.S * G.P);
    uint8_t* rd = take(4ull * G.S);
    uint8_t* rl = take(4ull * G.S);
    uint8_t* lc = take(4 * kMaxLevels);
    if (gs) {
        gs->bslot = reinterpret_cast<uint64_t*>(bslot);
        gs->bmask = bcap - 1;
        gs->bstate = bstate;
        gs->stream_bindings = reinterpret_cast<uint32_t*>(sb);
        gs->stream_max = reinterpret_cast<uint32_t*>(smx);
        gs->nmask = ncap - 1;
        for (uint32_t m = 1; m < L; ++m) {
            gs->nkeys[m] = reinterpret_cast<uint64_t*>(nk[m]);
            gs->ncounts[m] = reinterpret_cast<uint32_t*>(nc[m]);
            gs->nverdict[m] = nv[m];
            gs->nparent[m] = reinterpret_cast<uint32_t*>(np[m]);
            gs->ndirty[m] = reinterpret_cast<uint32_t*>(nd[m]);
            gs->nlist[m] = reinterpret_cast<uint32_t*>(nl[m]);
        }
        gs->rcounts = reinterpret_cast<uint32_t*>(rc);
        gs->rverdict = rv;
        gs->rdirty = reinterpret_cast<uint32_t*>(rd);
        gs->rlist = reinterpret_cast<uint32_t*>(rl);
        gs->list_cnt = reinterpret_cast<uint32_t*>(lc);
    }
    return off;
}

// table_bindings: bindings of all streams together the group's tables hold.
int32_t group_configure(ltl4c_ctx* ctx, GroupHost& G, const int32_t* props, int32_t n_props, uint32_t max_streams,
                        uint32_t max_bindings, uint64_t table_bindings, uint64_t max_batch) {
    int32_t s = check_props(ctx, props, n_props);
    if (s) return s;
    if (max_streams < 1 || max_bindings < 1 || table_bindings < 1)
        return fail(LTL4C_EINVAL, "max_streams and the binding limits must be >= 1");
    if (max_batch < 1 || max_batch > LTL4C_MAX_EVENTS) return fail(LTL4C_EUNSUPPORTED, "max_batch out of range");
    if (table_bindings > (1ull << 31)) return fail(LTL4C_EUNSUPPORTED, "the group's bindings exceed 2^31");
    const ltl4c_layout& L = ctx->layout;
    if (L.parent_events) return fail(LTL4C_EUNSUPPORTED, "stream groups do not take layouts with parent events");
    G.props.assign(props, props + n_props);
    G.P = (uint32_t)n_props;
    G.S = max_streams;
    G.max_bindings = max_bindings;
    G.table_bindings = table_bindings;
    G.max_batch = max_batch;
    G.V = 0;
    for (int32_t i = 0; i < n_props; ++i) G.V += ctx->monitors[ctx->props[props[i]].monitor].n_states;
    if (G.V > (uint32_t)kMaxProps)
        return fail(LTL4C_EUNSUPPORTED, "a stream group takes properties whose monitors have 16 states in total");
    const uint32_t sb = std::max<uint32_t>(1, bits_for(max_streams));
    G.g = geometry(L, sb, false, false, sort_threads(ctx->sort_variant) >= 512);
    if (G.g.cbits + G.g.key_bits_total + (G.g.excl ? 1 : 0) > 63)
        return fail(LTL4C_EUNSUPPORTED, "stream id, keys and class bits exceed 63 bits");
    G.sort_variant = ctx->sort_variant;
    G.scan_variant = ctx->scan_variant;
    G.lay_ws = L;
    G.lay_ws.n_keys = 1;
    Geometry g1 = G.g;
    g1.n_levels = 1;                    // the scan of a push numbers segments only
    std::vector<uint32_t> vstates;
    for (int32_t i = 0; i < n_props; ++i) {
        const uint32_t ns = ctx->monitors[ctx->props[props[i]].monitor].n_states;
        vstates.insert(vstates.end(), ns, ns);
    }
    G.sgroups = scan_groups(vstates);
    G.w = plan_workspace(G.lay_ws, g1, max_batch, G.V, (uint32_t)G.sgroups.size(), ctx->sort_variant, ctx->scan_variant);
    G.seg_keys_off = align256(G.w.total);
    G.ws_bytes = G.seg_keys_off + 8 * max_batch;
    G.state_bytes = group_state_layout(G, L.n_keys, nullptr, nullptr);
    G.total_bytes = G.state_bytes + G.ws_bytes + 4 * kChunkTableWords;
    return LTL4C_OK;
}

void group_free(GroupHost* G) {
    if (!G) return;
    if (G->copy_stream) (void)hipStreamSynchronize(G->copy_stream);
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(G->stage[i]);
        if (G->stage_free[i]) (void)hipEventDestroy(G->stage_free[i]);
        if (G->stage_ready[i]) (void)hipEventDestroy(G->stage_ready[i]);
    }
    if (G->copy_stream) (void)hipStreamDestroy(G->copy_stream);
    for (auto& p : G->pending) (void)hipEventDestroy(p.ev);
    for (auto e : G->spare_events) (void)hipEventDestroy(e);
    (void)hipFree(G->state);
    (void)hipFree(G->ws);
    (void)hipFree(G->chunk_dev);
    (void)hipHostFree(G->chunk_host);
    for (auto& e : G->ring_ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipFree(G->vplan);
    (void)hipFree(G->rplan);
    delete G;
}

int32_t get_group(ltl4c_ctx* ctx, int32_t id, GroupHost** out) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    if (id < 0 || id >= (int32_t)ctx->groups.size() || !ctx->groups[id]) return fail(LTL4C_ESEQ, "no such open group");
    *out = ctx->groups[id];
    return LTL4C_OK;
}

}  // namespace

extern "C" {

const char* ltl4c_last_error(void) { return g_last_error.c_str(); }

const char* ltl4c_status_str(int32_t s) {
    switch (s) {
        case LTL4C_OK: return "ok";
        case LTL4C_EINVAL: return "invalid argument";
        case LTL4C_ENOMEM: return "out of memory or workspace too small";
        case LTL4C_ECAPACITY: return "capacity exceeded";
        case LTL4C_EDEVICE: return "device error";
        case LTL4C_EADMIT: return "admission refused";
        case LTL4C_ESEQ: return "out of sequence";
        case LTL4C_EUNSUPPORTED: return "unsupported";
        case LTL4C_ERANGE: return "key wider than declared";
        default: return "unknown status";
    }
}

int32_t ltl4c_create(ltl4c_ctx** out, int32_t device) {
    if (!out) return fail(LTL4C_EINVAL, "out is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(LTL4C_EINVAL, "no such device");
    HIP_TRY(hipSetDevice(device));
    ltl4c_ctx* ctx = new ltl4c_ctx();
    ctx->device = device;
    hipError_t e = hipMalloc(&ctx->err_dev, 256);
    if (e == hipSuccess) e = hipMemset(ctx->err_dev, 0, 256);
    if (e == hipSuccess) e = scratch_address(device, &ctx->scratch);
    if (e != hipSuccess) {
        delete ctx;
        return fail(LTL4C_EDEVICE, std::string("context allocation: ") + hipGetErrorString(e));
    }
    *out = ctx;
    return LTL4C_OK;
}

int32_t ltl4c_destroy(ltl4c_ctx* ctx) {
    if (!ctx) return LTL4C_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    drop_plans(ctx);
    for (auto* G : ctx->groups) group_free(G);
    ctx->groups.clear();
    (void)hipFree(ctx->batch_chunk_dev);
    (void)hipHostFree(ctx->batch_chunk_host);
    if (ctx->batch_ev) (void)hipEventDestroy(ctx->batch_ev);
    for (auto& t : ctx->timed) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (auto e : ctx->free_events) (void)hipEventDestroy(e);
    for (auto* gh : ctx->graphs) {
        if (!gh) continue;
        if (gh->exec) (void)hipGraphExecDestroy(gh->exec);
        if (gh->graph) (void)hipGraphDestroy(gh->graph);
        (void)hipFree(gh->table_dev);
        delete gh;
    }
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    (void)hipFree(ctx->err_dev);
    delete ctx;
    return LTL4C_OK;
}

int32_t ltl4c_set_stream(ltl4c_ctx* ctx, void* hip_stream) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return LTL4C_OK;
}

int32_t ltl4c_set_layout(ltl4c_ctx* ctx, const ltl4c_layout* L) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    int32_t s = check_layout(L);
    if (s) return s;
    for (auto* G : ctx->groups)
        if (G) return fail(LTL4C_ESEQ, "close the open stream groups before changing the layout");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    drop_plans(ctx);
    ctx->layout = *L;
    ctx->has_layout = true;
    ctx->monitors.clear();
    ctx->props.clear();
    return LTL4C_OK;
}

int32_t ltl4c_add_monitor(ltl4c_ctx* ctx, const ltl4c_monitor* m, int32_t* id) {
    if (!ctx || !m || !id) return fail(LTL4C_EINVAL, "NULL argument");
    if (!ctx->has_layout) return fail(LTL4C_EINVAL, "set a layout first");
    if (m->n_states < 1 || m->n_states > LTL4C_MAX_STATES) return fail(LTL4C_EUNSUPPORTED, "n_states must be 1..16");
    if (m->n_classes != ctx->layout.n_classes) return fail(LTL4C_EINVAL, "monitor n_classes differs from the layout");
    if (m->q0 >= m->n_states) return fail(LTL4C_EINVAL, "q0 out of range");
    if (!m->delta || !m->label) return fail(LTL4C_EINVAL, "delta/label is NULL");
    MonitorHost h{m->n_states, m->n_classes, m->q0, {}, {}};
    h.delta.assign(m->delta, m->delta + (size_t)m->n_states * m->n_classes);
    h.label.assign(m->label, m->label + m->n_states);
    for (uint8_t d : h.delta)
        if (d >= m->n_states) return fail(LTL4C_EINVAL, "delta entry out of range");
    for (uint8_t l : h.label)
        if (!(l == LTL4C_BOT || l == LTL4C_BOT_P || l == LTL4C_TOP_P || l == LTL4C_TOP))
            return fail(LTL4C_EINVAL, "label must be an LTL4 verdict (F, Fp, Tp, T)");
    ctx->monitors.push_back(std::move(h));
    *id = (int32_t)ctx->monitors.size() - 1;
    return LTL4C_OK;
}

int32_t ltl4c_add_property(ltl4c_ctx* ctx, const ltl4c_property* p, int32_t* id) {
    if (!ctx || !p || !id) return fail(LTL4C_EINVAL, "NULL argument");
    if (!ctx->has_layout) return fail(LTL4C_EINVAL, "set a layout first");
    if (p->monitor < 0 || p->monitor >= (int32_t)ctx->monitors.size()) return fail(LTL4C_EINVAL, "unknown monitor id");
    if (p->n_levels != ctx->layout.n_keys) return fail(LTL4C_EINVAL, "n_levels must equal the layout's n_keys");
    for (uint32_t l = 0; l < p->n_levels; ++l) {
        const ltl4c_quant& q = p->q[l];
        if (q.kind > 1) return fail(LTL4C_EINVAL, "quantifier kind must be PERCENT or COUNT");
        if (q.op > 4) return fail(LTL4C_EINVAL, "comparison operator out of range");
        if (q.kind == LTL4C_Q_PERCENT && (q.den == 0 || q.num > q.den))
            return fail(LTL4C_EINVAL, "percentage constant must be num/den in [0, 1]");
    }
    ctx->props.push_back(*p);
    *id = (int32_t)ctx->props.size() - 1;
    return LTL4C_OK;
}

// ---- kernel schedules ---------------------------------------------------------
namespace {

uint32_t log2_floor(uint64_t n) {
    uint32_t b = 0;
    while (n >>= 1) ++b;
    return b;
}

// The shape class of a call, which tuned schedules are keyed by: the kind of
// call, the packed key bits (which fix the radix passes), the properties, the
// monitor size class, the tree levels and the trace size in powers of two.
SchedEntry shape_of(const ltl4c_ctx* ctx, int kind, uint64_t n, int32_t n_traces, const int32_t* props,
                    int32_t n_props) {
    SchedEntry e;
    e.kind = kind;
    uint32_t kb = 0;
    for (uint32_t m = 0; m < ctx->layout.n_keys; ++m) kb += ctx->layout.key_bits[m];
    e.levels = ctx->layout.n_keys;
    if (kind == 1) {
        kb += std::max<uint32_t>(1, bits_for((uint32_t)n_traces));
        e.levels += 1;
    }
    e.key_bits = kb;
    e.n_props = (uint32_t)n_props;
    for (uint32_t st : monitor_states(ctx, props, n_props))
        if (st > 8) e.big = 1;
    e.log2n = log2_floor(std::max<uint64_t>(n, 1));
    return e;
}

bool same_class(const SchedEntry& a, const SchedEntry& b) {
    return a.kind == b.kind && a.key_bits == b.key_bits && a.n_props == b.n_props && a.big == b.big &&
           a.levels == b.levels;
}

// The tuned entry of the same class whose trace size is nearest (at most a
// factor of 4 away), or null.
const SchedEntry* find_sched(const ltl4c_ctx* ctx, const SchedEntry& shape) {
    const SchedEntry* best = nullptr;
    uint32_t bd = 3;
    for (const auto& e : ctx->sched) {
        if (!same_class(e, shape)) continue;
        const uint32_t d = e.log2n > shape.log2n ? e.log2n - shape.log2n : shape.log2n - e.log2n;
        if (d < bd) {
            bd = d;
            best = &e;
        }
    }
    return best;
}

// For the duration of one call: the tuned schedule of its shape class, unless
// ltl4c_set_option pinned a tile; revert() returns to the context's own.
struct SchedScope {
    ltl4c_ctx* ctx;
    int sort0, scan0;
    SchedScope(ltl4c_ctx* c, const SchedEntry* e) : ctx(c), sort0(c->sort_variant), scan0(c->scan_variant) {
        if (e && !c->pin_sort) c->sort_variant = e->sort;
        if (e && !c->pin_scan) c->scan_variant = e->scan;
    }
    bool changed() const { return ctx->sort_variant != sort0 || ctx->scan_variant != scan0; }
    void revert() {
        ctx->sort_variant = sort0;
        ctx->scan_variant = scan0;
    }
    ~SchedScope() { revert(); }
};

uint64_t eval_ws_bytes(ltl4c_ctx* ctx, uint64_t n, const int32_t* props, int32_t n_props) {
    const bool ranked = needs_ranks(ctx->layout, n);
    const ltl4c_layout L = ranked ? rank_sized(ctx->layout, n) : ctx->layout;
    Geometry g = geometry(L, 0, false, true, sort_threads(ctx->sort_variant) >= 512);
    return (ranked ? rank_region(L, n, ctx->sort_variant).total : 0) +
           plan_workspace(L, g, n, (uint32_t)n_props, (uint32_t)scan_groups(monitor_states(ctx, props, n_props)).size(),
                          ctx->sort_variant, ctx->scan_variant)
               .total;
}

}  // namespace

// Enough for the context's schedule and for the tuned one of this shape, so
// that a workspace sized before or after tuning fits whichever runs.
int32_t ltl4c_workspace_bytes(ltl4c_ctx* ctx, uint64_t n_events, const int32_t* props, int32_t n_props,
                              uint64_t* bytes) {
    int32_t s = check_props(ctx, props, n_props);
    if (s) return s;
    if (!bytes) return fail(LTL4C_EINVAL, "bytes is NULL");
    if (n_events > LTL4C_MAX_EVENTS) return fail(LTL4C_EUNSUPPORTED, "too many events for one call");
    uint64_t b = eval_ws_bytes(ctx, n_events, props, n_props);
    SchedScope sc(ctx, find_sched(ctx, shape_of(ctx, 0, n_events, 0, props, n_props)));
    if (sc.changed()) b = std::max(b, eval_ws_bytes(ctx, n_events, props, n_props));
    *bytes = b;
    return LTL4C_OK;
}

// The evaluation pipeline after validation: zero, classify, radix passes,
// scan, counting per level, finalize.  g.n_levels tree levels; when a chunk
// table is given the chunk index (a trace id) is the top key.
static int32_t eval_core(ltl4c_ctx* ctx, const ltl4c_layout& L, const Geometry& g, const WsLayout& w, void* d_ws,
                         const void* d_records, uint64_t n, const Plan* plan, uint32_t P,
                         const std::vector<ScanGroup>& groups, const uint32_t* chunk_off,
                         const uint32_t* chunk_stream, uint32_t n_chunks, const ltl4c_result* out,
                         const uint32_t* const* rank = nullptr) {
    const uint32_t NL = g.n_levels;
    int32_t s = LTL4C_OK;
    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    uint32_t* z = reinterpret_cast<uint32_t*>(ws);
    uint32_t* scan_ticket = z + w.scan_ticket_off;
    uint32_t* root_counts = z + w.root_counts_off;
    uint32_t* sizes32 = z + w.sizes32_off;
    uint64_t* sizes64 = reinterpret_cast<uint64_t*>(z + w.sizes64_off);
    uint64_t* words_a = reinterpret_cast<uint64_t*>(ws + w.words_a_off);
    uint32_t* scan_status = z + w.scan_status_off;
    const hipStream_t st = ctx->stream;

    {
        ZeroArgs za{z, nullptr, 0, w.zero_words, 0};
        uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (w.zero_words + 255) / 256);
        s = launch(ctx, "zero", [&] { return launch_zero(za, blocks ? blocks : 1, st); });
        if (s) return s;
    }
    uint64_t* sorted = words_a;
    if (n > 0) {
        s = enqueue_front(ctx, L, g, w, ws, d_records, n, plan, chunk_off, chunk_stream, nullptr, n_chunks, true,
                          &sorted, ctx->sort_variant, rank);
        if (s) return s;
    }

    // parent events: the own events are the first n_own sorted words
    uint32_t* n_own = g.parent ? z + w.n_valid_off + 2 : nullptr;
    ParentArgs pa{};
    if (g.parent && n > 0) {
        pa.words = sorted;
        pa.n_kept = z + w.n_valid_off;
        pa.n_par = z + w.n_valid_off + 1;
        pa.n_own = n_own;
        s = launch(ctx, "parent", [&] { return launch_parent_counts(pa, st); });
        if (s) return s;
    }

    // per-instance arrays: the verdicts always exist (caller's or workspace)
    uint8_t* inst_verdict = out->inst_verdict ? out->inst_verdict : ws + w.inst_verdict_off;
    const uint64_t inst_stride = out->inst_verdict ? out->capacity : std::max<uint64_t>(n, 1);
    // per-level node arrays; node_start always lives in the workspace
    uint32_t* node_counts[kMaxLevels] = {nullptr, nullptr, nullptr, nullptr};
    uint64_t node_stride[kMaxLevels] = {0, 0, 0, 0};
    uint64_t node_limit[kMaxLevels] = {0, 0, 0, 0};
    uint32_t* node_start[kMaxLevels] = {nullptr, nullptr, nullptr, nullptr};
    for (uint32_t m = 1; m < NL; ++m) {
        node_start[m] = reinterpret_cast<uint32_t*>(ws + w.node_start_off[m]);
        if (out->node_counts[m]) {
            node_counts[m] = out->node_counts[m];
            node_stride[m] = out->capacity;
        } else {
            node_counts[m] = reinterpret_cast<uint32_t*>(ws + w.counts_off[m]);
            node_stride[m] = w.cap_node[m];
        }
        node_limit[m] = std::min(node_stride[m], w.cap_node[m]);
    }

    FinalizeArgs fa{};
    fa.n_props = P;
    fa.plan = plan;
    fa.root_counts = root_counts;
    fa.root_verdict = out->root_verdict;
    fa.root_counts_out = out->root_counts;
    fa.sizes_ws = sizes64;
    fa.sizes_out = out->sizes;
    fa.n_levels = NL;
    bool fused_finalize = false;
    if (n > 0) {
        ScanArgs sa{};
        sa.words = sorted;
        sa.n = (uint32_t)n;
        sa.n_dev = g.parent ? n_own : g.compact ? z + w.n_valid_off : nullptr;   // the first radix pass dropped excluded events
        sa.cbits = g.cbits + g.ibits;                        // where the key starts
        sa.class_mask = (1u << g.cbits) - 1u;
        sa.index_shift = g.cbits;
        sa.index_mask = g.ibits ? (uint32_t)((1ull << g.ibits) - 1u) : 0u;
        sa.n_levels = NL;
        for (uint32_t m = 1; m < NL; ++m) sa.prefix_shift[m] = sa.cbits + (g.key_bits_total - g.prefix_bits[m]);
        sa.valid_shift = sa.cbits + g.key_bits_total;
        sa.n_props_all = P;
        sa.plan = plan;
        sa.inst_verdict = inst_verdict;
        sa.inst_stride = inst_stride;
        sa.inst_limit = inst_stride;
        sa.inst_keys = out->inst_keys;
        for (uint32_t m = 1; m < NL; ++m) {
            sa.node_start[m] = node_start[m];
            sa.node_keys[m] = out->node_keys[m];
            sa.node_limit[m] = node_limit[m];
            sa.node_counts[m] = node_counts[m];
            sa.node_stride[m] = node_stride[m];
        }
        uint32_t* inst_parent = NL >= 2 ? reinterpret_cast<uint32_t*>(ws + w.inst_parent_off) : nullptr;
        sa.inst_parent = inst_parent;
        uint32_t* inst_start = reinterpret_cast<uint32_t*>(ws + w.inst_start_off);
        if (out->inst_conclusive) {
            sa.inst_conc = out->inst_conclusive;
            sa.inst_start = inst_start;
        }
        if (out->event_verdict) {
            // events that join no cluster keep "no instance"
            s = launch(ctx, "fill", [&] { return launch_fill_u8(out->event_verdict, LTL4C_NO_INSTANCE, (uint64_t)P * n, st); });
            if (s) return s;
            sa.event_verdict = out->event_verdict;
            sa.n_events = n;
        }
        sa.sizes = sizes64;
        sa.sizes32 = sizes32;
        sa.err = ctx->err_dev;
        // one launch per property group, each with its own look-back rows and
        // ticket; the first one also writes the numbering
        // The split map scan (reduce, spine, down sweep; its down sweep also
        // writes the verdict timeline on request).  With parent events it
        // numbers the own events (the verdicts come after).
        const bool split = ctx->scan_variant == kSplitScanVariant || ctx->scan_variant == kSplitScanVariant32;
        if (split) {
            if (!sa.n_dev) {
                // nothing is excluded: every word counts
                s = launch(ctx, "scan", [&] { return launch_set_u32(z + w.n_valid_off, (uint32_t)n, st); });
                if (s) return s;
                sa.n_dev = z + w.n_valid_off;
            }
            sa.desc = ws + w.ms_desc_off;
            sa.agg = reinterpret_cast<uint32_t*>(ws + w.ms_agg_off);
            sa.prefix = reinterpret_cast<uint32_t*>(ws + w.ms_prefix_off);
            sa.trec = reinterpret_cast<uint32_t*>(ws + w.ms_trec_off);
            sa.chunk_agg = reinterpret_cast<uint32_t*>(ws + w.ms_chunk_off);
            sa.chunk_pre = sa.chunk_agg + (uint64_t)kMsRec * (w.ms_tiles / kMsSpineThreads + 1);
            sa.tiles = w.ms_tiles;
        }
        // (with parent events only the numbering launch: the verdicts come after)
        for (size_t gi = 0; gi < (g.parent ? 1 : groups.size()); ++gi) {
            sa.n_props = groups[gi].cnt;
            std::memcpy(sa.prop_idx, groups[gi].idx, sizeof sa.prop_idx);
            sa.max_states = groups[gi].states;
            sa.structure = groups[gi].structure ? 1u : 0u;
            sa.status = scan_status + gi * 2ull * kScanRows * w.tiles_scan;
            sa.ticket = scan_ticket + gi;
            if (split) {
                sa.read_desc = gi > 0 ? 1u : 0u;    // the first launch wrote the descriptors
                const int items = ctx->scan_variant == kSplitScanVariant32 ? 32 : 16;
                s = launch(ctx, "scan", [&] { return launch_mapscan(sa, items, st); });
            } else {
                s = launch(ctx, "scan", [&] { return launch_scan(sa, ctx->scan_variant, st); });
            }
            if (s) return s;
        }

        if (g.parent) {
            // every instance's verdict with its parent events merged in
            pa.cbits = g.cbits;
            pa.class_mask = (1u << g.cbits) - 1u;
            pa.ibits = g.ibits;
            pa.index_mask = g.ibits ? (1ull << g.ibits) - 1ull : 0ull;
            pa.key_shift = g.cbits + g.ibits;
            pa.prefix_shift = pa.key_shift + L.key_bits[L.n_keys - 1];
            const uint32_t pbits = g.key_bits_total - g.stream_bits - L.key_bits[L.n_keys - 1];
            pa.prefix_mask = pbits ? (1ull << pbits) - 1ull : 0ull;
            pa.n_props = P;
            pa.plan = plan;
            pa.tree = reinterpret_cast<uint4*>(ws + w.pe_tree_off);
            for (uint32_t lv = 1; lv <= w.pe_levels; ++lv) {
                pa.tree_off[lv] = w.pe_tree_lvl[lv];
                pa.tree_cnt[lv] = w.pe_tree_cnt[lv];
            }
            pa.tile_agg = reinterpret_cast<uint4*>(ws + w.pe_tile_agg_off);
            pa.tile_prefix = reinterpret_cast<uint4*>(ws + w.pe_tile_prefix_off);
            pa.trec = reinterpret_cast<uint4*>(ws + w.pe_trec_off);
            pa.samples = reinterpret_cast<uint64_t*>(ws + w.pe_samples_off);
            pa.tile_heads = reinterpret_cast<uint32_t*>(ws + w.pe_tile_heads_off);
            pa.tile_head_prefix = reinterpret_cast<uint32_t*>(ws + w.pe_tile_hprefix_off);
            pa.inst_verdict = inst_verdict;
            pa.inst_stride = inst_stride;
            pa.inst_limit = inst_stride;
            pa.err = ctx->err_dev;
            s = launch(ctx, "parent", [&] { return launch_parent_samples(pa, st); });
            if (s) return s;
            for (uint32_t l0 = 0; l0 < w.pe_levels; l0 += kPeTreeLevelsPerLaunch) {
                const uint32_t nlev = std::min<uint32_t>(kPeTreeLevelsPerLaunch, w.pe_levels - l0);
                const uint64_t nodes0 = l0 ? w.pe_tree_cnt[l0] : n;
                s = launch(ctx, "parent", [&] { return launch_parent_tree(pa, l0, nlev, nodes0, st); });
                if (s) return s;
            }
            s = launch(ctx, "parent", [&] { return launch_parent_pass(pa, false, w.pe_tiles, st); });
            if (s) return s;
            s = launch(ctx, "parent", [&] { return launch_parent_spine(pa, st); });
            if (s) return s;
            s = launch(ctx, "parent", [&] { return launch_parent_pass(pa, true, w.pe_tiles, st); });
            if (s) return s;
        }
        if (out->inst_conclusive) {
            InstConclusiveArgs ia{};
            ia.inst_conc = out->inst_conclusive;
            ia.inst_start = inst_start;
            ia.n_inst = sizes32 + 0;
            ia.inst_limit = inst_stride;
            ia.inst_stride = inst_stride;
            ia.n_props = P;
            s = launch(ctx, "timeline", [&] { return launch_inst_conclusive(ia, st); });
            if (s) return s;
        }
        fused_finalize = NL >= 2;                             // the node-level root count ends with Def. 7
        for (int m = (int)NL - 1; m >= 0; --m) {
            CountArgs c{};
            c.level = (uint32_t)m;
            c.n_levels = NL;
            c.n_props = P;
            c.plan = plan;
            c.err = ctx->err_dev;
            if ((uint32_t)m + 1 == NL) {
                c.n_children = sizes32 + 0;
                c.child_limit = std::min<uint64_t>(inst_stride, n);
                c.child_verdict = inst_verdict;
                c.child_stride = inst_stride;
                c.child_parent = inst_parent;                 // null at the root
                c.items = 16;
            } else {
                c.items = 2;
                c.n_children = sizes32 + (m + 1);
                c.child_limit = node_limit[m + 1];
                c.child_counts = node_counts[m + 1];
                c.child_stride = node_stride[m + 1];
                c.child_verdict_out = out->node_verdict[m + 1];
            }
            if (m == 0) {
                c.counts = root_counts;
                c.stride = 1;
                c.node_limit = 1;
                if (fused_finalize) {
                    c.done = sizes32 + 32;
                    c.fin = fa;
                }
            } else {
                c.node_start = node_start[m];
                c.n_nodes = sizes32 + m;
                c.node_limit = node_limit[m];
                c.counts = node_counts[m];                    // zeroed by the scan as nodes appear
                c.stride = node_stride[m];
            }
            s = launch(ctx, "count", [&] { return launch_count(c, st); });
            if (s) return s;
        }
    }
    if (fused_finalize) return LTL4C_OK;
    s = launch(ctx, "finalize", [&] { return launch_finalize(fa, st); });
    return s;
}

// The property table of one evaluation, as the kernels read it.
static Plan host_plan(ltl4c_ctx* ctx, const int32_t* props, int32_t n_props) {
    Plan host;
    std::memset(&host, 0, sizeof host);
    for (int32_t i = 0; i < n_props; ++i) {
        const ltl4c_property& p = ctx->props[props[i]];
        host.prop[i] = make_prop(ctx->monitors[p.monitor], p);
    }
    std::memcpy(host.class_of_type, ctx->layout.class_of_type, 256);
    std::memcpy(host.key_present, ctx->layout.key_present, 256);
    return host;
}

// Dense ranks of every level's key values (see rank.hip): rank[m][i] for
// event i, and the value of every rank; the distinct counts land in the
// ranking area for the host to read.
static int32_t enqueue_ranks(ltl4c_ctx* ctx, const ltl4c_layout& L, const void* d_records, uint64_t n, uint8_t* area,
                             const RankRegion& rr, uint64_t* wa, uint64_t* wb) {
    const hipStream_t st = ctx->stream;
    uint32_t* z = reinterpret_cast<uint32_t*>(area + rr.zero_off);
    int32_t s = LTL4C_OK;
    for (uint32_t m = 0; m < L.n_keys && s == LTL4C_OK; ++m) {
        ZeroArgs za{z, nullptr, 0, rr.zero_words, 0};
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (rr.zero_words + 255) / 256);
        s = launch(ctx, "zero", [&] { return launch_zero(za, blocks ? blocks : 1, st); });
        if (s) return s;
        RankArgs ra{};
        ra.records = static_cast<const uint8_t*>(d_records);
        ra.n = n;
        ra.record_bytes = L.record_bytes;
        ra.type_dw = L.type_offset / 4;
        ra.type_shift = (L.type_offset % 4) * 8;
        ra.type_mask = L.type_bytes == 4 ? 0xFFFFFFFFu : ((1u << (8 * L.type_bytes)) - 1u);
        for (uint32_t t = 0; t < 256; ++t)
            if ((L.key_present[t] >> m) & 1u) ra.has_key[t >> 5] |= 1u << (t & 31u);
        ra.level = m;
        ra.key_dw = L.key_offset[m] / 4;
        ra.key_shift = (L.key_offset[m] % 4) * 8;
        ra.key_mask = L.key_bytes[m] == 4 ? 0xFFFFFFFFu : ((1u << (8 * L.key_bytes[m])) - 1u);
        ra.words = wa;
        ra.hist = z + rr.hist_w;
        ra.sorted = wa;
        ra.tile_cnt = reinterpret_cast<uint32_t*>(area + rr.tile_cnt_off);
        ra.tile_off = reinterpret_cast<uint32_t*>(area + rr.tile_off_off);
        ra.n_distinct = reinterpret_cast<uint32_t*>(area + rr.distinct_off) + m;
        ra.rank = reinterpret_cast<uint32_t*>(area + rr.rank_off[m]);
        ra.uniq = reinterpret_cast<uint32_t*>(area + rr.uniq_off[m]);
        s = launch(ctx, "rank", [&] { return launch_rank_prep(ra, st); });
        uint64_t* in = wa;
        uint64_t* outw = wb;
        for (uint32_t p = 0; p < 4 && s == LTL4C_OK; ++p) {
            SortPassArgs sa{};
            sa.in = in;
            sa.out = outw;
            sa.n = (uint32_t)n;
            sa.shift = 32 + 8 * p;
            sa.nbits = 8;
            sa.hist = z + rr.hist_w + 256 * p;
            sa.status = z + rr.status_w + (uint64_t)p * rr.tiles_sort * 256;
            sa.ticket = z + rr.ticket_w + p;
            sa.err = ctx->err_dev;
            s = launch(ctx, "rank", [&] { return launch_sort_pass(sa, ctx->sort_variant, 8, st); });
            std::swap(in, outw);
        }
        if (s == LTL4C_OK) s = launch(ctx, "rank", [&] { return launch_rank_scan(ra, st); });
    }
    return s;
}

// The values of the instances' and nodes' vectors, from their packed keys
// (through the rank tables when the keys were ranked).
static int32_t enqueue_key_values(ltl4c_ctx* ctx, const ltl4c_layout& L, const Geometry& g, const WsLayout& w,
                                  void* d_ws, uint64_t n, const ltl4c_result* out, const uint32_t* const* value_of) {
    const uint32_t* sizes32 = reinterpret_cast<const uint32_t*>(d_ws) + w.sizes32_off;
    (void)g;
    auto one = [&](const uint64_t* packed, uint32_t* dst, uint32_t level_of_count, uint32_t fields) {
        KeyValuesArgs ka{};
        ka.packed = packed;
        ka.n_dev = sizes32 + level_of_count;
        ka.limit = out->capacity;
        ka.n_fields = fields;
        uint32_t below = 0;
        for (int m = (int)fields - 1; m >= 0; --m) {
            ka.shift[m] = below;
            ka.mask[m] = (1ull << L.key_bits[m]) - 1ull;
            ka.uniq[m] = value_of[m];
            below += L.key_bits[m];
        }
        ka.uniq_cap = std::max<uint64_t>(n, 1);
        ka.out = dst;
        return launch(ctx, "key_values", [&] { return launch_key_values(ka, out->capacity, ctx->stream); });
    };
    int32_t s = LTL4C_OK;
    if (n > 0 && out->inst_key_values) s = one(out->inst_keys, out->inst_key_values, 0, L.n_keys);
    for (uint32_t m = 1; m < L.n_keys && s == LTL4C_OK; ++m)
        if (n > 0 && out->node_key_values[m]) s = one(out->node_keys[m], out->node_key_values[m], m, m);
    return s;
}

static int32_t eval_impl(ltl4c_ctx* ctx, const void* d_records, uint64_t n, const int32_t* props, int32_t n_props,
                         void* d_ws, uint64_t ws_bytes, const ltl4c_result* out, bool noalloc,
                         GraphHost* cap = nullptr);

int32_t ltl4c_eval(ltl4c_ctx* ctx, const void* d_records, uint64_t n, const int32_t* props, int32_t n_props,
                   void* d_ws, uint64_t ws_bytes, const ltl4c_result* out) {
    return eval_impl(ctx, d_records, n, props, n_props, d_ws, ws_bytes, out, false);
}

int32_t ltl4c_eval_noalloc(ltl4c_ctx* ctx, const void* d_records, uint64_t n, const int32_t* props, int32_t n_props,
                           const ltl4c_result* out) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    if (!ctx->scratch) return fail(LTL4C_EDEVICE, "the library's scratch memory has no address on this device");
    // the plan sits at the start of the scratch, the workspace after it
    const uint64_t plan_bytes = align256(sizeof(Plan));
    return eval_impl(ctx, d_records, n, props, n_props, ctx->scratch + plan_bytes, kNoAllocScratchBytes - plan_bytes,
                     out, true);
}

static int32_t capture_graph(ltl4c_ctx* ctx, GraphHost* gh, const std::function<int32_t()>& enqueue);

// cap: capture the kernel sequence into a graph instead of running it.
static int32_t eval_impl(ltl4c_ctx* ctx, const void* d_records, uint64_t n, const int32_t* props, int32_t n_props,
                         void* d_ws, uint64_t ws_bytes, const ltl4c_result* out, bool noalloc, GraphHost* cap) {
    int32_t s = check_props(ctx, props, n_props);
    if (s) return s;
    if (n > LTL4C_MAX_EVENTS) return fail(LTL4C_EUNSUPPORTED, "too many events for one call");
    if (n > 0 && !d_records) return fail(LTL4C_EINVAL, "records is NULL");
    if (!out || !out->root_verdict || !out->root_counts || !out->sizes)
        return fail(LTL4C_EINVAL, "root_verdict, root_counts and sizes are required");
    if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return fail(LTL4C_EINVAL, "workspace must be 256-byte aligned");
    // keys wider than the sort word: ranked first; the workspace is sized for
    // ranks of at most ceil(log2 n) bits and starts with the ranking area
    const bool ranked = needs_ranks(ctx->layout, n);
    ltl4c_layout L = ranked ? rank_sized(ctx->layout, n) : ctx->layout;
    const uint32_t P = (uint32_t)n_props;
    if (n > 0 && (reinterpret_cast<uintptr_t>(d_records) & 3))
        return fail(LTL4C_EINVAL, "records must be 4-byte aligned");
    SchedScope sc(ctx, find_sched(ctx, shape_of(ctx, 0, n, 0, props, n_props)));
    Geometry g = geometry(L, 0, false, true, sort_threads(ctx->sort_variant) >= 512);
    const std::vector<ScanGroup> groups = scan_groups(monitor_states(ctx, props, n_props));
    WsLayout w = plan_workspace(L, g, n, P, (uint32_t)groups.size(), ctx->sort_variant, ctx->scan_variant);
    uint64_t rbytes = ranked ? rank_region(L, n, ctx->sort_variant).total : 0;
    if (ws_bytes < rbytes + w.total && sc.changed()) {
        // a workspace sized for the context's own schedule: run that one
        sc.revert();
        g = geometry(L, 0, false, true, sort_threads(ctx->sort_variant) >= 512);
        w = plan_workspace(L, g, n, P, (uint32_t)groups.size(), ctx->sort_variant, ctx->scan_variant);
        rbytes = ranked ? rank_region(L, n, ctx->sort_variant).total : 0;
    }
    if (ws_bytes < rbytes + w.total) {
        if (!noalloc) return fail(LTL4C_ENOMEM, "workspace smaller than ltl4c_workspace_bytes()");
        char buf[200];
        std::snprintf(buf, sizeof buf,
                      "ltl4c_eval_noalloc: %llu events need %llu bytes of scratch; the library's scratch holds %llu "
                      "(use ltl4c_eval with a workspace)",
                      (unsigned long long)n, (unsigned long long)w.total, (unsigned long long)ws_bytes);
        return fail(LTL4C_ENOMEM, buf);
    }
    if ((out->inst_keys != nullptr) != (out->inst_verdict != nullptr))
        return fail(LTL4C_EINVAL, "inst_keys and inst_verdict are given together or not at all");
    if (out->inst_key_values && !out->inst_keys) return fail(LTL4C_EINVAL, "inst_key_values needs inst_keys");
    for (uint32_t m = 1; m < L.n_keys; ++m)
        if (out->node_key_values[m] && !out->node_keys[m])
            return fail(LTL4C_EINVAL, "node_key_values needs the node arrays of its level");
    const uint32_t* rank_of[kMaxLevels] = {nullptr, nullptr, nullptr, nullptr};
    const uint32_t* value_of[kMaxLevels] = {nullptr, nullptr, nullptr, nullptr};
    if (ranked) {
        if (noalloc || cap)
            return fail(LTL4C_EUNSUPPORTED, "keys wider than the sort word are ranked first, which waits for the "
                                            "device: not under graph capture or without allocation");
        HIP_TRY(hipSetDevice(ctx->device));
        uint8_t* ws8 = static_cast<uint8_t*>(d_ws);
        const RankRegion rr = rank_region(L, n, ctx->sort_variant);
        uint64_t* wa = reinterpret_cast<uint64_t*>(ws8 + rr.total + w.words_a_off);
        uint64_t* wb = reinterpret_cast<uint64_t*>(ws8 + rr.total + w.words_b_off);
        s = enqueue_ranks(ctx, ctx->layout, d_records, n, ws8, rr, wa, wb);
        if (s) return s;
        uint32_t distinct[kMaxLevels] = {0, 0, 0, 0};
        HIP_TRY(hipMemcpyAsync(distinct, ws8 + rr.distinct_off, sizeof distinct, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        for (uint32_t m = 0; m < L.n_keys; ++m) {
            L.key_bits[m] = std::max<uint32_t>(1, bits_for(std::max<uint32_t>(distinct[m], 1)));
            rank_of[m] = reinterpret_cast<const uint32_t*>(ws8 + rr.rank_off[m]);
            value_of[m] = reinterpret_cast<const uint32_t*>(ws8 + rr.uniq_off[m]);
        }
        // the evaluation proper, on the ranks, in the workspace after the ranking area
        g = geometry(L, 0, false, true, sort_threads(ctx->sort_variant) >= 512);
        w = plan_workspace(L, g, n, P, (uint32_t)groups.size(), ctx->sort_variant, ctx->scan_variant);
        d_ws = ws8 + rr.total;
        ws_bytes -= rr.total;
        if (g.cbits + g.key_bits_total + (g.excl ? 1 : 0) > 63)
            return fail(LTL4C_EUNSUPPORTED, "even ranked, the binding key plus class bits exceed 63 bits");
    }
    if (g.parent) {
        if (out->event_verdict || out->inst_conclusive)
            return fail(LTL4C_EUNSUPPORTED, "the verdict timeline is not available with parent events");
        // the parent events are searched by (parent prefix, trace index)
        g.ibits = std::max<uint32_t>(1, bits_for((uint32_t)std::max<uint64_t>(n, 1)));
        if (g.cbits + g.ibits + g.key_bits_total + 1 > 63)
            return fail(LTL4C_EUNSUPPORTED, "parent events: binding key, kind bit, class and trace index exceed 63 bits");
    }
    if (out->event_verdict) {
        // the trace index rides in the sort word between the class and the key
        g.ibits = std::max<uint32_t>(1, bits_for((uint32_t)std::max<uint64_t>(n, 1)));
        if (g.cbits + g.ibits + g.key_bits_total + (g.excl ? 1 : 0) > 63)
            return fail(LTL4C_EUNSUPPORTED, "event_verdict: binding key, class and trace index exceed 63 bits");
    }
    if (out->inst_conclusive) {
        if (!out->inst_verdict) return fail(LTL4C_EINVAL, "inst_conclusive needs inst_verdict");
        // T and F must be final: a conclusive state only leads to states of its label
        for (int32_t i = 0; i < n_props; ++i) {
            const MonitorHost& M = ctx->monitors[ctx->props[props[i]].monitor];
            for (uint32_t q = 0; q < M.n_states; ++q) {
                const uint8_t l = M.label[q];
                if (l != LTL4C_BOT && l != LTL4C_TOP) continue;
                for (uint32_t c = 0; c < M.n_classes; ++c)
                    if (M.label[M.delta[q * M.n_classes + c]] != l)
                        return fail(LTL4C_EINVAL, "inst_conclusive needs monitors whose T and F states are final");
            }
        }
    }
    bool any_optional = out->inst_verdict != nullptr;
    for (uint32_t m = 1; m < L.n_keys; ++m) {
        const bool k = out->node_keys[m] != nullptr, c = out->node_counts[m] != nullptr,
                   v = out->node_verdict[m] != nullptr;
        if (k != c || c != v)
            return fail(LTL4C_EINVAL, "node_keys, node_counts and node_verdict of a level go together");
        any_optional = any_optional || c;
    }
    if (any_optional && out->capacity == 0)
        return fail(LTL4C_EINVAL, "capacity must be > 0 when optional outputs are given");
    Plan* plan = nullptr;
    if (!noalloc) {
        s = get_plan(ctx, props, n_props, &plan);
        if (s) return s;
        HIP_TRY(hipSetDevice(ctx->device));
        auto enqueue = [&]() {
            int32_t e = eval_core(ctx, L, g, w, d_ws, d_records, n, plan, P, groups, nullptr, nullptr, 0, out,
                                  ranked ? rank_of : nullptr);
            if (e == LTL4C_OK) e = enqueue_key_values(ctx, L, g, w, d_ws, n, out, value_of);
            return e;
        };
        return cap ? capture_graph(ctx, cap, enqueue) : enqueue();
    }
    // no allocation: the plan travels inside kernel launches into the
    // scratch, and no profiling events are taken
    HIP_TRY(hipSetDevice(ctx->device));
    const Plan hp = host_plan(ctx, props, n_props);
    plan = reinterpret_cast<Plan*>(ctx->scratch);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&hp);
    static_assert(sizeof(Plan) % 4 == 0, "the plan is copied in 32-bit words");
    const uint32_t words = (uint32_t)(sizeof(Plan) / 4);
    ctx->no_timing = true;
    for (uint32_t at = 0; at < words && s == LTL4C_OK; at += kPutWords) {
        PutWords pw;
        pw.n = std::min<uint32_t>(kPutWords, words - at);
        std::memcpy(pw.w, src + at, 4ull * pw.n);
        s = launch(ctx, "put_words", [&] {
            return launch_put_words(reinterpret_cast<uint32_t*>(ctx->scratch) + at, pw, ctx->stream);
        });
    }
    if (s == LTL4C_OK) s = eval_core(ctx, L, g, w, d_ws, d_records, n, plan, P, groups, nullptr, nullptr, 0, out);
    if (s == LTL4C_OK) s = enqueue_key_values(ctx, L, g, w, d_ws, n, out, value_of);
    ctx->no_timing = false;
    return s;
}


// ---- batches of traces -----------------------------------------------------
namespace {

struct BatchLayout {
    Geometry g;
    WsLayout w;
    uint64_t root_off, keys_off, counts_off, verdict_off, cap1, total;
};

int32_t batch_layout(ltl4c_ctx* ctx, uint64_t n, int32_t n_traces, uint32_t P, uint32_t n_scan_groups,
                     BatchLayout* b) {
    const ltl4c_layout& L = ctx->layout;
    if (n_traces < 1 || n_traces > (int32_t)kMaxChunks) return fail(LTL4C_EUNSUPPORTED, "n_traces must be 1..4096");
    if (L.n_keys + 1 > (uint32_t)kMaxLevels)
        return fail(LTL4C_EUNSUPPORTED, "a batch takes properties with at most 3 quantifiers");
    if (L.parent_events) return fail(LTL4C_EUNSUPPORTED, "batches do not take layouts with parent events");
    if (n > LTL4C_MAX_EVENTS) return fail(LTL4C_EUNSUPPORTED, "too many events for one call");
    b->g = geometry(L, std::max<uint32_t>(1, bits_for((uint32_t)n_traces)), true, true,
                    sort_threads(ctx->sort_variant) >= 512);
    if (b->g.cbits + b->g.key_bits_total + (b->g.excl ? 1 : 0) > 63)
        return fail(LTL4C_EUNSUPPORTED, "trace id, keys and class bits exceed 63 bits");
    b->w = plan_workspace(L, b->g, n, P, n_scan_groups, ctx->sort_variant, ctx->scan_variant);
    b->cap1 = b->w.cap_node[1];
    uint64_t off = align256(b->w.total);
    b->root_off = off;    off = align256(off + 2048);     // outputs of the artificial root
    b->keys_off = off;    off = align256(off + 8 * b->cap1);
    b->counts_off = off;  off = align256(off + 24ull * P * b->cap1);
    b->verdict_off = off; off = align256(off + (uint64_t)P * b->cap1);
    b->total = off;
    return LTL4C_OK;
}

}  // namespace

int32_t ltl4c_batch_workspace_bytes(ltl4c_ctx* ctx, uint64_t n_events, int32_t n_traces, const int32_t* props,
                                    int32_t n_props, uint64_t* bytes) {
    int32_t s = check_props(ctx, props, n_props);
    if (s) return s;
    if (!bytes) return fail(LTL4C_EINVAL, "bytes is NULL");
    const uint32_t n_groups = (uint32_t)scan_groups(monitor_states(ctx, props, n_props)).size();
    BatchLayout b;
    s = batch_layout(ctx, n_events, n_traces, (uint32_t)n_props, n_groups, &b);
    if (s) return s;
    uint64_t total = b.total;
    SchedScope sc(ctx, find_sched(ctx, shape_of(ctx, 1, n_events, n_traces, props, n_props)));
    if (sc.changed() && batch_layout(ctx, n_events, n_traces, (uint32_t)n_props, n_groups, &b) == LTL4C_OK)
        total = std::max(total, b.total);
    *bytes = total;
    return LTL4C_OK;
}


// cap: capture the kernel sequence into a graph instead of running it; the
// trace table then lives in the graph's own device buffer.
static int32_t batch_impl(ltl4c_ctx* ctx, const void* d_records, const uint64_t* offsets, int32_t n_traces,
                          const int32_t* props, int32_t n_props, void* d_ws, uint64_t ws_bytes,
                          uint8_t* d_root_verdict, uint64_t* d_root_counts, GraphHost* cap) {
    int32_t s = check_props(ctx, props, n_props);
    if (s) return s;
    if (!offsets || !d_root_verdict || !d_root_counts) return fail(LTL4C_EINVAL, "NULL argument");
    if (n_traces < 1 || n_traces > (int32_t)kMaxChunks) return fail(LTL4C_EUNSUPPORTED, "n_traces must be 1..4096");
    if (offsets[0] != 0) return fail(LTL4C_EINVAL, "offsets[0] must be 0");
    for (int32_t t = 0; t < n_traces; ++t)
        if (offsets[t + 1] < offsets[t]) return fail(LTL4C_EINVAL, "offsets must be non-decreasing");
    const uint64_t n = offsets[n_traces];
    const uint32_t P = (uint32_t)n_props;
    const std::vector<ScanGroup> groups = scan_groups(monitor_states(ctx, props, n_props));
    SchedScope sc(ctx, find_sched(ctx, shape_of(ctx, 1, n, n_traces, props, n_props)));
    BatchLayout b;
    s = batch_layout(ctx, n, n_traces, P, (uint32_t)groups.size(), &b);
    if (s) return s;
    if (ws_bytes < b.total && sc.changed()) {
        sc.revert();
        s = batch_layout(ctx, n, n_traces, P, (uint32_t)groups.size(), &b);
        if (s) return s;
    }
    if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return fail(LTL4C_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < b.total) return fail(LTL4C_ENOMEM, "workspace smaller than ltl4c_batch_workspace_bytes()");
    if (n > 0 && (!d_records || (reinterpret_cast<uintptr_t>(d_records) & 3)))
        return fail(LTL4C_EINVAL, "records must be non-NULL and 4-byte aligned");
    Plan* plan = nullptr;
    s = get_plan(ctx, props, n_props, &plan, 1);
    if (s) return s;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!ctx->batch_chunk_dev) {
        HIP_TRY(hipMalloc(&ctx->batch_chunk_dev, 4 * (2 * kMaxChunks + 2)));
        HIP_TRY(hipHostMalloc(&ctx->batch_chunk_host, 4 * (2 * kMaxChunks + 2), hipHostMallocDefault));
        HIP_TRY(hipEventCreateWithFlags(&ctx->batch_ev, hipEventDisableTiming));
    }
    // trace table: chunk t is trace t
    const uint64_t table_bytes = 4ull * (2 * n_traces + 1);
    uint32_t* table = ctx->batch_chunk_dev;
    if (cap) {
        std::vector<uint32_t> h(2 * n_traces + 1);
        for (int32_t t = 0; t <= n_traces; ++t) h[t] = (uint32_t)offsets[t];
        for (int32_t t = 0; t < n_traces; ++t) h[n_traces + 1 + t] = (uint32_t)t;
        HIP_TRY(hipMalloc(&cap->table_dev, table_bytes));
        HIP_TRY(hipMemcpy(cap->table_dev, h.data(), table_bytes, hipMemcpyHostToDevice));
        table = static_cast<uint32_t*>(cap->table_dev);
    } else {
        HIP_TRY(hipEventSynchronize(ctx->batch_ev));
        uint32_t* h = ctx->batch_chunk_host;
        for (int32_t t = 0; t <= n_traces; ++t) h[t] = (uint32_t)offsets[t];
        for (int32_t t = 0; t < n_traces; ++t) h[n_traces + 1 + t] = (uint32_t)t;
        HIP_TRY(hipMemcpyAsync(ctx->batch_chunk_dev, h, table_bytes, hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipEventRecord(ctx->batch_ev, ctx->stream));
    }

    uint8_t* ws = static_cast<uint8_t*>(d_ws);
    ltl4c_result r{};
    r.root_verdict = ws + b.root_off;                                   // artificial root: unused
    r.root_counts = reinterpret_cast<uint64_t*>(ws + b.root_off + 256);
    r.sizes = reinterpret_cast<uint64_t*>(ws + b.root_off + 1024);
    r.capacity = b.cap1;
    r.node_keys[1] = reinterpret_cast<uint64_t*>(ws + b.keys_off);
    r.node_counts[1] = reinterpret_cast<uint32_t*>(ws + b.counts_off);
    r.node_verdict[1] = ws + b.verdict_off;
    BatchOutArgs o{};
    o.n_props = P;
    o.n_traces = (uint32_t)n_traces;
    o.plan = plan;
    o.n_nodes = reinterpret_cast<uint32_t*>(ws) + b.w.sizes32_off + 1;
    o.node_keys = r.node_keys[1];
    o.node_counts = r.node_counts[1];
    o.node_verdict = r.node_verdict[1];
    o.stride = b.cap1;
    o.verdict = d_root_verdict;
    o.counts = d_root_counts;
    auto enqueue = [&]() -> int32_t {
        int32_t e = eval_core(ctx, ctx->layout, b.g, b.w, d_ws, d_records, n, plan, P, groups, table, table + n_traces + 1,
                              (uint32_t)n_traces, &r);
        if (e) return e;
        return launch(ctx, "batch_out", [&] { return launch_batch_out(o, ctx->stream); });
    };
    return cap ? capture_graph(ctx, cap, enqueue) : enqueue();
}

int32_t ltl4c_eval_batch(ltl4c_ctx* ctx, const void* d_records, const uint64_t* offsets, int32_t n_traces,
                         const int32_t* props, int32_t n_props, void* d_ws, uint64_t ws_bytes,
                         uint8_t* d_root_verdict, uint64_t* d_root_counts) {
    return batch_impl(ctx, d_records, offsets, n_traces, props, n_props, d_ws, ws_bytes, d_root_verdict,
                      d_root_counts, nullptr);
}

int32_t ltl4c_wait(ltl4c_ctx* ctx) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    uint32_t err = 0;
    HIP_TRY(hipMemcpy(&err, ctx->err_dev, 4, hipMemcpyDeviceToHost));
    if (err) {
        HIP_TRY(hipMemset(ctx->err_dev, 0, 4));
        if (err & kErrSpin) return fail(LTL4C_EDEVICE, "a look-back wait exceeded its bound");
        if (err & kErrData)
            return fail(LTL4C_EDEVICE, "an internal consistency check failed on the device "
                                       "(a verdict outside 0..5 or a sort destination past the kept events)");
        if (err & kErrRange) return fail(LTL4C_ERANGE, "an event key exceeds its declared key_bits");
        if (err & kErrCapacity) return fail(LTL4C_ECAPACITY, "more instances or nodes than the capacity");
    }
    return LTL4C_OK;
}


int32_t ltl4c_set_memory_budget(ltl4c_ctx* ctx, uint64_t bytes) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    ctx->budget = bytes;
    return LTL4C_OK;
}

int32_t ltl4c_group_bytes(ltl4c_ctx* ctx, const int32_t* props, int32_t n_props, uint32_t max_streams,
                          uint32_t max_bindings, uint64_t max_batch, uint64_t* bytes) {
    if (!bytes) return fail(LTL4C_EINVAL, "bytes is NULL");
    GroupHost G;
    int32_t s = group_configure(ctx, G, props, n_props, max_streams, max_bindings,
                                (uint64_t)max_streams * max_bindings, max_batch);
    if (s) return s;
    *bytes = G.total_bytes;
    return LTL4C_OK;
}

static int32_t group_open_impl(ltl4c_ctx* ctx, const int32_t* props, int32_t n_props, uint32_t max_streams,
                               uint32_t max_bindings, uint64_t table_bindings, uint64_t max_batch, bool admit_all,
                               int32_t* group) {
    if (!group) return fail(LTL4C_EINVAL, "group is NULL");
    GroupHost* G = new GroupHost();
    int32_t s = group_configure(ctx, *G, props, n_props, max_streams, max_bindings, table_bindings, max_batch);
    if (s) {
        delete G;
        return s;
    }
    if (ctx->used + G->total_bytes > ctx->budget) {
        delete G;
        return fail(LTL4C_EADMIT, "the group does not fit the memory budget");
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipMalloc(&G->state, G->state_bytes);
    if (e == hipSuccess) e = hipMalloc(&G->ws, G->ws_bytes);
    if (e == hipSuccess) e = hipMalloc(&G->chunk_dev, 4 * kChunkTableWords);
    if (e == hipSuccess) e = hipHostMalloc(&G->chunk_host, 4 * kChunkTableWords * kChunkRing, hipHostMallocDefault);
    for (int i = 0; i < kChunkRing && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&G->ring_ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
        group_free(G);
        return fail(e == hipErrorOutOfMemory ? LTL4C_ENOMEM : LTL4C_EDEVICE,
                    std::string("group allocation: ") + hipGetErrorString(e));
    }
    // plans: the real properties, and one virtual property per (property, start state)
    Plan host;
    std::memset(&host, 0, sizeof host);
    std::memcpy(host.class_of_type, ctx->layout.class_of_type, 256);
    std::memcpy(host.key_present, ctx->layout.key_present, 256);
    Plan vhost = host;
    uint32_t v = 0;
    for (uint32_t p = 0; p < G->P; ++p) {
        const ltl4c_property& prop = ctx->props[G->props[p]];
        const MonitorHost& M = ctx->monitors[prop.monitor];
        host.prop[p] = make_prop(M, prop);
        G->gs.vbase[p] = v;
        for (uint32_t q = 0; q < M.n_states; ++q) {
            vhost.prop[v] = make_prop(M, prop);
            vhost.prop[v].q0 = q;
            ++v;
        }
    }
    e = hipMalloc(&G->rplan, sizeof(Plan));
    if (e == hipSuccess) e = hipMalloc(&G->vplan, sizeof(Plan));
    if (e == hipSuccess) e = hipMemcpy(G->rplan, &host, sizeof(Plan), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(G->vplan, &vhost, sizeof(Plan), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        group_free(G);
        return fail(LTL4C_EDEVICE, std::string("group plan upload: ") + hipGetErrorString(e));
    }
    const uint32_t L = ctx->layout.n_keys;
    group_state_layout(*G, L, G->state, &G->gs);
    GroupState& gs = G->gs;
    gs.n_props = G->P;
    gs.n_levels = L;
    gs.plan = G->rplan;
    for (uint32_t m = 1; m < L; ++m) gs.level_shift[m] = G->g.key_bits_total - G->g.prefix_bits[m];
    gs.stream_shift = G->g.key_bits_total - G->g.stream_bits;
    gs.max_streams = G->S;
    gs.err = ctx->err_dev;
    // empty tree: no keys, no verdicts yet, zero counts; then value every root
    const hipStream_t st = ctx->stream;
    e = hipMemsetAsync(G->state, 0, G->state_bytes, st);
    if (e == hipSuccess && admit_all) e = hipMemsetD32Async(gs.stream_max, (int)max_bindings, G->S, st);
    if (e == hipSuccess) e = launch_fill_u64(gs.bslot, 2 * (gs.bmask + 1), kEmptyKey, st);
    for (uint32_t m = 1; m < L && e == hipSuccess; ++m) {
        e = launch_fill_u64(gs.nkeys[m], gs.nmask + 1, kEmptyKey, st);
        if (e == hipSuccess) e = launch_fill_u8(gs.nverdict[m], (uint64_t)G->P * (gs.nmask + 1), kNoVerdict, st);
    }
    if (e == hipSuccess) e = launch_group_roots(gs, true, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        group_free(G);
        return fail(LTL4C_EDEVICE, std::string("group initialisation: ") + hipGetErrorString(e));
    }
    ctx->used += G->total_bytes;
    int32_t id = -1;
    for (size_t i = 0; i < ctx->groups.size(); ++i)
        if (!ctx->groups[i]) {
            id = (int32_t)i;
            break;
        }
    if (id < 0) {
        id = (int32_t)ctx->groups.size();
        ctx->groups.push_back(nullptr);
    }
    ctx->groups[id] = G;
    G->open.assign(G->S, admit_all ? 1 : 0);
    G->smax.assign(G->S, admit_all ? max_bindings : 0u);
    G->admitted = admit_all ? (uint64_t)G->S * max_bindings : 0;
    G->next_seq.assign(G->S, 0);
    G->done_seq.assign(G->S, 0);
    G->last_push.assign(G->S, std::chrono::steady_clock::now());
    *group = id;
    return LTL4C_OK;
}

int32_t ltl4c_group_open(ltl4c_ctx* ctx, const int32_t* props, int32_t n_props, uint32_t max_streams,
                         uint32_t max_bindings, uint64_t max_batch, int32_t* group) {
    return group_open_impl(ctx, props, n_props, max_streams, max_bindings, (uint64_t)max_streams * max_bindings,
                           max_batch, true, group);
}

int32_t ltl4c_group_open_pool(ltl4c_ctx* ctx, const int32_t* props, int32_t n_props, uint32_t max_streams,
                              uint64_t pool_bindings, uint64_t max_batch, int32_t* group) {
    if (pool_bindings < 1 || pool_bindings > (1ull << 31))
        return fail(LTL4C_EUNSUPPORTED, "pool_bindings must be in 1..2^31");
    return group_open_impl(ctx, props, n_props, max_streams, (uint32_t)std::min<uint64_t>(pool_bindings, 0xFFFFFFFFu),
                           pool_bindings, max_batch, false, group);
}

int32_t ltl4c_stream_open(ltl4c_ctx* ctx, int32_t group, uint32_t stream, uint32_t max_bindings, uint64_t first_seq) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    if (stream >= G->S) return fail(LTL4C_EINVAL, "stream id >= max_streams");
    if (max_bindings < 1) return fail(LTL4C_EINVAL, "max_bindings must be >= 1");
    if (G->open[stream]) return fail(LTL4C_ESEQ, "the stream is already open");
    if (G->admitted + max_bindings > G->table_bindings)
        return fail(LTL4C_EADMIT, "the group's binding pool cannot hold this stream's max_bindings");
    HIP_TRY(hipSetDevice(ctx->device));
    s = launch(ctx, "set_u32", [&] { return launch_set_u32(G->gs.stream_max + stream, max_bindings, ctx->stream); });
    if (s) return s;
    G->open[stream] = 1;
    G->smax[stream] = max_bindings;
    G->admitted += max_bindings;
    G->next_seq[stream] = G->done_seq[stream] = first_seq;
    G->last_push[stream] = std::chrono::steady_clock::now();
    return LTL4C_OK;
}

int32_t ltl4c_stream_close(ltl4c_ctx* ctx, int32_t group, uint32_t stream) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    if (stream >= G->S) return fail(LTL4C_EINVAL, "stream id >= max_streams");
    if (!G->open[stream]) return fail(LTL4C_ESEQ, "the stream is not open");
    HIP_TRY(hipSetDevice(ctx->device));
    s = launch(ctx, "group_purge", [&] { return launch_group_purge(G->gs, stream, ctx->stream); });
    if (s) return s;
    s = launch(ctx, "set_u32", [&] { return launch_set_u32(G->gs.stream_max + stream, 0u, ctx->stream); });
    if (s) return s;
    G->open[stream] = 0;
    G->admitted -= G->smax[stream];
    G->smax[stream] = 0;
    return LTL4C_OK;
}

// Completed pushes, oldest first, update the per-stream completed sequence numbers.
static int32_t drain_pending(GroupHost* G) {
    while (!G->pending.empty()) {
        hipError_t q = hipEventQuery(G->pending.front().ev);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return fail(LTL4C_EDEVICE, std::string("push completion: ") + hipGetErrorString(q));
        for (auto& sa : G->pending.front().seq_after) G->done_seq[sa.first] = std::max(G->done_seq[sa.first], sa.second);
        G->spare_events.push_back(G->pending.front().ev);
        G->pending.pop_front();
    }
    return LTL4C_OK;
}

int32_t ltl4c_stream_poll(ltl4c_ctx* ctx, int32_t group, uint32_t stream, uint64_t* next_seq, uint64_t* done_seq) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    if (stream >= G->S) return fail(LTL4C_EINVAL, "stream id >= max_streams");
    HIP_TRY(hipSetDevice(ctx->device));
    s = drain_pending(G);
    if (s) return s;
    if (next_seq) *next_seq = G->next_seq[stream];
    if (done_seq) *done_seq = G->done_seq[stream];
    return LTL4C_OK;
}

int32_t ltl4c_group_stalled(ltl4c_ctx* ctx, int32_t group, uint64_t idle_ns, uint32_t* streams, uint32_t capacity,
                            uint32_t* n_stalled) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    if (!n_stalled || (capacity && !streams)) return fail(LTL4C_EINVAL, "outputs are NULL");
    const auto now = std::chrono::steady_clock::now();
    uint32_t n = 0;
    for (uint32_t i = 0; i < G->S; ++i) {
        if (!G->open[i]) continue;
        const uint64_t idle = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(now - G->last_push[i]).count();
        if (idle >= idle_ns) {
            if (n < capacity) streams[n] = i;
            ++n;
        }
    }
    *n_stalled = n;
    return LTL4C_OK;
}

int32_t ltl4c_group_read_nodes(ltl4c_ctx* ctx, int32_t group, uint32_t level, uint64_t* d_keys, uint32_t* d_counts,
                               uint8_t* d_verdict, uint64_t capacity, uint64_t* d_n) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    if (level < 1 || level >= G->gs.n_levels) return fail(LTL4C_EINVAL, "level must be 1..n_levels-1");
    if (!d_keys || !d_counts || !d_verdict || !d_n) return fail(LTL4C_EINVAL, "outputs are NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    s = launch(ctx, "zero", [&] { return launch_set_u32(reinterpret_cast<uint32_t*>(d_n), 0u, ctx->stream); });
    if (s) return s;
    s = launch(ctx, "zero", [&] { return launch_set_u32(reinterpret_cast<uint32_t*>(d_n) + 1, 0u, ctx->stream); });
    if (s) return s;
    return launch(ctx, "group_nodes", [&] {
        return launch_group_nodes(G->gs, level, d_keys, d_counts, d_verdict, capacity, d_n, ctx->stream);
    });
}

int32_t ltl4c_group_close(ltl4c_ctx* ctx, int32_t group) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->used -= G->total_bytes;
    group_free(G);
    ctx->groups[group] = nullptr;
    return LTL4C_OK;
}

// Host memory of a push must be pinned (page-locked, allocated by HIP), so
// that the copy engine can read it while the host goes on.
static bool pinned_host(const void* p) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeHost;
}

// Host-side bookkeeping once a push is enqueued: sequence numbers, the
// completion event poll reads, the time of the stream's last push.
static int32_t note_push(ltl4c_ctx* ctx, GroupHost* G, const uint32_t* streams, int32_t n_chunks) {
    GroupHost::Pending pd;
    const auto now = std::chrono::steady_clock::now();
    for (int32_t i = 0; i < n_chunks; ++i) {
        const uint32_t st = streams[i];
        ++G->next_seq[st];
        G->last_push[st] = now;
    }
    for (int32_t i = 0; i < n_chunks; ++i) {
        const uint32_t st = streams[i];
        bool seen = false;
        for (auto& sa : pd.seq_after)
            if (sa.first == st) seen = true;
        if (!seen) pd.seq_after.emplace_back(st, G->next_seq[st]);
    }
    if (G->spare_events.empty()) {
        hipEvent_t e = nullptr;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        G->spare_events.push_back(e);
    }
    pd.ev = G->spare_events.back();
    G->spare_events.pop_back();
    HIP_TRY(hipEventRecord(pd.ev, ctx->stream));
    G->pending.push_back(std::move(pd));
    return drain_pending(G);
}

// Shared by the push entry points: chunk i holds sizes[i] records at
// chunk_ptr[i] (or at d_records + offset when chunk_ptr is NULL).  seqs, when
// given, are the chunks' sequence numbers (checked against each stream's
// next one).  from_host: chunk_ptr points to pinned host memory.
static int32_t capture_graph(ltl4c_ctx* ctx, GraphHost* gh, const std::function<int32_t()>& enqueue);

// cap: capture the push's kernel sequence into a graph (device chunks only)
// instead of running it; the chunk table then lives in the graph's own
// device buffer, and each replay counts as a push of the same chunks.
static int32_t group_push_impl(ltl4c_ctx* ctx, int32_t group, const void* d_records, const void* const* chunk_ptr,
                               const uint64_t* sizes, const uint32_t* streams, int32_t n_chunks,
                               const uint64_t* seqs = nullptr, bool from_host = false, GraphHost* cap = nullptr) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    if (cap && from_host) return fail(LTL4C_EINVAL, "a captured push takes device chunks only");
    if (n_chunks < 1 || n_chunks > (int32_t)kMaxChunks) return fail(LTL4C_EINVAL, "n_chunks must be 1..4096");
    if (!sizes || !streams) return fail(LTL4C_EINVAL, "chunk sizes / streams are NULL");
    uint64_t n = 0;
    bool vec_ok = ctx->layout.record_bytes == 16;
    for (int32_t i = 0; i < n_chunks; ++i) {
        if (streams[i] >= G->S) return fail(LTL4C_EINVAL, "stream id >= max_streams");
        if (!G->open[streams[i]]) return fail(LTL4C_ESEQ, "push to a stream that is not open");
        if (chunk_ptr && sizes[i] > 0) {
            const uintptr_t a = reinterpret_cast<uintptr_t>(chunk_ptr[i]);
            if (!a || (a & 3)) return fail(LTL4C_EINVAL, "chunk records must be non-NULL and 4-byte aligned");
            if (a & 15) vec_ok = false;
            if (from_host && !pinned_host(chunk_ptr[i]))
                return fail(LTL4C_EINVAL, "host chunks must be in pinned memory (hipHostMalloc)");
        }
        n += sizes[i];
    }
    if (seqs) {
        // every chunk must carry its stream's next sequence number: a smaller
        // one repeats a chunk, a larger one leaves a gap
        std::vector<std::pair<uint32_t, uint64_t>> expect;
        for (int32_t i = 0; i < n_chunks; ++i) {
            uint64_t* e = nullptr;
            for (auto& x : expect)
                if (x.first == streams[i]) e = &x.second;
            if (!e) {
                expect.emplace_back(streams[i], G->next_seq[streams[i]]);
                e = &expect.back().second;
            }
            if (seqs[i] != *e) {
                char buf[160];
                std::snprintf(buf, sizeof buf, "stream %u: chunk sequence number %llu, expected %llu (%s)", streams[i],
                              (unsigned long long)seqs[i], (unsigned long long)*e,
                              seqs[i] < *e ? "duplicate" : "gap");
                return fail(LTL4C_ESEQ, buf);
            }
            ++*e;
        }
    }
    if (n > G->max_batch) return fail(LTL4C_ECAPACITY, "batch larger than the group's max_batch");
    if (!chunk_ptr && n > 0 && (!d_records || (reinterpret_cast<uintptr_t>(d_records) & 3)))
        return fail(LTL4C_EINVAL, "records must be non-NULL and 4-byte aligned");
    HIP_TRY(hipSetDevice(ctx->device));
    if (n == 0) {
        if (cap) return fail(LTL4C_EINVAL, "a captured push needs events");
        return note_push(ctx, G, streams, n_chunks);
    }
    const hipStream_t st = ctx->stream;
    if (from_host) {
        // copy the chunks into one of two device staging buffers on the copy
        // stream (the buffer's previous push must have consumed it), then run
        // the push from there: the copy of one push overlaps the kernels of
        // the one before
        const uint64_t rb = ctx->layout.record_bytes;
        if (!G->copy_stream) {
            const uint64_t bytes = align256(G->max_batch * rb);
            if (ctx->used + 2 * bytes > ctx->budget)
                return fail(LTL4C_EADMIT, "host-memory staging does not fit the memory budget");
            hipError_t e = hipStreamCreateWithFlags(&G->copy_stream, hipStreamNonBlocking);
            for (int i = 0; i < 2 && e == hipSuccess; ++i) {
                e = hipMalloc(&G->stage[i], bytes);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&G->stage_free[i], hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&G->stage_ready[i], hipEventDisableTiming);
            }
            if (e != hipSuccess) return fail(LTL4C_ENOMEM, std::string("host-memory staging: ") + hipGetErrorString(e));
            G->stage_bytes = 2 * bytes;
            G->total_bytes += 2 * bytes;
            ctx->used += 2 * bytes;
        }
        const int b = G->stage_i;
        uint8_t* dst = G->stage[b];
        HIP_TRY(hipStreamWaitEvent(G->copy_stream, G->stage_free[b], 0));
        uint64_t off = 0;
        for (int32_t i = 0; i < n_chunks;) {
            // adjacent chunks in host memory go in one copy
            const uint8_t* src = static_cast<const uint8_t*>(chunk_ptr[i]);
            uint64_t len = sizes[i] * rb;
            int32_t j = i + 1;
            while (j < n_chunks && static_cast<const uint8_t*>(chunk_ptr[j]) == src + len) len += sizes[j++] * rb;
            if (len) HIP_TRY(hipMemcpyAsync(dst + off, src, len, hipMemcpyHostToDevice, G->copy_stream));
            off += len;
            i = j;
        }
        HIP_TRY(hipEventRecord(G->stage_ready[b], G->copy_stream));
        HIP_TRY(hipStreamWaitEvent(st, G->stage_ready[b], 0));
        d_records = dst;
        chunk_ptr = nullptr;
        vec_ok = true;
        G->stage_i ^= 1;
    }
    // packed chunk table [offsets n+1][streams n][pad][pointers n] through a
    // pinned ring slot, reused only after its copy has run (a captured push:
    // through the graph's own buffer)
    std::vector<uint32_t> cap_table;
    uint32_t* slot = G->chunk_host + (uint64_t)G->ring_i * kChunkTableWords;
    if (cap) {
        cap_table.assign(kChunkTableWords, 0u);
        slot = cap_table.data();
    } else {
        HIP_TRY(hipEventSynchronize(G->ring_ev[G->ring_i]));
    }
    uint64_t acc = 0;
    for (int32_t i = 0; i < n_chunks; ++i) {
        slot[i] = (uint32_t)acc;
        acc += sizes[i];
    }
    slot[n_chunks] = (uint32_t)acc;
    const uint64_t so = n_chunks + 1, po = (so + n_chunks + 1) & ~1ull;
    for (int32_t i = 0; i < n_chunks; ++i) slot[so + i] = streams[i];
    uint64_t words = so + n_chunks;
    if (chunk_ptr) {
        uint64_t* pp = reinterpret_cast<uint64_t*>(slot + po);
        for (int32_t i = 0; i < n_chunks; ++i) pp[i] = reinterpret_cast<uint64_t>(chunk_ptr[i]);
        words = po + 2ull * n_chunks;
    }
    uint32_t* table = G->chunk_dev;
    if (cap) {
        HIP_TRY(hipMalloc(&cap->table_dev, 4 * words));
        HIP_TRY(hipMemcpy(cap->table_dev, slot, 4 * words, hipMemcpyHostToDevice));
        table = static_cast<uint32_t*>(cap->table_dev);
    } else {
        HIP_TRY(hipMemcpyAsync(G->chunk_dev, slot, 4 * words, hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipEventRecord(G->ring_ev[G->ring_i], ctx->stream));
        G->ring_i = (G->ring_i + 1) % kChunkRing;
    }

    auto enqueue = [&]() -> int32_t {
        const hipStream_t st = ctx->stream;
        const ltl4c_layout& L = ctx->layout;
        const WsLayout& w = G->w;
        uint8_t* ws = G->ws;
        uint32_t* z = reinterpret_cast<uint32_t*>(ws);
        {
            ZeroArgs za{z, nullptr, 0, w.zero_words, 0};
            uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (w.zero_words + 255) / 256);
            s = launch(ctx, "zero", [&] { return launch_zero(za, blocks ? blocks : 1, st); });
            if (s) return s;
            ZeroArgs zl{G->gs.list_cnt, nullptr, 0, kMaxLevels, 0};
            s = launch(ctx, "zero", [&] { return launch_zero(zl, 1, st); });
            if (s) return s;
        }
        uint64_t* sorted = nullptr;
        s = enqueue_front(ctx, L, G->g, w, ws, d_records, n, G->vplan, table, table + so,
                          chunk_ptr ? reinterpret_cast<const uint64_t*>(table + po) : nullptr,
                          (uint32_t)n_chunks, chunk_ptr ? vec_ok : true, &sorted, G->sort_variant);
        if (s) return s;
        uint64_t* seg_keys = reinterpret_cast<uint64_t*>(ws + G->seg_keys_off);
        uint8_t* seg_state = ws + w.inst_verdict_off;
        uint32_t* sizes32 = z + w.sizes32_off;
        {
            ScanArgs sa{};
            sa.words = sorted;
            sa.n = (uint32_t)n;
            sa.cbits = G->g.cbits;
            sa.class_mask = (1u << G->g.cbits) - 1u;
            sa.n_levels = 1;
            sa.valid_shift = G->g.cbits + G->g.key_bits_total;
            sa.n_props_all = G->V;
            sa.plan = G->vplan;
            sa.inst_verdict = seg_state;
            sa.inst_stride = G->max_batch;
            sa.inst_limit = G->max_batch;
            sa.inst_keys = seg_keys;
            sa.sizes = reinterpret_cast<uint64_t*>(z + w.sizes64_off);
            sa.sizes32 = sizes32;
            sa.err = ctx->err_dev;
            sa.emit_state = 1;
            uint32_t* scan_status = z + w.scan_status_off;
            for (size_t gi = 0; gi < G->sgroups.size(); ++gi) {
                sa.n_props = G->sgroups[gi].cnt;
                std::memcpy(sa.prop_idx, G->sgroups[gi].idx, sizeof sa.prop_idx);
                sa.max_states = G->sgroups[gi].states;
                sa.structure = G->sgroups[gi].structure ? 1u : 0u;
                sa.status = scan_status + gi * 2ull * kScanRows * w.tiles_scan;
                sa.ticket = z + w.scan_ticket_off + gi;
                s = launch(ctx, "scan", [&] { return launch_scan(sa, G->scan_variant, st); });
                if (s) return s;
            }
        }
        GroupUpdateArgs ua{};
        ua.g = G->gs;
        ua.n_seg = sizes32;
        ua.seg_key = seg_keys;
        ua.seg_state = seg_state;
        ua.seg_stride = G->max_batch;
        s = launch(ctx, "group_update", [&] { return launch_group_update(ua, n, st); });
        if (s) return s;
        for (int m = (int)L.n_keys - 1; m >= 1; --m) {
            s = launch(ctx, "group_level", [&] { return launch_group_level(G->gs, (uint32_t)m, st); });
            if (s) return s;
        }
        s = launch(ctx, "group_roots", [&] { return launch_group_roots(G->gs, false, st); });
        if (s) return s;
        return LTL4C_OK;
    };
    if (cap) {
        s = capture_graph(ctx, cap, enqueue);
        if (s) return s;
        cap->group = group;
        cap->streams.assign(streams, streams + n_chunks);
        return LTL4C_OK;
    }
    s = enqueue();
    if (s) return s;
    if (from_host) HIP_TRY(hipEventRecord(G->stage_free[G->stage_i ^ 1], st));
    return note_push(ctx, G, streams, n_chunks);
}

int32_t ltl4c_group_push(ltl4c_ctx* ctx, int32_t group, const void* d_records, const uint64_t* offsets,
                         const uint32_t* streams, int32_t n_chunks) {
    if (!offsets) return fail(LTL4C_EINVAL, "offsets is NULL");
    if (n_chunks < 1 || n_chunks > (int32_t)kMaxChunks) return fail(LTL4C_EINVAL, "n_chunks must be 1..4096");
    if (offsets[0] != 0) return fail(LTL4C_EINVAL, "offsets[0] must be 0");
    std::vector<uint64_t> sizes(n_chunks);
    for (int32_t i = 0; i < n_chunks; ++i) {
        if (offsets[i + 1] < offsets[i]) return fail(LTL4C_EINVAL, "offsets must be non-decreasing");
        sizes[i] = offsets[i + 1] - offsets[i];
    }
    return group_push_impl(ctx, group, d_records, nullptr, sizes.data(), streams, n_chunks);
}

int32_t ltl4c_group_push_chunks(ltl4c_ctx* ctx, int32_t group, const void* const* d_chunks, const uint64_t* sizes,
                                const uint32_t* streams, int32_t n_chunks) {
    if (!d_chunks) return fail(LTL4C_EINVAL, "chunk pointers are NULL");
    return group_push_impl(ctx, group, nullptr, d_chunks, sizes, streams, n_chunks);
}

int32_t ltl4c_group_push_seq(ltl4c_ctx* ctx, int32_t group, const void* const* chunks, const uint64_t* sizes,
                             const uint32_t* streams, const uint64_t* seqs, int32_t n_chunks, int32_t is_device) {
    if (!chunks) return fail(LTL4C_EINVAL, "chunk pointers are NULL");
    if (!seqs) return fail(LTL4C_EINVAL, "sequence numbers are NULL");
    return group_push_impl(ctx, group, nullptr, chunks, sizes, streams, n_chunks, seqs, is_device == 0);
}

int32_t ltl4c_group_read(ltl4c_ctx* ctx, int32_t group, uint8_t* d_root_verdict, uint64_t* d_root_counts,
                         uint64_t* d_bindings) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    if (!d_root_verdict || !d_root_counts) return fail(LTL4C_EINVAL, "outputs are NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    return launch(ctx, "group_read",
                  [&] { return launch_group_read(G->gs, d_root_verdict, d_root_counts, d_bindings, ctx->stream); });
}

int32_t ltl4c_group_snapshot(ltl4c_ctx* ctx, int32_t group, void* host, uint64_t* bytes) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    if (!bytes) return fail(LTL4C_EINVAL, "bytes is NULL");
    if (!host) {
        *bytes = G->state_bytes;
        return LTL4C_OK;
    }
    if (*bytes < G->state_bytes) return fail(LTL4C_EINVAL, "snapshot buffer too small");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(host, G->state, G->state_bytes, hipMemcpyDeviceToHost));
    *bytes = G->state_bytes;
    return LTL4C_OK;
}

int32_t ltl4c_group_restore(ltl4c_ctx* ctx, int32_t group, const void* host, uint64_t bytes) {
    GroupHost* G = nullptr;
    int32_t s = get_group(ctx, group, &G);
    if (s) return s;
    if (!host || bytes != G->state_bytes) return fail(LTL4C_EINVAL, "snapshot size does not match this group");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipMemcpy(G->state, host, G->state_bytes, hipMemcpyHostToDevice));
    return LTL4C_OK;
}

int32_t ltl4c_set_option(ltl4c_ctx* ctx, int32_t option, int64_t value) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    switch (option) {
        case LTL4C_OPT_SORT_TILE:
            if (value < -1 || value >= kSortVariants) return fail(LTL4C_EINVAL, "sort tile variant out of range");
            ctx->pin_sort = value >= 0;
            ctx->sort_variant = value >= 0 ? (int)value : kDefaultSortVariant;
            return LTL4C_OK;
        case LTL4C_OPT_SCAN_TILE:
            if (value < -1 || value >= kScanVariants) return fail(LTL4C_EINVAL, "scan tile variant out of range");
            ctx->pin_scan = value >= 0;
            ctx->scan_variant = value >= 0 ? (int)value : kDefaultScanVariant;
            return LTL4C_OK;
        default:
            return fail(LTL4C_EINVAL, "unknown option");
    }
}

int32_t ltl4c_profile_enable(ltl4c_ctx* ctx, int32_t on) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    ctx->prof = on != 0;
    return LTL4C_OK;
}

int32_t ltl4c_profile_get(ltl4c_ctx* ctx, int32_t i, char* name_buf, int32_t name_len, double* total_ms,
                          uint64_t* launches) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    int32_t s = drain_profile(ctx);
    if (s) return s;
    if (i < 0 || i >= (int32_t)ctx->prof_acc.size()) return LTL4C_EINVAL;
    const auto& acc = ctx->prof_acc[i];
    if (name_buf && name_len > 0) {
        std::strncpy(name_buf, acc.first.c_str(), name_len - 1);
        name_buf[name_len - 1] = 0;
    }
    if (total_ms) *total_ms = acc.second.first;
    if (launches) *launches = acc.second.second;
    return LTL4C_OK;
}

int32_t ltl4c_profile_reset(ltl4c_ctx* ctx) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    int32_t s = drain_profile(ctx);
    ctx->prof_acc.clear();
    return s;
}

// ---- graphs: captured kernel sequences ----------------------------------------

// Runs `enqueue` with the context's launches redirected to a private stream
// in capture mode, and instantiates what it recorded.  Nothing runs; no
// profiling events are recorded into the graph.
static int32_t capture_graph(ltl4c_ctx* ctx, GraphHost* gh, const std::function<int32_t()>& enqueue) {
    if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    // work the caller enqueued before must not be reordered with the graph's
    // later replays: the capture only records, so no ordering is needed here
    const hipStream_t saved = ctx->stream;
    const bool saved_nt = ctx->no_timing;
    HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    ctx->stream = ctx->cap_stream;
    ctx->no_timing = true;
    const int32_t s = enqueue();
    ctx->stream = saved;
    ctx->no_timing = saved_nt;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (s) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess || !g) return fail(LTL4C_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    gh->graph = g;
    HIP_TRY(hipGraphInstantiate(&gh->exec, g, nullptr, nullptr, 0));
    return LTL4C_OK;
}

static int32_t keep_graph(ltl4c_ctx* ctx, GraphHost* gh, int32_t s, int32_t* graph) {
    if (s) {
        if (gh->exec) (void)hipGraphExecDestroy(gh->exec);
        if (gh->graph) (void)hipGraphDestroy(gh->graph);
        (void)hipFree(gh->table_dev);
        delete gh;
        return s;
    }
    int32_t id = -1;
    for (size_t i = 0; i < ctx->graphs.size(); ++i)
        if (!ctx->graphs[i]) id = (int32_t)i;
    if (id < 0) {
        id = (int32_t)ctx->graphs.size();
        ctx->graphs.push_back(nullptr);
    }
    ctx->graphs[id] = gh;
    *graph = id;
    return LTL4C_OK;
}

int32_t ltl4c_graph_eval(ltl4c_ctx* ctx, const void* d_records, uint64_t n_events, const int32_t* props,
                         int32_t n_props, void* d_ws, uint64_t ws_bytes, const ltl4c_result* out, int32_t* graph) {
    if (!ctx || !graph) return fail(LTL4C_EINVAL, "ctx or graph is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    GraphHost* gh = new GraphHost();
    const int32_t s = eval_impl(ctx, d_records, n_events, props, n_props, d_ws, ws_bytes, out, false, gh);
    return keep_graph(ctx, gh, s, graph);
}

int32_t ltl4c_graph_eval_batch(ltl4c_ctx* ctx, const void* d_records, const uint64_t* offsets, int32_t n_traces,
                               const int32_t* props, int32_t n_props, void* d_ws, uint64_t ws_bytes,
                               uint8_t* d_root_verdict, uint64_t* d_root_counts, int32_t* graph) {
    if (!ctx || !graph) return fail(LTL4C_EINVAL, "ctx or graph is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    GraphHost* gh = new GraphHost();
    const int32_t s = batch_impl(ctx, d_records, offsets, n_traces, props, n_props, d_ws, ws_bytes, d_root_verdict,
                                 d_root_counts, gh);
    return keep_graph(ctx, gh, s, graph);
}

int32_t ltl4c_graph_group_push(ltl4c_ctx* ctx, int32_t group, const void* const* d_chunks, const uint64_t* sizes,
                               const uint32_t* streams, int32_t n_chunks, int32_t* graph) {
    if (!ctx || !graph) return fail(LTL4C_EINVAL, "ctx or graph is NULL");
    if (!d_chunks) return fail(LTL4C_EINVAL, "chunk pointers are NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    GraphHost* gh = new GraphHost();
    const int32_t s = group_push_impl(ctx, group, nullptr, d_chunks, sizes, streams, n_chunks, nullptr, false, gh);
    return keep_graph(ctx, gh, s, graph);
}

int32_t ltl4c_graph_launch(ltl4c_ctx* ctx, int32_t graph) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    if (graph < 0 || graph >= (int32_t)ctx->graphs.size() || !ctx->graphs[graph])
        return fail(LTL4C_EINVAL, "unknown graph id");
    GraphHost* gh = ctx->graphs[graph];
    GroupHost* G = nullptr;
    if (gh->group >= 0) {
        int32_t s = get_group(ctx, gh->group, &G);
        if (s) return fail(LTL4C_EINVAL, "the graph's stream group was closed");
        for (uint32_t st : gh->streams)
            if (!G->open[st]) return fail(LTL4C_ESEQ, "the graph pushes to a stream that is not open");
    }
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipGraphLaunch(gh->exec, ctx->stream));
    if (G) return note_push(ctx, G, gh->streams.data(), (int32_t)gh->streams.size());
    return LTL4C_OK;
}

int32_t ltl4c_graph_destroy(ltl4c_ctx* ctx, int32_t graph) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    if (graph < 0 || graph >= (int32_t)ctx->graphs.size() || !ctx->graphs[graph])
        return fail(LTL4C_EINVAL, "unknown graph id");
    GraphHost* gh = ctx->graphs[graph];
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (gh->exec) (void)hipGraphExecDestroy(gh->exec);
    if (gh->graph) (void)hipGraphDestroy(gh->graph);
    (void)hipFree(gh->table_dev);
    delete gh;
    ctx->graphs[graph] = nullptr;
    return LTL4C_OK;
}

// ---- autotuning -------------------------------------------------------------

int32_t ltl4c_tune_workspace_bytes(ltl4c_ctx* ctx, uint64_t n_events, const uint64_t* offsets, int32_t n_traces,
                                   const int32_t* props, int32_t n_props, uint64_t* bytes) {
    int32_t s = check_props(ctx, props, n_props);
    if (s) return s;
    if (!bytes) return fail(LTL4C_EINVAL, "bytes is NULL");
    if (offsets && (n_traces < 1 || n_traces > (int32_t)kMaxChunks))
        return fail(LTL4C_EUNSUPPORTED, "n_traces must be 1..4096");
    const uint64_t n = offsets ? offsets[n_traces] : n_events;
    const int sv0 = ctx->sort_variant, cv0 = ctx->scan_variant;
    const bool ps0 = ctx->pin_sort, pc0 = ctx->pin_scan;
    ctx->pin_sort = ctx->pin_scan = true;
    uint64_t most = 0;
    for (int sv = 0; sv < kSortVariants && s == LTL4C_OK; ++sv)
        for (int cv = 0; cv < kScanVariants && s == LTL4C_OK; ++cv) {
            ctx->sort_variant = sv;
            ctx->scan_variant = cv;
            uint64_t b = 0;
            s = offsets ? ltl4c_batch_workspace_bytes(ctx, n, n_traces, props, n_props, &b)
                        : ltl4c_workspace_bytes(ctx, n, props, n_props, &b);
            most = std::max(most, b);
        }
    ctx->sort_variant = sv0;
    ctx->scan_variant = cv0;
    ctx->pin_sort = ps0;
    ctx->pin_scan = pc0;
    if (s) return s;
    *bytes = most;
    return LTL4C_OK;
}

int32_t ltl4c_tune(ltl4c_ctx* ctx, const void* d_records, uint64_t n_events, const uint64_t* offsets, int32_t n_traces,
                   const int32_t* props, int32_t n_props, void* d_ws, uint64_t ws_bytes, int32_t reps,
                   ltl4c_tuned* result) {
    int32_t s = check_props(ctx, props, n_props);
    if (s) return s;
    if (reps < 1 || reps > 1000) return fail(LTL4C_EINVAL, "reps must be 1..1000");
    if (offsets && (n_traces < 1 || n_traces > (int32_t)kMaxChunks))
        return fail(LTL4C_EUNSUPPORTED, "n_traces must be 1..4096");
    const bool batch = offsets != nullptr;
    const uint64_t n = batch ? offsets[n_traces] : n_events;
    HIP_TRY(hipSetDevice(ctx->device));
    // outputs of the timed calls
    const uint64_t cells = batch ? (uint64_t)n_traces * n_props : (uint64_t)n_props;
    uint8_t* outs = nullptr;
    HIP_TRY(hipMalloc(&outs, align256(cells) + 48 * cells + 1024));
    hipEvent_t ev[2] = {nullptr, nullptr};
    struct Restore {
        ltl4c_ctx* c;
        int sv, cv;
        bool ps, pc, prof;
        uint8_t* outs;
        hipEvent_t* ev;
        ~Restore() {
            c->sort_variant = sv;
            c->scan_variant = cv;
            c->pin_sort = ps;
            c->pin_scan = pc;
            c->prof = prof;
            (void)hipStreamSynchronize(c->stream);
            (void)hipFree(outs);
            for (int i = 0; i < 2; ++i)
                if (ev[i]) (void)hipEventDestroy(ev[i]);
        }
    } restore{ctx, ctx->sort_variant, ctx->scan_variant, ctx->pin_sort, ctx->pin_scan, ctx->prof, outs, ev};
    HIP_TRY(hipEventCreate(&ev[0]));
    HIP_TRY(hipEventCreate(&ev[1]));
    ctx->prof = false;
    ctx->pin_sort = ctx->pin_scan = true;      // the candidate is the schedule
    ltl4c_result r{};
    r.root_verdict = outs;
    r.root_counts = reinterpret_cast<uint64_t*>(outs + align256(cells));
    r.sizes = reinterpret_cast<uint64_t*>(outs + align256(cells) + 48 * cells);
    int32_t tried = 0;
    // median time of `reps` runs after one warm-up; +inf when the candidate's
    // workspace exceeds ws_bytes
    auto run = [&](int sv, int cv, double* med) -> int32_t {
        ctx->sort_variant = sv;
        ctx->scan_variant = cv;
        uint64_t need = 0;
        int32_t e = batch ? ltl4c_batch_workspace_bytes(ctx, n, n_traces, props, n_props, &need)
                          : ltl4c_workspace_bytes(ctx, n, props, n_props, &need);
        if (e) return e;
        if (need > ws_bytes) {
            *med = 1e300;
            return LTL4C_OK;
        }
        ++tried;
        std::vector<float> t;
        for (int i = 0; i <= reps; ++i) {
            HIP_TRY(hipEventRecord(ev[0], ctx->stream));
            e = batch ? ltl4c_eval_batch(ctx, d_records, offsets, n_traces, props, n_props, d_ws, ws_bytes,
                                         r.root_verdict, r.root_counts)
                      : ltl4c_eval(ctx, d_records, n, props, n_props, d_ws, ws_bytes, &r);
            if (e) return e;
            HIP_TRY(hipEventRecord(ev[1], ctx->stream));
            HIP_TRY(hipEventSynchronize(ev[1]));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));
            if (i > 0) t.push_back(ms);
        }
        std::sort(t.begin(), t.end());
        *med = 1e3 * t[t.size() / 2];
        return LTL4C_OK;
    };
    double def_us = 0.0;
    s = run(kDefaultSortVariant, kDefaultScanVariant, &def_us);
    if (s) return s;
    int bs = kDefaultSortVariant, bc = kDefaultScanVariant;
    double best = def_us;
    // coordinate descent: the radix tile with the default scan, then the
    // scan tile with that radix tile; a candidate must win by 1 %
    for (int sv = 0; sv < kSortVariants; ++sv) {
        if (sv == bs) continue;
        double u = 0.0;
        s = run(sv, bc, &u);
        if (s) return s;
        if (u < 0.99 * best) {
            best = u;
            bs = sv;
        }
    }
    for (int cv = 0; cv < kScanVariants; ++cv) {
        if (cv == bc) continue;
        double u = 0.0;
        s = run(bs, cv, &u);
        if (s) return s;
        if (u < 0.99 * best) {
            best = u;
            bc = cv;
        }
    }
    s = ltl4c_wait(ctx);
    if (s) return s;
    SchedEntry e = shape_of(ctx, batch ? 1 : 0, n, n_traces, props, n_props);
    e.sort = bs;
    e.scan = bc;
    e.us = best;
    e.default_us = def_us;
    bool replaced = false;
    for (auto& x : ctx->sched)
        if (same_class(x, e) && x.log2n == e.log2n) {
            x = e;
            replaced = true;
        }
    if (!replaced) ctx->sched.push_back(e);
    if (result) {
        result->sort_tile = bs;
        result->scan_tile = bc;
        result->tuned_us = best;
        result->default_us = def_us;
        result->candidates = tried;
    }
    return LTL4C_OK;
}

namespace {
std::string arch_of(int device) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// The number after "\"key\":" inside [b, e), or false.
bool json_num(const std::string& t, size_t b, size_t e, const char* key, double* out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = t.find(k, b);
    if (at == std::string::npos || at >= e) return false;
    char* end = nullptr;
    const double v = std::strtod(t.c_str() + at + k.size(), &end);
    if (end == t.c_str() + at + k.size()) return false;
    *out = v;
    return true;
}
}  // namespace

int32_t ltl4c_schedule_save(ltl4c_ctx* ctx, const char* path) {
    if (!ctx || !path) return fail(LTL4C_EINVAL, "ctx or path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(LTL4C_EINVAL, std::string("cannot write ") + path);
    std::fprintf(f, "{\"arch\": \"%s\", \"schedules\": [\n", arch_of(ctx->device).c_str());
    for (size_t i = 0; i < ctx->sched.size(); ++i) {
        const SchedEntry& e = ctx->sched[i];
        std::fprintf(f,
                     "  {\"batch\": %d, \"key_bits\": %u, \"props\": %u, \"big_monitors\": %u, \"levels\": %u, "
                     "\"log2_events\": %u, \"sort_tile\": %d, \"scan_tile\": %d, \"us\": %.2f, \"default_us\": %.2f}%s\n",
                     e.kind, e.key_bits, e.n_props, e.big, e.levels, e.log2n, e.sort, e.scan, e.us, e.default_us,
                     i + 1 < ctx->sched.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? LTL4C_OK : fail(LTL4C_EINVAL, std::string("cannot write ") + path);
}

int32_t ltl4c_schedule_load(ltl4c_ctx* ctx, const char* path, int32_t* n_loaded) {
    if (!ctx || !path) return fail(LTL4C_EINVAL, "ctx or path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(LTL4C_EINVAL, std::string("cannot read ") + path);
    std::string t;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) t.append(buf, k);
    std::fclose(f);
    int32_t loaded = 0;
    const size_t a = t.find("\"arch\":");
    const size_t q0 = a == std::string::npos ? a : t.find('"', a + 7);
    const size_t q1 = q0 == std::string::npos ? q0 : t.find('"', q0 + 1);
    if (q1 == std::string::npos) return fail(LTL4C_EINVAL, "schedule file without an arch");
    if (t.substr(q0 + 1, q1 - q0 - 1) == arch_of(ctx->device)) {
        size_t at = t.find('{', q1);
        while (at != std::string::npos) {
            const size_t end = t.find('}', at);
            if (end == std::string::npos) break;
            double v[8];
            const char* keys[8] = {"batch", "key_bits", "props", "big_monitors", "levels", "log2_events", "sort_tile",
                                   "scan_tile"};
            bool ok = true;
            for (int i = 0; i < 8 && ok; ++i) ok = json_num(t, at, end, keys[i], &v[i]);
            if (!ok || v[6] < 0 || v[6] >= kSortVariants || v[7] < 0 || v[7] >= kScanVariants || v[0] < 0 || v[0] > 1)
                return fail(LTL4C_EINVAL, "malformed schedule entry");
            SchedEntry e;
            e.kind = (int)v[0];
            e.key_bits = (uint32_t)v[1];
            e.n_props = (uint32_t)v[2];
            e.big = (uint32_t)v[3];
            e.levels = (uint32_t)v[4];
            e.log2n = (uint32_t)v[5];
            e.sort = (int)v[6];
            e.scan = (int)v[7];
            (void)json_num(t, at, end, "us", &e.us);
            (void)json_num(t, at, end, "default_us", &e.default_us);
            bool replaced = false;
            for (auto& x : ctx->sched)
                if (same_class(x, e) && x.log2n == e.log2n) {
                    x = e;
                    replaced = true;
                }
            if (!replaced) ctx->sched.push_back(e);
            ++loaded;
            at = t.find('{', end);
        }
    }
    if (n_loaded) *n_loaded = loaded;
    return LTL4C_OK;
}

int32_t ltl4c_schedule_clear(ltl4c_ctx* ctx) {
    if (!ctx) return fail(LTL4C_EINVAL, "ctx is NULL");
    ctx->sched.clear();
    return LTL4C_OK;
}

}  // extern "C"
