// The segmented transition-map scan (Def. 6: the state of every instance
// after its cluster, composed as maps so that a cluster may spread over any
// number of lanes and tiles), in three steps without look-back:
//   reduce  per tile of 4,096 or 8,192 sorted words: every thread composes the
//           maps of its 16 or 32 consecutive words (a head restarts from q0),
//           the block scans the threads in order; the tile's map per property
//           and its head counts per level go to `agg`, every thread's
//           exclusive prefix within the tile to `trec`;
//   spine   exclusive prefixes of the tile records in tile order: one block,
//           or, for many tiles, chunk compositions, their scan and the tile
//           prefixes of every chunk (three launches);
//   down    per tile: every thread starts from its prefix (tile prefix, then
//           its own), steps its states word by word and writes instance
//           verdicts, parents, numbering and nodes (and, on request, the
//           verdict timeline).
// Words are read as 16 or 32 consecutive 64-bit words per thread with 16-byte
// loads (no LDS staging).  The first reduce writes one descriptor byte per word
// (class, head and level-head flags); the down sweep and the launches of
// further property groups read those instead of the words.  No tile waits on
// another, so several tiles share a CU.
#include "internal.h"
#include "maps.h"

namespace ltl4c {

namespace {

constexpr uint32_t kAll = 0xFFFFFFFFu;

// Flags and classes of a thread's run of words: `cnt` valid words (a prefix of
// the run), head (a new instance), level-m heads (a new level-m node), classes
// packed 4 bits per word.
struct Run {
    uint32_t cnt, m_head, m_lvl[kMaxLevels];
    uint64_t cls[2];
};

// (selects rather than indexing, so that runs never leave registers)
__device__ __forceinline__ uint32_t run_class(const Run& r, int j) {
    return (uint32_t)((j < 16 ? r.cls[0] : r.cls[1]) >> (4 * (j & 15))) & 15u;
}

__device__ __forceinline__ uint32_t valid_mask(uint32_t cnt) { return cnt >= 32 ? kAll : (1u << cnt) - 1u; }

template <int ITEMS>
__device__ __forceinline__ Run run_from_words(const ScanArgs& a, uint64_t my0, uint32_t n) {
    // Loads are unconditional, so that all of them are in flight together:
    // the word buffers have room for a whole run past the last valid word.
    // A thread without valid words reads the first run instead (in bounds).
    Run r{};
    r.cnt = my0 < n ? (uint32_t)min<uint64_t>(ITEMS, n - my0) : 0u;
    const uint64_t ld0 = r.cnt ? my0 : 0;
    const uint64_t prev0 = a.words[ld0 > 0 ? ld0 - 1 : 0];
    uint64_t wv[ITEMS];
    const uint4* p = reinterpret_cast<const uint4*>(a.words + ld0);
#pragma unroll
    for (int k = 0; k < ITEMS / 2; ++k) {
        const uint4 v = p[k];
        wv[2 * k] = ((uint64_t)v.y << 32) | v.x;
        wv[2 * k + 1] = ((uint64_t)v.w << 32) | v.z;
    }
    const uint64_t hlim = 1ull << a.cbits;
    uint64_t llim[kMaxLevels];
#pragma unroll
    for (int m = 1; m < kMaxLevels; ++m) llim[m] = (uint32_t)m < a.n_levels ? 1ull << a.prefix_shift[m] : ~0ull;
    uint64_t prev = prev0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint64_t x = wv[j];
        const bool valid = (uint32_t)j < r.cnt;
        const bool first = my0 + j == 0;
        const uint64_t d = prev ^ x;
        prev = x;
        r.m_head |= (uint32_t)(valid && (first || d >= hlim)) << j;
#pragma unroll
        for (int m = 1; m < kMaxLevels; ++m)
            if ((uint32_t)m < a.n_levels) r.m_lvl[m] |= (uint32_t)(valid && (first || d >= llim[m])) << j;
        const uint64_t cj = (uint64_t)((uint32_t)x & a.class_mask) << (4 * (j & 15));
        if (j < 16) r.cls[0] |= cj;
        else r.cls[1] |= cj;
    }
    return r;
}

__device__ __forceinline__ uint32_t desc_byte(const Run& r, int j) {
    uint32_t b = run_class(r, j);
    b |= ((r.m_head >> j) & 1u) << 4;
#pragma unroll
    for (int m = 1; m < kMaxLevels; ++m) b |= ((r.m_lvl[m] >> j) & 1u) << (4 + m);
    return b;
}

template <int ITEMS>
__device__ __forceinline__ void store_desc(const ScanArgs& a, uint64_t my0, const Run& r) {
    if (r.cnt == ITEMS) {
        uint32_t d[ITEMS / 4];
#pragma unroll
        for (int i = 0; i < ITEMS / 4; ++i) d[i] = 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) d[j >> 2] |= desc_byte(r, j) << (8 * (j & 3));
        uint4* q = reinterpret_cast<uint4*>(a.desc + my0);
#pragma unroll
        for (int i = 0; i < ITEMS / 16; ++i) q[i] = make_uint4(d[4 * i], d[4 * i + 1], d[4 * i + 2], d[4 * i + 3]);
    } else {
        for (uint32_t j = 0; j < r.cnt; ++j) a.desc[my0 + j] = (uint8_t)desc_byte(r, (int)j);
    }
}

// Four words' descriptor bytes (one dword) at once: the low nibbles packed
// into 16 bits (the classes), the high nibbles as a transposed 4 x 4 bit
// matrix, so that nibble f holds flag f (head, level-1..3 head) of the four
// words.
__device__ __forceinline__ uint32_t pack_nibbles(uint32_t x) {   // nibbles at bits 0, 8, 16, 24
    x = (x | (x >> 4)) & 0x00FF00FFu;
    return (x | (x >> 8)) & 0xFFFFu;
}
__device__ __forceinline__ uint32_t transpose4x4(uint32_t y) {   // bit 4k + f -> bit 4f + k
    uint32_t t = ((y >> 3) ^ y) & 0x0A0Au;
    y ^= t ^ (t << 3);
    t = ((y >> 6) ^ y) & 0x00CCu;
    return y ^ t ^ (t << 6);
}

template <int ITEMS>
__device__ __forceinline__ Run run_from_desc(const ScanArgs& a, uint64_t my0, uint32_t n) {
    // (the descriptor buffer has room for a whole run past the last word)
    Run r{};
    r.cnt = my0 < n ? (uint32_t)min<uint64_t>(ITEMS, n - my0) : 0u;
    const uint4* q = reinterpret_cast<const uint4*>(a.desc + (r.cnt ? my0 : 0));
#pragma unroll
    for (int i = 0; i < ITEMS / 16; ++i) {
        const uint4 v = q[i];
        uint32_t d[4] = {v.x, v.y, v.z, v.w};
        if (r.cnt < ITEMS) {
            // the bytes of words past the end read as 0
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t s0 = 16u * i + 4u * k;
                d[k] = s0 >= r.cnt ? 0u : s0 + 4u > r.cnt ? d[k] & ((1u << (8u * (r.cnt - s0))) - 1u) : d[k];
            }
        }
        uint64_t c = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c |= (uint64_t)pack_nibbles(d[k] & 0x0F0F0F0Fu) << (16 * k);
            const uint32_t f = transpose4x4(pack_nibbles((d[k] >> 4) & 0x0F0F0F0Fu));
            const int at = 16 * i + 4 * k;
            r.m_head |= (f & 15u) << at;
#pragma unroll
            for (int m = 1; m < kMaxLevels; ++m) r.m_lvl[m] |= ((f >> (4 * m)) & 15u) << at;
        }
        r.cls[i] = c;
    }
    return r;
}

// The composed map of a run per property: a head restarts the monitor at q0.
// FULL: every word of the run is valid (all threads but the trace's last).
template <int PMAX, int MW, int ITEMS, bool FULL>
__device__ __forceinline__ void run_maps_t(const Run& r, uint32_t P, const uint32_t (*s_cm)[16][MW],
                                           const uint32_t* s_q0, BMap<MW>* f) {
    const uint32_t valid = FULL ? kAll : valid_mask(r.cnt);
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        f[p] = bm_identity<MW>();
        if (p > 0 && p >= (int)P) continue;    // (a launch has at least one property)
        const BMap<MW> start = bm_const<MW>(s_q0[p]);
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const BMap<MW> cm = bm_load<MW>(s_cm[p][run_class(r, j)]);
            const BMap<MW> g = bm_compose<MW>(cm, ((r.m_head >> j) & 1u) ? start : f[p]);
            if (FULL || ((valid >> j) & 1u)) f[p] = g;
        }
    }
}
template <int PMAX, int MW, int ITEMS>
__device__ __forceinline__ void run_maps(const Run& r, uint32_t P, const uint32_t (*s_cm)[16][MW], const uint32_t* s_q0,
                                         BMap<MW>* f) {
    // (four 16-state maps keep the one path: the second copy costs them registers)
    if (PMAX * MW <= 8 && r.cnt == ITEMS) run_maps_t<PMAX, MW, ITEMS, true>(r, P, s_cm, s_q0, f);
    else run_maps_t<PMAX, MW, ITEMS, false>(r, P, s_cm, s_q0, f);
}

// The class maps of the launch's properties, one table word per thread
// (PMAX * 16 * MW <= 256 = the block), plus q0 and the packed labels: read
// into registers first (the loads overlap the block's data loads), stored to
// LDS afterwards.
struct TableRegs {
    uint32_t cm, q0, lab0, lab1;
};

// prop_idx[p] for a thread-dependent p, by selects over kernel-argument
// scalars (indexing the argument array would be a vector load)
template <int PMAX>
__device__ __forceinline__ uint32_t prop_index(const ScanArgs& a, uint32_t p) {
    uint32_t r = a.prop_idx[0];
#pragma unroll
    for (int q = 1; q < PMAX; ++q)
        if (p == (uint32_t)q) r = a.prop_idx[q];
    return r;
}

template <int PMAX, int MW>
__device__ __forceinline__ TableRegs read_tables(const ScanArgs& a) {
    static_assert(PMAX * 16 * MW <= kMsThreads, "one table word per thread");
    TableRegs t{0, 0, 0, 0};
    const uint32_t P = a.n_props, i = threadIdx.x;
    if (i < P * 16 * MW) {
        const uint32_t p = i / (16 * MW), c = (i / MW) % 16, k = i % MW;
        t.cm = a.plan->prop[prop_index<PMAX>(a, p)].bmap[c][k];
    }
    if (i < P) {
        const PropDev& pd = a.plan->prop[prop_index<PMAX>(a, i)];
        t.q0 = pd.q0;
        t.lab0 = pd.blabel[0];
        t.lab1 = pd.blabel[1];
    }
    return t;
}

template <int PMAX, int MW>
__device__ __forceinline__ void store_tables(const ScanArgs& a, const TableRegs& t, uint32_t (*s_cm)[16][MW],
                                             uint32_t* s_q0, uint32_t (*s_lab)[2]) {
    const uint32_t P = a.n_props, i = threadIdx.x;
    if (i < P * 16 * MW) s_cm[i / (16 * MW)][(i / MW) % 16][i % MW] = t.cm;
    if (i < P) {
        s_q0[i] = t.q0;
        if (s_lab) {
            s_lab[i][0] = t.lab0;
            s_lab[i][1] = t.lab1;
        }
    }
}

// Block-wide ordered scan of one map per property and four counts per
// thread: on return `excl` and `cexcl` hold this thread's exclusive prefix
// within the block, `tot` / `ctot` (valid in every thread) the block's total.
// With PACK, the counts of a tile (below 2^16) travel two to a word, and the
// second word only when there are more than two levels.  The wave totals are
// scanned once, by wave 0 (row WAVES of s_wm / s_wc receives the block total),
// so no thread composes more than log2(WAVES) of them.
template <int PMAX, int MW, int THREADS, bool PACK = false>
__device__ __forceinline__ void block_scan(uint32_t P, const BMap<MW>* f, const uint32_t* cnt, BMap<MW>* excl,
                                           uint32_t* cexcl, BMap<MW>* tot, uint32_t* ctot,
                                           uint32_t (*s_wm)[THREADS / 64 + 1][MW], uint32_t (*s_wc)[THREADS / 64 + 1],
                                           uint32_t levels = 4) {
    constexpr int WAVES = THREADS / 64;
    constexpr int NC = PACK ? 2 : 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t c[4];
    if (PACK) {
        c[0] = cnt[0] | (cnt[1] << 16);
        c[1] = cnt[2] | (cnt[3] << 16);
    } else {
        c[0] = cnt[0], c[1] = cnt[1], c[2] = cnt[2], c[3] = cnt[3];
    }
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        BMap<MW> v = f[p];
        if (p < (int)P) v = bm_wave_incl_scan<MW>(v);
        excl[p] = bm_wave_shr1<MW>(v);
        if (lane == 63)
#pragma unroll
            for (int k = 0; k < MW; ++k) s_wm[p][w][k] = v.d[k];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        uint32_t x = c[k];
        if ((uint32_t)k * (4 / NC) < levels) x = wave_incl_sum(x);    // counts of absent levels stay zero
        cexcl[k] = x - c[k];
        if (lane == 63) s_wc[k][w] = x;
    }
    __syncthreads();
    if (w == 0) {
        // wave 0: exclusive scan of the wave totals, in place; the block total
        // goes to row WAVES
#pragma unroll
        for (int p = 0; p < PMAX; ++p) {
            if (p >= (int)P) continue;
            BMap<MW> v = lane < WAVES ? bm_load<MW>(s_wm[p][lane]) : bm_identity<MW>();
            v = bm_wave_incl_scan<MW>(v);
            const BMap<MW> ex = bm_wave_shr1<MW>(v);
            if (lane < WAVES) {
#pragma unroll
                for (int k = 0; k < MW; ++k) s_wm[p][lane][k] = ex.d[k];
            }
            if (lane == WAVES - 1)
#pragma unroll
                for (int k = 0; k < MW; ++k) s_wm[p][WAVES][k] = v.d[k];
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const uint32_t c0 = lane < WAVES ? s_wc[k][lane] : 0u;
            const uint32_t x = wave_incl_sum(c0);
            if (lane < WAVES) s_wc[k][lane] = x - c0;
            if (lane == WAVES - 1) s_wc[k][WAVES] = x;
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (p >= (int)P) {
            tot[p] = bm_identity<MW>();
            continue;
        }
        excl[p] = bm_compose<MW>(excl[p], bm_load<MW>(s_wm[p][w]));
        tot[p] = bm_load<MW>(s_wm[p][WAVES]);
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        cexcl[k] += s_wc[k][w];
        ctot[k] = s_wc[k][WAVES];
    }
    if (PACK) {
#pragma unroll
        for (int k = 1; k >= 0; --k) {
            cexcl[2 * k + 1] = cexcl[k] >> 16;
            cexcl[2 * k] = cexcl[k] & 0xFFFFu;
            ctot[2 * k + 1] = ctot[k] >> 16;
            ctot[2 * k] = ctot[k] & 0xFFFFu;
        }
    }
}

}  // namespace

template <int PMAX, int MW, int ITEMS>
__global__ __launch_bounds__(kMsThreads) void k_ms_reduce(ScanArgs a) {
    constexpr uint32_t TILE = kMsThreads * ITEMS;
    __shared__ uint32_t s_cm[PMAX][16][MW];
    __shared__ uint32_t s_q0[PMAX];
    __shared__ uint32_t s_wm[PMAX][kMsThreads / 64 + 1][MW];
    __shared__ uint32_t s_wc[4][kMsThreads / 64 + 1];
    const uint32_t n = *a.n_dev;
    const uint64_t base = (uint64_t)blockIdx.x * TILE;
    if (base >= n) return;                       // the whole block: no word of this tile
    const uint64_t my0 = base + (uint64_t)threadIdx.x * ITEMS;
    Run r = a.read_desc ? run_from_desc<ITEMS>(a, my0, n) : run_from_words<ITEMS>(a, my0, n);
    const TableRegs tr = read_tables<PMAX, MW>(a);
    store_tables<PMAX, MW>(a, tr, s_cm, s_q0, nullptr);
    if (!a.read_desc && a.desc && r.cnt) store_desc<ITEMS>(a, my0, r);
    __syncthreads();
    BMap<MW> f[PMAX], excl[PMAX], tot[PMAX];
    run_maps<PMAX, MW, ITEMS>(r, a.n_props, s_cm, s_q0, f);
    uint32_t cnt[4], cexcl[4], ctot[4];
    cnt[0] = __popc(r.m_head);
#pragma unroll
    for (int m = 1; m < 4; ++m) cnt[m] = __popc(r.m_lvl[m]);
    block_scan<PMAX, MW, kMsThreads, true>(a.n_props, f, cnt, excl, cexcl, tot, ctot, s_wm, s_wc, a.n_levels);
    // this thread's exclusive prefix within the tile, for the down sweep
    // (rows of consecutive threads: coalesced)
    const uint64_t row = (uint64_t)a.tiles * kMsThreads, at = (uint64_t)blockIdx.x * kMsThreads + threadIdx.x;
    a.trec[at] = cexcl[0] | (cexcl[1] << 16);
    a.trec[row + at] = cexcl[2] | (cexcl[3] << 16);
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
        if (p < (int)a.n_props)
#pragma unroll
            for (int k = 0; k < MW; ++k) a.trec[(2 + MW * p + k) * row + at] = excl[p].d[k];
    if (threadIdx.x < kMsRec) {
        const uint32_t k = threadIdx.x;
        uint32_t v = 0;
        if (k < 4) {
            v = ctot[k];
        } else {
            const uint32_t p = (k - 4) / MW, d = (k - 4) % MW;
#pragma unroll
            for (int q = 0; q < PMAX; ++q)
#pragma unroll
                for (int e = 0; e < MW; ++e)
                    if ((uint32_t)q == p && (uint32_t)e == d) v = tot[q].d[e];
        }
        a.agg[(uint64_t)blockIdx.x * kMsRec + k] = v;
    }
}

// Exclusive prefixes of the tile records (maps composed in tile order, head
// counts summed).  Records go in passes of kSpineThreads x (up to 4) records:
// each thread loads its chunk's records at once (16-byte loads, all in flight
// together), composes them, the block scans the thread totals, and the running
// prefix carries from pass to pass.  MODE 0: one block over all tiles (one
// pass up to 16M words).  Above a few passes the work is spread: MODE 1, block
// b composes the tiles of chunk b (a.spine_chunk tiles) into a chunk record;
// MODE 2, one block scans the chunk records; MODE 3, block b writes the tile
// prefixes of chunk b, starting from the chunk's prefix.
constexpr int kSpineThreads = kMsSpineThreads;

template <int NW>
__host__ __device__ constexpr int spine_chunk_items() { return NW <= 8 ? 4 : NW <= 12 ? 2 : 1; }

template <int PMAX, int MW, int ITEMS, int MODE>
__global__ __launch_bounds__(kSpineThreads) void k_ms_spine(ScanArgs a) {
    constexpr uint32_t TILE = kMsThreads * ITEMS;
    constexpr int NW = 4 + PMAX * MW;            // record words in use
    constexpr int kSpineChunk = spine_chunk_items<NW>();    // records held in registers
    constexpr int NQ = (NW + 3) / 4;             // 16-byte parts of a record (records are 80 bytes)
    static_assert(kMsRec % 4 == 0 && NQ * 4 <= kMsRec, "records load as whole 16-byte parts");
    __shared__ uint32_t s_wm[PMAX][kSpineThreads / 64 + 1][MW];
    __shared__ uint32_t s_wc[4][kSpineThreads / 64 + 1];
    __shared__ uint32_t s_carry[NW];
    const uint32_t n = *a.n_dev;
    const uint32_t tiles = (n + TILE - 1) / TILE;
    const uint32_t P = a.n_props;
    const uint32_t nchunks = MODE == 0 ? 1u : (tiles + a.spine_chunk - 1) / a.spine_chunk;
    uint32_t r0 = 0, r1 = tiles;                 // the records this block scans
    const uint32_t* in = a.agg;
    uint32_t* out = a.prefix;
    if (MODE == 1 || MODE == 3) {
        r0 = blockIdx.x * a.spine_chunk;
        r1 = min(tiles, r0 + a.spine_chunk);
        if (r0 >= r1) return;
    } else if (MODE == 2) {
        r1 = nchunks;
        in = a.chunk_agg;
        out = a.chunk_pre;
    }
    if (threadIdx.x < NW) {
        uint32_t v = threadIdx.x < 4 ? 0u : bm_identity<MW>().d[(threadIdx.x - 4) % MW];
        if (MODE == 3) v = a.chunk_pre[(uint64_t)blockIdx.x * kMsRec + threadIdx.x];
        s_carry[threadIdx.x] = v;
    }
    __syncthreads();
    for (uint32_t pass0 = r0; pass0 < r1; pass0 += kSpineThreads * kSpineChunk) {
        const uint32_t t0 = pass0 + threadIdx.x * kSpineChunk;
        const uint32_t cnt = t0 < r1 ? min<uint32_t>(kSpineChunk, r1 - t0) : 0u;
        // unconditional loads of clamped records: all of them in flight together
        uint32_t rec[kSpineChunk][NQ * 4];
#pragma unroll
        for (int i = 0; i < kSpineChunk; ++i) {
            const uint32_t t = min(t0 + (uint32_t)i, r1 - 1u);
            const uint4* src = reinterpret_cast<const uint4*>(in + (uint64_t)t * kMsRec);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const uint4 v = src[q];
                rec[i][4 * q] = v.x;
                rec[i][4 * q + 1] = v.y;
                rec[i][4 * q + 2] = v.z;
                rec[i][4 * q + 3] = v.w;
            }
        }
        BMap<MW> f[PMAX], excl[PMAX], tot[PMAX];
        uint32_t c[4] = {0, 0, 0, 0}, cexcl[4], ctot[4];
#pragma unroll
        for (int p = 0; p < PMAX; ++p) f[p] = bm_identity<MW>();
#pragma unroll
        for (int i = 0; i < kSpineChunk; ++i) {
            const bool inr = (uint32_t)i < cnt;
#pragma unroll
            for (int p = 0; p < PMAX; ++p)
                if (p < (int)P && inr) f[p] = bm_compose<MW>(bm_load<MW>(&rec[i][4 + MW * p]), f[p]);
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] += inr ? rec[i][k] : 0u;
        }
        block_scan<PMAX, MW, kSpineThreads>(P, f, c, excl, cexcl, tot, ctot, s_wm, s_wc);
        if (MODE != 1) {
            // this thread's prefix: the carry from earlier passes, then the block's
            BMap<MW> acc[PMAX];
            uint32_t cc[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) cc[k] = s_carry[k] + cexcl[k];
#pragma unroll
            for (int p = 0; p < PMAX; ++p) acc[p] = bm_compose<MW>(excl[p], bm_load<MW>(&s_carry[4 + MW * p]));
#pragma unroll
            for (int i = 0; i < kSpineChunk; ++i) {
                if ((uint32_t)i >= cnt) continue;
                uint32_t* o = out + (uint64_t)(t0 + i) * kMsRec;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    o[k] = cc[k];
                    cc[k] += rec[i][k];
                }
#pragma unroll
                for (int p = 0; p < PMAX; ++p) {
                    if (p >= (int)P) continue;
#pragma unroll
                    for (int k = 0; k < MW; ++k) o[4 + MW * p + k] = acc[p].d[k];
                    acc[p] = bm_compose<MW>(bm_load<MW>(&rec[i][4 + MW * p]), acc[p]);
                }
            }
        }
        __syncthreads();                         // every thread has read the carry
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) s_carry[k] += ctot[k];
#pragma unroll
            for (int p = 0; p < PMAX; ++p) {
                const BMap<MW> nc = bm_compose<MW>(tot[p], bm_load<MW>(&s_carry[4 + MW * p]));
#pragma unroll
                for (int k = 0; k < MW; ++k) s_carry[4 + MW * p + k] = nc.d[k];
            }
        }
        __syncthreads();
    }
    // the chunk's record: its composition (the carry started at the identity)
    if (MODE == 1 && threadIdx.x < NW) a.chunk_agg[(uint64_t)blockIdx.x * kMsRec + threadIdx.x] = s_carry[threadIdx.x];
}

// TL: the instantiation that also walks the verdict timeline (its registers
// stay out of the plain sweep's occupancy)
template <int PMAX, int MW, int ITEMS, bool TL>
__global__ __launch_bounds__(kMsThreads) void k_ms_down(ScanArgs a) {
    constexpr uint32_t TILE = kMsThreads * ITEMS;
    constexpr bool kParents = PMAX <= 4;         // LDS room to stage parent ids
    constexpr uint32_t kIvStride = TILE + 1;
    __shared__ uint32_t s_cm[PMAX][16][MW];
    __shared__ uint32_t s_q0[PMAX], s_lab[PMAX][2];
    __shared__ uint32_t s_red[2][kMsThreads / 64];
    // staging: verdict bytes [P][tile + 1], then 16-bit parent offsets [tile + 1]
    __shared__ uint32_t s_stage[(PMAX * kIvStride + 3) / 4 + (kParents ? (kIvStride + 1) / 2 : 0)];
    const uint32_t n = *a.n_dev;
    const uint64_t base = (uint64_t)blockIdx.x * TILE;
    if (base >= n) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t P = a.n_props, L = a.n_levels;
    const bool structure = kParents && a.structure != 0;
    const uint64_t my0 = base + (uint64_t)tid * ITEMS;
    // every load first, so that they are all in flight together: tables,
    // this thread's prefix within the tile (reduce), the tile's (spine), the
    // descriptors and the one after them
    const uint64_t row = (uint64_t)a.tiles * kMsThreads, at = (uint64_t)blockIdx.x * kMsThreads + tid;
    const uint32_t c01 = a.trec[at], c23 = a.trec[row + at];
    BMap<MW> tex[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
#pragma unroll
        for (int k = 0; k < MW; ++k) tex[p].d[k] = a.trec[(2 + MW * p + k) * row + at];
    const uint32_t* pre = a.prefix + (uint64_t)blockIdx.x * kMsRec;
    uint32_t tcnt[4], pmap[PMAX][MW];
#pragma unroll
    for (int k = 0; k < 4; ++k) tcnt[k] = pre[k];
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
#pragma unroll
        for (int k = 0; k < MW; ++k) pmap[p][k] = pre[4 + MW * p + k];
    const uint32_t next_desc = a.desc[(my0 < n ? my0 : 0) + ITEMS];
    const Run r = run_from_desc<ITEMS>(a, my0, n);
    const TableRegs tr = read_tables<PMAX, MW>(a);
    // an instance ends where the next word is absent or a head
    const bool next_head = my0 + ITEMS < n ? ((next_desc >> 4) & 1u) != 0 : true;
    store_tables<PMAX, MW>(a, tr, s_cm, s_q0, s_lab);
    __syncthreads();
    uint32_t cexcl[4] = {c01 & 0xFFFFu, c01 >> 16, c23 & 0xFFFFu, c23 >> 16};
    uint32_t cur[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        cur[p] = 0;
        if (p < (int)P) cur[p] = bm_at<MW>(bm_compose<MW>(tex[p], bm_load<MW>(pmap[p])), 0);
    }
    const bool timeline = TL && (a.inst_conc || a.event_verdict);
    uint32_t cur0[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) cur0[p] = cur[p];
    const uint32_t valid = valid_mask(r.cnt);
    const uint32_t m_end = r.cnt ? valid & ((r.m_head >> 1) | ((next_head ? 1u : 0u) << (r.cnt - 1u))) : 0u;
    uint8_t* s_iv = reinterpret_cast<uint8_t*>(s_stage);
    uint16_t* s_par = reinterpret_cast<uint16_t*>(s_stage + (PMAX * kIvStride + 3) / 4);
    const uint32_t id_base = tcnt[0];
    const uint32_t m_par = L >= 4 ? r.m_lvl[3] : L == 3 ? r.m_lvl[2] : r.m_lvl[1];
    // parents are level-(L-1) nodes: id = the tile's count before it + a local offset
    const uint32_t lpar = L >= 4 ? 3u : L == 3 ? 2u : 1u;
    const uint32_t par_tile = tcnt[lpar] - 1u, par_local = cexcl[lpar];
    uint32_t my_lo = 0xFFFFFFFFu, my_hi = 0u, err = 0;
    // First every word's state, without branches (the class maps' LDS reads
    // do not wait on the instance bookkeeping): 4 bits per word and property.
    uint64_t st[PMAX][ITEMS / 16];
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
#pragma unroll
        for (int h = 0; h < ITEMS / 16; ++h) st[p][h] = 0;
#pragma clang loop unroll(full)
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t c = run_class(r, j);
        const bool hd = (r.m_head >> j) & 1u;
#pragma clang loop unroll(full)
        for (int p = 0; p < PMAX; ++p) {    // (a launch has at least one property)
            if (p > 0 && p >= (int)P) continue;
            cur[p] = bm_at<MW>(bm_load<MW>(s_cm[p][c]), hd ? s_q0[p] : cur[p]);
            st[p][j >> 4] |= (uint64_t)cur[p] << (4 * (j & 15));
        }
    }
    // Then the instances ending in the run, one loop step per end.
    for (uint32_t rest = m_end; rest != 0u; rest &= rest - 1u) {
        const uint32_t j = (uint32_t)__ffs(rest) - 1u;
        const uint32_t upto = j == 31u ? kAll : (2u << j) - 1u;
        const uint32_t slot = cexcl[0] + __popc(r.m_head & upto);     // 1-based, within the tile
        const uint64_t id = (uint64_t)id_base + slot - 1u;
        if (id < a.inst_limit) {
            const uint32_t sh = 4u * (j & 15u);
#pragma clang loop unroll(full)
            for (int p = 0; p < PMAX; ++p) {
                if (p > 0 && p >= (int)P) continue;
                // both halves shifted before the choice, and kept apart so that
                // the choice is not turned into an indexed register array
                uint32_t s0 = (uint32_t)(st[p][0] >> sh) & 15u, s1 = (uint32_t)(st[p][ITEMS / 16 - 1] >> sh) & 15u;
                asm("" : "+v"(s0), "+v"(s1));
                const uint32_t q = ITEMS > 16 && j >= 16u ? s1 : s0;
                s_iv[p * kIvStride + slot] = (s_lab[p][q >> 3] >> (4 * (q & 7u))) & 15u;
            }
            if (kParents && L >= 2) s_par[slot] = (uint16_t)(par_local + __popc(m_par & upto));
            my_lo = min(my_lo, (uint32_t)id);
            my_hi = max(my_hi, (uint32_t)id + 1u);
            if (structure && a.inst_keys) a.inst_keys[id] = a.words[my0 + j] >> a.cbits;
        } else {
            err |= kErrCapacity;
        }
    }
    // On request, the verdict timeline: a second walk from the thread's
    // starting states.  Conclusive verdicts are final (Def. 5), so the monitor
    // enters a conclusive state at most once per instance: the word where it
    // does writes its 1-based sorted position (the head's position when q0
    // itself is conclusive), the word ending an instance that never got there
    // writes kNever; k_inst_conclusive turns positions into prefix lengths.
    // The verdict after every event goes to the event's trace index, which
    // rides in the word between class and key.
    if (timeline) {
        // trace indices of the thread's words: all loads in flight at once,
        // then one taken per step and the rest moved down a register
        uint32_t evi[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) evi[k] = 0;
        if (a.event_verdict) {
            const uint4* wp = reinterpret_cast<const uint4*>(a.words + (r.cnt ? my0 : 0));
#pragma unroll
            for (int k = 0; k < ITEMS / 2; ++k) {
                const uint4 v = wp[k];
                evi[2 * k] = (uint32_t)((((uint64_t)v.y << 32) | v.x) >> a.index_shift) & a.index_mask;
                evi[2 * k + 1] = (uint32_t)((((uint64_t)v.w << 32) | v.z) >> a.index_shift) & a.index_mask;
            }
        }
        // the states come from the first walk (4 bits per word), the labels
        // of the states from registers
        uint32_t lab[PMAX][2], q0v[PMAX], prev[PMAX];
#pragma unroll
        for (int p = 0; p < PMAX; ++p) {
            lab[p][0] = s_lab[p][0];
            lab[p][1] = s_lab[p][1];
            q0v[p] = s_q0[p];
            prev[p] = cur0[p];
        }
#pragma unroll 1
        for (uint32_t j = 0; j < r.cnt; ++j) {
            const uint32_t sh = 4u * (j & 15u);
            const bool hd = (r.m_head >> j) & 1u, end = (m_end >> j) & 1u;
            const uint32_t upto = j == 31u ? kAll : (2u << j) - 1u;
            const uint64_t id = (uint64_t)id_base + cexcl[0] + __popc(r.m_head & upto) - 1u;
            const uint32_t pos = (uint32_t)(my0 + j);
            const bool conc_out = a.inst_conc && id < a.inst_limit;
            if (conc_out && hd && structure) a.inst_start[id] = pos;
            const uint64_t ev = evi[0];
#pragma unroll
            for (int k = 0; k + 1 < ITEMS; ++k) evi[k] = evi[k + 1];
#pragma clang loop unroll(full)
            for (int p = 0; p < PMAX; ++p) {
                if (p > 0 && p >= (int)P) continue;
                // both halves shifted before the choice, kept apart (no
                // indexed register array)
                uint32_t s0 = (uint32_t)(st[p][0] >> sh) & 15u, s1 = (uint32_t)(st[p][ITEMS / 16 - 1] >> sh) & 15u;
                asm("" : "+v"(s0), "+v"(s1));
                const uint32_t post = ITEMS > 16 && j >= 16u ? s1 : s0;
                const uint32_t pre = hd ? q0v[p] : prev[p];
                prev[p] = post;
                const uint32_t lpost = ((post < 8u ? lab[p][0] : lab[p][1]) >> (4u * (post & 7u))) & 15u;
                if (a.event_verdict) a.event_verdict[a.prop_idx[p] * a.n_events + ev] = (uint8_t)lpost;
                if (!conc_out) continue;
                uint32_t* out = a.inst_conc + a.prop_idx[p] * a.inst_stride + id;
                const uint32_t lpre = ((pre < 8u ? lab[p][0] : lab[p][1]) >> (4u * (pre & 7u))) & 15u;
                const bool cpre = lpre == 0u || lpre == 5u, cpost = lpost == 0u || lpost == 5u;
                if (hd && cpre) *out = pos;
                else if (cpost && !cpre) *out = pos + 1u;
                if (end && !cpost) *out = kNever;
            }
        }
    }
    // nodes of levels 1.. open at their first word (a level-m head is also a
    // level-(m+1) head); few words do: a loop over them
    if (structure && L >= 2) {
        for (uint32_t rest = m_par; rest != 0u; rest &= rest - 1u) {
            const int j = __ffs(rest) - 1;
            const uint32_t upto = j == 31 ? kAll : (2u << j) - 1u;
#pragma unroll
            for (int m = kMaxLevels - 1; m >= 1; --m) {
                if (m >= (int)L || !((r.m_lvl[m] >> j) & 1u)) continue;
                const uint64_t id = (uint64_t)tcnt[m] + cexcl[m] + __popc(r.m_lvl[m] & upto) - 1u;
                const int mc = m < 3 ? m + 1 : 3;
                const uint32_t child = m == (int)L - 1 ? tcnt[0] + cexcl[0] + __popc(r.m_head & upto) - 1u
                                                       : tcnt[mc] + cexcl[mc] + __popc(r.m_lvl[mc] & upto) - 1u;
                if (id < a.node_limit[m]) {
                    a.node_start[m][id] = child;
                    if (a.node_keys[m]) a.node_keys[m][id] = a.words[my0 + j] >> a.prefix_shift[m];
                    uint32_t* cn = a.node_counts[m];
                    if (cn)
                        for (uint32_t p = 0; p < a.n_props_all; ++p) {
                            uint2* q = reinterpret_cast<uint2*>(cn + (p * a.node_stride[m] + id) * 6);
                            q[0] = make_uint2(0u, 0u);
                            q[1] = make_uint2(0u, 0u);
                            q[2] = make_uint2(0u, 0u);
                        }
                } else {
                    err |= kErrCapacity;
                }
            }
        }
    }
    if (err) atomicOr(a.err, err);
    // the instances ending in this tile have consecutive ids: write their
    // verdicts (and parents) contiguously from LDS
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        my_lo = min(my_lo, (uint32_t)__shfl_xor(my_lo, off, 64));
        my_hi = max(my_hi, (uint32_t)__shfl_xor(my_hi, off, 64));
    }
    if (lane == 0) {
        s_red[0][w] = my_lo;
        s_red[1][w] = my_hi;
    }
    __syncthreads();
    uint32_t lo = s_red[0][0], hi = s_red[1][0];
    for (int i = 1; i < kMsThreads / 64; ++i) {
        lo = min(lo, s_red[0][i]);
        hi = max(hi, s_red[1][i]);
    }
    if (lo < hi) {
        const uint32_t cnt_iv = hi - lo, slot0 = lo + 1u - id_base;
        for (uint32_t p = 0; p < P; ++p)
            for (uint32_t i = tid; i < cnt_iv; i += kMsThreads)
                a.inst_verdict[a.prop_idx[p] * a.inst_stride + lo + i] = s_iv[p * kIvStride + slot0 + i];
        if (structure && a.inst_parent && L >= 2)
            for (uint32_t i = tid; i < cnt_iv; i += kMsThreads) a.inst_parent[lo + i] = par_tile + s_par[slot0 + i];
    }
    // the thread holding the last word publishes the totals
    if (structure && r.cnt && my0 + r.cnt == n) {
        const uint32_t cnt[4] = {(uint32_t)__popc(r.m_head), (uint32_t)__popc(r.m_lvl[1]), (uint32_t)__popc(r.m_lvl[2]),
                                 (uint32_t)__popc(r.m_lvl[3])};
#pragma unroll
        for (int m = 0; m < kMaxLevels; ++m) {
            if (m >= (int)L) break;
            const uint32_t tot_m = tcnt[m] + cexcl[m] + cnt[m];
            a.sizes[m] = tot_m;
            a.sizes32[m] = tot_m;
        }
    }
}

template <int PMAX, int MW, int ITEMS>
static void launch_ms_t(const ScanArgs& a, hipStream_t s) {
    const uint32_t tiles = (uint32_t)((a.n + kMsThreads * ITEMS - 1) / (kMsThreads * ITEMS));
    const dim3 grid(tiles ? tiles : 1);
    ScanArgs r = a;
    r.tiles = tiles;
    hipLaunchKernelGGL((k_ms_reduce<PMAX, MW, ITEMS>), grid, dim3(kMsThreads), 0, s, r);
    // one spine block takes kSpineThreads x chunk records per pass; beyond two
    // passes the chunks are spread over blocks
    constexpr uint32_t kPass = (uint32_t)kSpineThreads * spine_chunk_items<4 + PMAX * MW>();
    if (tiles <= 2 * kPass || !a.chunk_agg || !a.chunk_pre) {
        hipLaunchKernelGGL((k_ms_spine<PMAX, MW, ITEMS, 0>), dim3(1), dim3(kSpineThreads), 0, s, r);
    } else {
        r.spine_chunk = kPass;
        const uint32_t nchunks = (tiles + kPass - 1) / kPass;
        hipLaunchKernelGGL((k_ms_spine<PMAX, MW, ITEMS, 1>), dim3(nchunks), dim3(kSpineThreads), 0, s, r);
        hipLaunchKernelGGL((k_ms_spine<PMAX, MW, ITEMS, 2>), dim3(1), dim3(kSpineThreads), 0, s, r);
        hipLaunchKernelGGL((k_ms_spine<PMAX, MW, ITEMS, 3>), dim3(nchunks), dim3(kSpineThreads), 0, s, r);
    }
    ScanArgs d = r;
    d.read_desc = 1;
    if (a.inst_conc || a.event_verdict) hipLaunchKernelGGL((k_ms_down<PMAX, MW, ITEMS, true>), grid, dim3(kMsThreads), 0, s, d);
    else hipLaunchKernelGGL((k_ms_down<PMAX, MW, ITEMS, false>), grid, dim3(kMsThreads), 0, s, d);
}

template <int ITEMS>
static void launch_ms_items(const ScanArgs& a, hipStream_t s) {
    if (a.max_states <= 8) {
        if (a.n_props <= 1) launch_ms_t<1, 2, ITEMS>(a, s);
        else if (a.n_props <= 2) launch_ms_t<2, 2, ITEMS>(a, s);
        else if (a.n_props <= 4) launch_ms_t<4, 2, ITEMS>(a, s);
        else launch_ms_t<8, 2, ITEMS>(a, s);
    } else {
        if (a.n_props <= 1) launch_ms_t<1, 4, ITEMS>(a, s);
        else if (a.n_props <= 2) launch_ms_t<2, 4, ITEMS>(a, s);
        else launch_ms_t<4, 4, ITEMS>(a, s);
    }
}

// items: words per thread, 16 (4,096-word tiles) or 32 (8,192-word tiles).
// The workspace arrays are sized for 16 (the more tiles).
hipError_t launch_mapscan(const ScanArgs& a, int items, hipStream_t s) {
    if (a.n_props < 1 || a.n_props > (a.max_states <= 8 ? 8u : 4u) || (a.structure && a.n_props > 4) || !a.n_dev ||
        !a.desc || !a.agg || !a.prefix || !a.trec || (items != 16 && items != 32))
        return hipErrorInvalidValue;
    if (items == 16) launch_ms_items<16>(a, s);
    else launch_ms_items<32>(a, s);
    return hipGetLastError();
}

}  // namespace ltl4c
