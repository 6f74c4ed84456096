// Parent events: events that carry the keys of every quantifier level but the
// innermost one join the cluster u^D of every instance D under their parent,
// at their place in trace order (the proxy-cache case study of Section 5,
// where per-video cache events bear on every request of the video).
//
// After the radix sort the own events (full value vectors, kind bit 0) come
// first, sorted by (key, trace index), and the parent events (kind bit 1) after
// them, sorted by (parent prefix, trace index): the "parent array" P.  The
// structure scan numbers the instances and nodes from the own events alone.
// Here every instance's verdict is recomputed with its parent events merged
// in:
//   * G_i, the number of parent-array entries ordered before own event i by
//     (prefix, trace index); an instance's own events split its parent's run
//     of P at the G_i into gaps.  Within an instance the G_i grow, and so do
//     the run starts along the sorted own events, so each thread finds them by
//     galloping forward from the previous bound (one full binary search per
//     thread run);
//   * the map of each gap is the composition of the class maps of its parent
//     events, taken from a segment tree over P (level L node q composes the
//     entries [q 2^L, (q+1) 2^L)), built eight levels per launch in LDS;
//   * own event i contributes F_i = M_c o [gap before it], a head the
//     constant map of F_i(q0); an inclusive scan of the F_i (reduce per
//     tile, a parallel spine over the tiles, down sweep) gives the state
//     after every own event, and the trailing gap of the parent's run,
//     applied at an instance's last own event, its final state.
#include "internal.h"

namespace ltl4c {

namespace {

struct Map16 {
    uint32_t d[4];
};

__device__ __forceinline__ Map16 m_identity() {
    Map16 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = 0x03020100u + 0x04040404u * (uint32_t)i;
    return r;
}

__device__ __forceinline__ Map16 m_const(uint32_t s) {
    Map16 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = s * 0x01010101u;
    return r;
}

// g o f: f first, byte q of the result is g[f[q]]
__device__ __forceinline__ Map16 m_compose(const Map16& g, const Map16& f) {
    Map16 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // low half where the state is below 8, high half elsewhere; the last
        // permute picks per byte on bit 3 of the state
        const uint32_t sel = f.d[i];
        const uint32_t lo = __builtin_amdgcn_perm(g.d[1], g.d[0], sel);
        const uint32_t hi = __builtin_amdgcn_perm(g.d[3], g.d[2], sel ^ 0x08080808u);
        r.d[i] = __builtin_amdgcn_perm(hi, lo, ((sel >> 1) & 0x04040404u) | 0x03020100u);
    }
    return r;
}

// byte q of a map (byte permutes, not an indexed register array, which the
// compiler would place in scratch memory)
__device__ __forceinline__ uint32_t m_at(const Map16& g, uint32_t q) {
    const uint32_t lo = __builtin_amdgcn_perm(g.d[1], g.d[0], q & 7u);
    const uint32_t hi = __builtin_amdgcn_perm(g.d[3], g.d[2], q & 7u);
    return ((q & 8u) ? hi : lo) & 0xFFu;
}

__device__ __forceinline__ Map16 m_from(const uint4& v) {
    Map16 r;
    r.d[0] = v.x;
    r.d[1] = v.y;
    r.d[2] = v.z;
    r.d[3] = v.w;
    return r;
}

__device__ __forceinline__ uint4 m_to(const Map16& m) { return make_uint4(m.d[0], m.d[1], m.d[2], m.d[3]); }

__device__ __forceinline__ Map16 m_shfl_up(const Map16& v, int off) {
    Map16 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = __shfl_up(v.d[i], off, 64);
    return r;
}

// (prefix, trace index) of a sorted word; the parent array is in this order
__device__ __forceinline__ uint64_t search_key(const ParentArgs& a, uint64_t w) {
    const uint64_t prefix = (w >> a.prefix_shift) & a.prefix_mask;
    return (prefix << a.ibits) | ((w >> a.cbits) & a.index_mask);
}

__device__ __forceinline__ uint64_t prefix_of(const ParentArgs& a, uint64_t w) {
    return (w >> a.prefix_shift) & a.prefix_mask;
}

// number of parent-array entries whose search key is below `target`, from
// the block's copy of the sample table (sample i is the key of entry
// i * stride, all ones past the end): a search in LDS narrows the answer to
// one stride, then a binary search in memory.
__device__ __forceinline__ uint32_t lower_bound_sampled(const ParentArgs& a, const uint64_t* par, uint32_t k,
                                                        const uint64_t* samp, uint64_t target) {
    if (k == 0) return 0;
    const uint32_t stride = (k + kPeSamples - 1) / kPeSamples;
    uint32_t lo = 0, hi = kPeSamples;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (samp[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    if (lo == 0) return 0;
    uint32_t l = (lo - 1) * stride + 1, r = min(lo * stride, k);
    while (l < r) {
        const uint32_t mid = (l + r) >> 1;
        if (search_key(a, par[mid]) < target) l = mid + 1;
        else r = mid;
    }
    return l;
}

// The same, given that every entry before g is below `target`: probes at g
// and then at doubling distances, and a binary search in the last interval,
// so a bound that moved by d entries costs about 2 log2(d + 1) loads (one
// when it did not move).
__device__ __forceinline__ uint32_t gallop(const ParentArgs& a, const uint64_t* par, uint32_t k, uint32_t g,
                                           uint64_t target) {
    uint64_t lo = g, step = 1, hi = k;
    while (lo < k) {
        const uint64_t probe = lo + step - 1;
        if (probe >= k) break;
        if (search_key(a, par[probe]) >= target) {
            hi = probe;
            break;
        }
        lo = probe + 1;
        step <<= 1;
    }
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (search_key(a, par[mid]) < target) lo = mid + 1;
        else hi = mid;
    }
    return (uint32_t)lo;
}

// search key of parent entry g, all ones past the end
__device__ __forceinline__ uint64_t key_at(const ParentArgs& a, const uint64_t* par, uint32_t k, uint32_t g) {
    return g < k ? search_key(a, par[g]) : ~0ull;
}

// level L node q of the segment tree of property p (level 0: the class map of
// the entry, from the block's copy of the property's class maps)
__device__ __forceinline__ Map16 tree_node(const ParentArgs& a, const uint4* cm, const uint64_t* par, uint32_t p,
                                           uint32_t L, uint64_t q) {
    if (L == 0) return m_from(cm[(uint32_t)par[q] & a.class_mask]);
    return m_from(a.tree[a.tree_off[L] + (uint64_t)p * a.tree_cnt[L] + q]);
}

// composition of the class maps of parent-array entries [l, r), in order.
// Up to kPeShortGap entries: their words are loaded together and their maps
// composed from LDS; longer gaps walk the segment tree.
__device__ __forceinline__ Map16 range_map(const ParentArgs& a, const uint4* cm, const uint64_t* par, uint32_t p,
                                           uint32_t l, uint32_t r) {
    if (r - l <= (uint32_t)kPeShortGap) {
        uint32_t c[kPeShortGap];
#pragma unroll
        for (int j = 0; j < kPeShortGap; ++j) c[j] = (uint32_t)par[min(l + (uint32_t)j, r - 1u)] & a.class_mask;
        Map16 m = m_identity();
#pragma unroll
        for (int j = 0; j < kPeShortGap; ++j)
            if (l + (uint32_t)j < r) m = m_compose(m_from(cm[c[j]]), m);
        return m;
    }
    Map16 left = m_identity(), right = m_identity();
    uint32_t L = 0;
    while (l < r) {
        if (l & 1u) {
            left = m_compose(tree_node(a, cm, par, p, L, l), left);
            ++l;
        }
        if (r & 1u) {
            --r;
            right = m_compose(right, tree_node(a, cm, par, p, L, r));
        }
        l >>= 1;
        r >>= 1;
        ++L;
    }
    return m_compose(right, left);
}

// One thread's run of own events: loaded to registers, its trace indices
// later staged in LDS (row j of column tid holds event j's), its classes and
// prefix ordinals (0 for the first event's prefix, one more at every change)
// kept as nibbles, its head and end flags as bits.
struct PeRun {
    uint64_t my0;
    uint32_t cnt;
    uint32_t heads, ends;                // bit j
    uint32_t cls[2], pord[2];            // nibble j of the pair
    uint64_t wprev;                      // the word before the run
    uint64_t w[kPeItems];
};

__device__ __forceinline__ uint32_t nibble(const uint32_t* v, uint32_t j) {
    return ((j < 8u ? v[0] : v[1]) >> (4 * (j & 7u))) & 15u;
}

__device__ __forceinline__ void load_run(const ParentArgs& a, uint32_t n_own, uint64_t my0, PeRun& r) {
    r.my0 = my0;
    r.cnt = my0 < n_own ? (uint32_t)min<uint64_t>(kPeItems, n_own - my0) : 0u;
    // unconditional loads (the word buffers are padded past the last tile)
    const uint64_t ld0 = r.cnt ? my0 : 0;
    const uint4* src = reinterpret_cast<const uint4*>(a.words + ld0);
#pragma unroll
    for (int q = 0; q < kPeItems / 2; ++q) {
        const uint4 v = src[q];
        r.w[2 * q] = (uint64_t)v.x | ((uint64_t)v.y << 32);
        r.w[2 * q + 1] = (uint64_t)v.z | ((uint64_t)v.w << 32);
    }
    r.wprev = a.words[ld0 ? ld0 - 1 : 0];
    const uint64_t wnext = a.words[ld0 + kPeItems];
    r.heads = r.ends = 0;
    r.cls[0] = r.cls[1] = r.pord[0] = r.pord[1] = 0;
    uint32_t ord = 0;
#pragma unroll
    for (int j = 0; j < kPeItems; ++j) {
        const uint64_t key = r.w[j] >> a.key_shift;
        const uint64_t kp = (j ? r.w[j - 1] : r.wprev) >> a.key_shift;
        const uint64_t kn = (j + 1 < kPeItems ? r.w[j + 1] : wnext) >> a.key_shift;
        const bool valid = (uint32_t)j < r.cnt;
        const bool head = valid && (my0 + j == 0 || kp != key);
        const bool end = valid && (my0 + j + 1 == n_own || kn != key);
        r.heads |= (head ? 1u : 0u) << j;
        r.ends |= (end ? 1u : 0u) << j;
        if (j && prefix_of(a, r.w[j]) != prefix_of(a, r.w[j - 1])) ++ord;
        r.cls[j >> 3] |= ((uint32_t)r.w[j] & a.class_mask) << (4 * (j & 7));
        r.pord[j >> 3] |= ord << (4 * (j & 7));
    }
}

// The search over the parent array along a run: the parent's run [rs, re)
// of the current prefix and the bound g of the last event.  Prefixes grow
// along the sorted own events and the bounds grow within an instance, so
// every search gallops forward from a known lower bound.  A short run (at
// most kPeShortRun entries, the usual case) is read once when its prefix is
// entered, its trace indices and classes kept in registers: bounds are then
// counts of smaller trace indices and gap maps come from the block's class
// maps, without memory traffic.  On a long run a bound that did not move
// costs no load either (the key at g is kept).
struct PeWalk {
    uint64_t pf;
    uint32_t ord;                        // prefix ordinal of pf within the thread's run
    uint32_t rs, re, g;
    uint64_t gkey;                       // long run: search key at g, all ones at re
    uint32_t rcls;                       // short run: class of entry rs + j in bits 4j..
    uint32_t tix[kPeShortRun];           // short run: trace index of entry rs + j

    __device__ __forceinline__ bool is_short() const { return re - rs <= (uint32_t)kPeShortRun; }

    // the run of prefix pj, searched from `from` (a lower bound of its start;
    // `exact` when it is the start): the first kPeShortRun + 1 entries are
    // read together, and only a longer run is searched further
    __device__ __forceinline__ void enter(const ParentArgs& a, const uint64_t* par, uint32_t k, uint64_t pj,
                                          uint32_t from, bool exact) {
        pf = pj;
        rs = exact ? from : gallop(a, par, k, from, pj << a.ibits);
        uint64_t wj[kPeShortRun + 1];
        const uint32_t last = k ? k - 1u : 0u;
#pragma unroll
        for (int j = 0; j <= kPeShortRun; ++j) wj[j] = k ? par[min(rs + (uint32_t)j, last)] : 0ull;
        uint32_t n = 0;
#pragma unroll
        for (int j = 0; j <= kPeShortRun; ++j)
            n += (rs + (uint32_t)j < k && prefix_of(a, wj[j]) == pj) ? 1u : 0u;
        rcls = 0;
        if (n <= (uint32_t)kPeShortRun) {
            re = rs + n;
#pragma unroll
            for (int j = 0; j < kPeShortRun; ++j) {
                tix[j] = (uint32_t)j < n ? (uint32_t)((wj[j] >> a.cbits) & a.index_mask) : 0xFFFFFFFFu;
                rcls |= ((uint32_t)j < n ? ((uint32_t)wj[j] & a.class_mask) : 0u) << (4 * j);
            }
        } else {
            re = gallop(a, par, k, rs + kPeShortRun + 1, (pj + 1) << a.ibits);
        }
    }

    __device__ __forceinline__ void reset_to_run_start(const ParentArgs& a, const uint64_t* par) {
        g = rs;
        gkey = is_short() ? ~0ull : key_at(a, par, re, rs);
    }

    // start of a run: a search in the sample table for the first prefix, then
    // the bound of the event before the run when it belongs to the same
    // instance
    __device__ __forceinline__ void start(const ParentArgs& a, const uint64_t* par, uint32_t k, const PeRun& r,
                                          const uint64_t* samp) {
        const uint64_t pj = prefix_of(a, r.w[0]);
        ord = 0;
        enter(a, par, k, pj, r.cnt ? lower_bound_sampled(a, par, k, samp, pj << a.ibits) : 0u, r.cnt != 0);
        reset_to_run_start(a, par);
        if (r.cnt && !(r.heads & 1u)) advance(a, par, (uint32_t)((r.wprev >> a.cbits) & a.index_mask));
    }

    // g becomes the bound of an own event of the current instance with trace
    // index t
    __device__ __forceinline__ void advance(const ParentArgs& a, const uint64_t* par, uint32_t t) {
        if (is_short()) {
            uint32_t c = 0;
#pragma unroll
            for (int j = 0; j < kPeShortRun; ++j) c += tix[j] < t ? 1u : 0u;
            g = rs + c;
            return;
        }
        const uint64_t target = (pf << a.ibits) | t;
        if (gkey < target) {
            g = gallop(a, par, re, g + 1, target);
            gkey = key_at(a, par, re, g);       // all ones at the run end
        }
    }

    // own event j of the run, with trace index t: returns lo, the start of the
    // gap before it; g becomes its G.  A head with a new prefix reads its word
    // again for the prefix.
    __device__ __forceinline__ uint32_t step(const ParentArgs& a, const uint64_t* par, uint32_t k, const PeRun& r,
                                             uint32_t j, uint32_t t, bool head) {
        if (head) {
            const uint32_t oj = nibble(r.pord, j);
            if (oj != ord) {
                ord = oj;
                enter(a, par, k, prefix_of(a, a.words[r.my0 + j]), re, false);
            }
            reset_to_run_start(a, par);
        }
        const uint32_t lo = g;
        advance(a, par, t);
        return lo;
    }

    // composition of the class maps of the run's entries [l, r) (l <= r)
    __device__ __forceinline__ Map16 gap_map(const ParentArgs& a, const uint4* cm, const uint64_t* par, uint32_t p,
                                             uint32_t l, uint32_t r) const {
        if (!is_short()) return range_map(a, cm, par, p, l, r);
        Map16 m = m_identity();
        for (uint32_t e = l; e < r; ++e) m = m_compose(m_from(cm[(rcls >> (4 * (e - rs))) & 15u]), m);
        return m;
    }

    // the same, applied to one state
    __device__ __forceinline__ uint32_t gap_at(const ParentArgs& a, const uint4* cm, const uint64_t* par, uint32_t p,
                                               uint32_t l, uint32_t r, uint32_t st) const {
        if (!is_short()) return m_at(range_map(a, cm, par, p, l, r), st);
        for (uint32_t e = l; e < r; ++e) st = m_at(m_from(cm[(rcls >> (4 * (e - rs))) & 15u]), st);
        return st;
    }
};

// inclusive scan of (map, count) over the block, thread order; returns the
// thread's inclusive value and leaves the wave totals in s_map / s_cnt
__device__ __forceinline__ void block_scan(Map16& v, uint32_t& c, uint4* s_map, uint32_t* s_cnt) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const Map16 o = m_shfl_up(v, off);
        const uint32_t oc = __shfl_up(c, off, 64);
        if (lane >= off) {
            v = m_compose(v, o);
            c += oc;
        }
    }
    if (lane == 63) {
        s_map[w] = m_to(v);
        s_cnt[w] = c;
    }
    __syncthreads();
}

}  // namespace

// n_own = kept - parent events (both counted by classify)
__global__ void k_pe_counts(ParentArgs a) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *a.n_own = *a.n_kept - *a.n_par;
}

// The sample table: entry i * stride of the parent array (stride =
// ceil(k / kPeSamples)), all ones past the end.
__global__ __launch_bounds__(256) void k_pe_samples(ParentArgs a) {
    const uint32_t k = *a.n_par;
    const uint64_t* par = a.words + *a.n_own;
    const uint32_t stride = k ? (k + kPeSamples - 1) / kPeSamples : 1u;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < (uint32_t)kPeSamples; i += gridDim.x * blockDim.x) {
        const uint64_t at = (uint64_t)i * stride;
        a.samples[i] = at < k ? search_key(a, par[at]) : ~0ull;
    }
}

// Levels L0+1 .. L0+nlev of the segment tree of property blockIdx.y, from
// level L0: each block takes 256 level-L0 nodes and halves them in LDS.  A
// missing right child counts as the identity.
__global__ __launch_bounds__(256) void k_pe_tree(ParentArgs a, uint32_t L0, uint32_t nlev) {
    __shared__ uint4 s[256];
    __shared__ uint4 s_cm[16];
    const uint32_t p = blockIdx.y;
    if (threadIdx.x < 16) {
        const uint32_t* m = a.plan->prop[p].bmap[threadIdx.x];
        s_cm[threadIdx.x] = make_uint4(m[0], m[1], m[2], m[3]);
    }
    __syncthreads();
    const uint32_t k = *a.n_par;
    const uint64_t* par = a.words + *a.n_own;
    const uint64_t cnt0 = ((uint64_t)k + (1ull << L0) - 1) >> L0;
    const uint32_t t = threadIdx.x;
    for (uint64_t b = blockIdx.x; b * 256 < cnt0; b += gridDim.x) {
        const uint64_t q = b * 256 + t;
        Map16 m = q < cnt0 ? tree_node(a, s_cm, par, p, L0, q) : m_identity();
        for (uint32_t l = 1; l <= nlev; ++l) {
            if (t < (256u >> (l - 1))) s[t] = m_to(m);
            __syncthreads();
            if (t < (256u >> l)) {
                m = m_compose(m_from(s[2 * t + 1]), m_from(s[2 * t]));
                const uint32_t L = L0 + l;
                const uint64_t node = b * (256u >> l) + t;
                if (node < (((uint64_t)k + (1ull << L) - 1) >> L))
                    a.tree[a.tree_off[L] + (uint64_t)p * a.tree_cnt[L] + node] = m_to(m);
            }
            __syncthreads();
        }
    }
}

// DOWN = false: per tile and property, every thread's run map (into trec)
// and the tile's composition, and the tile's head count.  DOWN = true: the
// states at the instance ends, from the spine's tile prefixes and the run
// maps; verdicts written by instance number.
template <bool DOWN>
__global__ __launch_bounds__(kPeThreads) void k_pe_pass(ParentArgs a) {
    __shared__ uint32_t s_t[kPeItems][kPeThreads];
    __shared__ uint4 s_cm[kMaxProps][16];
    __shared__ uint8_t s_iv[kPeTile + 4];
    __shared__ uint32_t s_red[2][kPeThreads / 64];
    __shared__ uint4 s_map[kPeThreads / 64];
    __shared__ uint32_t s_cnt[kPeThreads / 64];
    const uint32_t n_own = *a.n_own, k = *a.n_par;
    const uint64_t* par = a.words + n_own;
    const uint32_t tile = blockIdx.x;
    const uint64_t base = (uint64_t)tile * kPeTile;
    if (base >= n_own) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (uint32_t i = tid; i < a.n_props * 16u; i += kPeThreads) {
        const uint32_t* m = a.plan->prop[i >> 4].bmap[i & 15u];
        s_cm[i >> 4][i & 15u] = make_uint4(m[0], m[1], m[2], m[3]);
    }
    // the sample table of the parent array first occupies the LDS rows of the
    // trace indices
    static_assert(kPeSamples * 8 <= kPeItems * kPeThreads * 4, "samples share LDS with the trace indices");
    uint64_t* s_samp = reinterpret_cast<uint64_t*>(&s_t[0][0]);
    for (uint32_t i = tid; i < (uint32_t)kPeSamples; i += kPeThreads) s_samp[i] = a.samples[i];
    PeRun r;
    load_run(a, n_own, base + (uint64_t)tid * kPeItems, r);
    __syncthreads();
    PeWalk w0;
    w0.start(a, par, k, r, s_samp);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPeItems; ++j) s_t[j][tid] = (uint32_t)((r.w[j] >> a.cbits) & a.index_mask);
    __syncthreads();
    const uint64_t row = (uint64_t)gridDim.x * kPeThreads;
    if (!DOWN) {
        for (uint32_t p = 0; p < a.n_props; ++p) {
            const uint4* cm = s_cm[p];
            const uint32_t q0 = a.plan->prop[p].q0;
            Map16 agg = m_identity();
            PeWalk wk = w0;
            if (r.heads == 0) {
                // no instance begins in the run: compose the maps of its events
                for (uint32_t j = 0; j < r.cnt; ++j) {
                    const uint32_t lo = wk.step(a, par, k, r, j, s_t[j][tid], false);
                    Map16 f = m_from(cm[nibble(r.cls, j)]);
                    if (lo < wk.g) f = m_compose(f, wk.gap_map(a, cm, par, p, lo, wk.g));
                    agg = m_compose(f, agg);
                }
            } else {
                // the last head's map is constant, so the run's map is the
                // constant of the state reached from q0 at that head
                uint32_t st = q0;
                for (uint32_t j = 31u - __clz(r.heads); j < r.cnt; ++j) {
                    const uint32_t lo = wk.step(a, par, k, r, j, s_t[j][tid], (r.heads >> j) & 1u);
                    if (lo < wk.g) st = wk.gap_at(a, cm, par, p, lo, wk.g, st);
                    st = m_at(m_from(cm[nibble(r.cls, j)]), st);
                }
                agg = m_const(st);
            }
            a.trec[(uint64_t)p * row + (uint64_t)tile * kPeThreads + tid] = m_to(agg);
            uint32_t c = __popc(r.heads);
            block_scan(agg, c, s_map, s_cnt);
            if (tid == 0) {
                Map16 t = m_identity();
                uint32_t tc = 0;
                for (int i = 0; i < kPeThreads / 64; ++i) {
                    t = m_compose(m_from(s_map[i]), t);
                    tc += s_cnt[i];
                }
                a.tile_agg[(uint64_t)tile * a.n_props + p] = m_to(t);
                if (p == 0) a.tile_heads[tile] = tc;
            }
            __syncthreads();             // s_map is reused by the next property
        }
        return;
    }
    for (uint32_t p = 0; p < a.n_props; ++p) {
        const PropDev& pd = a.plan->prop[p];
        const uint4* cm = s_cm[p];
        Map16 v = m_from(a.trec[(uint64_t)p * row + (uint64_t)tile * kPeThreads + tid]);
        uint32_t c = __popc(r.heads);
        block_scan(v, c, s_map, s_cnt);
        // exclusive prefix: tile prefix, earlier waves, earlier lanes
        Map16 pre = m_from(a.tile_prefix[(uint64_t)tile * a.n_props + p]);
        uint32_t id = a.tile_head_prefix[tile];
        for (int i = 0; i < w; ++i) {
            pre = m_compose(m_from(s_map[i]), pre);
            id += s_cnt[i];
        }
        const Map16 ex = m_shfl_up(v, 1);
        const uint32_t exc = __shfl_up(c, 1, 64);
        if (lane > 0) {
            pre = m_compose(ex, pre);
            id += exc;
        }
        __syncthreads();                 // s_map is reused by the next property
        const uint32_t lab0 = pd.blabel[0], lab1 = pd.blabel[1];
        uint32_t st = m_at(pre, pd.q0);  // state before this thread's first event
        // the instances ending in the tile have consecutive numbers, from
        // the one holding its first event (heads before the tile, minus one):
        // their verdicts are staged in LDS and written out contiguously
        const uint32_t inst0 = a.tile_head_prefix[tile] - 1u;
        uint32_t my_lo = 0xFFFFFFFFu, my_hi = 0;
        PeWalk wk = w0;
        for (uint32_t j = 0; j < r.cnt; ++j) {
            const bool head = (r.heads >> j) & 1u;
            const uint32_t lo = wk.step(a, par, k, r, j, s_t[j][tid], head);
            if (head) {
                st = pd.q0;
                ++id;
            }
            if (lo < wk.g) st = wk.gap_at(a, cm, par, p, lo, wk.g, st);
            st = m_at(m_from(cm[nibble(r.cls, j)]), st);
            if ((r.ends >> j) & 1u) {
                // the trailing gap: the parent's entries after the last own event
                uint32_t fin = st;
                if (wk.g < wk.re) fin = wk.gap_at(a, cm, par, p, wk.g, wk.re, fin);
                const uint32_t inst = id - 1u;
                s_iv[inst - inst0] = (uint8_t)((((fin & 8u) ? lab1 : lab0) >> (4 * (fin & 7u))) & 15u);
                my_lo = min(my_lo, inst);
                my_hi = max(my_hi, inst + 1u);
            }
        }
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
        for (int i = 1; i < kPeThreads / 64; ++i) {
            lo = min(lo, s_red[0][i]);
            hi = max(hi, s_red[1][i]);
        }
        if (lo < hi) {
            if ((uint64_t)hi > a.inst_limit) {
                if (tid == 0) atomicOr(a.err, kErrCapacity);
                hi = (uint32_t)min<uint64_t>(hi, a.inst_limit);
            }
            for (uint32_t i = lo + tid; i < hi; i += kPeThreads)
                a.inst_verdict[(uint64_t)p * a.inst_stride + i] = s_iv[i - inst0];
        }
        __syncthreads();                 // s_iv and s_red are reused by the next property
    }
}

// Exclusive prefixes of the tile aggregates in tile order: block p < n_props
// scans property p's maps, block n_props the head counts.  Each thread
// composes a contiguous chunk of tiles, a block scan joins the chunks, and
// the threads walk their chunks again to write the prefixes.
__global__ __launch_bounds__(kPeSpineThreads) void k_pe_spine(ParentArgs a) {
    __shared__ uint4 s_map[kPeSpineThreads / 64];
    __shared__ uint32_t s_cnt[kPeSpineThreads / 64];
    const uint32_t n_own = *a.n_own;
    const uint32_t tiles = (n_own + kPeTile - 1) / kPeTile;
    const uint32_t p = blockIdx.x;
    const bool counts = p == a.n_props;
    const uint32_t chunk = (tiles + kPeSpineThreads - 1) / kPeSpineThreads;
    const uint32_t t0 = threadIdx.x * chunk, t1 = min(tiles, t0 + chunk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    Map16 v = m_identity();
    uint32_t c = 0;
    for (uint32_t i = t0; i < t1; ++i) {
        if (counts) c += a.tile_heads[i];
        else v = m_compose(m_from(a.tile_agg[(uint64_t)i * a.n_props + p]), v);
    }
    block_scan(v, c, s_map, s_cnt);
    Map16 pre = m_identity();
    uint32_t cpre = 0;
    for (int i = 0; i < w; ++i) {
        pre = m_compose(m_from(s_map[i]), pre);
        cpre += s_cnt[i];
    }
    const Map16 ex = m_shfl_up(v, 1);
    const uint32_t exc = __shfl_up(c, 1, 64);
    if (lane > 0) {
        pre = m_compose(ex, pre);
        cpre += exc;
    }
    for (uint32_t i = t0; i < t1; ++i) {
        if (counts) {
            a.tile_head_prefix[i] = cpre;
            cpre += a.tile_heads[i];
        } else {
            const uint64_t at = (uint64_t)i * a.n_props + p;
            a.tile_prefix[at] = m_to(pre);
            pre = m_compose(m_from(a.tile_agg[at]), pre);
        }
    }
}

hipError_t launch_parent_counts(const ParentArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_pe_counts, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_parent_samples(const ParentArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_pe_samples, dim3(kPeSamples / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_parent_tree(const ParentArgs& a, uint32_t level0, uint32_t nlev, uint64_t max_nodes0,
                              hipStream_t s) {
    const uint64_t want = (max_nodes0 + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 1024 ? (want ? want : 1) : 1024);
    hipLaunchKernelGGL(k_pe_tree, dim3(blocks, a.n_props), dim3(256), 0, s, a, level0, nlev);
    return hipGetLastError();
}

hipError_t launch_parent_pass(const ParentArgs& a, bool down, uint64_t max_tiles, hipStream_t s) {
    const dim3 grid((uint32_t)(max_tiles ? max_tiles : 1));
    if (down) hipLaunchKernelGGL(k_pe_pass<true>, grid, dim3(kPeThreads), 0, s, a);
    else hipLaunchKernelGGL(k_pe_pass<false>, grid, dim3(kPeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_parent_spine(const ParentArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_pe_spine, dim3(a.n_props + 1), dim3(kPeSpineThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace ltl4c
