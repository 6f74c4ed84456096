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
        const uint32_t sel = f.d[i], s7 = sel & 0x07070707u;
        const uint32_t lo = __builtin_amdgcn_perm(g.d[1], g.d[0], s7);
        const uint32_t hi = __builtin_amdgcn_perm(g.d[3], g.d[2], s7);
        const uint32_t t = (sel >> 3) & 0x01010101u, m = (t << 8) - t;
        r.d[i] = (hi & m) | (lo & ~m);
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

__device__ __forceinline__ Map16 m_class(const PropDev& pd, uint32_t c) {
    Map16 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = pd.bmap[c][i];
    return r;
}

// delta(q, c) of a class map, for one state
__device__ __forceinline__ uint32_t class_at(const PropDev& pd, uint32_t c, uint32_t q) {
    return (pd.bmap[c][q >> 2] >> (8 * (q & 3u))) & 0xFFu;
}

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

// number of parent-array entries whose search key is below `target`
__device__ __forceinline__ uint32_t lower_bound(const ParentArgs& a, const uint64_t* par, uint32_t k, uint64_t target) {
    uint32_t lo = 0, hi = k;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (search_key(a, par[mid]) < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
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

// level L node q of the segment tree of property p (level 0: a class map)
__device__ __forceinline__ Map16 tree_node(const ParentArgs& a, const PropDev& pd, const uint64_t* par, uint32_t p,
                                           uint32_t L, uint64_t q) {
    if (L == 0) return m_class(pd, (uint32_t)par[q] & a.class_mask);
    return m_from(a.tree[a.tree_off[L] + (uint64_t)p * a.tree_cnt[L] + q]);
}

// composition of the class maps of parent-array entries [l, r), in order
__device__ __forceinline__ Map16 range_map(const ParentArgs& a, const PropDev& pd, const uint64_t* par, uint32_t p,
                                        uint32_t l, uint32_t r) {
    Map16 left = m_identity(), right = m_identity();
    uint32_t L = 0;
    while (l < r) {
        if (l & 1u) {
            left = m_compose(tree_node(a, pd, par, p, L, l), left);
            ++l;
        }
        if (r & 1u) {
            --r;
            right = m_compose(right, tree_node(a, pd, par, p, L, r));
        }
        l >>= 1;
        r >>= 1;
        ++L;
    }
    return m_compose(right, left);
}

// One thread's run of own events, staged in LDS (row j + 1 of column tid is
// its event j, row 0 the word before the run, row kPeItems + 1 the word
// after it), with its head and end flags and the start of its gap search:
// the parent's run start `rs` of the first event's prefix (a binary search)
// and `g`, the bound G of the event before the run when it belongs to the
// same instance.
struct PeRun {
    uint32_t cnt;
    uint32_t heads, ends;                // bit j
    uint64_t pf;                         // prefix of the first event
    uint32_t rs, g;
};

__device__ __forceinline__ void load_run(const ParentArgs& a, uint32_t n_own, uint32_t k, const uint64_t* par,
                                         uint64_t my0, uint64_t (*s_w)[kPeThreads], PeRun& r) {
    const int tid = threadIdx.x;
    r.cnt = my0 < n_own ? (uint32_t)min<uint64_t>(kPeItems, n_own - my0) : 0u;
    // unconditional loads (the word buffers are padded past the last tile)
    const uint64_t ld0 = r.cnt ? my0 : 0;
    uint64_t w[kPeItems];
    const uint4* src = reinterpret_cast<const uint4*>(a.words + ld0);
#pragma unroll
    for (int q = 0; q < kPeItems / 2; ++q) {
        const uint4 v = src[q];
        w[2 * q] = (uint64_t)v.x | ((uint64_t)v.y << 32);
        w[2 * q + 1] = (uint64_t)v.z | ((uint64_t)v.w << 32);
    }
    const uint64_t wprev = a.words[ld0 ? ld0 - 1 : 0];
    const uint64_t wnext = a.words[ld0 + kPeItems];
    r.heads = r.ends = 0;
#pragma unroll
    for (int j = 0; j < kPeItems; ++j) {
        const uint64_t key = w[j] >> a.key_shift;
        const uint64_t kp = (j ? w[j - 1] : wprev) >> a.key_shift;
        const uint64_t kn = (j + 1 < kPeItems ? w[j + 1] : wnext) >> a.key_shift;
        const bool valid = (uint32_t)j < r.cnt;
        const bool head = valid && (my0 + j == 0 || kp != key);
        const bool end = valid && (my0 + j + 1 == n_own || kn != key);
        r.heads |= (head ? 1u : 0u) << j;
        r.ends |= (end ? 1u : 0u) << j;
        s_w[j + 1][tid] = w[j];
    }
    s_w[0][tid] = wprev;
    s_w[kPeItems + 1][tid] = wnext;
    r.pf = prefix_of(a, w[0]);
    r.rs = r.cnt ? lower_bound(a, par, k, r.pf << a.ibits) : 0u;
    r.g = (r.cnt && !(r.heads & 1u)) ? gallop(a, par, k, r.rs, search_key(a, wprev)) : r.rs;
}

// The walk over a run: for each own event, its word, flags and the gap
// [lo, g) of parent entries before it; the run starts and bounds move
// forward by galloping.
struct PeWalk {
    uint64_t pf;
    uint32_t rs, g;
    __device__ __forceinline__ explicit PeWalk(const PeRun& r) : pf(r.pf), rs(r.rs), g(r.g) {}
    // returns lo; g becomes G of the event
    __device__ __forceinline__ uint32_t step(const ParentArgs& a, const uint64_t* par, uint32_t k, uint64_t x,
                                             bool head) {
        if (head) {
            const uint64_t pj = prefix_of(a, x);
            if (pj != pf) {
                rs = gallop(a, par, k, rs, pj << a.ibits);
                pf = pj;
            }
            g = rs;
        }
        const uint32_t lo = g;
        g = gallop(a, par, k, g, search_key(a, x));
        return lo;
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

// Levels L0+1 .. L0+nlev of the segment tree of property blockIdx.y, from
// level L0: each block takes 256 level-L0 nodes and halves them in LDS.  A
// missing right child counts as the identity.
__global__ __launch_bounds__(256) void k_pe_tree(ParentArgs a, uint32_t L0, uint32_t nlev) {
    __shared__ uint4 s[256];
    const uint32_t p = blockIdx.y;
    const PropDev& pd = a.plan->prop[p];
    const uint32_t k = *a.n_par;
    const uint64_t* par = a.words + *a.n_own;
    const uint64_t cnt0 = ((uint64_t)k + (1ull << L0) - 1) >> L0;
    const uint32_t t = threadIdx.x;
    for (uint64_t b = blockIdx.x; b * 256 < cnt0; b += gridDim.x) {
        const uint64_t q = b * 256 + t;
        Map16 m = q < cnt0 ? tree_node(a, pd, par, p, L0, q) : m_identity();
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
    __shared__ uint64_t s_w[kPeItems + 2][kPeThreads];
    __shared__ uint4 s_map[kPeThreads / 64];
    __shared__ uint32_t s_cnt[kPeThreads / 64];
    const uint32_t n_own = *a.n_own, k = *a.n_par;
    const uint64_t* par = a.words + n_own;
    const uint32_t tile = blockIdx.x;
    const uint64_t base = (uint64_t)tile * kPeTile;
    if (base >= n_own) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    PeRun r;
    load_run(a, n_own, k, par, base + (uint64_t)tid * kPeItems, s_w, r);
    const uint64_t row = (uint64_t)gridDim.x * kPeThreads;
    if (!DOWN) {
        for (uint32_t p = 0; p < a.n_props; ++p) {
            const PropDev& pd = a.plan->prop[p];
            Map16 agg = m_identity();
            PeWalk wk(r);
            for (uint32_t j = 0; j < r.cnt; ++j) {
                const uint64_t x = s_w[j + 1][tid];
                const bool head = (r.heads >> j) & 1u;
                const uint32_t lo = wk.step(a, par, k, x, head);
                Map16 f = m_class(pd, (uint32_t)x & a.class_mask);
                if (lo < wk.g) f = m_compose(f, range_map(a, pd, par, p, lo, wk.g));
                if (head) f = m_const(m_at(f, pd.q0));
                agg = m_compose(f, agg);
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
        uint32_t st = m_at(pre, pd.q0);  // state before this thread's first event
        PeWalk wk(r);
        for (uint32_t j = 0; j < r.cnt; ++j) {
            const uint64_t x = s_w[j + 1][tid];
            const bool head = (r.heads >> j) & 1u;
            const uint32_t lo = wk.step(a, par, k, x, head);
            if (head) {
                st = pd.q0;
                ++id;
            }
            if (lo < wk.g) st = m_at(range_map(a, pd, par, p, lo, wk.g), st);
            st = class_at(pd, (uint32_t)x & a.class_mask, st);
            if ((r.ends >> j) & 1u) {
                // the trailing gap: the parent's entries after the last own event
                const uint32_t hi = gallop(a, par, k, wk.g, (prefix_of(a, x) + 1) << a.ibits);
                uint32_t fin = st;
                if (wk.g < hi) fin = m_at(range_map(a, pd, par, p, wk.g, hi), fin);
                const uint64_t inst = (uint64_t)id - 1u;
                if (inst < a.inst_limit) a.inst_verdict[(uint64_t)p * a.inst_stride + inst] = pd.label[fin & 15u];
                else atomicOr(a.err, kErrCapacity);
            }
        }
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
