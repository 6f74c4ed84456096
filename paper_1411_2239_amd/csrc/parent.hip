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
//     (prefix, trace index), is found by binary search; an instance's own
//     events split its parent's run of P at G_i into gaps;
//   * the map of each gap is the composition of the class maps of its parent
//     events, taken from a segment tree over P (level L node q composes the
//     entries [q 2^L, (q+1) 2^L));
//   * own event i contributes F_i = [trailing gap at the instance end] o M_c
//     o [gap before it], a head contributes the constant map of F_i(q0); an
//     inclusive scan of the F_i (reduce per tile, sequential spine, down
//     sweep) gives the final state at every instance end.
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

__device__ __forceinline__ uint32_t m_at(const Map16& g, uint32_t q) {
    return (g.d[q >> 2] >> (8 * (q & 3u))) & 0xFFu;
}

__device__ __forceinline__ Map16 m_load(const uint4* p) {
    const uint4 v = *p;
    Map16 r;
    r.d[0] = v.x;
    r.d[1] = v.y;
    r.d[2] = v.z;
    r.d[3] = v.w;
    return r;
}

__device__ __forceinline__ void m_store(uint4* p, const Map16& m) { *p = make_uint4(m.d[0], m.d[1], m.d[2], m.d[3]); }

__device__ __forceinline__ Map16 m_class(const PropDev& pd, uint32_t c) {
    Map16 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r.d[i] = pd.bmap[c][i];
    return r;
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

// level L node q of the segment tree of property p (level 0: a class map)
__device__ __forceinline__ Map16 tree_node(const ParentArgs& a, const PropDev& pd, const uint64_t* par, uint32_t p,
                                           uint32_t L, uint32_t q) {
    if (L == 0) return m_class(pd, (uint32_t)par[q] & a.class_mask);
    return m_load(a.tree + a.tree_off[L] + (uint64_t)p * a.tree_cnt[L] + q);
}

// composition of the class maps of parent-array entries [l, r), in order
__device__ Map16 range_map(const ParentArgs& a, const PropDev& pd, const uint64_t* par, uint32_t p, uint32_t l,
                           uint32_t r) {
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

}  // namespace

// n_own = kept - parent events (both counted by classify)
__global__ void k_pe_counts(ParentArgs a) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *a.n_own = *a.n_kept - *a.n_par;
}

// Level L >= 1 of the segment tree, for property blockIdx.y.
__global__ __launch_bounds__(256) void k_pe_tree(ParentArgs a, uint32_t L) {
    const uint32_t p = blockIdx.y;
    const PropDev& pd = a.plan->prop[p];
    const uint32_t k = *a.n_par;
    const uint64_t* par = a.words + *a.n_own;
    const uint32_t cnt = (uint32_t)((k + (1ull << L) - 1) >> L);
    const uint32_t half = 1u << (L - 1);
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
        const Map16 lo = tree_node(a, pd, par, p, L - 1, 2 * q);
        Map16 r = lo;
        if ((uint64_t)(2 * q + 1) * half < k) r = m_compose(tree_node(a, pd, par, p, L - 1, 2 * q + 1), lo);
        m_store(a.tree + a.tree_off[L] + (uint64_t)p * a.tree_cnt[L] + q, r);
    }
}

// The map F_i of own event i (see the file header) and its head flag.
__device__ __forceinline__ Map16 event_map(const ParentArgs& a, const PropDev& pd, const uint64_t* par, uint32_t k,
                                           uint32_t p, uint32_t n_own, uint32_t i, uint64_t x, uint32_t g_prev_in,
                                           bool have_prev, uint32_t* g_out, bool* head_out) {
    const uint64_t key = x >> a.key_shift;
    const bool head = i == 0 || (a.words[i - 1] >> a.key_shift) != key;
    const bool end = i + 1 == n_own || (a.words[i + 1] >> a.key_shift) != key;
    const uint64_t prefix = (x >> a.prefix_shift) & a.prefix_mask;
    const uint32_t gi = a.g_in ? a.g_in[i] : lower_bound(a, par, k, search_key(a, x));
    uint32_t gp;
    if (head) gp = lower_bound(a, par, k, prefix << a.ibits);
    else if (have_prev) gp = g_prev_in;
    else gp = a.g_in ? a.g_in[i - 1] : lower_bound(a, par, k, search_key(a, a.words[i - 1]));
    Map16 f = m_compose(m_class(pd, (uint32_t)x & a.class_mask), range_map(a, pd, par, p, gp, gi));
    if (end) f = m_compose(range_map(a, pd, par, p, gi, lower_bound(a, par, k, (prefix + 1) << a.ibits)), f);
    if (head) f = m_const(m_at(f, pd.q0));
    *g_out = gi;
    *head_out = head;
    return f;
}

// DOWN = false: per tile and property, the composition of the tile's F_i and
// its head count (and G_i into g_out).  DOWN = true: the states at the
// instance ends, from the spine's tile prefixes; verdicts written by id.
template <bool DOWN>
__global__ __launch_bounds__(kPeThreads) void k_pe_pass(ParentArgs a) {
    __shared__ uint32_t s_wmap[kPeThreads / 64][4];
    __shared__ uint32_t s_wcnt[kPeThreads / 64];
    const uint32_t p = blockIdx.y;
    const PropDev& pd = a.plan->prop[p];
    const uint32_t n_own = *a.n_own, k = *a.n_par;
    const uint64_t* par = a.words + n_own;
    const uint32_t tile = blockIdx.x;
    const uint64_t base = (uint64_t)tile * kPeTile;
    if (base >= n_own) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t my0 = base + (uint64_t)tid * kPeItems;
    const uint32_t cnt = my0 < n_own ? (uint32_t)min<uint64_t>(kPeItems, n_own - my0) : 0u;
    // this thread's run: its composed map and head count
    Map16 agg = m_identity();
    uint32_t heads = 0, gprev = 0;
    for (uint32_t j = 0; j < cnt; ++j) {
        const uint32_t i = (uint32_t)(my0 + j);
        uint32_t gi;
        bool hd;
        const Map16 f = event_map(a, pd, par, k, p, n_own, i, a.words[i], gprev, j > 0, &gi, &hd);
        if (!DOWN && p == 0 && a.g_out) a.g_out[i] = gi;
        gprev = gi;
        heads += hd ? 1u : 0u;
        agg = m_compose(f, agg);
    }
    // block-wide exclusive scan of the runs (thread order = event order)
    Map16 v = agg;
    uint32_t c = heads;
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
#pragma unroll
        for (int i = 0; i < 4; ++i) s_wmap[w][i] = v.d[i];
        s_wcnt[w] = c;
    }
    __syncthreads();
    if (!DOWN) {
        if (tid == 0) {
            Map16 t = m_identity();
            uint32_t tc = 0;
            for (int i = 0; i < kPeThreads / 64; ++i) {
                Map16 wm;
#pragma unroll
                for (int d = 0; d < 4; ++d) wm.d[d] = s_wmap[i][d];
                t = m_compose(wm, t);
                tc += s_wcnt[i];
            }
            m_store(a.tile_agg + (uint64_t)tile * a.n_props + p, t);
            if (p == 0) a.tile_heads[tile] = tc;
        }
        return;
    }
    // exclusive prefix of this thread: tile prefix, earlier waves, earlier lanes
    Map16 pre = m_load(a.tile_prefix + (uint64_t)tile * a.n_props + p);
    uint32_t id_base = a.tile_head_prefix[tile];
    for (int i = 0; i < w; ++i) {
        Map16 wm;
#pragma unroll
        for (int d = 0; d < 4; ++d) wm.d[d] = s_wmap[i][d];
        pre = m_compose(wm, pre);
        id_base += s_wcnt[i];
    }
    const Map16 ex = m_shfl_up(v, 1);
    const uint32_t exc = __shfl_up(c, 1, 64);
    if (lane > 0) {
        pre = m_compose(ex, pre);
        id_base += exc;
    }
    uint32_t st = m_at(pre, pd.q0);      // state before this thread's first event
    uint32_t id = id_base;               // heads before it
    gprev = 0;
    for (uint32_t j = 0; j < cnt; ++j) {
        const uint32_t i = (uint32_t)(my0 + j);
        const uint64_t x = a.words[i];
        uint32_t gi;
        bool hd;
        const Map16 f = event_map(a, pd, par, k, p, n_own, i, x, gprev, j > 0, &gi, &hd);
        gprev = gi;
        if (hd) ++id;
        st = m_at(f, st);
        const bool end = i + 1 == n_own || (a.words[i + 1] >> a.key_shift) != (x >> a.key_shift);
        if (end) {
            const uint64_t inst = (uint64_t)id - 1u;
            if (inst < a.inst_limit) {
                const uint8_t lab = pd.label[st & 15u];
                a.inst_verdict[(uint64_t)p * a.inst_stride + inst] = lab;
            } else {
                atomicOr(a.err, kErrCapacity);
            }
        }
    }
}

// Exclusive prefixes of the tile aggregates, one thread per property (and the
// head counts on thread n_props), in tile order.
__global__ void k_pe_spine(ParentArgs a) {
    const uint32_t n_own = *a.n_own;
    const uint32_t tiles = (n_own + kPeTile - 1) / kPeTile;
    const uint32_t t = threadIdx.x;
    if (t < a.n_props) {
        Map16 pre = m_identity();
        for (uint32_t i = 0; i < tiles; ++i) {
            m_store(a.tile_prefix + (uint64_t)i * a.n_props + t, pre);
            pre = m_compose(m_load(a.tile_agg + (uint64_t)i * a.n_props + t), pre);
        }
    } else if (t == a.n_props) {
        uint32_t s = 0;
        for (uint32_t i = 0; i < tiles; ++i) {
            a.tile_head_prefix[i] = s;
            s += a.tile_heads[i];
        }
    }
}

hipError_t launch_parent_counts(const ParentArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_pe_counts, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_parent_tree(const ParentArgs& a, uint32_t level, uint64_t max_nodes, hipStream_t s) {
    const uint64_t want = (max_nodes + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 1024 ? (want ? want : 1) : 1024);
    hipLaunchKernelGGL(k_pe_tree, dim3(blocks, a.n_props), dim3(256), 0, s, a, level);
    return hipGetLastError();
}

hipError_t launch_parent_pass(const ParentArgs& a, bool down, uint64_t max_tiles, hipStream_t s) {
    const dim3 grid((uint32_t)(max_tiles ? max_tiles : 1), a.n_props);
    if (down) hipLaunchKernelGGL(k_pe_pass<true>, grid, dim3(kPeThreads), 0, s, a);
    else hipLaunchKernelGGL(k_pe_pass<false>, grid, dim3(kPeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_parent_spine(const ParentArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_pe_spine, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace ltl4c
