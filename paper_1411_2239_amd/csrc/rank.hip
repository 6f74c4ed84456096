// Key ranking for composite keys wider than the sort word: the values of
// each quantifier level are replaced by their dense rank among the values of
// that level occurring in the trace.  Ranks keep order and equality, so the
// clusters (Eq. 5), the lexicographic order of value vectors and the tree of
// Section 2.4 are the same as with the raw values; only the bits shrink to
// ceil(log2(distinct values)) per level.
//
// Per level: (value << 32 | event index) words, LSD radix passes over the
// value bits (the library's radix pass), then a head count of the sorted
// values (reduce per tile, spine, down sweep) that gives every event its rank
// and every rank its value.
#include "internal.h"

namespace ltl4c {

__device__ __forceinline__ uint32_t rank_field(const RankArgs& a, uint64_t i) {
    const uint32_t* rec = reinterpret_cast<const uint32_t*>(a.records + i * a.record_bytes);
    const uint32_t t = (rec[a.type_dw] >> a.type_shift) & a.type_mask;
    // a type without this key (or beyond the table) contributes the value 0,
    // which at most adds one rank; such events never use theirs
    if (t > 255u || !((a.has_key[t >> 5] >> (t & 31u)) & 1u)) return 0u;
    return (rec[a.key_dw] >> a.key_shift) & a.key_mask;
}

// words[i] = value << 32 | i, and the histograms of the four 8-bit digits
__global__ __launch_bounds__(1024) void k_rank_prep(RankArgs a) {
    __shared__ uint32_t s_hist[4 * 256];
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = rank_field(a, i);
        a.words[i] = ((uint64_t)v << 32) | i;
#pragma unroll
        for (int p = 0; p < 4; ++p) atomicAdd(&s_hist[p * 256 + ((v >> (8 * p)) & 255u)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) {
        const uint32_t v = s_hist[i];
        if (v) atomicAdd(a.hist + i, v);
    }
}

// Heads of the sorted values (a value different from the one before) in
// thread-blocked runs of kRankItems; returns this thread's head mask.
__device__ __forceinline__ uint32_t rank_heads(const RankArgs& a, uint64_t my0, uint32_t cnt, uint32_t* vals) {
    uint32_t m = 0;
    uint32_t prev = my0 > 0 ? (uint32_t)(a.sorted[my0 - 1] >> 32) : 0u;
    for (uint32_t j = 0; j < cnt; ++j) {
        const uint32_t v = (uint32_t)(a.sorted[my0 + j] >> 32);
        vals[j] = v;
        if (my0 + j == 0 || v != prev) m |= 1u << j;
        prev = v;
    }
    return m;
}

// block-wide exclusive sum of one count per thread (thread order), and the total
__device__ __forceinline__ uint32_t rank_block_excl(uint32_t c, uint32_t* total) {
    __shared__ uint32_t s_w[kRankThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(x, off, 64);
        if (lane >= off) x += o;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int i = 0; i < kRankThreads / 64; ++i) {
        if (i < w) before += s_w[i];
        tot += s_w[i];
    }
    *total = tot;
    return before + x - c;
}

__global__ __launch_bounds__(kRankThreads) void k_rank_tiles(RankArgs a) {
    const uint64_t base = (uint64_t)blockIdx.x * kRankTile;
    const uint64_t my0 = base + (uint64_t)threadIdx.x * kRankItems;
    const uint32_t cnt = my0 < a.n ? (uint32_t)min<uint64_t>(kRankItems, a.n - my0) : 0u;
    uint32_t vals[kRankItems];
    const uint32_t m = cnt ? rank_heads(a, my0, cnt, vals) : 0u;
    uint32_t total;
    (void)rank_block_excl(__popc(m), &total);
    if (threadIdx.x == 0) a.tile_cnt[blockIdx.x] = total;
}

__global__ void k_rank_spine(RankArgs a, uint32_t tiles) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t s = 0;
    for (uint32_t t = 0; t < tiles; ++t) {
        a.tile_off[t] = s;
        s += a.tile_cnt[t];
    }
    *a.n_distinct = s;
}

__global__ __launch_bounds__(kRankThreads) void k_rank_apply(RankArgs a) {
    const uint64_t base = (uint64_t)blockIdx.x * kRankTile;
    const uint64_t my0 = base + (uint64_t)threadIdx.x * kRankItems;
    const uint32_t cnt = my0 < a.n ? (uint32_t)min<uint64_t>(kRankItems, a.n - my0) : 0u;
    uint32_t vals[kRankItems];
    const uint32_t m = cnt ? rank_heads(a, my0, cnt, vals) : 0u;
    uint32_t total;
    const uint32_t before = rank_block_excl(__popc(m), &total);
    uint32_t r = a.tile_off[blockIdx.x] + before;     // heads before this thread's run
    for (uint32_t j = 0; j < cnt; ++j) {
        if ((m >> j) & 1u) {
            a.uniq[r] = vals[j];
            ++r;
        }
        const uint32_t idx = (uint32_t)a.sorted[my0 + j];
        a.rank[idx] = r - 1u;
    }
}

// Values of the vectors of instances (n_levels values each) and of the
// nodes of one level (level values each), from their packed keys.
__global__ __launch_bounds__(256) void k_key_values(KeyValuesArgs a) {
    const uint32_t n = (uint32_t)min<uint64_t>(*a.n_dev, a.limit);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint64_t k = a.packed[i];
        for (uint32_t m = 0; m < a.n_fields; ++m) {
            const uint32_t r = (uint32_t)((k >> a.shift[m]) & a.mask[m]);
            a.out[(uint64_t)i * a.n_fields + m] = !a.uniq[m] ? r : r < a.uniq_cap ? a.uniq[m][r] : 0xFFFFFFFFu;
        }
    }
}

hipError_t launch_rank_prep(const RankArgs& a, hipStream_t s) {
    const uint64_t want = (a.n + 1023) / 1024;
    const uint32_t blocks = (uint32_t)(want < 512 ? (want ? want : 1) : 512);
    hipLaunchKernelGGL(k_rank_prep, dim3(blocks), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rank_scan(const RankArgs& a, hipStream_t s) {
    const uint32_t tiles = (uint32_t)((a.n + kRankTile - 1) / kRankTile);
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rank_tiles, dim3(tiles), dim3(kRankThreads), 0, s, a);
    hipLaunchKernelGGL(k_rank_spine, dim3(1), dim3(64), 0, s, a, tiles);
    hipLaunchKernelGGL(k_rank_apply, dim3(tiles), dim3(kRankThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_key_values(const KeyValuesArgs& a, uint64_t max_n, hipStream_t s) {
    const uint64_t want = (max_n + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 2048 ? (want ? want : 1) : 2048);
    hipLaunchKernelGGL(k_key_values, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ltl4c
