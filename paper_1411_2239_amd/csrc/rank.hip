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

// This thread's kRankItems sorted words (thread-blocked, 16-byte loads
// issued together; the word buffers are padded past the last tile), split into
// values and event indices, and the heads among them (a value different from
// the one before); returns the head mask.
__device__ __forceinline__ uint32_t rank_heads(const RankArgs& a, uint64_t my0, uint32_t cnt, uint32_t* vals,
                                               uint32_t* idx) {
    const uint64_t ld0 = cnt ? my0 : 0;
    const uint4* src = reinterpret_cast<const uint4*>(a.sorted + ld0);
#pragma unroll
    for (int q = 0; q < kRankItems / 2; ++q) {
        const uint4 v = src[q];
        idx[2 * q] = v.x;
        vals[2 * q] = v.y;
        idx[2 * q + 1] = v.z;
        vals[2 * q + 1] = v.w;
    }
    const uint32_t prev = (uint32_t)(a.sorted[ld0 ? ld0 - 1 : 0] >> 32);
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < kRankItems; ++j) {
        const uint32_t before = j ? vals[j - 1] : prev;
        const bool head = (uint32_t)j < cnt && (my0 + j == 0 || vals[j] != before);
        m |= (head ? 1u : 0u) << j;
    }
    return m;
}

// block-wide exclusive sum of one count per thread (thread order), and the total
template <int THREADS>
__device__ __forceinline__ uint32_t rank_block_excl(uint32_t c, uint32_t* total) {
    __shared__ uint32_t s_w[THREADS / 64];
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
    for (int i = 0; i < THREADS / 64; ++i) {
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
    uint32_t vals[kRankItems], idx[kRankItems];
    const uint32_t m = rank_heads(a, my0, cnt, vals, idx);
    uint32_t total;
    (void)rank_block_excl<kRankThreads>(__popc(m), &total);
    if (threadIdx.x == 0) a.tile_cnt[blockIdx.x] = total;
}

// Exclusive prefix of the tiles' head counts, and the number of distinct
// values: each thread sums a contiguous chunk of tiles, a block scan joins
// the chunks, and the threads walk their chunks again.
__global__ __launch_bounds__(kRankSpineThreads) void k_rank_spine(RankArgs a, uint32_t tiles) {
    const uint32_t chunk = (tiles + kRankSpineThreads - 1) / kRankSpineThreads;
    const uint32_t t0 = min(tiles, threadIdx.x * chunk), t1 = min(tiles, t0 + chunk);
    uint32_t c = 0;
    for (uint32_t t = t0; t < t1; ++t) c += a.tile_cnt[t];
    uint32_t total;
    uint32_t s = rank_block_excl<kRankSpineThreads>(c, &total);
    for (uint32_t t = t0; t < t1; ++t) {
        a.tile_off[t] = s;
        s += a.tile_cnt[t];
    }
    if (threadIdx.x == 0) *a.n_distinct = total;
}

__global__ __launch_bounds__(kRankThreads) void k_rank_apply(RankArgs a) {
    const uint64_t base = (uint64_t)blockIdx.x * kRankTile;
    const uint64_t my0 = base + (uint64_t)threadIdx.x * kRankItems;
    const uint32_t cnt = my0 < a.n ? (uint32_t)min<uint64_t>(kRankItems, a.n - my0) : 0u;
    uint32_t vals[kRankItems], idx[kRankItems];
    const uint32_t m = rank_heads(a, my0, cnt, vals, idx);
    uint32_t total;
    const uint32_t before = rank_block_excl<kRankThreads>(__popc(m), &total);
    uint32_t r = a.tile_off[blockIdx.x] + before;     // heads before this thread's run
#pragma unroll
    for (int j = 0; j < kRankItems; ++j) {
        if ((uint32_t)j >= cnt) continue;
        if ((m >> j) & 1u) {
            a.uniq[r] = vals[j];
            ++r;
        }
        a.rank[idx[j]] = r - 1u;
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
    hipLaunchKernelGGL(k_rank_spine, dim3(1), dim3(kRankSpineThreads), 0, s, a, tiles);
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
