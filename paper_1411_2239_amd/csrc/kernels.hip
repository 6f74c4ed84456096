// HIP kernels of the LTL4-C hot path for gfx950 (CDNA4, wave64).
//
//   k_classify   valuation extraction epsilon(u_i, K) (Section 4.1, the map
//                step of SortTrace in Algorithm 1): record -> letter (event
//                class) and packed binding key; builds the radix histograms
//                of every sort pass in the same read.
//   k_sort_pass  one stable LSD radix pass (ParallelSort of Algorithm 1) on
//                8- or 9-bit digits: single-pass "onesweep" ranking with wave
//                ballots, LDS-staged scatter and decoupled look-back across
//                tiles; the first pass may drop events that join no cluster.
//   k_scan       Distribute / ProcessBuffer of Algorithm 1 as a flat scan:
//                composes byte-packed transition maps (a segment head is the
//                constant map to delta(q0, c)), so each instance's final
//                state lambda(delta(q0, u^D)) (Def. 6) is found without one
//                thread per monitor; also the compaction (ParallelCompact)
//                into instance and node numbering.
//   k_count_leaves, k_count
//                ApplyQuantifiers of Algorithm 1 for one level: the 6-bin
//                count vector v of every quantifier submonitor (Def. 8) from
//                its children's verdicts (Def. 7 at every child node); at the
//                root the last block also runs Def. 7 at the root.
//   k_finalize   Def. 7 at the root of a one-level tree.
#include "internal.h"
#include "maps.h"

namespace ltl4c {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ld_acquire_flag(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) { return wave_incl_sum(v); }

// Exclusive scan of one value per thread over threads 0..255 of the block
// (every thread of the block must call it; threads >= 256 get garbage).
__device__ __forceinline__ uint32_t block256_excl_scan(uint32_t v, uint32_t* s_tmp /*[4]*/, uint32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t incl = wave_incl_scan_u32(v);
    if (lane == 63 && w < 4) s_tmp[w] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (int i = 0; i < w && i < 4; ++i) pre += s_tmp[i];
    *total = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
    __syncthreads();
    return pre + incl - v;
}

// Exclusive scans of two values over the threads of waves 0..NB-1 in one
// pass (later waves contribute zeros).  One barrier: s_tmp[0..NB) then holds
// the wave totals of v0 and s_tmp[NB..2NB) those of v1, and the caller must
// not write s_tmp again before its next barrier.
template <int NB>
__device__ __forceinline__ uint2 block_excl_scan2(uint32_t v0, uint32_t v1, uint32_t* s_tmp /*[2 NB]*/) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t i0 = wave_incl_scan_u32(v0), i1 = wave_incl_scan_u32(v1);
    if (lane == 63 && w < NB) {
        s_tmp[w] = i0;
        s_tmp[NB + w] = i1;
    }
    __syncthreads();
    uint32_t p0 = 0, p1 = 0;
    for (int i = 0; i < w && i < NB; ++i) {
        p0 += s_tmp[i];
        p1 += s_tmp[NB + i];
    }
    return make_uint2(p0 + i0 - v0, p1 + i1 - v1);
}

// Eq. 6 and Def. 7 (device restatement; exact integers).
__device__ __forceinline__ bool cmp_op(uint64_t a, uint32_t op, uint64_t b) {
    switch (op) {
        case 0: return a < b;
        case 1: return a <= b;
        case 2: return a > b;
        case 3: return a >= b;
        default: return a == b;
    }
}

__device__ __forceinline__ bool constraint_S(uint32_t kind, uint32_t op, uint32_t num, uint32_t den,
                                             uint64_t k, uint64_t n) {
    if (kind == 0) return cmp_op(k * (uint64_t)den, op, (uint64_t)num * n);   // percentage
    return cmp_op(k, op, (uint64_t)num);                                       // instance count
}

// Table 1 and the rule for A=1, extended to every operator: can no
// extension move the count of T children out of the constraint?
__device__ __forceinline__ bool forever_sat(uint32_t kind, uint32_t op, uint32_t num, uint32_t den,
                                            uint64_t top, uint64_t bot) {
    if (kind == 1) return (op == 2 && top > num) || (op == 3 && top >= num);
    const bool zero = num == 0, one = num == den;
    switch (op) {
        case 3: return zero;
        case 2: return zero && top >= 1;
        case 1: return one;
        case 0: return one && bot >= 1;
        default: return false;
    }
}

// Can no extension bring the count of non-F children into the constraint?
__device__ __forceinline__ bool forever_viol(uint32_t kind, uint32_t op, uint32_t num, uint32_t den,
                                             uint64_t top, uint64_t bot) {
    if (kind == 1) return ((op == 4 || op == 1) && top > num) || (op == 0 && top >= num);
    const bool zero = num == 0, one = num == den;
    switch (op) {
        case 3: return one && bot >= 1;
        case 2: return one;
        case 1: return zero && top >= 1;
        case 0: return zero;
        default: return (one && bot >= 1) || (zero && top >= 1);
    }
}

// Def. 7: the highest truth value whose condition holds.
__device__ __forceinline__ uint32_t valuate(const PropDev& P, int m, const uint32_t* v) {
    const uint32_t kind = P.kind[m], op = P.op[m], num = P.num[m], den = P.den[m];
    const uint64_t n = (uint64_t)v[0] + v[1] + v[2] + v[3] + v[4] + v[5];
    const uint64_t t = v[5];                 // {T}
    const uint64_t tc = t + v[4];            // {T, Tc}
    const uint64_t tp = tc + v[3];           // {T, Tc, Tp}
    const uint64_t nf2 = tp + v[2];          // B6 - {F, Fc}
    const uint64_t nf1 = nf2 + v[1];         // B6 - {F}
    if (constraint_S(kind, op, num, den, t, n) && forever_sat(kind, op, num, den, t, v[0])) return 5;
    if (constraint_S(kind, op, num, den, tc, n)) return 4;
    if (constraint_S(kind, op, num, den, tp, n)) return 3;
    if (constraint_S(kind, op, num, den, nf2, n)) return 2;
    if (!constraint_S(kind, op, num, den, nf1, n) && forever_viol(kind, op, num, den, t, v[0])) return 0;
    return 1;
}

// ---------------------------------------------------------------------------
// zero fill (look-back flags, histograms, counters; counts of a level)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zero(ZeroArgs a) {
    const uint64_t n = a.n_dev ? min<uint64_t>(*a.n_dev, a.limit) * a.mult : a.n_words;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // 16-byte stores over the aligned part, then the last words one by one
    const uint64_t head = (reinterpret_cast<uintptr_t>(a.ptr) & 15) == 0 ? n / 4 : 0;
    uint4* p4 = reinterpret_cast<uint4*>(a.ptr);
    for (uint64_t i = t0; i < head; i += stride) p4[i] = make_uint4(0u, 0u, 0u, 0u);
    for (uint64_t i = head * 4 + t0; i < n; i += stride) a.ptr[i] = 0u;
}

// ---------------------------------------------------------------------------
// classify: record -> (binding key, class) word + radix histograms
// ---------------------------------------------------------------------------
template <int RDW>
__device__ __forceinline__ void load_record(const uint8_t* rec, uint32_t* dw) {
    if constexpr (RDW == 4) {
        uint4 r = *reinterpret_cast<const uint4*>(rec);
        dw[0] = r.x; dw[1] = r.y; dw[2] = r.z; dw[3] = r.w;
    } else if constexpr (RDW == 3) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(rec);
        dw[0] = p[0]; dw[1] = p[1]; dw[2] = p[2];
    }
}

// A data predicate: an unsigned comparison of a record field with a constant.
__device__ __forceinline__ bool pred_holds(uint32_t op, uint32_t x, uint32_t v) {
    switch (op) {
        case 0: return x < v;
        case 1: return x <= v;
        case 2: return x > v;
        case 3: return x >= v;
        case 4: return x == v;
        default: return x != v;
    }
}

// NK: the number of key levels when fixed at compile time (0: a.n_keys)
template <int RDW, bool GROUP, bool PRED, int NK>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_classify(ClassifyArgs a) {
    __shared__ uint8_t s_cls[256];
    __shared__ uint8_t s_kp[256];
    __shared__ uint32_t s_hist[kHistWords];     // [n_pass][1 << digit_bits]
    __shared__ uint32_t s_nvalid;
    __shared__ uint32_t s_coff[GROUP ? kMaxChunks + 1 : 1];
    __shared__ uint32_t s_cstream[GROUP ? kMaxChunks : 1];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) {
        s_cls[i] = a.plan->class_of_type[i];
        s_kp[i] = a.plan->key_present[i];
    }
    const uint32_t n_hist = a.n_pass << a.digit_bits, dmask = (1u << a.digit_bits) - 1u;
    for (uint32_t i = threadIdx.x; i < n_hist; i += blockDim.x) s_hist[i] = 0;
    if (threadIdx.x == 0) s_nvalid = 0;
    if constexpr (GROUP) {
        for (uint32_t i = threadIdx.x; i <= a.n_chunks; i += blockDim.x) s_coff[i] = a.chunk_off[i];
        for (uint32_t i = threadIdx.x; i < a.n_chunks; i += blockDim.x) s_cstream[i] = a.chunk_stream[i];
    }
    __syncthreads();
    uint32_t err = 0, kept = 0, npar = 0;
    const int nk = NK ? NK : (int)a.n_keys;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // Records of one grid-stride step are loaded before any is processed, so
    // that each thread keeps U loads in flight.
    constexpr int U = RDW > 0 ? 4 : 1;
    constexpr int NDW = RDW > 0 ? RDW : 1;
    auto process = [&](uint64_t i, uint32_t t, const uint32_t* f, uint32_t pm, uint32_t chunk) {
        bool ok = !(a.check_type_range && t > 255u);
        const uint32_t t8 = t & 255u;
        const uint32_t kpm = s_kp[t8] & a.need_mask;
        // a parent event: every key but the innermost, which it takes as 0
        const bool par = ok && kpm == a.parent_mask;
        ok = ok && (kpm == a.need_mask || par);
        uint64_t key = 0;
        uint32_t over = 0;
#pragma unroll
        for (int m = 0; m < kMaxLevels; ++m) {
            if (m < nk) {
                const uint32_t b = a.key_bits[m];
                const uint32_t v = par && m + 1 == nk ? 0u : a.rank[m] ? a.rank[m][i] : f[m];
                over |= b < 32 ? (v >> b) : 0u;
                key = (key << b) | v;
            }
        }
        if (ok && over) err |= kErrRange;
        if (par) {
            key |= 1ull << a.stream_shift;
            ++npar;
        }
        if constexpr (GROUP) key |= (uint64_t)s_cstream[chunk] << a.stream_shift;
        // [key][trace index, when asked for][class]
        const uint64_t word = ok ? ((key << (a.cbits + a.ibits)) | (a.ibits ? i << a.cbits : 0ull) |
                                    (s_cls[t8] + (pm << a.pred_class_shift)))
                                 : (1ull << a.excl_shift);
        a.words[i] = word;
        // with n_valid set the first radix pass drops excluded events, so
        // they enter no histogram
        if (ok || !a.n_valid) {
            kept += ok;
            for (uint32_t p = 0; p < a.n_pass; ++p)
                atomicAdd(&s_hist[(p << a.digit_bits) + ((uint32_t)(word >> (a.sort_shift + a.digit_bits * p)) & dmask)], 1u);
        }
    };
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < a.n; i0 += U * stride) {
        uint32_t dw[U][NDW];
        uint32_t chunk[U];
        const uint8_t* rec_ptr[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + u * stride;
            chunk[u] = 0;
            rec_ptr[u] = a.records + i * a.record_bytes;
            if (i >= a.n) continue;
            if constexpr (GROUP) {
                // chunk c with s_coff[c] <= i < s_coff[c+1]
                uint32_t lo = 0, hi = a.n_chunks;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_coff[mid] <= (uint32_t)i) lo = mid; else hi = mid;
                }
                chunk[u] = lo;
                if (a.chunk_ptr)
                    rec_ptr[u] = reinterpret_cast<const uint8_t*>(a.chunk_ptr[lo]) + (i - s_coff[lo]) * a.record_bytes;
            }
            if constexpr (RDW > 0) load_record<RDW>(rec_ptr[u], dw[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + u * stride;
            if (i >= a.n) continue;
            uint32_t t, f[kMaxLevels], pm = 0;
            if constexpr (RDW > 0) {
                t = (dw[u][a.type_dw] >> a.type_shift) & a.type_mask;
#pragma unroll
                for (int m = 0; m < kMaxLevels; ++m)
                    f[m] = m < nk ? (dw[u][a.key_dw[m]] >> a.key_shift[m]) & a.key_mask[m] : 0u;
                if (PRED) {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        if (q < (int)a.n_preds)
                            pm |= (uint32_t)pred_holds(a.pred_op[q], (dw[u][a.pred_dw[q]] >> a.pred_shift[q]) & a.pred_mask[q],
                                                       a.pred_val[q]) << q;
                }
            } else {
                const uint32_t* rec = reinterpret_cast<const uint32_t*>(rec_ptr[u]);
                t = (rec[a.type_dw] >> a.type_shift) & a.type_mask;
#pragma unroll
                for (int m = 0; m < kMaxLevels; ++m)
                    f[m] = m < nk ? (rec[a.key_dw[m]] >> a.key_shift[m]) & a.key_mask[m] : 0u;
                if (PRED) {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        if (q < (int)a.n_preds)
                            pm |= (uint32_t)pred_holds(a.pred_op[q], (rec[a.pred_dw[q]] >> a.pred_shift[q]) & a.pred_mask[q],
                                                       a.pred_val[q]) << q;
                }
            }
            process(i, t, f, pm, chunk[u]);
        }
    }
    if (err) atomicOr(a.err, err);
    if (a.n_par) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) npar += __shfl_xor(npar, off, 64);
        if ((threadIdx.x & 63) == 0 && npar) atomicAdd(a.n_par, npar);
    }
    if (a.n_valid) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) kept += __shfl_xor(kept, off, 64);
        if ((threadIdx.x & 63) == 0 && kept) atomicAdd(&s_nvalid, kept);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n_hist; i += blockDim.x) {
        const uint32_t v = s_hist[i];
        if (v) atomicAdd(a.hist + i, v);
    }
    if (a.n_valid && threadIdx.x == 0 && s_nvalid) atomicAdd(a.n_valid, s_nvalid);
}

// ---------------------------------------------------------------------------
// one stable radix pass (onesweep: rank in-tile, look back across tiles)
// ---------------------------------------------------------------------------
constexpr uint32_t kFlagAgg = 1u << 30, kFlagInc = 2u << 30, kValMask = (1u << 30) - 1;
constexpr int kSortLookWindow = 4;
constexpr bool kSortSpinSleep = true;    // back off while a predecessor has not published

// 16-item tiles are held to 128 VGPRs (two 512-thread blocks per CU), 8-item
// tiles to 80 (three).  Tiles above 8192 words are written out in PHASES
// parts through an LDS buffer of CHUNK words.  RB is the digit width of the
// kernel (8: 256 buckets, 9: 512); one thread owns each bucket.
template <int THREADS, int ITEMS, int RB>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(ITEMS <= 8 ? 6 : ITEMS <= 12 ? 5 : ITEMS <= 16 ? 4 : 2)))
void k_sort_pass(SortPassArgs a) {
    constexpr int B = 1 << RB;
    constexpr int NB = B / 64;                 // waves whose threads own a bucket
    constexpr int TILE = THREADS * ITEMS;
    constexpr int WAVES = THREADS / 64;
    constexpr int PHASES = TILE <= 16384 ? 1 : (TILE + 8191) / 8192;
    constexpr int CHUNK = TILE / PHASES;
    // 512 buckets: the per-wave counters and the key buffer share LDS (keys
    // are placed once every position is known), which keeps two 512 x 16
    // blocks on a CU
    constexpr bool kShare = RB > 8;
    constexpr int CNT64 = WAVES * B / 2;       // per-wave counters, in 64-bit words
    static_assert(THREADS >= B, "one thread per bucket");
    static_assert(CHUNK * PHASES == TILE, "phases split the tile evenly");
    static_assert(!kShare || PHASES == 1, "shared counters need the whole tile in LDS");
    __shared__ uint64_t s_buf[kShare ? (CHUNK > CNT64 ? CHUNK : CNT64) : CHUNK + CNT64];
    uint64_t* s_keys = s_buf;
    uint32_t* s_wcnt = reinterpret_cast<uint32_t*>(s_buf + (kShare ? 0 : CHUNK));   // [WAVES][B]
    __shared__ uint32_t s_gbase[B];
    __shared__ uint32_t s_tmp[2 * NB];
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(a.ticket, 1u);
    for (int i = tid; i < WAVES * B; i += THREADS) s_wcnt[i] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = (uint64_t)tile * TILE;
    // words read and written: the first pass of a dropping sort reads all n
    // and keeps n_valid; the later passes read and write n_valid
    const uint32_t n_out = a.n_valid ? *a.n_valid : a.n;
    const uint32_t n_in = a.drop_excl ? a.n : n_out;
    if (base >= n_in) return;                  // the whole block: no word of this tile
    const uint64_t wbase = base + (uint64_t)w * (ITEMS * 64) + lane;   // item r of this lane: wbase + 64 r
    // items r with 64 r < rem are inside the array
    const uint32_t rem = wbase < n_in ? (uint32_t)min<uint64_t>(n_in - wbase, ITEMS * 64) : 0u;
    const uint32_t dmask = (1u << a.nbits) - 1u;
    const uint64_t lt = (1ull << lane) - 1ull;

    uint64_t key[ITEMS];
    uint32_t dr[ITEMS];   // digit in bits 0..RB-1; rank inside the wave, later the tile position, from bit RB on
    uint32_t vm = 0;      // items this lane keeps
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        key[r] = (uint32_t)r * 64 < rem ? a.in[wbase + (uint64_t)r * 64] : 0ull;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
        if ((uint32_t)r * 64 < rem && !(a.drop_excl && (key[r] >> a.excl_shift) != 0)) vm |= 1u << r;
    uint32_t h = 0;
    if (tid < B) h = a.hist[tid];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) dr[r] = (uint32_t)(key[r] >> a.shift) & dmask;
    // rank inside the wave: lanes with the same digit found by one ballot per
    // digit bit (bits above nbits are zero in every lane and keep every lane);
    // per-wave counters in LDS carry the count across rounds
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const bool valid = (vm >> r) & 1u;
        const uint32_t d = dr[r];
        const uint64_t vb = __ballot(valid);
        uint32_t x_lo = 0, x_hi = 0;           // lanes whose digit differs from mine
        uint32_t sb[RB];                       // bit b of d in all 32 bits
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            sb[b] = (uint32_t)__builtin_amdgcn_sbfe((int32_t)d, b, 1);
            asm("" : "+v"(sb[b]));             // ballot on sb itself, not on a second extract of the bit
        }
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const uint64_t bb = __ballot(sb[b] != 0u);
            // x |= sb ^ bb, one three-input bit operation per half
            x_lo = __builtin_amdgcn_bitop3_b32(x_lo, sb[b], (uint32_t)bb, 0xF6);
            x_hi = __builtin_amdgcn_bitop3_b32(x_hi, sb[b], (uint32_t)(bb >> 32), 0xF6);
        }
        const uint64_t m = vb & ~(((uint64_t)x_hi << 32) | x_lo);
        const uint32_t below = (uint32_t)__popcll(m & lt);
        const uint32_t prev = s_wcnt[w * B + d];
        dr[r] = d | ((prev + below) << RB);
        if (valid && below == 0) s_wcnt[w * B + d] = prev + (uint32_t)__popcll(m);
    }
    __syncthreads();
    // per bucket: publish this tile's count, then tile and global offsets
    uint32_t tot = 0;
    if (tid < B) {
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) tot += s_wcnt[ww * B + tid];
        st_flag(a.status + (uint64_t)tile * B + tid, (tile == 0 ? kFlagInc : kFlagAgg) | tot);
    }
    const uint2 ex = block_excl_scan2<NB>(tot, h, s_tmp);
    const uint32_t lstart = ex.x, gexcl = ex.y;
    uint32_t tile_n = 0;                       // words this tile keeps
#pragma unroll
    for (int i = 0; i < NB; ++i) tile_n += s_tmp[i];
    if (tid < B) {
        // each thread reads and rewrites only its own bucket's column
        uint32_t run = lstart;
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) {
            const uint32_t c = s_wcnt[ww * B + tid];
            s_wcnt[ww * B + tid] = run;
            run += c;
        }
    }
    __syncthreads();
    // tile position of every kept key; a tile that fits the LDS buffer is
    // ordered there before the look-back, so that the waves without a bucket
    // do it while the others wait on their predecessors
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t d = dr[r] & (B - 1);
        dr[r] = d | ((s_wcnt[w * B + d] + (dr[r] >> RB)) << RB);
    }
    if (kShare) __syncthreads();               // the counters' LDS becomes the key buffer
    if (PHASES == 1) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r)
            if (((vm >> r) & 1u) && (dr[r] >> RB) < (uint32_t)CHUNK) s_keys[dr[r] >> RB] = key[r];
    }
    if (tid < B) {
        uint32_t prefix = 0;
        if (tile > 0) {
            // windowed look-back: one round trip fetches kSortLookWindow
            // predecessors of this bucket (consecutive buckets: coalesced)
            int64_t j = (int64_t)tile - 1;
            uint32_t spins = 0;
            bool done = false;
            while (!done) {
                uint32_t sv[kSortLookWindow];
#pragma unroll
                for (int k = 0; k < kSortLookWindow; ++k)
                    sv[k] = j - k >= 0 ? ld_acquire_flag(a.status + (uint64_t)(j - k) * B + tid) : kFlagInc;
                int used = 0;
                bool stop = false;
#pragma unroll
                for (int k = 0; k < kSortLookWindow; ++k) {
                    if (done || stop) continue;
                    if ((sv[k] >> 30) == 0u) { stop = true; continue; }   // not published yet: poll again from here
                    prefix += sv[k] & kValMask;
                    used = k + 1;
                    if ((sv[k] & ~kValMask) == kFlagInc) done = true;
                }
                j -= used;
                if (!done && j < 0) done = true;
                if (!done && used == 0) {
                    if (++spins > kSpinLimit) {
                        atomicOr(a.err, kErrSpin);
                        break;
                    }
                    if (kSortSpinSleep) __builtin_amdgcn_s_sleep(1);
                }
            }
            st_flag(a.status + (uint64_t)tile * B + tid, kFlagInc | (prefix + tot));
        }
        s_gbase[tid] = gexcl + prefix - lstart;     // destination of tile position i of bucket d: s_gbase[d] + i
    }
    __syncthreads();
#pragma unroll
    for (int ph = 0; ph < PHASES; ++ph) {
        const uint32_t lo_pos = (uint32_t)ph * CHUNK;
        if (PHASES > 1) {
            if (ph > 0) __syncthreads();
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) {
                const uint32_t rel = (dr[r] >> RB) - lo_pos;
                if (((vm >> r) & 1u) && rel < (uint32_t)CHUNK) s_keys[rel] = key[r];
            }
            __syncthreads();
        }
        const uint32_t hi_pos = min<uint32_t>(tile_n, lo_pos + CHUNK);
        for (uint32_t i = lo_pos + tid; i < hi_pos; i += THREADS) {
            const uint64_t k = s_keys[i - lo_pos];
            const uint32_t d = (uint32_t)(k >> a.shift) & dmask;
            const uint64_t dst = (uint64_t)(uint32_t)(s_gbase[d] + i);
            if (dst < n_out) a.out[dst] = k;
            else atomicOr(a.err, kErrData);
        }
    }
}

// ---------------------------------------------------------------------------
// segmented transition-map scan
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pad_idx(uint32_t i) { return i + (i >> 4); }

// A new level-m node starts with empty counts (its counting runs later).
__device__ __forceinline__ void zero_node_counts(const ScanArgs& a, int m, uint64_t id) {
    uint32_t* c = a.node_counts[m];
    if (!c) return;
    for (uint32_t p = 0; p < a.n_props_all; ++p) {
        uint2* q = reinterpret_cast<uint2*>(c + (p * a.node_stride[m] + id) * 6);
        q[0] = make_uint2(0u, 0u);
        q[1] = make_uint2(0u, 0u);
        q[2] = make_uint2(0u, 0u);
    }
}

// One launch scans a group of up to PMAX properties whose monitors have at
// most 4 MW states (PMAX * MW <= 16); the structure outputs (instance and node
// numbering, parent ids, node-count zeroing, keys, sizes) come from one
// launch with at most 4 properties.
//
// Look-back records are structure-of-arrays: row r of the aggregates of tile
// t is st[r * tiles + t], row r of the inclusive values st[(kScanRows + r) *
// tiles + t].  Rows 0..3 are the instance / node counts, row 4 + MW p + k the
// dword k of property p's map, so that the lanes of one wave reading one row
// of 64 consecutive tiles read one contiguous 256-byte span.  Every word
// carries its own validity bit 31 (counts stay below 2^30 and map bytes below
// 16): readers need no fence.
//
// Every instance is held to 128 VGPRs so that 16 waves share a CU (two
// 512-thread blocks, or one 1024-thread block); the 4 x 16-state instance
// spills a few words, and still runs faster so.
template <int PMAX, int MW, int THREADS>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_scan(ScanArgs a) {
    static_assert(PMAX * MW <= 16 && 4 + PMAX * MW <= kScanRows, "look-back record of at most 20 words");
    constexpr bool kParents = PMAX <= 4;       // LDS room to stage parent ids
    constexpr int TILE = THREADS * kScanItems;
    constexpr int WAVES = THREADS / 64;
    constexpr int NW = 4 + MW * PMAX;          // record words in use (at most)
    __shared__ uint64_t s_w[TILE + TILE / 16 + 1];
    __shared__ uint32_t s_cm[PMAX][16][MW];
    __shared__ uint32_t s_q0[PMAX], s_lab[PMAX][2];
    __shared__ uint32_t s_wtot[PMAX][WAVES][MW];
    __shared__ uint32_t s_ctot[2][WAVES];
    __shared__ uint32_t s_tprefix[PMAX][MW];
    __shared__ uint32_t s_tagg[PMAX][MW];
    __shared__ uint32_t s_cagg[4];
    __shared__ uint32_t s_tcnt[4];
    __shared__ uint64_t s_prev, s_next;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_red[2][WAVES];

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t P = a.n_props;               // properties of this launch
    const bool structure = kParents && a.structure != 0;
    if (tid == 0) s_tile = atomicAdd(a.ticket, 1u);
    for (uint32_t i = tid; i < P * 16 * MW; i += THREADS) {
        const uint32_t p = i / (16 * MW), c = (i / MW) % 16, k = i % MW;
        s_cm[p][c][k] = a.plan->prop[a.prop_idx[p]].bmap[c][k];
    }
    if (tid < (int)P) {
        const PropDev& pd = a.plan->prop[a.prop_idx[tid]];
        s_q0[tid] = pd.q0;
        s_lab[tid][0] = pd.blabel[0];
        s_lab[tid][1] = pd.blabel[1];
    }
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = (uint64_t)tile * TILE;
    const uint64_t kInvalid = ~0ull;
    const uint32_t n = a.n_dev ? *a.n_dev : a.n;    // the look-back rows stay laid out for a.n
    if (base >= n) return;                         // the whole block: no word of this tile
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const uint64_t idx = base + r * THREADS + tid;
        s_w[pad_idx(r * THREADS + tid)] = idx < n ? a.words[idx] : kInvalid;
    }
    if (tid == 0) s_prev = base > 0 ? a.words[base - 1] : kInvalid;
    if (tid == 1) s_next = base + TILE < n ? a.words[base + TILE] : kInvalid;
    __syncthreads();

    uint64_t wv[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) wv[j] = s_w[pad_idx(tid * kScanItems + j)];
    const uint64_t wp = tid == 0 ? s_prev : s_w[pad_idx(tid * kScanItems - 1)];
    const uint64_t wn = tid == THREADS - 1 ? s_next : s_w[pad_idx(tid * kScanItems + kScanItems)];
    const bool has_prev = base + (uint64_t)tid * kScanItems > 0;
    const uint32_t cb = a.cbits, vs = a.valid_shift, L = a.n_levels;
    const uint32_t cmask = a.class_mask;    // the class; cb is where the key starts

    // per-event flags as bit masks (excluded events sort last, so the valid
    // events of a thread are a prefix of its run).  Branch-free: with d the
    // previous word XOR this one, a change of the packed keys above bit s
    // shows as d >= 2^s.
    const uint64_t vlim = 1ull << vs, hlim = 1ull << cb;
    uint64_t llim[kMaxLevels];
#pragma unroll
    for (int m = 1; m < kMaxLevels; ++m) llim[m] = (uint32_t)m < L ? 1ull << a.prefix_shift[m] : ~0ull;
    uint32_t m_valid = 0, m_head = 0, m_end = 0, m_lvl[kMaxLevels] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t x = wv[j];
        const bool valid = x < vlim;
        const bool first = j == 0 && !has_prev;
        const uint64_t d = (j == 0 ? wp : wv[j - 1]) ^ x;
        m_valid |= (uint32_t)valid << j;
        m_head |= (uint32_t)(valid && (first || d >= hlim)) << j;
#pragma unroll
        for (int m = 1; m < kMaxLevels; ++m)
            if ((uint32_t)m < L) m_lvl[m] |= (uint32_t)(valid && (first || d >= llim[m])) << j;
    }
    {
        // an instance ends where the next word is excluded, absent or of another key
        const uint32_t cont = m_valid & ~m_head;             // valid words that continue the previous one
        const bool cont_next = wn < vlim && (wn ^ wv[kScanItems - 1]) < hlim;
        m_end = m_valid & ~((cont >> 1) | ((uint32_t)cont_next << (kScanItems - 1)));
    }
    // the class of each word, 4 bits apiece: the words themselves are not
    // needed in registers after this point
    uint64_t cls = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) cls |= (uint64_t)((uint32_t)wv[j] & cmask) << (4 * j);
    uint32_t cnt[4];
    cnt[0] = __popc(m_head);
#pragma unroll
    for (int m = 1; m < 4; ++m) cnt[m] = (uint32_t)m < L ? __popc(m_lvl[m]) : 0u;

    // run summaries (a head restarts the monitor from q0), then a
    // wave-inclusive scan of them in lane order
    BMap<MW> excl[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        BMap<MW> f = bm_identity<MW>();
        if (p < (int)P) {
            const BMap<MW> start = bm_const<MW>(s_q0[p]);
#pragma unroll
            for (int j = 0; j < kScanItems; ++j) {
                // excluded / absent words leave f alone
                const BMap<MW> cm = bm_load<MW>(s_cm[p][(uint32_t)(cls >> (4 * j)) & 15u]);
                const BMap<MW> g = bm_compose<MW>(cm, ((m_head >> j) & 1u) ? start : f);
                if ((m_valid >> j) & 1u) f = g;
            }
        }
        BMap<MW> v = f;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const BMap<MW> o = bm_shfl_up<MW>(v, off);
            if (lane >= off) v = bm_compose<MW>(v, o);
        }
        const BMap<MW> e = bm_shfl_up<MW>(v, 1);
        excl[p] = lane == 0 ? bm_identity<MW>() : e;
        if (lane == 63)
#pragma unroll
            for (int k = 0; k < MW; ++k) s_wtot[p][w][k] = v.d[k];
    }
    // head counts two to a word in 16-bit fields (a tile holds at most 8192
    // words, so no field carries into the next); levels 2-3 only when present
    uint32_t cexcl[4];
    uint32_t pe[2] = {0u, 0u};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && L <= 2) break;
        const uint32_t pk = cnt[2 * k] | (cnt[2 * k + 1] << 16);
        const uint32_t incl = wave_incl_scan_u32(pk);
        pe[k] = incl - pk;
        if (lane == 63) s_ctot[k][w] = incl;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PMAX; ++p) {
        if (p >= (int)P) continue;
        BMap<MW> pre = bm_identity<MW>();
        for (int i = 0; i < w; ++i) pre = bm_compose<MW>(bm_load<MW>(s_wtot[p][i]), pre);
        excl[p] = bm_compose<MW>(excl[p], pre);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && L <= 2) break;
        for (int i = 0; i < w; ++i) pe[k] += s_ctot[k][i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) cexcl[k] = (pe[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
    if (tid < (int)P) {
        BMap<MW> t = bm_identity<MW>();
        for (int i = 0; i < WAVES; ++i) t = bm_compose<MW>(bm_load<MW>(s_wtot[tid][i]), t);
#pragma unroll
        for (int k = 0; k < MW; ++k) s_tagg[tid][k] = t.d[k];
    }
    if (tid >= 32 && tid < 34) {
        const int k = tid - 32;
        uint32_t sum = 0;
        if (k == 0 || L > 2)
            for (int i = 0; i < WAVES; ++i) sum += s_ctot[k][i];
        s_cagg[2 * k] = sum & 0xFFFFu;
        s_cagg[2 * k + 1] = sum >> 16;
    }
    __syncthreads();

    // publish the aggregate (tile 0: the inclusive value), then look back
    // with one lane per predecessor tile (wave 0)
    if (w == 0) {
        const uint32_t n_tiles = (uint32_t)((a.n + TILE - 1) / TILE);
        uint32_t* st = a.status;
        const uint32_t nw = 4 + MW * P;
        const uint32_t kValid = 1u << 31;
        if (lane < (int)nw) {
            const uint32_t pay = lane < 4 ? s_cagg[lane] : s_tagg[(lane - 4) / MW][(lane - 4) % MW];
            const uint32_t row = (tile == 0 ? kScanRows : 0) + lane;
            __hip_atomic_store(st + (uint64_t)row * n_tiles + tile, kValid | pay, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        BMap<MW> acc[PMAX];
        uint32_t accc[4] = {0, 0, 0, 0};
#pragma unroll
        for (int p = 0; p < PMAX; ++p) acc[p] = bm_identity<MW>();
        int64_t j = (int64_t)tile - 1;
        uint32_t spins = 0;
        while (j >= 0) {
            const int64_t t = j - lane;
            uint32_t vi[NW], va[NW];
            bool inc_ok = true, agg_ok = true;
#pragma unroll
            for (int r = 0; r < NW; ++r) {
                vi[r] = va[r] = kValid;
                if (r < (int)nw && t >= 0) {
                    vi[r] = __hip_atomic_load(st + (uint64_t)(kScanRows + r) * n_tiles + t, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    va[r] = __hip_atomic_load(st + (uint64_t)r * n_tiles + t, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                }
                inc_ok = inc_ok && (vi[r] & kValid);
                agg_ok = agg_ok && (va[r] & kValid);
            }
            // lanes past tile 0 read as inclusive identities; tile 0 itself
            // only ever publishes an inclusive record
            const uint64_t incm = __ballot(inc_ok);
            const uint64_t nrm = __ballot(!inc_ok && !agg_ok);
            const int first_inc = incm ? __ffsll((unsigned long long)incm) - 1 : 64;
            const int first_nr = nrm ? __ffsll((unsigned long long)nrm) - 1 : 64;
            const bool done = first_inc < first_nr;
            const int take = done ? first_inc + 1 : first_nr;
            const bool mine = lane < take;
            // fold lanes [0, take): the nearest tile is applied last
            BMap<MW> m[PMAX];
#pragma unroll
            for (int p = 0; p < PMAX; ++p)
#pragma unroll
                for (int k = 0; k < MW; ++k) {
                    const uint32_t x = (inc_ok ? vi[4 + MW * p + k] : va[4 + MW * p + k]) & ~kValid;
                    m[p].d[k] = (mine && p < (int)P) ? x : 0x03020100u + 0x04040404u * (uint32_t)k;
                }
            uint32_t c[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] = mine ? (inc_ok ? vi[k] : va[k]) & ~kValid : 0u;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
                for (int p = 0; p < PMAX; ++p) {
                    const BMap<MW> o = bm_shfl_down<MW>(m[p], off);
                    if (lane + off < 64) m[p] = bm_compose<MW>(m[p], o);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t o = __shfl_down(c[k], off, 64);
                    if (lane + off < 64) c[k] += o;
                }
            }
#pragma unroll
            for (int p = 0; p < PMAX; ++p) acc[p] = bm_compose<MW>(acc[p], bm_bcast<MW>(m[p], 0));
#pragma unroll
            for (int k = 0; k < 4; ++k) accc[k] += __shfl(c[k], 0, 64);
            j -= take;
            if (done) break;
            if (take == 0) {
                if (++spins > kSpinLimit) {
                    if (lane == 0) atomicOr(a.err, kErrSpin);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (tile > 0 && lane < (int)nw) {
            uint32_t pay;
            if (lane < 4) {
                pay = accc[lane] + s_cagg[lane];
            } else {
                const int p = (lane - 4) / MW, k = (lane - 4) % MW;
                BMap<MW> incl = bm_identity<MW>();
#pragma unroll
                for (int q = 0; q < PMAX; ++q)
                    if (q == p) incl = bm_compose<MW>(bm_load<MW>(s_tagg[q]), acc[q]);
                pay = incl.d[0];
#pragma unroll
                for (int i = 1; i < MW; ++i)
                    if (i == k) pay = incl.d[i];
            }
            __hip_atomic_store(st + (uint64_t)(kScanRows + lane) * n_tiles + tile, kValid | pay, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane < (int)P)
#pragma unroll
            for (int q = 0; q < PMAX; ++q)
                if (q == lane)
#pragma unroll
                    for (int k = 0; k < MW; ++k) s_tprefix[q][k] = acc[q].d[k];
        if (lane < 4) s_tcnt[lane] = accc[lane];
    }
    __syncthreads();

    // second walk: final state at every instance end; numbering of nodes
    uint32_t cur[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
        cur[p] = p < (int)P ? bm_at<MW>(bm_compose<MW>(excl[p], bm_load<MW>(s_tprefix[p])), 0) : 0u;
    // staging in the word buffer (free now): verdict bytes [P][TILE + 1],
    // then parent ids [TILE + 1]
    uint8_t* s_iv = reinterpret_cast<uint8_t*>(s_w);
    constexpr uint32_t kIvStride = TILE + 1;
    static_assert(PMAX * kIvStride + (kParents ? 4 * kIvStride + 4 : 0) <= sizeof(s_w), "staging fits the word buffer");
    uint32_t* s_par = reinterpret_cast<uint32_t*>(s_iv + ((PMAX * kIvStride + 3) & ~3u));
    const uint32_t id_base = s_tcnt[0];
    // parents are level-(L-1) nodes: their heads, and the id before this thread's first
    const uint32_t m_par = L >= 4 ? m_lvl[3] : L == 3 ? m_lvl[2] : m_lvl[1];
    const uint32_t par_base = (L >= 4 ? s_tcnt[3] + cexcl[3] : L == 3 ? s_tcnt[2] + cexcl[2] : s_tcnt[1] + cexcl[1]) - 1u;
    uint32_t my_lo = 0xFFFFFFFFu, my_hi = 0u;
    uint32_t err = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint32_t c = (uint32_t)(cls >> (4 * j)) & 15u;
        const bool hd = (m_head >> j) & 1u;
#pragma unroll
        for (int p = 0; p < PMAX; ++p)
            if (p < (int)P) cur[p] = bm_at<MW>(bm_load<MW>(s_cm[p][c]), hd ? s_q0[p] : cur[p]);
        if ((m_end >> j) & 1u) {
            // instances of this thread so far, from its head count
            const uint32_t upto = (2u << j) - 1u;
            const uint32_t slot = cexcl[0] + __popc(m_head & upto);
            const uint64_t id = (uint64_t)id_base + slot - 1u;
            if (id < a.inst_limit) {
#pragma unroll
                for (int p = 0; p < PMAX; ++p)
                    if (p < (int)P)
                        s_iv[p * kIvStride + slot] =
                            a.emit_state ? cur[p] : (s_lab[p][cur[p] >> 3] >> (4 * (cur[p] & 7u))) & 15u;
                if (kParents && L >= 2) s_par[slot] = par_base + __popc(m_par & upto);
                my_lo = min(my_lo, (uint32_t)id);
                my_hi = max(my_hi, (uint32_t)id + 1u);
                if (structure && a.inst_keys) a.inst_keys[id] = a.words[base + (uint64_t)tid * kScanItems + j] >> cb;
            } else {
                err |= kErrCapacity;
            }
        }
    }
    // On request, the verdict timeline of every instance: the first prefix
    // whose verdict is conclusive (T or F).  Those verdicts are final (Def. 5),
    // so the monitor enters a conclusive state at most once per instance: the
    // word where it does writes its 1-based sorted position (or the head's
    // position, when q0 itself is conclusive), the word ending an instance
    // that never got there writes kNever.  Positions become counts of the
    // instance's words in k_inst_conclusive.  Also on request, the verdict
    // after every event, stored at the event's trace index.
    if (a.inst_conc || a.event_verdict) {
        uint32_t st[PMAX];
#pragma unroll
        for (int p = 0; p < PMAX; ++p)
            st[p] = p < (int)P ? bm_at<MW>(bm_compose<MW>(excl[p], bm_load<MW>(s_tprefix[p])), 0) : 0u;
        auto label = [&](int p, uint32_t q) { return (s_lab[p][q >> 3] >> (4 * (q & 7u))) & 15u; };
#pragma unroll 1
        for (int j = 0; j < kScanItems; ++j) {
            if (!((m_valid >> j) & 1u)) break;
            const uint32_t c = (uint32_t)(cls >> (4 * j)) & 15u;
            const bool hd = (m_head >> j) & 1u, end = (m_end >> j) & 1u;
            const uint64_t id = (uint64_t)id_base + cexcl[0] + __popc(m_head & ((2u << j) - 1u)) - 1u;
            const uint32_t pos = (uint32_t)(base + (uint64_t)tid * kScanItems + j);
            const bool conc_out = a.inst_conc && id < a.inst_limit;
            if (conc_out && hd && structure) a.inst_start[id] = pos;
            // the event's trace index rides in the word between class and key
            const uint64_t ev = a.event_verdict ? (a.words[pos] >> a.index_shift) & a.index_mask : 0ull;
#pragma unroll
            for (int p = 0; p < PMAX; ++p) {
                if (p >= (int)P) continue;
                const uint32_t pre = hd ? s_q0[p] : st[p];
                const uint32_t post = bm_at<MW>(bm_load<MW>(s_cm[p][c]), pre);
                st[p] = post;
                const uint32_t lpost = label(p, post);
                if (a.event_verdict) a.event_verdict[a.prop_idx[p] * a.n_events + ev] = (uint8_t)lpost;
                if (!conc_out) continue;
                uint32_t* out = a.inst_conc + a.prop_idx[p] * a.inst_stride + id;
                const uint32_t lpre = label(p, pre);
                const bool cpre = lpre == 0u || lpre == 5u, cpost = lpost == 0u || lpost == 5u;
                if (hd && cpre) *out = pos;
                else if (cpost && !cpre) *out = pos + 1u;
                if (end && !cpost) *out = kNever;
            }
        }
    }
    // nodes of levels 1.. open at their first word; every such word is a
    // level-(L-1) head, and a level-m head is also a level-(m+1) head
    if (structure && L >= 2) {
        // few words open nodes: loop over them, the word read again from memory
        for (uint32_t rest = m_par; rest != 0u; rest &= rest - 1u) {
            const int j = __ffs(rest) - 1;
            const uint32_t upto = (2u << j) - 1u;
            const uint64_t x = a.words[base + (uint64_t)tid * kScanItems + j];
#pragma unroll
            for (int m = kMaxLevels - 1; m >= 1; --m) {
                if (m >= (int)L || !((m_lvl[m] >> j) & 1u)) continue;
                const uint64_t id = (uint64_t)s_tcnt[m] + cexcl[m] + __popc(m_lvl[m] & upto) - 1u;
                const int mc = m < 3 ? m + 1 : 3;
                const uint32_t child = m == (int)L - 1 ? s_tcnt[0] + cexcl[0] + __popc(m_head & upto) - 1u
                                                       : s_tcnt[mc] + cexcl[mc] + __popc(m_lvl[mc] & upto) - 1u;
                if (id < a.node_limit[m]) {
                    a.node_start[m][id] = child;
                    if (a.node_keys[m]) a.node_keys[m][id] = x >> a.prefix_shift[m];
                    zero_node_counts(a, m, id);
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
    for (int i = 1; i < WAVES; ++i) {
        lo = min(lo, s_red[0][i]);
        hi = max(hi, s_red[1][i]);
    }
    if (lo < hi) {
        const uint32_t cnt_iv = hi - lo, slot0 = lo + 1u - id_base;
        for (uint32_t p = 0; p < P; ++p)
            for (uint32_t i = tid; i < cnt_iv; i += THREADS)
                a.inst_verdict[a.prop_idx[p] * a.inst_stride + lo + i] = s_iv[p * kIvStride + slot0 + i];
        if (structure && a.inst_parent)
            for (uint32_t i = tid; i < cnt_iv; i += THREADS) a.inst_parent[lo + i] = s_par[slot0 + i];
    }
    // the thread holding the last event publishes the totals
    const uint64_t my0 = base + (uint64_t)tid * kScanItems;
    if (structure && my0 <= n - 1 && n - 1 < my0 + kScanItems) {
#pragma unroll
        for (int m = 0; m < kMaxLevels; ++m) {
            if (m >= (int)L) break;
            const uint32_t tot = s_tcnt[m] + cexcl[m] + cnt[m];
            a.sizes[m] = tot;
            a.sizes32[m] = tot;
        }
    }
}

// Byte fill: the per-event verdicts start as "no instance" (events that join
// no cluster are never visited by the scan).
__global__ __launch_bounds__(256) void k_fill_u8(uint8_t* p, uint8_t v, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n16 = (reinterpret_cast<uintptr_t>(p) & 15) == 0 ? n / 16 : 0;
    const uint32_t v4 = 0x01010101u * v;
    uint4* p16 = reinterpret_cast<uint4*>(p);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p16[i] = make_uint4(v4, v4, v4, v4);
    for (uint64_t i = n16 * 16 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Verdict timeline, second step: a sorted position p of the first conclusive
// word becomes p - start, the number of the instance's words consumed (0 when
// its empty prefix is already conclusive); kNever stays.
__global__ __launch_bounds__(256) void k_inst_conclusive(InstConclusiveArgs a) {
    const uint64_t n = min<uint64_t>(*a.n_inst, a.inst_limit);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t start = a.inst_start[i];
        for (uint32_t p = 0; p < a.n_props; ++p) {
            uint32_t* o = a.inst_conc + p * a.inst_stride + i;
            const uint32_t v = *o;
            if (v != kNever) *o = v - start;
        }
    }
}

// ---------------------------------------------------------------------------
// counting for one level
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t node_of(const uint32_t* start, uint32_t nn, uint32_t c) {
    // last node j with start[j] <= c
    uint32_t lo = 0, hi = nn;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (start[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// Def. 7 at the root and the sizes, by threads 0..63; `counts` read coherently.
__device__ __forceinline__ void finalize_root(const FinalizeArgs& a) {
    const uint32_t p = threadIdx.x;
    if (p <= a.n_levels) a.sizes_out[p] = p < a.n_levels ? a.sizes_ws[p] : 0ull;
    if (p >= a.n_props) return;
    uint32_t v[6];
#pragma unroll
    for (int b = 0; b < 6; ++b)
        v[b] = __hip_atomic_load(a.root_counts + p * 6 + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.root_verdict[p] = (uint8_t)valuate(a.plan->prop[p], 0, v);
    for (int b = 0; b < 6; ++b) a.root_counts_out[p * 6 + b] = v[b];
}

__global__ void k_finalize(FinalizeArgs a) { finalize_root(a); }

// Children are read in strided order (consecutive threads take consecutive
// children; all loads of a tile are issued before any is used) and counted
// into an LDS window of kCountWindow parents.  Children are in parent order,
// so the lanes of one wave with one parent form a run: six ballots give every
// run's bin counts and the first lane of each run adds them.
__device__ __forceinline__ void count_add(const CountArgs& a, uint32_t* s_cnt, uint32_t p, uint32_t lo, uint32_t nn,
                                          uint32_t node, uint32_t q, uint32_t v) {
    const uint32_t slot = node - lo;
    if (slot < (uint32_t)kCountWindow)
        atomicAdd(&s_cnt[(p * kCountWindow + slot) * 6 + q], v);
    else if (node < nn)
        atomicAdd(&a.counts[((uint64_t)p * a.stride + node) * 6 + q], v);
}

__device__ __forceinline__ void count_child(const CountArgs& a, uint32_t* s_cnt, uint32_t p, uint32_t lo, uint32_t nn,
                                            bool valid, uint32_t node, uint32_t b) {
    const int lane = threadIdx.x & 63;
    const uint64_t vm = __ballot(valid);
    if (vm == 0) return;
    uint64_t bq[6];
#pragma unroll
    for (uint32_t q = 0; q < 6; ++q) bq[q] = __ballot(valid && b == q);
    const uint32_t pn = __shfl_up(node, 1, 64);
    const bool head = valid && (lane == 0 || pn != node);
    const uint64_t heads = __ballot(head);
    if (__popcll(heads) == 1) {
        // one parent for the whole wave: lanes 0..5 add one bin each
        const uint32_t node0 = __shfl(node, __ffsll((unsigned long long)heads) - 1, 64);
        uint32_t mine = 0;
#pragma unroll
        for (uint32_t q = 0; q < 6; ++q)
            if (lane == (int)q) mine = (uint32_t)__popcll(bq[q]);
        if (lane < 6 && mine) count_add(a, s_cnt, p, lo, nn, node0, (uint32_t)lane, mine);
    } else if (head) {
        const uint64_t later = heads & ~((2ull << lane) - 1ull);
        const int end = later ? __ffsll((unsigned long long)later) - 1 : 64;
        const uint64_t run = (end == 64 ? ~0ull : ((1ull << end) - 1ull)) & ~((1ull << lane) - 1ull);
#pragma unroll
        for (uint32_t q = 0; q < 6; ++q) {
            const uint32_t cnt = (uint32_t)__popcll(bq[q] & run);
            if (cnt) count_add(a, s_cnt, p, lo, nn, node, q, cnt);
        }
    }
}

template <int ITEMS>
__global__ __launch_bounds__(kCountThreads) void k_count(CountArgs a) {
    __shared__ uint32_t s_cnt[kMaxProps * kCountWindow * 6];
    __shared__ uint32_t s_lo;
    const int tid = threadIdx.x;
    const uint32_t P = a.n_props;
    const uint32_t nch_all = *a.n_children;
    const uint32_t nn_all = a.level == 0 ? 1u : *a.n_nodes;
    const uint32_t nch = (uint32_t)min<uint64_t>(nch_all, a.child_limit);
    const uint32_t nn = (uint32_t)min<uint64_t>(nn_all, a.level == 0 ? 1ull : a.node_limit);
    const bool leaves = a.level + 1 == a.n_levels;
    constexpr uint32_t kTile = kCountThreads * ITEMS;
    const uint32_t ntiles = (nch + kTile - 1) / kTile;
    if (blockIdx.x == 0 && tid == 0 && (nch < nch_all || nn < nn_all)) atomicOr(a.err, kErrCapacity);
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t c0 = tile * kTile;
        for (uint32_t i = tid; i < P * kCountWindow * 6; i += kCountThreads) s_cnt[i] = 0;
        if (tid == 0)
            s_lo = a.level == 0 ? 0u : a.child_parent ? a.child_parent[c0] : node_of(a.node_start, nn, c0);
        uint32_t node[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t c = c0 + k * kCountThreads + tid;
            node[k] = 0;
            if (c < nch && a.level > 0) node[k] = a.child_parent ? a.child_parent[c] : node_of(a.node_start, nn, c);
        }
        __syncthreads();
        const uint32_t lo = s_lo;
        for (uint32_t p = 0; p < P; ++p) {
            uint32_t b[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const uint32_t c = c0 + k * kCountThreads + tid;
                b[k] = 6u;
                if (c < nch) {
                    if (leaves) {
                        b[k] = a.child_verdict[p * a.child_stride + c];
                    } else {
                        b[k] = valuate(a.plan->prop[p], (int)a.level + 1, a.child_counts + (p * a.child_stride + c) * 6);
                        if (a.child_verdict_out) a.child_verdict_out[p * a.child_stride + c] = (uint8_t)b[k];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const uint32_t c = c0 + k * kCountThreads + tid;
                const bool valid = c < nch;
                if (valid && b[k] > 5u) {
                    atomicOr(a.err, kErrData);
                    b[k] = 6u;
                }
                count_child(a, s_cnt, p, lo, nn, valid, node[k], b[k]);
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < P * kCountWindow * 6; i += kCountThreads) {
            const uint32_t v = s_cnt[i];
            if (!v) continue;
            const uint32_t p = i / (kCountWindow * 6), slot = (i / 6) % kCountWindow, b = i % 6;
            const uint32_t node = lo + slot;
            if (node < nn) atomicAdd(&a.counts[((uint64_t)p * a.stride + node) * 6 + b], v);
        }
        __syncthreads();
    }
    if (a.done) {
        // the last block to finish values the root
        __shared__ uint32_t s_last;
        __threadfence();
        __syncthreads();
        if (tid == 0) s_last = atomicAdd(a.done, 1u) == gridDim.x - 1 ? 1u : 0u;
        __syncthreads();
        if (s_last) {
            __threadfence();
            finalize_root(a.fin);
        }
    }
}
// Counting of leaf verdicts: every thread takes 16 consecutive children (the
// verdict bytes and parent ids are read as 16-byte vectors where aligned),
// accumulates each run of children with one parent in a packed register of
// six 5-bit bins and adds the run once, into the LDS window of kCountWindow
// parents or, beyond it, to global memory.
__device__ __forceinline__ void leaf_flush(const CountArgs& a, uint32_t* s_cnt, uint32_t p, uint32_t lo, uint32_t nn,
                                           uint32_t node, uint32_t acc) {
    if (!acc) return;
    const uint32_t slot = node - lo;
#pragma unroll
    for (uint32_t q = 0; q < 6; ++q) {
        const uint32_t v = (acc >> (5 * q)) & 31u;
        if (!v) continue;
        if (slot < (uint32_t)kCountWindow)
            atomicAdd(&s_cnt[(p * kCountWindow + slot) * 6 + q], v);
        else if (node < nn)
            atomicAdd(&a.counts[((uint64_t)p * a.stride + node) * 6 + q], v);
    }
}

__global__ __launch_bounds__(kCountThreads) void k_count_leaves(CountArgs a) {
    __shared__ uint32_t s_cnt[kMaxProps * kCountWindow * 6];
    __shared__ uint32_t s_lo;
    const int tid = threadIdx.x;
    const uint32_t P = a.n_props;
    const uint32_t nch_all = *a.n_children;
    const uint32_t nn_all = a.level == 0 ? 1u : *a.n_nodes;
    const uint32_t nch = (uint32_t)min<uint64_t>(nch_all, a.child_limit);
    const uint32_t nn = (uint32_t)min<uint64_t>(nn_all, a.level == 0 ? 1ull : a.node_limit);
    constexpr uint32_t kItems = 16, kTile = kCountThreads * kItems;
    const uint32_t ntiles = (nch + kTile - 1) / kTile;
    if (blockIdx.x == 0 && tid == 0 && (nch < nch_all || nn < nn_all)) atomicOr(a.err, kErrCapacity);
    uint32_t err = 0;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t c0 = tile * kTile;
        for (uint32_t i = tid; i < P * kCountWindow * 6; i += kCountThreads) s_cnt[i] = 0;
        if (tid == 0) s_lo = a.level == 0 ? 0u : a.child_parent[c0];
        const uint32_t cb = c0 + tid * kItems;
        const uint32_t cnt = cb < nch ? min(kItems, nch - cb) : 0u;
        uint32_t par[kItems];
        if (a.level == 0) {
#pragma unroll
            for (uint32_t k = 0; k < kItems; ++k) par[k] = 0;
        } else if (cnt == kItems) {
            const uint4* pv = reinterpret_cast<const uint4*>(a.child_parent + cb);   // cb is a multiple of 16
#pragma unroll
            for (uint32_t k = 0; k < kItems / 4; ++k) {
                const uint4 x = pv[k];
                par[4 * k] = x.x;
                par[4 * k + 1] = x.y;
                par[4 * k + 2] = x.z;
                par[4 * k + 3] = x.w;
            }
        } else {
#pragma unroll
            for (uint32_t k = 0; k < kItems; ++k) par[k] = k < cnt ? a.child_parent[cb + k] : 0u;
        }
        __syncthreads();
        const uint32_t lo = s_lo;
        for (uint32_t p = 0; p < P && cnt > 0; ++p) {
            const uint8_t* vp = a.child_verdict + p * a.child_stride + cb;
            uint32_t vw[kItems / 4];
            if (cnt == kItems && (reinterpret_cast<uintptr_t>(vp) & 15u) == 0) {
                const uint4 x = *reinterpret_cast<const uint4*>(vp);
                vw[0] = x.x;
                vw[1] = x.y;
                vw[2] = x.z;
                vw[3] = x.w;
            } else {
#pragma unroll
                for (uint32_t k = 0; k < kItems / 4; ++k) vw[k] = 0;
                for (uint32_t k = 0; k < cnt; ++k) vw[k >> 2] |= (uint32_t)vp[k] << (8 * (k & 3));
            }
            uint32_t cur = par[0], acc = 0;
#pragma unroll
            for (uint32_t k = 0; k < kItems; ++k) {
                if (k >= cnt) break;
                if (par[k] != cur) {
                    leaf_flush(a, s_cnt, p, lo, nn, cur, acc);
                    cur = par[k];
                    acc = 0;
                }
                const uint32_t b = (vw[k >> 2] >> (8 * (k & 3))) & 0xFFu;
                if (b > 5u) err |= kErrData;
                else acc += 1u << (5 * b);
            }
            leaf_flush(a, s_cnt, p, lo, nn, cur, acc);
        }
        __syncthreads();
        for (uint32_t i = tid; i < P * kCountWindow * 6; i += kCountThreads) {
            const uint32_t v = s_cnt[i];
            if (!v) continue;
            const uint32_t p = i / (kCountWindow * 6), slot = (i / 6) % kCountWindow, b = i % 6;
            const uint32_t node = lo + slot;
            if (node < nn) atomicAdd(&a.counts[((uint64_t)p * a.stride + node) * 6 + b], v);
        }
        __syncthreads();
    }
    if (err) atomicOr(a.err, err);
}


// ---------------------------------------------------------------------------
// online monitoring: incremental update of a stream group's monitor tree
// (Section 4: online mode; SpawnMonitors / AddToTree of Algorithm 1 become
// hash-table inserts, ApplyQuantifiers a re-valuation of the touched nodes)
// ---------------------------------------------------------------------------
// Bit mixer of the table's hash: the 64-bit finalizer ("fmix64") of Austin
// Appleby's public-domain MurmurHash3, with its published shift and multiplier
// constants.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// Insert-or-find `key` in an open-addressing table; returns its slot and
// whether this call inserted it, or ~0 when the table is full.  Within one
// kernel a slot only changes from empty (or dead: a slot of a closed stream)
// to a key, so probes read through the caches: a stale copy can only show a
// free slot, and the compare-and-swap that claims it returns the slot's real
// content.  A key may sit past a dead slot (it was inserted before that slot
// died), so a free slot is only claimed once the walk has reached an empty
// one: the key is then absent, and it is put into the first free slot of its
// probe sequence.  Slots before that one never become free during a kernel,
// so concurrent inserts of one key race for the same slot and the loser sees
// the winner's key.  A lost race with another key restarts the walk.
// Keys sit `stride` words apart (a slot may carry data after its key).
__device__ uint64_t table_slot(uint64_t* keys, uint32_t stride, uint64_t mask, uint64_t key, bool* fresh) {
    const uint64_t h0 = mix64(key) & mask;
    for (uint32_t attempt = 0; attempt < 64; ++attempt) {
        uint64_t h = h0, dead = ~0ull, probe = 0;
        for (; probe <= mask; ++probe) {
            const uint64_t k = __hip_atomic_load(keys + h * stride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (k == key) {
                *fresh = false;
                return h;
            }
            if (k == kDeadKey) {
                if (dead == ~0ull) dead = h;
            } else if (k == kEmptyKey) {
                break;
            }
            h = (h + 1) & mask;
        }
        const bool use_dead = dead != ~0ull;
        if (!use_dead && probe > mask) break;             // full: no empty and no dead slot
        const uint64_t at = use_dead ? dead : h;
        const uint64_t expect = use_dead ? kDeadKey : kEmptyKey;
        const uint64_t prev = atomicCAS(reinterpret_cast<unsigned long long*>(keys + at * stride), expect, key);
        if (prev == expect) {
            *fresh = true;
            return at;
        }
        if (prev == key) {
            *fresh = false;
            return at;
        }
    }
    *fresh = false;
    return ~0ull;
}

// Put node `slot` of `level` on the level's dirty list once.  Called by every
// lane of a wave (want: this lane has a node to mark); the appends of a wave
// share one atomic on the list length.  A dirty flag only goes from 0 to 1
// within a kernel, so a cached read of 1 is final and skips the exchange.
__device__ __forceinline__ void mark_nodes(const GroupState& g, uint32_t level, bool want, uint32_t slot) {
    const int lane = threadIdx.x & 63;
    uint32_t* dirty = level == 0 ? g.rdirty : g.ndirty[level];
    uint32_t* list = level == 0 ? g.rlist : g.nlist[level];
    bool mine = false;
    if (want)
        mine = __hip_atomic_load(dirty + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0u &&
               atomicExch(dirty + slot, 1u) == 0u;
    const uint64_t m = __ballot(mine);
    if (m == 0) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(g.list_cnt + level, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    if (mine) list[base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = slot;
}

__device__ __forceinline__ uint32_t* counts_of(const GroupState& g, uint32_t level, uint32_t slot, uint32_t p) {
    if (level == 0) return g.rcounts + ((uint64_t)slot * g.n_props + p) * 6;
    return g.ncounts[level] + ((uint64_t)p * (g.nmask + 1) + slot) * 6;
}

// One thread per binding segment of the pushed chunks.  Segments are in key
// order, so the lanes of a wave whose bindings share a parent node form a
// run: its count changes are summed by ballots and applied once per run.
__global__ __launch_bounds__(256) void k_group_update(GroupUpdateArgs a) {
    const GroupState& g = a.g;
    const uint32_t nseg = *a.n_seg;
    const uint32_t L = g.n_levels;
    const uint32_t plevel = L - 1;
    const int lane = threadIdx.x & 63;
    for (uint32_t base = blockIdx.x * blockDim.x; base < nseg; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        bool ok = i < nseg;
        uint64_t b = 0, aux = 0;                                 // aux: parent | states of properties 0..3
        bool fresh = false;
        uint32_t parent = 0;
        if (ok) {
            const uint64_t key = a.seg_key[i];
            const uint32_t stream = (uint32_t)(key >> g.stream_shift);
            b = table_slot(g.bslot, 2, g.bmask, key, &fresh);
            if (b == ~0ull || stream >= g.max_streams) {
                atomicOr(g.err, kErrCapacity);
                ok = false;
            } else if (fresh) {
                if (L == 1) {
                    parent = stream;
                } else {
                    // find or create the chain of quantifier nodes above this binding
                    bool nf = false;
                    uint64_t slot = table_slot(g.nkeys[L - 1], 1, g.nmask, key >> g.level_shift[L - 1], &nf);
                    if (slot == ~0ull) {
                        atomicOr(g.err, kErrCapacity);
                        ok = false;
                    } else {
                        parent = (uint32_t)slot;
                        for (uint32_t m = L - 1; nf && m >= 1; --m) {
                            if (m == 1) {
                                g.nparent[1][slot] = stream;
                                break;
                            }
                            bool pf = false;
                            const uint64_t ps = table_slot(g.nkeys[m - 1], 1, g.nmask, key >> g.level_shift[m - 1], &pf);
                            if (ps == ~0ull) {
                                atomicOr(g.err, kErrCapacity);
                                break;
                            }
                            g.nparent[m][slot] = (uint32_t)ps;
                            slot = ps;
                            nf = pf;
                        }
                    }
                }
            } else {
                aux = g.bslot[2 * b + 1];
                parent = (uint32_t)aux;
            }
        }
        const uint64_t okm = __ballot(ok);
        {
            // new bindings per stream: one atomic per run of lanes with one stream
            const uint32_t stream = ok ? (uint32_t)(a.seg_key[i] >> g.stream_shift) : 0u;
            const uint32_t ps = __shfl_up(stream, 1, 64);
            const bool sprev = lane > 0 && ((okm >> (lane - 1)) & 1ull);
            const bool shead = ok && (!sprev || ps != stream);
            const uint64_t sheads = __ballot(shead);
            const uint64_t freshm = __ballot(ok && fresh);
            if (shead && freshm) {
                const uint64_t later = sheads & ~((2ull << lane) - 1ull);
                const int end = later ? __ffsll((unsigned long long)later) - 1 : 64;
                const uint64_t srun = (end == 64 ? ~0ull : ((1ull << end) - 1ull)) & ~((1ull << lane) - 1ull);
                const uint32_t nf = (uint32_t)__popcll(freshm & srun);
                if (nf && atomicAdd(g.stream_bindings + stream, nf) + nf > g.stream_max[stream])
                    atomicOr(g.err, kErrCapacity);
            }
        }
        // runs of lanes with one parent (all lanes take part in the ballots)
        const uint32_t pn = __shfl_up(parent, 1, 64);
        const bool prev_ok = lane > 0 && ((okm >> (lane - 1)) & 1ull);
        const bool head = ok && (!prev_ok || pn != parent);
        const uint64_t heads = __ballot(head);
        uint64_t run = 0;
        if (head) {
            const uint64_t later = heads & ~((2ull << lane) - 1ull);
            const int end = later ? __ffsll((unsigned long long)later) - 1 : 64;
            run = (end == 64 ? ~0ull : ((1ull << end) - 1ull)) & ~((1ull << lane) - 1ull) & okm;
        }
        bool touched_run = false;
        uint64_t aux_new = (uint64_t)parent;
        for (uint32_t p = 0; p < g.n_props; ++p) {
            const PropDev& P = g.plan->prop[p];
            uint32_t v_old = 6u, v_new = 6u;                       // 6: no change in this lane
            if (ok) {
                uint8_t* sp = p >= 4 ? g.bstate + (uint64_t)(p - 4) * (g.bmask + 1) + b : nullptr;
                const uint32_t s_old = fresh ? P.q0 : p < 4 ? (uint32_t)(aux >> (32 + 8 * p)) & 0xFFu : *sp;
                const uint32_t s_new = a.seg_state[(uint64_t)(g.vbase[p] + s_old) * a.seg_stride + i];
                if (p < 4) aux_new |= (uint64_t)s_new << (32 + 8 * p);
                else *sp = (uint8_t)s_new;
                const uint32_t vn = P.label[s_new];
                if (fresh) {
                    v_new = vn;
                } else {
                    const uint32_t vo = P.label[s_old];
                    if (vo != vn) {
                        v_old = vo;
                        v_new = vn;
                    }
                }
            }
            uint32_t delta[6];
#pragma unroll
            for (uint32_t q = 0; q < 6; ++q) {
                const uint64_t plus = __ballot(v_new == q), minus = __ballot(v_old == q);
                delta[q] = (uint32_t)__popcll(plus & run) - (uint32_t)__popcll(minus & run);
            }
            if (head) {
                uint32_t* c = counts_of(g, plevel, parent, p);
#pragma unroll
                for (uint32_t q = 0; q < 6; ++q)
                    if (delta[q]) {
                        atomicAdd(c + q, delta[q]);                // two's complement: a negative delta subtracts
                        touched_run = true;
                    }
            }
        }
        if (ok) g.bslot[2 * b + 1] = aux_new;
        mark_nodes(g, plevel, head && touched_run, parent);
    }
}

// Re-valuate the dirty nodes of one level (>= 1) and pass changed verdicts up.
__global__ __launch_bounds__(256) void k_group_level(GroupState g, uint32_t level) {
    const uint32_t n = g.list_cnt[level];
    for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        bool touched = false;
        uint32_t parent = 0;
        if (i < n) {
            const uint32_t slot = g.nlist[level][i];
            g.ndirty[level][slot] = 0u;
            parent = g.nparent[level][slot];
            for (uint32_t p = 0; p < g.n_props; ++p) {
                const uint32_t v = valuate(g.plan->prop[p], (int)level, counts_of(g, level, slot, p));
                uint8_t* vp = g.nverdict[level] + (uint64_t)p * (g.nmask + 1) + slot;
                const uint32_t v_old = *vp;
                if (v_old == v) continue;
                *vp = (uint8_t)v;
                uint32_t* c = counts_of(g, level - 1, parent, p);
                if (v_old != kNoVerdict) atomicSub(c + v_old, 1u);
                atomicAdd(c + v, 1u);
                touched = true;
            }
        }
        mark_nodes(g, level - 1, touched, parent);
    }
}

// Def. 7 at every dirty stream root (or at all roots).
__global__ __launch_bounds__(256) void k_group_roots(GroupState g, uint32_t all) {
    const uint32_t n = all ? g.max_streams : g.list_cnt[0];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t s = all ? i : g.rlist[i];
        g.rdirty[s] = 0u;
        for (uint32_t p = 0; p < g.n_props; ++p)
            g.rverdict[(uint64_t)s * g.n_props + p] = (uint8_t)valuate(g.plan->prop[p], 0, counts_of(g, 0, s, p));
    }
}

__global__ __launch_bounds__(256) void k_group_read(GroupState g, uint8_t* verdict, uint64_t* counts,
                                                    uint64_t* bindings) {
    const uint32_t n = g.max_streams * g.n_props;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        verdict[i] = g.rverdict[i];
        for (int b = 0; b < 6; ++b) counts[(uint64_t)i * 6 + b] = g.rcounts[(uint64_t)i * 6 + b];
        if (bindings && i % g.n_props == 0) bindings[i / g.n_props] = g.stream_bindings[i / g.n_props];
    }
}

// Close stream `stream`: its bindings and quantifier nodes become dead slots
// (free for later inserts, with cleared data), its root counts and binding
// count return to zero and its root is valued on the empty tree again.
__global__ __launch_bounds__(256) void k_group_purge(GroupState g, uint32_t stream) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t b = t0; b <= g.bmask; b += stride) {
        const uint64_t k = g.bslot[2 * b];
        if (k >= kDeadKey || (uint32_t)(k >> g.stream_shift) != stream) continue;
        g.bslot[2 * b] = kDeadKey;
        g.bslot[2 * b + 1] = 0;
        for (uint32_t p = 4; p < g.n_props; ++p) g.bstate[(uint64_t)(p - 4) * (g.bmask + 1) + b] = 0;
    }
    for (uint32_t m = 1; m < g.n_levels; ++m) {
        const uint32_t sh = g.stream_shift - g.level_shift[m];
        for (uint64_t j = t0; j <= g.nmask; j += stride) {
            const uint64_t k = g.nkeys[m][j];
            if (k >= kDeadKey || (uint32_t)(k >> sh) != stream) continue;
            g.nkeys[m][j] = kDeadKey;
            for (uint32_t p = 0; p < g.n_props; ++p) {
                uint32_t* c = counts_of(g, m, (uint32_t)j, p);
                for (int q = 0; q < 6; ++q) c[q] = 0u;
                g.nverdict[m][(uint64_t)p * (g.nmask + 1) + j] = kNoVerdict;
            }
            g.nparent[m][j] = 0u;
            g.ndirty[m][j] = 0u;
        }
    }
    if (t0 == 0) {
        g.stream_bindings[stream] = 0u;
        g.rdirty[stream] = 0u;
        for (uint32_t p = 0; p < g.n_props; ++p) {
            uint32_t* c = counts_of(g, 0, stream, p);
            for (int q = 0; q < 6; ++q) c[q] = 0u;
            g.rverdict[(uint64_t)stream * g.n_props + p] = (uint8_t)valuate(g.plan->prop[p], 0, c);
        }
    }
}

// The live quantifier nodes of one level (>= 1), in table order: key (the
// packed stream id and key prefix), 6-bin counts and verdict per property.
__global__ __launch_bounds__(256) void k_group_nodes(GroupState g, uint32_t level, uint64_t* keys, uint32_t* counts,
                                                     uint8_t* verdict, uint64_t capacity, uint64_t* n_out) {
    const int lane = threadIdx.x & 63;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base <= g.nmask; base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = base + threadIdx.x;
        const uint64_t k = j <= g.nmask ? g.nkeys[level][j] : kEmptyKey;
        const bool live = k < kDeadKey && g.nverdict[level][j] != kNoVerdict;
        const uint64_t m = __ballot(live);
        if (m == 0) continue;
        const int leader = __ffsll((unsigned long long)m) - 1;
        unsigned long long at = 0;
        if (lane == leader) at = atomicAdd(reinterpret_cast<unsigned long long*>(n_out), (unsigned long long)__popcll(m));
        at = __shfl(at, leader, 64);
        if (!live) continue;
        const uint64_t o = at + (uint64_t)__popcll(m & ((1ull << lane) - 1ull));
        if (o >= capacity) {
            atomicOr(g.err, kErrCapacity);
            continue;
        }
        keys[o] = k;
        for (uint32_t p = 0; p < g.n_props; ++p) {
            const uint32_t* c = counts_of(g, level, (uint32_t)j, p);
            for (int q = 0; q < 6; ++q) counts[((uint64_t)p * capacity + o) * 6 + q] = c[q];
            verdict[(uint64_t)p * capacity + o] = g.nverdict[level][(uint64_t)p * (g.nmask + 1) + j];
        }
    }
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

__global__ __launch_bounds__(64) void k_put_words(uint32_t* dst, PutWords a) {
    for (uint32_t i = threadIdx.x; i < a.n; i += blockDim.x) dst[i] = a.w[i];
}

// One thread per trace of a batch.
__global__ __launch_bounds__(256) void k_batch_out(BatchOutArgs a) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_traces) return;
    const uint32_t nn = min<uint64_t>(*a.n_nodes, a.stride);
    uint32_t lo = 0, hi = nn;                 // first node with key >= t
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.node_keys[mid] < t) lo = mid + 1; else hi = mid;
    }
    const bool has = lo < nn && a.node_keys[lo] == t;
    const uint32_t zero[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t p = 0; p < a.n_props; ++p) {
        const uint32_t* c = has ? a.node_counts + ((uint64_t)p * a.stride + lo) * 6 : zero;
        a.verdict[(uint64_t)t * a.n_props + p] =
            has ? a.node_verdict[(uint64_t)p * a.stride + lo] : (uint8_t)valuate(a.plan->prop[p], 1, zero);
        for (int b = 0; b < 6; ++b) a.counts[((uint64_t)t * a.n_props + p) * 6 + b] = c[b];
    }
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_u8(uint8_t* p, uint64_t n, uint8_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_zero(const ZeroArgs& a, uint32_t blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int RDW, bool GROUP>
static void launch_classify_t(const ClassifyArgs& a, uint32_t blocks, hipStream_t s) {
    if (a.n_preds > 0) hipLaunchKernelGGL((k_classify<RDW, GROUP, true, 0>), dim3(blocks), dim3(1024), 0, s, a);
    else if (RDW == 4 && !GROUP && a.n_keys == 2) hipLaunchKernelGGL((k_classify<RDW, GROUP, false, 2>), dim3(blocks), dim3(1024), 0, s, a);
    else if (RDW == 4 && !GROUP && a.n_keys == 1) hipLaunchKernelGGL((k_classify<RDW, GROUP, false, 1>), dim3(blocks), dim3(1024), 0, s, a);
    else hipLaunchKernelGGL((k_classify<RDW, GROUP, false, 0>), dim3(blocks), dim3(1024), 0, s, a);
}

hipError_t launch_classify(const ClassifyArgs& a, hipStream_t s) {
    const uint64_t want = (a.n + 1023) / 1024;
    const uint32_t blocks = (uint32_t)(want < 512 ? (want ? want : 1) : 512);
    const bool group = a.chunk_off != nullptr;
    if (a.record_bytes == 16 && (reinterpret_cast<uintptr_t>(a.records) & 15) == 0 && a.vec_ok) {
        if (group) launch_classify_t<4, true>(a, blocks, s);
        else launch_classify_t<4, false>(a, blocks, s);
    } else if (a.record_bytes == 12) {
        if (group) launch_classify_t<3, true>(a, blocks, s);
        else launch_classify_t<3, false>(a, blocks, s);
    } else {
        if (group) launch_classify_t<0, true>(a, blocks, s);
        else launch_classify_t<0, false>(a, blocks, s);
    }
    return hipGetLastError();
}

uint32_t sort_tile(int variant) {
    switch (variant) {
        case 1: return 512 * 16;
        case 2: return 256 * 24;
        case 3: return 256 * 8;
        case 4: return 512 * 8;
        case 5: return 512 * 12;
        case 6: return 1024 * 16;
        default: return 256 * 16;
    }
}

uint32_t sort_threads(int variant) { return variant == 6 ? 1024u : variant == 1 || variant == 4 || variant == 5 ? 512u : 256u; }

hipError_t launch_sort_pass(const SortPassArgs& a, int variant, uint32_t digit_bits, hipStream_t s) {
    const uint32_t tile = sort_tile(variant);
    const uint32_t tiles = (a.n + tile - 1) / tile;
    if (digit_bits == 9) {
        switch (variant) {
            case 1: hipLaunchKernelGGL((k_sort_pass<512, 16, 9>), dim3(tiles), dim3(512), 0, s, a); break;
            case 4: hipLaunchKernelGGL((k_sort_pass<512, 8, 9>), dim3(tiles), dim3(512), 0, s, a); break;
            case 5: hipLaunchKernelGGL((k_sort_pass<512, 12, 9>), dim3(tiles), dim3(512), 0, s, a); break;
            case 6: hipLaunchKernelGGL((k_sort_pass<1024, 16, 9>), dim3(tiles), dim3(1024), 0, s, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (digit_bits != 8) return hipErrorInvalidValue;
    switch (variant) {
        case 1: hipLaunchKernelGGL((k_sort_pass<512, 16, 8>), dim3(tiles), dim3(512), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_sort_pass<256, 24, 8>), dim3(tiles), dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_sort_pass<256, 8, 8>), dim3(tiles), dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_sort_pass<512, 8, 8>), dim3(tiles), dim3(512), 0, s, a); break;
        case 5: hipLaunchKernelGGL((k_sort_pass<512, 12, 8>), dim3(tiles), dim3(512), 0, s, a); break;
        case 6: hipLaunchKernelGGL((k_sort_pass<1024, 16, 8>), dim3(tiles), dim3(1024), 0, s, a); break;
        default: hipLaunchKernelGGL((k_sort_pass<256, 16, 8>), dim3(tiles), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

template <int T>
static void launch_scan_t(const ScanArgs& a, hipStream_t s) {
    const uint32_t tiles = (a.n + T * kScanItems - 1) / (T * kScanItems);
    if (a.max_states <= 8) {
        if (a.n_props <= 1)
            hipLaunchKernelGGL((k_scan<1, 2, T>), dim3(tiles), dim3(T), 0, s, a);
        else if (a.n_props <= 2)
            hipLaunchKernelGGL((k_scan<2, 2, T>), dim3(tiles), dim3(T), 0, s, a);
        else if (a.n_props <= 4)
            hipLaunchKernelGGL((k_scan<4, 2, T>), dim3(tiles), dim3(T), 0, s, a);
        else
            hipLaunchKernelGGL((k_scan<8, 2, T>), dim3(tiles), dim3(T), 0, s, a);
    } else {
        if (a.n_props <= 1)
            hipLaunchKernelGGL((k_scan<1, 4, T>), dim3(tiles), dim3(T), 0, s, a);
        else if (a.n_props <= 2)
            hipLaunchKernelGGL((k_scan<2, 4, T>), dim3(tiles), dim3(T), 0, s, a);
        else
            hipLaunchKernelGGL((k_scan<4, 4, T>), dim3(tiles), dim3(T), 0, s, a);
    }
}

// Variant 3 picks per launch: 1024-thread tiles for launches whose maps take
// at most 4 dwords per event (fewer tiles, a shorter look-back chain), 512
// otherwise.  Workspace is sized for the smaller tile.
uint32_t scan_tile(int variant) { return (variant == 2 ? 1024u : variant == 0 ? 256u : 512u) * kScanItems; }

hipError_t launch_scan(const ScanArgs& a, int variant, hipStream_t s) {
    if (a.n_props < 1 || a.n_props > (a.max_states <= 8 ? 8u : 4u) || (a.structure && a.n_props > 4))
        return hipErrorInvalidValue;
    if (variant >= 3) {     // per launch (the split scan's look-back fallback too)
        const uint32_t mw = a.max_states <= 8 ? 2u : 4u;
        const uint32_t pmax = a.n_props <= 1 ? 1u : a.n_props <= 2 ? 2u : a.n_props <= 4 ? 4u : 8u;
        variant = mw * pmax <= 4 ? 2 : 1;
    }
    if (variant == 2) launch_scan_t<1024>(a, s);
    else if (variant == 1) launch_scan_t<512>(a, s);
    else launch_scan_t<256>(a, s);
    return hipGetLastError();
}

hipError_t launch_count(const CountArgs& a, hipStream_t s) {
    // the root level takes one child per thread: more blocks in flight
    const uint32_t items = a.items >= 16 ? 16 : a.level == 0 ? 1 : 2;
    const uint64_t tile = (uint64_t)kCountThreads * items;
    const uint64_t want = (a.child_limit + tile - 1) / tile;
    const uint32_t blocks = (uint32_t)(want < 2048 ? (want ? want : 1) : 2048);
    if (items == 16)
        hipLaunchKernelGGL(k_count_leaves, dim3(blocks), dim3(kCountThreads), 0, s, a);
    else if (items == 1)
        hipLaunchKernelGGL(k_count<1>, dim3(blocks), dim3(kCountThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_count<2>, dim3(blocks), dim3(kCountThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, uint64_t n, hipStream_t s) {
    const uint64_t want = (n / 16 + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 2048 ? (want ? want : 1) : 2048);
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_inst_conclusive(const InstConclusiveArgs& a, hipStream_t s) {
    const uint64_t want = (a.inst_limit + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 2048 ? (want ? want : 1) : 2048);
    hipLaunchKernelGGL(k_inst_conclusive, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace ltl4c

namespace ltl4c {

hipError_t launch_group_update(const GroupUpdateArgs& a, uint64_t max_seg, hipStream_t s) {
    const uint64_t want = (max_seg + 255) / 256;
    const uint32_t blocks = (uint32_t)(want < 2048 ? (want ? want : 1) : 2048);
    hipLaunchKernelGGL(k_group_update, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_group_level(const GroupState& g, uint32_t level, hipStream_t s) {
    hipLaunchKernelGGL(k_group_level, dim3(512), dim3(256), 0, s, g, level);
    return hipGetLastError();
}

hipError_t launch_group_roots(const GroupState& g, bool all, hipStream_t s) {
    hipLaunchKernelGGL(k_group_roots, dim3(64), dim3(256), 0, s, g, all ? 1u : 0u);
    return hipGetLastError();
}

hipError_t launch_group_read(const GroupState& g, uint8_t* verdict, uint64_t* counts, uint64_t* bindings,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_group_read, dim3(64), dim3(256), 0, s, g, verdict, counts, bindings);
    return hipGetLastError();
}

hipError_t launch_group_purge(const GroupState& g, uint32_t stream, hipStream_t s) {
    hipLaunchKernelGGL(k_group_purge, dim3(512), dim3(256), 0, s, g, stream);
    return hipGetLastError();
}

hipError_t launch_group_nodes(const GroupState& g, uint32_t level, uint64_t* keys, uint32_t* counts, uint8_t* verdict,
                              uint64_t capacity, uint64_t* n_out, hipStream_t s) {
    hipLaunchKernelGGL(k_group_nodes, dim3(512), dim3(256), 0, s, g, level, keys, counts, verdict, capacity, n_out);
    return hipGetLastError();
}

hipError_t launch_put_words(uint32_t* dst, const PutWords& a, hipStream_t s) {
    hipLaunchKernelGGL(k_put_words, dim3(1), dim3(64), 0, s, dst, a);
    return hipGetLastError();
}

hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u8, dim3(1024), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace ltl4c

namespace ltl4c {

hipError_t launch_batch_out(const BatchOutArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_out, dim3((a.n_traces + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ltl4c
