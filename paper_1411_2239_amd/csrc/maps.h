// Transition maps of LTL4 monitors as packed bytes (see the comment below),
// shared by the map-scan kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ltl4c {

// Maps over at most 8 (MW = 2) or 16 (MW = 4) states: MW dwords whose byte q
// holds the image of state q.  The composition g∘f (f applied first) picks,
// for every byte of f, the byte of g it names: one byte permute per dword for
// 8 states; for 16 states two permutes (the low and the high half of g) and a
// third that picks per byte on bit 3 of the selector.  No constant-map
// special cases are needed.
template <int MW>
struct BMap {
    uint32_t d[MW];
};

template <int MW>
__device__ __forceinline__ BMap<MW> bm_identity() {
    BMap<MW> r;
#pragma unroll
    for (int i = 0; i < MW; ++i) r.d[i] = 0x03020100u + 0x04040404u * (uint32_t)i;
    return r;
}
template <int MW>
__device__ __forceinline__ BMap<MW> bm_const(uint32_t s) {
    BMap<MW> r;
#pragma unroll
    for (int i = 0; i < MW; ++i) r.d[i] = s * 0x01010101u;
    return r;
}
template <int MW>
__device__ __forceinline__ BMap<MW> bm_compose(const BMap<MW>& g, const BMap<MW>& f) {
    BMap<MW> r;
#pragma unroll
    for (int i = 0; i < MW; ++i) {
        if constexpr (MW == 2) {
            r.d[i] = __builtin_amdgcn_perm(g.d[1], g.d[0], f.d[i]);
        } else {
            // lo is right in the bytes whose state is below 8, hi (selector
            // bytes 8..15 turned into 0..7) in the others; a third permute picks
            // byte k of lo, or byte k of hi (pair index k + 4) where bit 3 of the
            // state is set.  All full-rate instructions (a byte mask built as
            // t * 255 compiles to a quarter-rate multiply).
            const uint32_t sel = f.d[i];
            const uint32_t lo = __builtin_amdgcn_perm(g.d[1], g.d[0], sel);
            const uint32_t hi = __builtin_amdgcn_perm(g.d[3], g.d[2], sel ^ 0x08080808u);
            const uint32_t pick = ((sel >> 1) & 0x04040404u) | 0x03020100u;
            r.d[i] = __builtin_amdgcn_perm(hi, lo, pick);
        }
    }
    return r;
}
template <int MW>
__device__ __forceinline__ uint32_t bm_at(const BMap<MW>& g, uint32_t q) {
    if constexpr (MW == 2) {
        return __builtin_amdgcn_perm(g.d[1], g.d[0], q) & 0xFFu;
    } else {
        const uint32_t lo = __builtin_amdgcn_perm(g.d[1], g.d[0], q & 7u);
        const uint32_t hi = __builtin_amdgcn_perm(g.d[3], g.d[2], q & 7u);
        return ((q & 8u) ? hi : lo) & 0xFFu;
    }
}
// Wave-wide inclusive scans with DPP row operations (GFX9 DPP controls:
// row_shr:n = 0x110 + n within rows of 16 lanes, row_bcast:15 = 0x142 sends
// lane 15 of a row to the next row, row_bcast:31 = 0x143 sends lane 31 to rows
// 2 and 3, wave_shr:1 = 0x138).  A lane whose source is outside its row, or
// whose row the row mask leaves out, keeps `old`: the operation's identity.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, CTRL, ROW_MASK, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    v += dpp_mov<0x111, 0xF>(0u, v);
    v += dpp_mov<0x112, 0xF>(0u, v);
    v += dpp_mov<0x114, 0xF>(0u, v);
    v += dpp_mov<0x118, 0xF>(0u, v);
    v += dpp_mov<0x142, 0xA>(0u, v);
    v += dpp_mov<0x143, 0xC>(0u, v);
    return v;
}

template <int MW, int CTRL, int ROW_MASK>
__device__ __forceinline__ BMap<MW> bm_dpp(const BMap<MW>& v) {
    const BMap<MW> id = bm_identity<MW>();
    BMap<MW> r;
#pragma unroll
    for (int i = 0; i < MW; ++i) r.d[i] = dpp_mov<CTRL, ROW_MASK>(id.d[i], v.d[i]);
    return r;
}

// inclusive scan of maps in lane order (a later lane's map applies after)
template <int MW>
__device__ __forceinline__ BMap<MW> bm_wave_incl_scan(BMap<MW> v) {
    v = bm_compose<MW>(v, bm_dpp<MW, 0x111, 0xF>(v));
    v = bm_compose<MW>(v, bm_dpp<MW, 0x112, 0xF>(v));
    v = bm_compose<MW>(v, bm_dpp<MW, 0x114, 0xF>(v));
    v = bm_compose<MW>(v, bm_dpp<MW, 0x118, 0xF>(v));
    v = bm_compose<MW>(v, bm_dpp<MW, 0x142, 0xA>(v));
    v = bm_compose<MW>(v, bm_dpp<MW, 0x143, 0xC>(v));
    return v;
}

// the previous lane's value (lane 0: the identity map)
template <int MW>
__device__ __forceinline__ BMap<MW> bm_wave_shr1(const BMap<MW>& v) {
    return bm_dpp<MW, 0x138, 0xF>(v);
}

template <int MW>
__device__ __forceinline__ BMap<MW> bm_shfl_up(const BMap<MW>& v, int off) {
    BMap<MW> r;
#pragma unroll
    for (int i = 0; i < MW; ++i) r.d[i] = __shfl_up(v.d[i], off, 64);
    return r;
}
template <int MW>
__device__ __forceinline__ BMap<MW> bm_shfl_down(const BMap<MW>& v, int off) {
    BMap<MW> r;
#pragma unroll
    for (int i = 0; i < MW; ++i) r.d[i] = __shfl_down(v.d[i], off, 64);
    return r;
}
template <int MW>
__device__ __forceinline__ BMap<MW> bm_bcast(const BMap<MW>& v, int src) {
    BMap<MW> r;
#pragma unroll
    for (int i = 0; i < MW; ++i) r.d[i] = __shfl(v.d[i], src, 64);
    return r;
}
template <int MW>
__device__ __forceinline__ BMap<MW> bm_load(const uint32_t* p) {
    BMap<MW> r;
#pragma unroll
    for (int i = 0; i < MW; ++i) r.d[i] = p[i];
    return r;
}

}  // namespace ltl4c
