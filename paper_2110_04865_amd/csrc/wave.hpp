// Wave64 and workgroup primitives for gfx950, plus the single-pass
// decoupled look-back prefix used by every order-preserving compaction
// (Merrill and Garland, "Single-pass Parallel Prefix Scan with Decoupled
// Look-back", NVIDIA tech report NVR-2016-002; restated for 64-lane waves).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msf {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// ---- DPP lane moves (GFX9 encodings; no LDS traffic) -----------------------
// row_shr:n = 0x110 + n (within rows of 16 lanes), row_bcast:15 = 0x142 (lane
// 15 of a row to the next row), row_bcast:31 = 0x143 (lane 31 to rows 2-3),
// wave_shl:1 = 0x130 (lane l reads l+1), wave_shr:1 = 0x138 (lane l reads
// l-1).  Lanes without a source, or in rows outside ROW_MASK, read `old`.
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114,
              DPP_ROW_SHR8 = 0x118, DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143,
              DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v, uint32_t old = 0)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v, uint64_t old = 0)
{
    const uint32_t lo = dpp_u32<CTRL, ROW_MASK>((uint32_t)v, (uint32_t)old);
    const uint32_t hi = dpp_u32<CTRL, ROW_MASK>((uint32_t)(v >> 32), (uint32_t)(old >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The same for any 4- or 8-byte type (bits moved unchanged).
template <int CTRL, int ROW_MASK = 0xF, typename T>
__device__ __forceinline__ T dpp_move(T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte lanes only");
    T r;
    if constexpr (sizeof(T) == 4) {
        uint32_t u;
        __builtin_memcpy(&u, &v, 4);
        u = dpp_u32<CTRL, ROW_MASK>(u);
        __builtin_memcpy(&r, &u, 4);
    } else {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        u = dpp_u64<CTRL, ROW_MASK>(u);
        __builtin_memcpy(&r, &u, 8);
    }
    return r;
}

// Inclusive prefix sum over the 64 lanes (all lanes active): Hillis-Steele
// inside each row of 16, then the row totals carried by row broadcasts.
template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v)
{
    v += dpp_move<DPP_ROW_SHR1>(v);
    v += dpp_move<DPP_ROW_SHR2>(v);
    v += dpp_move<DPP_ROW_SHR4>(v);
    v += dpp_move<DPP_ROW_SHR8>(v);
    v += dpp_move<DPP_ROW_BCAST15, 0xA>(v);
    v += dpp_move<DPP_ROW_BCAST31, 0xC>(v);
    return v;
}

// Lane 63's value, in every lane.
template <typename T>
__device__ __forceinline__ T lane63(T v)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte lanes only");
    T r;
    if constexpr (sizeof(T) == 4) {
        uint32_t u;
        __builtin_memcpy(&u, &v, 4);
        u = (uint32_t)__builtin_amdgcn_readlane((int)u, 63);
        __builtin_memcpy(&r, &u, 4);
    } else {
        uint64_t u;
        __builtin_memcpy(&u, &v, 8);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
        u = ((uint64_t)hi << 32) | lo;
        __builtin_memcpy(&r, &u, 8);
    }
    return r;
}

// Sum over the 64 lanes, in every lane (all lanes active).
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    return lane63(wave_incl_sum(v));
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint64_t o = __shfl_xor(v, d, 64);
        v = o < v ? o : v;
    }
    return v;
}

// Exclusive prefix sum over a workgroup of NT threads (NT/64 waves).
// Returns this thread's exclusive prefix; *total receives the block sum.
// `lds` must hold NT/64 + 1 elements.  Contains __syncthreads().
template <int NT, typename T>
__device__ __forceinline__ T block_excl_sum(T v, T *lds, T *total)
{
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6;
    T inc = wave_incl_sum(v);
    if (__lane_id() == 63) lds[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T s = 0;
        for (int i = 0; i < NW; ++i) {
            T t = lds[i];
            lds[i] = s;
            s += t;
        }
        lds[NW] = s;
    }
    __syncthreads();
    T r = lds[w] + inc - v;
    *total = lds[NW];
    __syncthreads();  // lds may be reused right after
    return r;
}

// ---- decoupled look-back ---------------------------------------------------
// status[t] = flag << 62 | value; flag 1 = tile aggregate, 2 = inclusive
// prefix.  The status array must be zero before the launch, and tiles must
// be numbered in the order they start (take them from an atomic ticket), so
// a tile only ever waits on tiles that are already running or done.

constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_PRE = 2ull << 62;
constexpr uint64_t LB_VAL = (1ull << 62) - 1ull;

__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by all 64 lanes of ONE wave.  Returns the exclusive prefix of
// `tile` (identical in every lane) and publishes its inclusive prefix.
__device__ __forceinline__ uint64_t lookback(uint64_t *status, uint32_t tile, uint64_t agg)
{
    const int lane = __lane_id();
    if (tile == 0) {
        if (lane == 0) lb_store(status, LB_PRE | agg);
        return 0;
    }
    if (lane == 0) lb_store(status + tile, LB_AGG | agg);
    uint64_t excl = 0;
    int64_t base = (int64_t)tile - 1;
    for (;;) {
        const int64_t t = base - lane;
        uint64_t s = LB_PRE;  // virtual tile before 0: prefix 0
        if (t >= 0) s = __hip_atomic_load(status + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t flag = (uint32_t)(s >> 62);
        const uint64_t pmask = __ballot(flag == 2u);
        const uint64_t zmask = __ballot(flag == 0u);
        const int first = pmask ? (int)__builtin_ctzll(pmask) : 64;
        const uint64_t need = (first >= 63) ? ~0ull : ((2ull << first) - 1ull);
        if (zmask & need) {
            __builtin_amdgcn_s_sleep(1);
            continue;  // a needed predecessor has not published yet
        }
        uint64_t v = (lane <= first) ? (s & LB_VAL) : 0ull;
        excl += wave_sum(v);
        if (first < 64) break;
        base -= 64;
    }
    if (lane == 0) lb_store(status + tile, LB_PRE | (excl + agg));
    return excl;
}

// ---- ordered compaction of a tile into up to two lists ---------------------
// Every thread of an NT-thread block passes its counts (ca, cb) of items
// going to lists a and b.  Returns this thread's first output index in each
// list; *total receives the running totals (a << 31 | b) after this tile.
// Tile ids come from an atomic ticket (see lookback).  `lds` holds NT/64+1
// u64; `s_pre` one u64.  Contains __syncthreads().
template <int NT>
__device__ __forceinline__ void tile_offsets2(uint32_t tile, uint32_t ca, uint32_t cb,
                                              uint64_t *status, uint64_t *lds, uint64_t *s_pre,
                                              uint32_t *oa, uint32_t *ob, uint64_t *total)
{
    constexpr uint64_t M31 = (1ull << 31) - 1ull;
    const uint64_t mine = ((uint64_t)ca << 31) | (uint64_t)cb;
    uint64_t btot;
    const uint64_t ex = block_excl_sum<NT>(mine, lds, &btot);
    if (threadIdx.x < 64) {
        const uint64_t pre = lookback(status, tile, btot);
        if (threadIdx.x == 0) *s_pre = pre;
    }
    __syncthreads();
    const uint64_t pre = *s_pre;
    *oa = (uint32_t)((pre >> 31) + (ex >> 31));
    *ob = (uint32_t)((pre & M31) + (ex & M31));
    *total = pre + btot;
}

// Block-wide sum (all threads get it).  `lds` holds NT/64+1 elements.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T *lds)
{
    T tot;
    block_excl_sum<NT>(v, lds, &tot);
    return tot;
}

}  // namespace msf
