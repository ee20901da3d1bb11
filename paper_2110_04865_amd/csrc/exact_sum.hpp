// Exact forest weights.
//
// The paper's algorithm returns the sum of the weights of the edges that
// hook (Algorithm 2).  For uint32 weights that sum is an exact u64.  For
// float32 weights the result is the exact real sum rounded once to the
// nearest double (ties to even), which does not depend on the order of the
// additions: every float32 is an integer multiple of 2^-149 (the smallest
// subnormal), so each weight is added exactly into signed 32-bit digits of
// a fixed-point number, and the digits are rounded once at the end.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msf.h"
#include "wave.hpp"

namespace msf {

constexpr int ACC_DIGITS = 10;  // 320 bits: 2^-149 .. beyond 2^128 (float max) x 2^31 terms

struct WSum {
    uint64_t su = 0;
    int64_t acc[ACC_DIGITS] = {};
    uint32_t pinf = 0, ninf = 0;
};

// Add one float32 weight given by its raw bits.
__device__ __forceinline__ void wsum_add_bits(WSum &ws, uint32_t b)
{
    const uint32_t ex = (b >> 23) & 0xFFu;
    const bool neg = (b >> 31) != 0;
    if (ex == 0xFFu) {
        if (neg) ++ws.ninf;
        else ++ws.pinf;
        return;
    }
    const uint64_t mant = ex ? ((b & 0x7FFFFFu) | 0x800000u) : (b & 0x7FFFFFu);
    const uint32_t sh = ex ? ex - 1u : 0u;  // value = mant * 2^(sh-149)
    const uint64_t x = mant << (sh & 31u);
    const uint32_t di = sh >> 5;
    const int64_t lo = (int64_t)(x & 0xFFFFFFFFull), hi = (int64_t)(x >> 32);
#pragma unroll
    for (int d = 0; d < ACC_DIGITS; ++d) {
        const int64_t add = (d == (int)di) ? lo : ((d == (int)di + 1) ? hi : 0);
        ws.acc[d] += neg ? -add : add;
    }
}

// Add one weight given by its order-preserving key (the high word of an
// edge key): uint32 weights are their own key; for float32 the map is
// undone (keys >= 2^31 were non-negative floats).
template <int WT>
__device__ __forceinline__ void wsum_add(WSum &ws, uint32_t wkey)
{
    if (WT == MSF_W_U32) {
        ws.su += wkey;
        return;
    }
    wsum_add_bits(ws, (wkey & 0x80000000u) ? (wkey & 0x7FFFFFFFu) : ~wkey);
}

// Workgroup sum of every thread's WSum into out[j * stride], j < WS_WORDS
// (thread 0 writes: u64 sum, ACC_DIGITS digits, +inf and -inf counts).
// `lds` holds (NT/64) * (ACC_DIGITS + 1) int64; contains __syncthreads().
constexpr int WS_WORDS = ACC_DIGITS + 3;

template <int NT, int WT>
__device__ __forceinline__ void wsum_block(WSum &ws, int64_t *lds, int64_t *out, uint32_t stride)
{
    constexpr int W = ACC_DIGITS + 1;
    const int wv = threadIdx.x >> 6;
    if (WT == MSF_W_U32) {
        const uint64_t v = wave_sum(ws.su);
        if (__lane_id() == 0) lds[wv * W] = (int64_t)v;
    } else {
        // a weight touches two adjacent digits: reduce only digits some
        // lane uses (the ballot is uniform across the wave)
#pragma unroll
        for (int d = 0; d < ACC_DIGITS; ++d) {
            const int64_t v = __ballot(ws.acc[d] != 0) ? wave_sum(ws.acc[d]) : 0;
            if (__lane_id() == 0) lds[wv * W + d] = v;
        }
        const uint32_t pi = __ballot(ws.pinf != 0) ? wave_sum(ws.pinf) : 0u;
        const uint32_t ni = __ballot(ws.ninf != 0) ? wave_sum(ws.ninf) : 0u;
        if (__lane_id() == 0) lds[wv * W + ACC_DIGITS] = ((int64_t)pi << 32) | ni;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    int64_t o[WS_WORDS] = {};
    for (int i = 0; i < NT / 64; ++i) {
        if (WT == MSF_W_U32) {
            o[0] += lds[i * W];
        } else {
            for (int d = 0; d < ACC_DIGITS; ++d) o[1 + d] += lds[i * W + d];
            o[1 + ACC_DIGITS] += (int64_t)(uint32_t)(lds[i * W + ACC_DIGITS] >> 32);
            o[2 + ACC_DIGITS] += lds[i * W + ACC_DIGITS] & 0xFFFFFFFFll;
        }
    }
    for (int j = 0; j < WS_WORDS; ++j) out[(size_t)j * stride] = o[j];
}

// The total as a double: for uint32 weights the u64 sum converted (correctly
// rounded); for float32 the signed digits carried into a two's-complement
// number of ACC_DIGITS*32 bits and rounded once to nearest, ties to even;
// NaN if both infinities occur, else the infinity that occurs.
__device__ inline double exact_total_f64(uint64_t su, const int64_t *acc, uint32_t pinf,
                                         uint32_t ninf, int wt)
{
    if (wt == MSF_W_U32) return (double)su;
    if (pinf || ninf)
        return (pinf && ninf) ? __builtin_nan("") : (pinf ? __builtin_inf() : -__builtin_inf());
    uint32_t dig[ACC_DIGITS];
    int64_t carry = 0;
    for (int d = 0; d < ACC_DIGITS; ++d) {
        const int64_t v = acc[d] + carry;
        dig[d] = (uint32_t)(v & 0xFFFFFFFFll);
        carry = v >> 32;  // arithmetic shift: floor division
    }
    const bool neg = carry < 0;
    if (neg) {
        uint64_t c1 = 1;
        for (int d = 0; d < ACC_DIGITS; ++d) {
            const uint64_t v = (uint64_t)(uint32_t)~dig[d] + c1;
            dig[d] = (uint32_t)v;
            c1 = v >> 32;
        }
    }
    int top = -1;
    for (int d = ACC_DIGITS - 1; d >= 0 && top < 0; --d)
        if (dig[d]) top = d * 32 + 31 - __builtin_clz(dig[d]);
    double out = 0.0;
    if (top >= 0) {
        auto bit = [&](int i) -> uint32_t { return i < 0 ? 0u : (dig[i >> 5] >> (i & 31)) & 1u; };
        uint64_t q = 0;
        const int lo = top - 52;  // lowest kept bit
        int scale = lo;           // value = q * 2^(scale - 149)
        if (lo < 0) {
            scale = 0;
            for (int i = top; i >= 0; --i) q = (q << 1) | bit(i);
        } else {
            for (int i = top; i >= lo; --i) q = (q << 1) | bit(i);
            const uint32_t rb = bit(lo - 1);
            uint32_t sticky = 0;
            for (int i = lo - 2; i >= 0 && !sticky; --i) sticky |= bit(i);
            if (rb && (sticky || (q & 1u))) {
                ++q;
                if (q == (1ull << 53)) {
                    q >>= 1;
                    ++scale;
                }
            }
        }
        out = ldexp((double)q, scale - 149);
    }
    return neg ? -out : out;
}

}  // namespace msf
