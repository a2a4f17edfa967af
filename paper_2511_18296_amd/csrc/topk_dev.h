// topk_dev.h -- device helpers of exact top-k selection shared by the
// single-array top-k (topk.hip) and the per-model segmented top-k of the
// batched kernel (batch.hip): the order-preserving 64-bit item key, the
// wave-aggregated append and the parallel boundary-digit search.
#pragma once
#include <float.h>
#include <math.h>

#include "internal.h"

namespace mps {

__device__ __forceinline__ uint32_t ord_f32(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float unord_f32(uint32_t o) {
    const uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}

// Key of an item with the given score and flags; false if it does not
// qualify (flags filter, NaN score).
__device__ __forceinline__ bool key_from(float score, uint8_t f, int64_t i, uint8_t req,
                                         uint8_t forbid, uint64_t &key) {
    // -0 + +0 = +0: both zeros compare equal, as in IEEE comparison
    const float s = score + 0.0f;
    if ((f & req) != req || (f & forbid) != 0 || isnan(s)) return false;
    key = ((uint64_t)ord_f32(s) << 32) | (uint64_t)(0xffffffffu - (uint32_t)i);
    return true;
}

__device__ __forceinline__ bool item_key(const float *score, const uint8_t *flags, int64_t i,
                                         uint8_t req, uint8_t forbid, uint64_t &key) {
    return key_from(score[i], flags[i], i, req, forbid, key);
}

// Append `key` where pred holds: one atomic per wave, positions by prefix
// popcount (the order inside the buffer is irrelevant: keys are sorted last).
// Every lane of the wave must call it.
__device__ __forceinline__ void wave_append(bool pred, uint64_t key, uint64_t *buf,
                                            int32_t *cnt) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (int32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (pred) {
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        buf[base + (int32_t)__popcll(mask & below)] = key;
    }
}

// The digit at which the running count from the top bin reaches k_rem, in an
// LDS histogram h of nb bins (nb a multiple of 256).  res = {digit or -1,
// count strictly above it, total}.  Called by every thread of the block
// (blockDim a multiple of 64, at least 256): threads 0..255 own slices of
// nb/256 bins counted from the top, a wave-level inclusive scan plus the
// four wave totals give each slice its running count, and the one slice
// whose range contains k_rem walks its bins.
__device__ inline void select_digit(const uint32_t *h, int nb, int32_t k_rem, uint32_t *part,
                             int32_t *res) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int per = nb >> 8;
    uint32_t c = 0;
    if (tid < 256)
        for (int j = 0; j < per; ++j) c += h[nb - 1 - (tid * per + j)];
    uint32_t x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (tid < 256 && lane == 63) part[tid >> 6] = x;
    if (tid == 0) {
        res[0] = -1;
        res[1] = 0;
    }
    __syncthreads();
    if (tid < 256) {
        uint32_t off = 0;
        for (int w = 0; w < (tid >> 6); ++w) off += part[w];
        const uint32_t incl = x + off, excl = incl - c;
        if (excl < (uint32_t)k_rem && (uint32_t)k_rem <= incl) {
            uint32_t r = excl;
            for (int j = 0; j < per; ++j) {
                const int bin = nb - 1 - (tid * per + j);
                if (r + h[bin] >= (uint32_t)k_rem) {
                    res[0] = bin;
                    res[1] = (int32_t)r;
                    break;
                }
                r += h[bin];
            }
        }
        if (tid == 255) res[2] = (int32_t)incl;
    }
    __syncthreads();
}

}  // namespace mps
