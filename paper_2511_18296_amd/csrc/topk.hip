// topk.hip -- exact top-k of scored moves (the per-thread-block argmax
// reduction of Alg. 5, generalised to the k best moves and made
// deterministic: no floating-point atomics, a total order on items).
//
// Each qualifying item i gets the 64-bit key
//   key = ord(score) << 32 | (0xffffffff - i)
// where ord maps floats to unsigned integers monotonically.  Keys are unique
// and "larger key" = "better item" (higher score, then smaller index), so the
// top k items are the k largest keys.  A most-significant-digit radix select
// (digits of 11/11/10 bits per 32-bit half) finds them with integer
// histograms; survivors of each level are compacted; the final k keys are
// sorted in LDS with a bitonic network.
#include <float.h>
#include <math.h>

#include "internal.h"

namespace mps {

constexpr int kBins = 2048;
constexpr int kLevels = 6;
__constant__ int c_shift[kLevels] = {53, 42, 32, 21, 10, 0};
__constant__ int c_bits[kLevels] = {11, 11, 10, 11, 11, 10};

struct TopkCtrl {
    uint64_t pad0;
    int32_t k_rem;      // how many keys are still to be chosen
    int32_t n_out;      // keys chosen so far (in out[])
    int32_t n_cand[2];  // survivors per ping-pong buffer
    int32_t sel;        // selected digit of the current level
    int32_t take_all;   // every survivor of the level qualifies
    int32_t pad1[2];
};

struct TopkWs {
    TopkCtrl *ctrl;
    uint32_t *hist;   // [kBins]
    uint64_t *out;    // [k]
    uint64_t *cand0;  // [n]
    uint64_t *cand1;  // [n]
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t topk_ws_bytes(int64_t n, int32_t k) {
    size_t nn = n > 0 ? (size_t)n : 1;
    return a256(sizeof(TopkCtrl)) + a256(sizeof(uint32_t) * kBins) +
           a256(sizeof(uint64_t) * (size_t)k) + 2 * a256(sizeof(uint64_t) * nn);
}

static TopkWs carve_ws(void *ws, int64_t n, int32_t k) {
    char *p = (char *)ws;
    size_t nn = n > 0 ? (size_t)n : 1;
    TopkWs w;
    w.ctrl = (TopkCtrl *)p;
    p += a256(sizeof(TopkCtrl));
    w.hist = (uint32_t *)p;
    p += a256(sizeof(uint32_t) * kBins);
    w.out = (uint64_t *)p;
    p += a256(sizeof(uint64_t) * (size_t)k);
    w.cand0 = (uint64_t *)p;
    p += a256(sizeof(uint64_t) * nn);
    w.cand1 = (uint64_t *)p;
    return w;
}

__device__ __forceinline__ uint32_t ord_f32(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float unord_f32(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(u);
}

__device__ __forceinline__ bool item_key(const float *score, const uint8_t *flags, int64_t i,
                                         uint8_t req, uint8_t forbid, uint64_t &key) {
    const uint8_t f = flags[i];
    // -0 + +0 = +0: both zeros compare equal, as in IEEE comparison
    const float s = score[i] + 0.0f;
    if ((f & req) != req || (f & forbid) != 0 || isnan(s)) return false;
    key = ((uint64_t)ord_f32(s) << 32) | (uint64_t)(0xffffffffu - (uint32_t)i);
    return true;
}

__global__ void k_topk_init(TopkWs w, int32_t k) {
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) w.hist[i] = 0;
    if (threadIdx.x == 0) {
        w.ctrl->k_rem = k;
        w.ctrl->n_out = 0;
        w.ctrl->n_cand[0] = 0;
        w.ctrl->n_cand[1] = 0;
        w.ctrl->sel = 0;
        w.ctrl->take_all = 0;
    }
}

__device__ __forceinline__ int digit_of(uint64_t key, int level) {
    return (int)((key >> c_shift[level]) & ((1ull << c_bits[level]) - 1ull));
}

__device__ void flush_hist(uint32_t *lh, uint32_t *gh) {
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) {
        uint32_t c = lh[i];
        if (c) atomicAdd(gh + i, c);
    }
}

// Level 0 histogram straight from the scores.
__global__ void __launch_bounds__(256) k_hist_src(const float *score, const uint8_t *flags,
                                                  int64_t n, uint8_t req, uint8_t forbid,
                                                  TopkWs w) {
    __shared__ uint32_t lh[kBins];
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) lh[i] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t key;
        if (item_key(score, flags, i, req, forbid, key)) atomicAdd(&lh[digit_of(key, 0)], 1u);
    }
    flush_hist(lh, w.hist);
}

// Histogram of level `level` over the survivors in cand (count at *cnt).
__global__ void __launch_bounds__(256) k_hist_cand(const uint64_t *cand, const int32_t *cnt,
                                                   int level, TopkWs w) {
    __shared__ uint32_t lh[kBins];
    const int64_t n = *cnt;
    if (w.ctrl->take_all || n == 0 || (int64_t)blockIdx.x * blockDim.x >= n) return;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) lh[i] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&lh[digit_of(cand[i], level)], 1u);
    flush_hist(lh, w.hist);
}

// Pick the digit at which the running count from the top reaches k_rem.
// 256 threads, 8 bins each.  Clears the histogram for the next level.
__global__ void __launch_bounds__(256) k_select(TopkWs w, int level, int32_t n_survivors_known,
                                                const int32_t *n_surv) {
    __shared__ uint32_t part[256];
    __shared__ int32_t sel_s, above_s, total_s;
    const int tid = threadIdx.x;
    TopkCtrl *c = w.ctrl;
    if (c->take_all) return;
    const int nb = 1 << c_bits[level];
    const int per = nb / 256 > 0 ? nb / 256 : 1;
    // thread tid owns bins [tid*per, tid*per+per) counted from the top
    uint32_t loc = 0;
    for (int j = 0; j < per; ++j) {
        int bin = nb - 1 - (tid * per + j);
        if (bin >= 0) loc += w.hist[bin];
    }
    part[tid] = loc;
    __syncthreads();
    if (tid == 0) {
        const int32_t k_rem = c->k_rem;
        uint32_t run = 0;
        int32_t sel = -1, above = 0;
        for (int t = 0; t < 256 && sel < 0; ++t) {
            if (run + part[t] >= (uint32_t)k_rem) {
                for (int j = 0; j < per; ++j) {
                    int bin = nb - 1 - (t * per + j);
                    if (bin < 0) break;
                    uint32_t h = w.hist[bin];
                    if (run + h >= (uint32_t)k_rem) {
                        sel = bin;
                        above = (int32_t)run;
                        break;
                    }
                    run += h;
                }
            } else {
                run += part[t];
            }
        }
        uint32_t total = 0;
        for (int t = 0; t < 256; ++t) total += part[t];
        sel_s = sel;
        above_s = above;
        total_s = (int32_t)total;
    }
    __syncthreads();
    for (int i = tid; i < kBins; i += 256) w.hist[i] = 0;
    if (tid == 0) {
        if (sel_s < 0 || total_s <= c->k_rem) {
            c->take_all = 1;   // every survivor is in the top k
        } else {
            c->sel = sel_s;
            c->k_rem -= above_s;
        }
    }
    (void)n_survivors_known;
    (void)n_surv;
}

__device__ __forceinline__ void push(uint64_t *buf, int32_t *cnt, uint64_t key) {
    int32_t j = atomicAdd(cnt, 1);
    buf[j] = key;
}

// Level 0 compaction from the scores: digit above the selected one -> out,
// equal -> cand0.  With take_all every qualifying item goes to out.
__global__ void __launch_bounds__(256) k_compact_src(const float *score, const uint8_t *flags,
                                                     int64_t n, uint8_t req, uint8_t forbid,
                                                     TopkWs w) {
    TopkCtrl *c = w.ctrl;
    const int take_all = c->take_all;
    const int sel = c->sel;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t key;
        if (!item_key(score, flags, i, req, forbid, key)) continue;
        const int d = digit_of(key, 0);
        if (take_all || d > sel) push(w.out, &c->n_out, key);
        else if (d == sel) push(w.cand0, &c->n_cand[0], key);
    }
}

// Later levels: survivors of src -> out (digit above) or dst (digit equal).
// At the last level (all 64 bits consumed) keys are unique, so digits equal
// to the selection are taken too.
__global__ void __launch_bounds__(256) k_compact_cand(int level, int src_i, TopkWs w) {
    TopkCtrl *c = w.ctrl;
    const uint64_t *src = src_i ? w.cand1 : w.cand0;
    uint64_t *dst = src_i ? w.cand0 : w.cand1;
    int32_t *dcnt = &c->n_cand[src_i ^ 1];
    const int64_t n = c->n_cand[src_i];
    const int take_all = c->take_all;
    const int sel = c->sel;
    const bool last = level == kLevels - 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = src[i];
        const int d = digit_of(key, level);
        if (take_all || d > sel || (last && d == sel)) push(w.out, &c->n_out, key);
        else if (d == sel) push(dst, dcnt, key);
    }
}

// Reset the destination counter before a level writes into it (also after a
// take_all, so that later levels see an empty buffer).
__global__ void k_reset_cnt(TopkWs w, int which) {
    if (threadIdx.x == 0) w.ctrl->n_cand[which] = 0;
}

// Sort the chosen keys (descending) and write the results.  1024 threads.
__global__ void __launch_bounds__(1024) k_topk_final(TopkWs w, int32_t k, int64_t *idx,
                                                     float *top_score, int32_t *count) {
    extern __shared__ uint64_t keys[];
    const int tid = threadIdx.x;
    int32_t n = w.ctrl->n_out;
    if (n > k) n = k;   // cannot happen; guards the buffer
    int32_t P = 1;
    while (P < n) P <<= 1;
    for (int i = tid; i < P; i += blockDim.x) keys[i] = i < n ? w.out[i] : 0ull;
    __syncthreads();
    for (int32_t size = 2; size <= P; size <<= 1) {
        for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int32_t i = tid; i < P; i += blockDim.x) {
                int32_t j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    uint64_t a = keys[i], b = keys[j];
                    if (desc ? (a < b) : (a > b)) {
                        keys[i] = b;
                        keys[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < k; i += blockDim.x) {
        if (i < n) {
            uint64_t key = keys[i];
            idx[i] = (int64_t)(0xffffffffu - (uint32_t)(key & 0xffffffffull));
            if (top_score) top_score[i] = unord_f32((uint32_t)(key >> 32));
        } else {
            idx[i] = -1;
            if (top_score) top_score[i] = -INFINITY;
        }
    }
    if (tid == 0) *count = n;
}

hipError_t launch_topk(const float *score, const uint8_t *flags, int64_t n, int32_t k,
                       uint8_t req, uint8_t forbid, int64_t *idx, float *top_score,
                       int32_t *count, void *ws, hipStream_t st) {
    TopkWs w = carve_ws(ws, n, k);
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, st, w, k);
    int64_t g = (n + 256 * 8 - 1) / (256 * 8);
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    int64_t gc = (n + 255) / 256;
    if (gc < 1) gc = 1;
    if (gc > 2048) gc = 2048;
    hipLaunchKernelGGL(k_hist_src, dim3((unsigned)g), dim3(256), 0, st, score, flags, n, req,
                       forbid, w);
    hipLaunchKernelGGL(k_select, dim3(1), dim3(256), 0, st, w, 0, 0, nullptr);
    hipLaunchKernelGGL(k_compact_src, dim3((unsigned)g), dim3(256), 0, st, score, flags, n,
                       req, forbid, w);
    int src = 0;
    for (int level = 1; level < kLevels; ++level) {
        const int32_t *cnt = &w.ctrl->n_cand[src];
        hipLaunchKernelGGL(k_hist_cand, dim3((unsigned)gc), dim3(256), 0, st,
                           src ? w.cand1 : w.cand0, cnt, level, w);
        hipLaunchKernelGGL(k_select, dim3(1), dim3(256), 0, st, w, level, 0, nullptr);
        hipLaunchKernelGGL(k_reset_cnt, dim3(1), dim3(64), 0, st, w, src ^ 1);
        hipLaunchKernelGGL(k_compact_cand, dim3((unsigned)gc), dim3(256), 0, st, level, src, w);
        src ^= 1;
    }
    size_t lds = 0;
    int32_t P = 1;
    while (P < k) P <<= 1;
    lds = sizeof(uint64_t) * (size_t)P;
    hipLaunchKernelGGL(k_topk_final, dim3(1), dim3(1024), lds, st, w, k, idx, top_score, count);
    return hipGetLastError();
}

}  // namespace mps
