// topk.hip -- exact top-k of scored moves (the per-thread-block argmax
// reduction of Alg. 5, generalised to the k best moves and made
// deterministic: no floating-point atomics, a total order on items).
//
// Each qualifying item i gets the 64-bit key
//   key = ord(score) << 32 | (0xffffffff - i)
// where ord maps floats to unsigned integers monotonically (-0 and +0 equal).
// Keys are unique and "larger key" = "better item" (higher score, then smaller
// index), so the top k items are the k largest keys.  A most-significant-
// digit radix select finds them:
//   1. histogram of the top 11 bits over all items (every workgroup adds its
//      LDS histogram to one of four replicas);
//   2. every workgroup of one more pass sums the replicas and picks the
//      boundary digit (the same in all), then moves its items above the
//      boundary digit to the output and items on it to a candidate buffer
//      (wave-aggregated appends);
//   3. one workgroup refines the candidates digit by digit (11/10/11/11/10
//      more bits) until every remaining candidate is needed, and appends them
//      to the chosen keys: exactly the top min(k, total); it then clears the
//      histogram and counters for the next call;
//   4. each chosen key's rank is the number of chosen keys above it, counted
//      by a grid of workgroups against all chosen keys in LDS, and the key is
//      written at its rank.
// Four launches in all; every count is an integer, so the result does not
// depend on thread timing.  The workspace's first topk_ws_zero_bytes() bytes
// must be zero when a call starts (the caller clears them once, before the
// first call; every call leaves them zero).
#include <float.h>
#include <math.h>

#include "topk_dev.h"

namespace mps {

constexpr int kBins = 2048;
constexpr int kLevels = 6;
constexpr int kRefineThreads = 1024;
__constant__ int c_shift[kLevels] = {53, 42, 32, 21, 10, 0};
__constant__ int c_bits[kLevels] = {11, 11, 10, 11, 11, 10};

constexpr int kRep = 4;   // replicas of the level-0 histogram and counters

// Zero between calls (cleared by the refinement launch of each call, and by
// the caller before the first call): the level-0 histogram replicas and the
// append counters of the level-0 compaction.
struct TopkZero {
    uint32_t hist[kRep][kBins];
    int32_t out_next[kRep];    // next free slot of each replica's output region
    int32_t cand_next[kRep];   // next free slot of each replica's candidate region
};

struct TopkCtrl {
    int32_t k_rem;      // how many keys are still to be chosen
    int32_t n_out;      // keys chosen at level 0 (in out[])
    int32_t n_cand;     // candidates on the boundary digit after level 0
    int32_t take_all;   // every qualifying item is in the top k
    int32_t n_final;    // keys of the result, all in out[]
};

struct TopkWs {
    TopkZero *z;
    TopkCtrl *ctrl;
    uint64_t *out;    // [k]
    uint64_t *cand0;  // [n]
    uint64_t *cand1;  // [n]
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t topk_ws_zero_bytes() { return a256(sizeof(TopkZero)); }

size_t topk_ws_bytes(int64_t n, int32_t k) {
    const size_t nn = n > 0 ? (size_t)n : 1;
    return topk_ws_zero_bytes() + a256(sizeof(TopkCtrl)) + a256(sizeof(uint64_t) * (size_t)k) +
           2 * a256(sizeof(uint64_t) * nn);
}

static TopkWs carve_ws(void *ws, int64_t n, int32_t k) {
    char *p = (char *)ws;
    const size_t nn = n > 0 ? (size_t)n : 1;
    TopkWs w;
    w.z = (TopkZero *)p;
    p += topk_ws_zero_bytes();
    w.ctrl = (TopkCtrl *)p;
    p += a256(sizeof(TopkCtrl));
    w.out = (uint64_t *)p;
    p += a256(sizeof(uint64_t) * (size_t)k);
    w.cand0 = (uint64_t *)p;
    p += a256(sizeof(uint64_t) * nn);
    w.cand1 = (uint64_t *)p;
    return w;
}

__device__ __forceinline__ int digit_of(uint64_t key, int level) {
    return (int)((key >> c_shift[level]) & ((1ull << c_bits[level]) - 1ull));
}

// Items per thread of the two full passes; a workgroup covers a contiguous
// range of 256 * kItems items and issues all their loads before using them.
constexpr int kItems = 8;

// Level-0 histogram over all items: workgroup g adds its LDS histogram to
// replica g % kRep (spreading the global atomics over kRep copies).
__global__ void __launch_bounds__(256) k_hist0(const float *score, const uint8_t *flags,
                                               int64_t n, uint8_t req, uint8_t forbid,
                                               TopkWs w) {
    __shared__ uint32_t lh[kBins];
    for (int i = threadIdx.x; i < kBins; i += 256) lh[i] = 0;
    const int64_t base = (int64_t)blockIdx.x * 256 * kItems + threadIdx.x;
    uint64_t key[kItems];
    bool q[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = base + 256 * u;
        q[u] = i < n && item_key(score, flags, i, req, forbid, key[u]);
    }
    __syncthreads();
    // one LDS atomic per item (grouping the lanes of a digit by ballot first
    // measured slower: the scores of a wave spread over many digits)
#pragma unroll
    for (int u = 0; u < kItems; ++u)
        if (q[u]) atomicAdd(&lh[digit_of(key[u], 0)], 1u);
    __syncthreads();
    uint32_t *rep = w.z->hist[blockIdx.x % kRep];
    for (int i = threadIdx.x; i < kBins; i += 256) {
        const uint32_t c = lh[i];
        if (c) atomicAdd(rep + i, c);
    }
}

// Level-0 selection and compaction.  Every workgroup first repeats the same
// selection from the histogram replicas (so no separate launch has to
// publish it): the boundary digit, and per replica the sizes of its output
// and candidate regions, laid out back to back (replica r's counts are
// exactly the items workgroups g = r (mod kRep) append, which cover the same
// items as in the histogram launch).  Then items above the boundary digit
// go to out, items on it to cand0 (all qualifying items to out with
// take_all): each workgroup counts its items in LDS, reserves its ranges
// with one atomic per buffer on its replica's counters, then writes.
// Workgroup 0 records the selection for the refinement.
__global__ void __launch_bounds__(256) k_compact0(const float *score, const uint8_t *flags,
                                                  int64_t n, uint8_t req, uint8_t forbid,
                                                  int32_t k, TopkWs w) {
    __shared__ uint32_t lh[kBins];
    __shared__ uint32_t part[256];
    __shared__ int32_t res[3];
    __shared__ int32_t reg_out[kRep], reg_cand[kRep];
    __shared__ int32_t cnt[2], base_s[2];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * 256 * kItems + tid;
    uint64_t key[kItems];
    bool q[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = base + 256 * u;
        q[u] = i < n && item_key(score, flags, i, req, forbid, key[u]);
    }
    // the replicas: thread tid owns bins tid + 256 j, all loads in flight together
    constexpr int kPer = kBins / 256;
    uint32_t hr[kPer][kRep];
#pragma unroll
    for (int j = 0; j < kPer; ++j)
#pragma unroll
        for (int r = 0; r < kRep; ++r) hr[j][r] = w.z->hist[r][tid + 256 * j];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        uint32_t c = 0;
#pragma unroll
        for (int r = 0; r < kRep; ++r) c += hr[j][r];
        lh[tid + 256 * j] = c;
    }
    if (tid < 2) cnt[tid] = 0;
    __syncthreads();
    select_digit(lh, kBins, k, part, res);
    const bool take_all = res[0] < 0 || res[2] <= k;
    const int sel = take_all ? -1 : res[0];
    if (tid < 2 * kRep) part[tid] = 0u;
    __syncthreads();
    {
        uint32_t above[kRep], equal[kRep];
#pragma unroll
        for (int r = 0; r < kRep; ++r) {
            above[r] = 0u;
            equal[r] = 0u;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int b = tid + 256 * j;
#pragma unroll
            for (int r = 0; r < kRep; ++r) {
                above[r] += b > sel ? hr[j][r] : 0u;
                equal[r] += b == sel ? hr[j][r] : 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < kRep; ++r) {
            if (above[r]) atomicAdd(&part[r], above[r]);
            if (equal[r]) atomicAdd(&part[kRep + r], equal[r]);
        }
    }
    __syncthreads();
    if (tid == 0) {
        int32_t oa = 0, oc = 0;
        for (int r = 0; r < kRep; ++r) {
            reg_out[r] = oa;
            reg_cand[r] = oc;
            oa += (int32_t)part[r];
            oc += (int32_t)part[kRep + r];
        }
        if (blockIdx.x == 0) {
            w.ctrl->n_out = oa;
            w.ctrl->n_cand = take_all ? 0 : oc;
            w.ctrl->take_all = take_all ? 1 : 0;
            w.ctrl->k_rem = take_all ? k : k - res[1];
        }
    }
    // local positions
    int32_t pos[kItems];
    int8_t dst[kItems];
    const int lane = tid & 63;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int d = q[u] ? digit_of(key[u], 0) : -1;
        const bool to_out = q[u] && (take_all || d > sel);
        const bool to_cand = q[u] && !take_all && d == sel;
        dst[u] = to_out ? 0 : (to_cand ? 1 : -1);
        pos[u] = -1;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const uint64_t mask = __ballot(dst[u] == b);
            if (mask == 0) continue;
            const int leader = __ffsll((unsigned long long)mask) - 1;
            int32_t wb = 0;
            if (lane == leader) wb = atomicAdd(&cnt[b], (int32_t)__popcll(mask));
            wb = __shfl(wb, leader);
            if (dst[u] == b) pos[u] = wb + (int32_t)__popcll(mask & below);
        }
    }
    __syncthreads();
    if (tid < 2) {
        const int r = blockIdx.x % kRep;
        int32_t *next = tid == 0 ? &w.z->out_next[r] : &w.z->cand_next[r];
        const int32_t reg = tid == 0 ? reg_out[r] : reg_cand[r];
        base_s[tid] = reg + (cnt[tid] ? atomicAdd(next, cnt[tid]) : 0);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        if (dst[u] == 0) w.out[base_s[0] + pos[u]] = key[u];
        else if (dst[u] == 1) w.cand0[base_s[1] + pos[u]] = key[u];
    }
}

// One workgroup: while the candidates on the boundary digit are more than the
// keys still needed, refine them by the next digit; then every remaining
// candidate is needed, and the chosen keys plus the remaining candidates are
// exactly the top min(k, total) (keys are unique).
constexpr int kRU = 8;   // candidates per thread in flight in the refinement
__global__ void __launch_bounds__(kRefineThreads) k_refine(TopkWs w) {
    __shared__ uint32_t lh[kBins];
    __shared__ uint32_t part[256];
    __shared__ int32_t res[3];
    __shared__ int32_t n_src_s, n_dst_s, n_out_s, k_rem_s;
    const int tid = threadIdx.x;
    const TopkCtrl *c = w.ctrl;
    if (tid == 0) {
        n_src_s = c->n_cand;
        n_out_s = c->n_out;
        k_rem_s = c->k_rem;
    }
    __syncthreads();
    uint64_t *src = w.cand0, *dst = w.cand1;
    for (int level = 1; level < kLevels; ++level) {
        const int32_t ns = n_src_s;
        // stop once every remaining candidate is needed
        if (ns == 0 || ns <= k_rem_s) break;
        const int nb = 1 << c_bits[level];
        for (int i = tid; i < nb; i += kRefineThreads) lh[i] = 0;
        if (tid == 0) n_dst_s = 0;
        __syncthreads();
        // candidates in chunks of kRU per thread, every load of a chunk in
        // flight before the first use
        for (int32_t c0 = 0; c0 < ns; c0 += kRU * kRefineThreads) {
            uint64_t key[kRU];
#pragma unroll
            for (int u = 0; u < kRU; ++u) {
                const int32_t i = c0 + tid + u * kRefineThreads;
                key[u] = i < ns ? src[i] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < kRU; ++u)
                if (c0 + tid + u * kRefineThreads < ns) atomicAdd(&lh[digit_of(key[u], level)], 1u);
        }
        __syncthreads();
        const int32_t k_rem = k_rem_s;
        select_digit(lh, nb, k_rem, part, res);
        const bool take_all = res[0] < 0 || res[2] <= k_rem;
        const int sel = res[0];
        const bool last = level == kLevels - 1;
        // digit above -> out; equal -> dst (keys are unique, so at the last
        // level the equal digit is taken as well)
        for (int32_t c0 = 0; c0 < ns; c0 += kRU * kRefineThreads) {
            uint64_t key[kRU];
#pragma unroll
            for (int u = 0; u < kRU; ++u) {
                const int32_t i = c0 + tid + u * kRefineThreads;
                key[u] = i < ns ? src[i] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < kRU; ++u) {
                const bool in = c0 + tid + u * kRefineThreads < ns;
                const int d = in ? digit_of(key[u], level) : -1;
                const bool to_out = in && (take_all || d > sel || (last && d == sel));
                const bool to_dst = in && !take_all && !last && d == sel;
                wave_append(to_out, key[u], w.out, &n_out_s);
                wave_append(to_dst, key[u], dst, &n_dst_s);
            }
        }
        __threadfence_block();
        __syncthreads();
        if (tid == 0) {
            if (!take_all) k_rem_s = k_rem - res[1];
            n_src_s = take_all ? 0 : n_dst_s;
        }
        __syncthreads();
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    __threadfence_block();
    __syncthreads();
    // every remaining candidate is chosen: append them after the others
    const int32_t no = n_out_s, ns = n_src_s;
    for (int32_t c0 = 0; c0 < ns; c0 += kRU * kRefineThreads) {
        uint64_t key[kRU];
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            const int32_t i = c0 + tid + u * kRefineThreads;
            key[u] = i < ns ? src[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            const int32_t i = c0 + tid + u * kRefineThreads;
            if (i < ns) w.out[no + i] = key[u];
        }
    }
    if (tid == 0) w.ctrl->n_final = no + ns;
    // the level-0 histogram and counters are no longer read in this call:
    // leave them zero for the next one
    uint32_t *z = (uint32_t *)w.z;
    for (size_t i = tid; i < sizeof(TopkZero) / 4; i += kRefineThreads) z[i] = 0u;
}

// Rank of each chosen key = the number of chosen keys above it (keys are
// unique, so ranks are a permutation of 0 .. n_final-1), and the key written
// at its rank.  Workgroup g takes keys [16 g, 16 g + 16): thread (j, q)
// counts, for key j, the chosen keys above it among the key pairs 32 m + 2 q,
// 32 m + 2 q + 1 (all chosen keys staged in LDS, zero-padded to a multiple
// of 32; no key is 0), and the sixteen counts of a key are added.  Entries
// past n_final get -1 / -inf.
constexpr int kRankKeys = 16;
__global__ void __launch_bounds__(256) k_rank(TopkWs w, int32_t k, int64_t *idx,
                                              float *top_score, int32_t *count) {
    extern __shared__ __align__(16) uint64_t keys[];   // [k rounded up to 32]
    __shared__ uint32_t part[16][kRankKeys];
    const int32_t tot = w.ctrl->n_final;
    const int32_t tot32 = (tot + 31) & ~31;
    const int tid = threadIdx.x;
    {
        // every load in flight before the first store: key pairs tid + 256 u
        // (out[] is allocated in whole 256-byte units, so pairs up to tot32
        // stay inside it; entries from tot on are replaced by 0)
        constexpr int kPairs = (MPS_MAX_TOPK + 511) / 512;
        ulonglong2 buf[kPairs];
#pragma unroll
        for (int u = 0; u < kPairs; ++u) {
            const int32_t j = 2 * (tid + 256 * u);
            buf[u] = j < tot32 ? *(const ulonglong2 *)(w.out + j) : make_ulonglong2(0ull, 0ull);
        }
#pragma unroll
        for (int u = 0; u < kPairs; ++u) {
            const int32_t j = 2 * (tid + 256 * u);
            if (j < tot32) {
                ulonglong2 v = buf[u];
                if (j >= tot) v.x = 0ull;
                if (j + 1 >= tot) v.y = 0ull;
                *(ulonglong2 *)(keys + j) = v;
            }
        }
    }
    __syncthreads();
    const int kj = tid & (kRankKeys - 1), q = tid >> 4;
    const int32_t i = blockIdx.x * kRankKeys + kj;
    const uint64_t me = i < tot ? keys[i] : ~0ull;
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    int32_t j = 2 * q;
    for (; j + 32 < tot32; j += 64) {
        const ulonglong2 a = *(const ulonglong2 *)(keys + j);
        const ulonglong2 b = *(const ulonglong2 *)(keys + j + 32);
        c0 += a.x > me ? 1u : 0u;
        c1 += a.y > me ? 1u : 0u;
        c2 += b.x > me ? 1u : 0u;
        c3 += b.y > me ? 1u : 0u;
    }
    if (j < tot32) {
        const ulonglong2 a = *(const ulonglong2 *)(keys + j);
        c0 += a.x > me ? 1u : 0u;
        c1 += a.y > me ? 1u : 0u;
    }
    part[q][kj] = (c0 + c1) + (c2 + c3);
    __syncthreads();
    if (tid < kRankKeys) {
        const int32_t ii = blockIdx.x * kRankKeys + tid;
        if (ii < tot) {
            uint32_t r = 0;
            for (int u = 0; u < 16; ++u) r += part[u][tid];
            const uint64_t key = keys[ii];
            idx[r] = (int64_t)(0xffffffffu - (uint32_t)(key & 0xffffffffull));
            if (top_score) top_score[r] = unord_f32((uint32_t)(key >> 32));
        } else if (ii < k) {
            idx[ii] = -1;
            if (top_score) top_score[ii] = -INFINITY;
        }
        if (ii == 0) *count = tot;
    }
}

hipError_t launch_topk(const float *score, const uint8_t *flags, int64_t n, int32_t k,
                       uint8_t req, uint8_t forbid, int64_t *idx, float *top_score,
                       int32_t *count, void *ws, hipStream_t st) {
    const TopkWs w = carve_ws(ws, n, k);
    int64_t g = (n + 256 * kItems - 1) / (256 * kItems);
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_hist0, dim3((unsigned)g), dim3(256), 0, st, score, flags, n, req, forbid,
                       w);
    hipLaunchKernelGGL(k_compact0, dim3((unsigned)g), dim3(256), 0, st, score, flags, n, req,
                       forbid, k, w);
    hipLaunchKernelGGL(k_refine, dim3(1), dim3(kRefineThreads), 0, st, w);
    hipLaunchKernelGGL(k_rank, dim3((unsigned)((k + kRankKeys - 1) / kRankKeys)), dim3(256),
                       sizeof(uint64_t) * (size_t)((k + 31) & ~31), st, w, k, idx, top_score,
                       count);
    return hipGetLastError();
}

}  // namespace mps
