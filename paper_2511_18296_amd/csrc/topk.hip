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
//      LDS histogram to one of eight replicas); one workgroup then picks the
//      boundary digit;
//   2. one pass moves items above the boundary digit to the output and items
//      on it to a candidate buffer (wave-aggregated appends);
//   3. one workgroup refines the candidates digit by digit (11/10/11/11/10
//      more bits) until every remaining candidate is needed, and appends
//      them to the chosen keys: exactly the top min(k, total);
//   4. each chosen key's rank is the number of chosen keys above it,
//      counted tile against tile by a grid of workgroups, and the key is
//      written at its rank.
// Seven launches in all; every count is an integer, so the result does not
// depend on thread timing.
#include <float.h>
#include <math.h>
#include <stdio.h>

#include <mutex>

#include "topk_dev.h"

namespace mps {

constexpr int kBins = 2048;
constexpr int kLevels = 6;
constexpr int kRefineThreads = 1024;
__constant__ int c_shift[kLevels] = {53, 42, 32, 21, 10, 0};
__constant__ int c_bits[kLevels] = {11, 11, 10, 11, 11, 10};

constexpr int kRep = 8;   // replicas of the level-0 histogram and counters

struct TopkCtrl {
    int32_t k_rem;      // how many keys are still to be chosen
    int32_t n_out;      // keys chosen so far (in out[])
    int32_t n_cand;     // candidates on the boundary digit after level 0
    int32_t sel;        // boundary digit of level 0
    int32_t take_all;   // every qualifying item is in the top k
    int32_t out_next[kRep];    // next free slot of each replica's output region
    int32_t cand_next[kRep];   // next free slot of each replica's candidate region
    int32_t n_final;           // keys of the result, all in out[]
};

struct TopkWs {
    TopkCtrl *ctrl;
    uint32_t *hist;   // [kRep][kBins]
    uint64_t *out;    // [k]
    uint64_t *cand0;  // [n]
    uint64_t *cand1;  // [n]
    uint32_t *rank_part;   // [ceil(k/256)][k] partial ranks
};

constexpr int kRankTile = 256;   // keys per rank workgroup and per comparison tile

__host__ __device__ inline int32_t rank_tiles(int32_t k) { return (k + kRankTile - 1) / kRankTile; }

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t topk_ws_bytes(int64_t n, int32_t k) {
    const size_t nn = n > 0 ? (size_t)n : 1;
    return a256(sizeof(TopkCtrl)) + a256(sizeof(uint32_t) * kBins * kRep) +
           a256(sizeof(uint64_t) * (size_t)k) + 2 * a256(sizeof(uint64_t) * nn) +
           a256(sizeof(uint32_t) * (size_t)rank_tiles(k) * k);
}

static TopkWs carve_ws(void *ws, int64_t n, int32_t k) {
    char *p = (char *)ws;
    const size_t nn = n > 0 ? (size_t)n : 1;
    TopkWs w;
    w.ctrl = (TopkCtrl *)p;
    p += a256(sizeof(TopkCtrl));
    w.hist = (uint32_t *)p;
    p += a256(sizeof(uint32_t) * kBins * kRep);
    w.out = (uint64_t *)p;
    p += a256(sizeof(uint64_t) * (size_t)k);
    w.cand0 = (uint64_t *)p;
    p += a256(sizeof(uint64_t) * nn);
    w.cand1 = (uint64_t *)p;
    p += a256(sizeof(uint64_t) * nn);
    w.rank_part = (uint32_t *)p;
    return w;
}

__device__ __forceinline__ int digit_of(uint64_t key, int level) {
    return (int)((key >> c_shift[level]) & ((1ull << c_bits[level]) - 1ull));
}

__global__ void k_topk_init(TopkWs w, int32_t k) {
    for (int i = threadIdx.x; i < kBins * kRep; i += blockDim.x) w.hist[i] = 0;
    if (threadIdx.x == 0) {
        w.ctrl->k_rem = k;
        w.ctrl->n_out = 0;
        w.ctrl->n_cand = 0;
        w.ctrl->sel = 0;
        w.ctrl->take_all = 0;
    }
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
    // scores crowd into few digits: one LDS atomic per distinct digit of a
    // wave (lanes grouped by ballot) instead of one per lane
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int d = q[u] ? digit_of(key[u], 0) : -1;
        uint64_t pending = __ballot(d >= 0);
        while (pending) {
            const int leader = __ffsll((unsigned long long)pending) - 1;
            const int dl = __shfl(d, leader);
            const uint64_t same = __ballot(d == dl);
            if (lane == leader) atomicAdd(&lh[dl], (uint32_t)__popcll(same));
            pending &= ~same;
        }
    }
    __syncthreads();
    uint32_t *rep = w.hist + (size_t)(blockIdx.x % kRep) * kBins;
    for (int i = threadIdx.x; i < kBins; i += 256) {
        const uint32_t c = lh[i];
        if (c) atomicAdd(rep + i, c);
    }
}

// One workgroup after the histogram launch: sum the replicas, select the
// boundary digit and lay out the output and candidate regions of each
// replica back to back (replica r's counts are exactly the items workgroups
// g = r (mod kRep) of the compaction will append, which covers the same
// items per workgroup).
__global__ void __launch_bounds__(256) k_select0(TopkWs w) {
    __shared__ uint32_t lh[kBins];
    __shared__ uint32_t part[256];
    __shared__ int32_t res[3];
    for (int i = threadIdx.x; i < kBins; i += 256) {
        uint32_t c = 0;
        for (int r = 0; r < kRep; ++r)
            c += __hip_atomic_load(w.hist + (size_t)r * kBins + i, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        lh[i] = c;
    }
    __syncthreads();
    const int32_t k_rem = w.ctrl->k_rem;
    select_digit(lh, kBins, k_rem, part, res);
    const bool take_all = res[0] < 0 || res[2] <= k_rem;
    const int sel = take_all ? -1 : res[0];
    // per-replica region sizes: items above sel (all items with take_all)
    // and items on sel; every thread takes its bins of every replica (all
    // loads in flight together) and the sums meet in LDS
    if (threadIdx.x < 2 * kRep) part[threadIdx.x] = 0u;
    __syncthreads();
    {
        constexpr int kPer = kBins / 256;
        uint32_t above[kRep], equal[kRep];
#pragma unroll
        for (int r = 0; r < kRep; ++r) {
            above[r] = 0u;
            equal[r] = 0u;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int b = threadIdx.x + 256 * j;
#pragma unroll
            for (int r = 0; r < kRep; ++r) {
                const uint32_t h = __hip_atomic_load(w.hist + (size_t)r * kBins + b,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                above[r] += b > sel ? h : 0u;
                equal[r] += b == sel ? h : 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < kRep; ++r) {
            if (above[r]) atomicAdd(&part[r], above[r]);
            if (equal[r]) atomicAdd(&part[kRep + r], equal[r]);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t oa = 0, oc = 0;
        for (int r = 0; r < kRep; ++r) {
            w.ctrl->out_next[r] = oa;
            w.ctrl->cand_next[r] = oc;
            oa += (int32_t)part[r];
            oc += (int32_t)part[kRep + r];
        }
        w.ctrl->n_out = oa;
        w.ctrl->n_cand = oc;
        w.ctrl->take_all = take_all ? 1 : 0;
        w.ctrl->sel = sel;
        if (!take_all) w.ctrl->k_rem = k_rem - res[1];
    }
}

// Items above the boundary digit -> out; on it -> cand0 (all qualifying items
// -> out with take_all).  Each workgroup counts its items in LDS, reserves its
// ranges with one atomic per buffer on its replica's counters, then writes.
__global__ void __launch_bounds__(256) k_compact0(const float *score, const uint8_t *flags,
                                                  int64_t n, uint8_t req, uint8_t forbid,
                                                  TopkWs w) {
    __shared__ int32_t cnt[2], base_s[2];
    const int take_all = w.ctrl->take_all;
    const int sel = w.ctrl->sel;
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    const int64_t base = (int64_t)blockIdx.x * 256 * kItems + threadIdx.x;
    uint64_t key[kItems];
    bool q[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = base + 256 * u;
        q[u] = i < n && item_key(score, flags, i, req, forbid, key[u]);
    }
    __syncthreads();
    // local positions
    int32_t pos[kItems];
    int8_t dst[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int d = q[u] ? digit_of(key[u], 0) : -1;
        const bool to_out = q[u] && (take_all || d > sel);
        const bool to_cand = q[u] && !take_all && d == sel;
        dst[u] = to_out ? 0 : (to_cand ? 1 : -1);
        pos[u] = -1;
        const int lane = threadIdx.x & 63;
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
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
    if (threadIdx.x < 2) {
        const int r = blockIdx.x % kRep;
        int32_t *next = threadIdx.x == 0 ? &w.ctrl->out_next[r] : &w.ctrl->cand_next[r];
        base_s[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(next, cnt[threadIdx.x]) : 0;
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

__global__ void __launch_bounds__(kRefineThreads) k_refine(TopkWs w) {
    __shared__ uint32_t lh[kBins];
    __shared__ uint32_t part[256];
    __shared__ int32_t res[3];
    __shared__ int32_t n_src_s, n_dst_s, n_out_s, k_rem_s;
    const int tid = threadIdx.x;
    const TopkCtrl *c = w.ctrl;
    if (tid == 0) {
        n_src_s = c->take_all ? 0 : c->n_cand;
        n_out_s = c->n_out;
        k_rem_s = c->k_rem;
    }
    __syncthreads();
    uint64_t *src = w.cand0, *dst = w.cand1;
    for (int level = 1; level < kLevels; ++level) {
        const int32_t ns = n_src_s;
        // stop once every remaining candidate is needed: the sort then
        // takes exactly the k chosen keys
        if (ns == 0 || ns <= k_rem_s) break;
        const int nb = 1 << c_bits[level];
        for (int i = tid; i < nb; i += kRefineThreads) lh[i] = 0;
        if (tid == 0) n_dst_s = 0;
        __syncthreads();
        for (int32_t i = tid; i < ns; i += kRefineThreads)
            atomicAdd(&lh[digit_of(src[i], level)], 1u);
        __syncthreads();
        const int32_t k_rem = k_rem_s;
        select_digit(lh, nb, k_rem, part, res);
        const bool take_all = res[0] < 0 || res[2] <= k_rem;
        const int sel = res[0];
        const bool last = level == kLevels - 1;
        // digit above -> out; equal -> dst (keys are unique, so at the last
        // level the equal digit is taken as well)
        const int32_t n_up = ((ns + 63) / 64) * 64;
        for (int32_t i = tid; i < n_up; i += kRefineThreads) {
            const bool in = i < ns;
            const uint64_t key = in ? src[i] : 0ull;
            const int d = in ? digit_of(key, level) : -1;
            const bool to_out = in && (take_all || d > sel || (last && d == sel));
            const bool to_dst = in && !take_all && !last && d == sel;
            wave_append(to_out, key, w.out, &n_out_s);
            wave_append(to_dst, key, dst, &n_dst_s);
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
    for (int32_t i = tid; i < ns; i += kRefineThreads) w.out[no + i] = src[i];
    if (tid == 0) w.ctrl->n_final = no + ns;
}

// Rank of each chosen key = the number of chosen keys above it (keys are
// unique, so ranks are a permutation of 0 .. n_final-1).  Workgroup (x, y)
// compares keys [x*256, x*256+256) with the keys of tile y staged in LDS.
__global__ void __launch_bounds__(kRankTile) k_rank_part(TopkWs w, int32_t k) {
    __shared__ uint64_t tile[kRankTile];
    const int32_t tot = w.ctrl->n_final;
    const int32_t tid = threadIdx.x;
    const int32_t i = blockIdx.x * kRankTile + tid;
    const int32_t j = blockIdx.y * kRankTile + tid;
    tile[tid] = j < tot ? w.out[j] : 0ull;   // 0 is below every key
    const uint64_t me = i < tot ? w.out[i] : ~0ull;
    __syncthreads();
    uint32_t c = 0;
#pragma unroll 16
    for (int32_t t = 0; t < kRankTile; ++t) c += tile[t] > me ? 1u : 0u;
    if (i < k) w.rank_part[(size_t)blockIdx.y * k + i] = c;
}

// Each chosen key goes to its rank; entries past n_final get -1 / -inf.
__global__ void __launch_bounds__(kRankTile) k_rank_scatter(TopkWs w, int32_t k, int64_t *idx,
                                                            float *top_score, int32_t *count) {
    const int32_t tot = w.ctrl->n_final;
    const int32_t i = blockIdx.x * kRankTile + threadIdx.x;
    if (i < tot) {
        uint32_t r = 0;
        const int32_t nt = rank_tiles(k);
        for (int32_t t = 0; t < nt; ++t) r += w.rank_part[(size_t)t * k + i];
        const uint64_t key = w.out[i];
        idx[r] = (int64_t)(0xffffffffu - (uint32_t)(key & 0xffffffffull));
        if (top_score) top_score[r] = unord_f32((uint32_t)(key >> 32));
    } else if (i < k) {
        idx[i] = -1;
        if (top_score) top_score[i] = -INFINITY;
    }
    if (i == 0) *count = tot;
}

hipError_t launch_topk(const float *score, const uint8_t *flags, int64_t n, int32_t k,
                       uint8_t req, uint8_t forbid, int64_t *idx, float *top_score,
                       int32_t *count, void *ws, hipStream_t st) {
    const TopkWs w = carve_ws(ws, n, k);
    hipLaunchKernelGGL(k_topk_init, dim3(1), dim3(256), 0, st, w, k);
    int64_t g = (n + 256 * kItems - 1) / (256 * kItems);
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_hist0, dim3((unsigned)g), dim3(256), 0, st, score, flags, n, req, forbid,
                       w);
    hipLaunchKernelGGL(k_select0, dim3(1), dim3(256), 0, st, w);
    hipLaunchKernelGGL(k_compact0, dim3((unsigned)g), dim3(256), 0, st, score, flags, n, req,
                       forbid, w);
    hipLaunchKernelGGL(k_refine, dim3(1), dim3(kRefineThreads), 0, st, w);
    const unsigned nt = (unsigned)rank_tiles(k);
    hipLaunchKernelGGL(k_rank_part, dim3(nt, nt), dim3(kRankTile), 0, st, w, k);
    hipLaunchKernelGGL(k_rank_scatter, dim3(nt), dim3(kRankTile), 0, st, w, k, idx, top_score,
                       count);
    return hipGetLastError();
}

}  // namespace mps

// ---- top-k with a library-owned workspace ------------------------------------
// The selection above with its workspace in a device array of this library
// instead of a caller buffer, for callers that cannot allocate.  The array is
// sized for kNoAllocMaxN items and k <= MPS_MAX_TOPK; each device holds its
// own copy for the life of the process.  k_topk_init clears what must start
// at zero on every call, so no call depends on what the previous one left.

namespace mps {

constexpr int64_t kNoAllocMaxN = (int64_t)1 << 21;
constexpr size_t ca256(size_t x) { return (x + 255) & ~(size_t)255; }
// the layout carve_ws makes for (kNoAllocMaxN, MPS_MAX_TOPK)
constexpr size_t kScratchBytes =
    ca256(sizeof(TopkCtrl)) + ca256(sizeof(uint32_t) * kBins * kRep) +
    ca256(sizeof(uint64_t) * MPS_MAX_TOPK) + 2 * ca256(sizeof(uint64_t) * kNoAllocMaxN) +
    ca256(sizeof(uint32_t) * ((MPS_MAX_TOPK + kRankTile - 1) / kRankTile) * MPS_MAX_TOPK);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of this device's copy of `scratch` (the host-side name is
// only a stand-in and must never reach a kernel).  Looked up once per device.
static hipError_t scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace mps

extern "C" mps_status mps_topk_noalloc(const float *score, const uint8_t *flags, int64_t n,
                                       int32_t k, uint8_t require, uint8_t forbid,
                                       int64_t *idx, float *top_score, int32_t *count,
                                       void *stream) {
    using namespace mps;
    char msg[160];
    if (k < 1 || k > MPS_MAX_TOPK) {
        snprintf(msg, sizeof(msg), "k must be in 1..%d (got %d)", MPS_MAX_TOPK, k);
        return report_error(MPS_E_INVALID_ARG, msg);
    }
    if (n < 0 || n > kNoAllocMaxN) {
        snprintf(msg, sizeof(msg),
                 "n = %lld exceeds the %lld items the library-owned top-k workspace holds",
                 (long long)n, (long long)kNoAllocMaxN);
        return report_error(MPS_E_INVALID_ARG, msg);
    }
    if ((n > 0 && (!score || !flags)) || !idx || !count)
        return report_error(MPS_E_INVALID_ARG, "score, flags, idx and count are required");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        snprintf(msg, sizeof(msg), "no usable current device (%s)", hipGetErrorString(e));
        return report_error(MPS_E_DEVICE, msg);
    }
    void *ws = nullptr;
    e = scratch_address(dev, &ws);
    if (e != hipSuccess) {
        snprintf(msg, sizeof(msg), "address of the top-k scratch: %s", hipGetErrorString(e));
        return report_error(MPS_E_DEVICE, msg);
    }
    e = launch_topk(score, flags, n, k, require, forbid, idx, top_score, count, ws,
                    (hipStream_t)stream);
    if (e != hipSuccess) {
        snprintf(msg, sizeof(msg), "topk: %s", hipGetErrorString(e));
        return report_error(MPS_E_DEVICE, msg);
    }
    return MPS_OK;
}
