// greedy.hip -- the greedy initializer (Alg. 3 with every uncertainty factor
// equal to 1): blocks in descending value density take their earliest
// feasible period.
//
// Value density is the block's expected value m_b = mean_s v[s][b] (FP64,
// the per-block statistic of the model).  Order: m_b descending, block index
// ascending on ties.  Starting from "nothing mined", a block is placed in the
// earliest period t < T in which
//   every predecessor is already placed in t or earlier,
//   M[t] + ton_b <= mine_cap, and
//   O[t][s] + ton_b <= proc_cap in every scenario s in which b is ore
// (the PREC_OK, MINE_OK and PROC_OK conditions of the move (b, t) against the
// partial schedule; an unplaced block counts as never mined, so a successor
// of b cannot be placed before b and needs no check).  Blocks that find no
// period stay unplaced; passes over the unplaced blocks, in the same order,
// repeat until one places nothing.
//
// Execution:
// 1. the order: a bitonic sort of (key, index) pairs, where key is an
//    order-preserving integer image of m_b -- stages with a stride of 2,048
//    or more run as one launch each over global memory, the others inside a
//    workgroup in LDS;
// 2. the walk: one workgroup of kGW waves.  O[t][s] and M[t] live in LDS
//    (FP64, summed in placement order, so every capacity decision is the
//    sequential one bit for bit).  For each block every wave reads the
//    block's predecessor periods itself (no barrier and, with the schedule
//    mirrored in LDS, no global load on the skip path); the periods from the
//    predecessor bound up are checked eight at a time, one per wave, each
//    wave testing every scenario with one ballot; the earliest feasible one
//    is applied to the LDS state and to p.
#include "internal.h"

namespace mps {

constexpr int kGW = 8;                 // waves of the walk
constexpr int kGT = 64 * kGW;
constexpr int kSortLocal = 2048;       // elements sorted per workgroup in LDS
constexpr int kSortThreads = kSortLocal / 2;
constexpr int kMaxPred = 16;           // predecessor lanes of a block (>= MPS_MAX_DEGREE)
static_assert(kMaxPred >= MPS_MAX_DEGREE, "one lane per predecessor");

struct SortItem {
    uint64_t key;
    uint32_t idx;
    uint32_t pad;
};

// "a comes first": larger key, then smaller index.
__device__ __forceinline__ bool first(const SortItem &a, const SortItem &b) {
    return a.key > b.key || (a.key == b.key && a.idx < b.idx);
}

__device__ __forceinline__ uint64_t ord64(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Keys of the blocks; padding items (index >= N) go after every block.
__global__ void k_greedy_keys(const double *mb, int64_t N, int64_t n2, SortItem *a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    SortItem it;
    it.key = i < N ? ord64(mb[i]) : 0ull;
    it.idx = i < N ? (uint32_t)i : 0xffffffffu;
    it.pad = 0;
    a[i] = it;
}

__device__ __forceinline__ void cmp_swap(SortItem &x, SortItem &y, bool asc) {
    // asc: the item that comes first ends at the lower position
    if (first(y, x) == asc) {
        const SortItem t = x;
        x = y;
        y = t;
    }
}

// In LDS: for kk == 0 every stage of sizes 2..kSortLocal; otherwise the
// stages of size kk with strides kSortLocal/2 .. 1.
__global__ void __launch_bounds__(kSortThreads) k_sort_local(SortItem *a, int64_t kk) {
    __shared__ SortItem s[kSortLocal];
    const int64_t base = (int64_t)blockIdx.x * kSortLocal;
    const int tid = threadIdx.x;
    s[tid] = a[base + tid];
    s[tid + kSortThreads] = a[base + tid + kSortThreads];
    __syncthreads();
    auto stage = [&](int64_t k, int j) {
        const int i = 2 * tid - (tid & (j - 1));   // lower element of this thread's pair
        const int l = i + j;
        const bool asc = ((base + i) & k) == 0;
        cmp_swap(s[i], s[l], asc);
        __syncthreads();
    };
    if (kk == 0) {
        for (int k = 2; k <= kSortLocal; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) stage(k, j);
    } else {
        for (int j = kSortLocal >> 1; j > 0; j >>= 1) stage(kk, j);
    }
    a[base + tid] = s[tid];
    a[base + tid + kSortThreads] = s[tid + kSortThreads];
}

// One stage of size k and stride j >= kSortLocal over global memory.
__global__ void k_sort_global(SortItem *a, int64_t k, int64_t j) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = 2 * t - (t & (j - 1));
    const int64_t l = i + j;
    SortItem x = a[i], y = a[l];
    cmp_swap(x, y, (i & k) == 0);
    a[i] = x;
    a[l] = y;
}

__global__ void k_greedy_unplace(DevModel m, int8_t *p, const SortItem *a, int32_t *order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.N) return;
    p[i] = (int8_t)m.T;
    order[i] = (int32_t)a[i].idx;
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, not for its global loads in flight (the coming list ids).
__device__ __forceinline__ void greedy_lds_sync() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0); vmcnt, expcnt untouched
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Most visits of a pass skip their block (a predecessor is still unplaced),
// so a visit first decides that from what needs no global load on its path:
// the block id (the list is read 64 ids at a time, the next 64 meanwhile),
// its predecessor ids (grid arithmetic, or the lists) and their periods
// (kLP: the schedule mirrored in LDS, one byte per block).  Only a block that
// may be placed loads its tonnage and ore words.  Without kLP (N too large
// for LDS) the periods are read from p after full barriers.
template <bool kLP>
__global__ void __launch_bounds__(kGT) k_greedy_walk(DevModel m, int8_t *p, int32_t *list0,
                                                     int32_t *list1, int32_t max_pass,
                                                     int32_t *out) {
    extern __shared__ double lds[];
    const int32_t T = m.T, S = m.S;
    double *O = lds;                       // [T][S]
    double *Ml = O + (size_t)T * S;        // [T]
    int8_t *pl = (int8_t *)(Ml + T);       // [N] when kLP
    __shared__ int32_t best_s[kGW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t i = tid; i < (int64_t)T * S; i += kGT) O[i] = 0.0;
    for (int t = tid; t < T; t += kGT) Ml[t] = 0.0;
    if (kLP)
        for (int64_t i = tid; i < m.N; i += kGT) pl[i] = (int8_t)T;   // all unplaced
    __syncthreads();
    auto sync = [&]() {
        if (kLP)
            greedy_lds_sync();
        else
            __syncthreads();
    };
    const int32_t G = (S + 255) / 256;     // groups of 256 scenarios
    int32_t *cur = list0, *nxt = list1;
    int32_t ncur = (int32_t)m.N;
    int32_t passes = 0;
    int64_t placed = 0;

    while (passes < max_pass) {
        ++passes;
        int32_t nn = 0;
        int64_t now = 0;
        // list ids [base, base + 64) in ids, the next 64 in flight in ids_next
        int32_t base = 0;
        int32_t ids = lane < ncur ? cur[lane] : -1;
        int32_t ids_next = 64 + lane < ncur ? cur[64 + lane] : -1;
        for (int32_t i = 0; i < ncur; ++i) {
            if (i == base + 64) {
                base += 64;
                ids = ids_next;
                ids_next = base + 64 + lane < ncur ? cur[base + 64 + lane] : -1;
            }
            const int32_t b = __builtin_amdgcn_readlane(ids, i - base);
            // earliest admissible period: every predecessor placed, at or before t
            const int64_t pid = lane < MPS_MAX_DEGREE ? nbr(m, b, lane, true) : -1;
            int32_t lo = pid >= 0 ? (int32_t)(kLP ? pl[pid] : p[pid]) : 0;
            for (int o = 1; o < kMaxPred; o <<= 1) lo = max(lo, __shfl_xor(lo, o));
            lo = __builtin_amdgcn_readfirstlane(lo);
            int32_t tb = T;
            double ton = 0.0;
            if (lo < T) {
                ton = m.ton64[b];
                uint32_t ore0[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int32_t s = lane + 64 * j;
                    ore0[j] = s < S ? m.ore[(int64_t)(s >> 5) * m.N + b] : 0u;
                }
                for (int32_t t0 = lo; t0 < T && tb == T; t0 += kGW) {
                    const int32_t t = t0 + wave;
                    bool bad = true;
                    if (t < T) {
                        bad = !(Ml[t] + ton <= m.mcap);
                        const double *Ot = O + (size_t)t * S;
                        for (int32_t g = 0; g < G && !bad; ++g) {
                            uint32_t orw[4];
                            if (g == 0) {
#pragma unroll
                                for (int j = 0; j < 4; ++j) orw[j] = ore0[j];
                            } else {
#pragma unroll
                                for (int j = 0; j < 4; ++j) {
                                    const int32_t s = g * 256 + lane + 64 * j;
                                    orw[j] = s < S ? m.ore[(int64_t)(s >> 5) * m.N + b] : 0u;
                                }
                            }
                            bool v = false;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const int32_t s = g * 256 + lane + 64 * j;
                                if (s < S && ((orw[j] >> (s & 31)) & 1u))
                                    v = v || !(Ot[s] + ton <= m.pcap);
                            }
                            bad = __ballot(v) != 0ull;
                        }
                    }
                    if (lane == 0) best_s[wave] = bad ? T : t;
                    sync();
                    int32_t bt = T;
#pragma unroll
                    for (int w = 0; w < kGW; ++w) bt = min(bt, best_s[w]);
                    tb = bt;
                    sync();   // best_s is rewritten by the next round
                }
            }
            if (tb < T) {
                double *Ot = O + (size_t)tb * S;
                for (int32_t s = tid; s < S; s += kGT)
                    if ((m.ore[(int64_t)(s >> 5) * m.N + b] >> (s & 31)) & 1u) Ot[s] += ton;
                if (tid == 0) {
                    Ml[tb] += ton;
                    p[b] = (int8_t)tb;
                    if (kLP) pl[b] = (int8_t)tb;
                }
                ++now;
                sync();
            } else {
                if (tid == 0) nxt[nn] = b;
                ++nn;
            }
        }
        // the next pass reads the list wave 0 has just written
        __syncthreads();
        placed += now;
        int32_t *t = cur;
        cur = nxt;
        nxt = t;
        ncur = nn;
        if (now == 0) break;
    }
    if (tid == 0) {
        out[0] = passes;
        out[1] = (int32_t)placed;
    }
}

size_t greedy_ws_bytes(const DevModel &m) {
    int64_t n2 = kSortLocal;
    while (n2 < m.N) n2 <<= 1;
    return (size_t)n2 * sizeof(SortItem) + 2 * 4 * (size_t)m.N + 256;
}

size_t greedy_lds_bytes(const DevModel &m) {
    return 8 * ((size_t)m.T * m.S + m.T) + 64;   // + the round results (static)
}

static size_t greedy_lds_map_bytes(const DevModel &m) {
    return greedy_lds_bytes(m) + (size_t)m.N;
}

hipError_t launch_greedy(const DevModel &m, int8_t *p, int32_t max_pass, void *ws,
                         int32_t *out, hipStream_t st) {
    int64_t n2 = kSortLocal;
    while (n2 < m.N) n2 <<= 1;
    char *c = (char *)ws;
    SortItem *a = (SortItem *)c;
    c += (size_t)n2 * sizeof(SortItem);
    int32_t *l0 = (int32_t *)c;
    int32_t *l1 = l0 + m.N;
    hipLaunchKernelGGL(k_greedy_keys, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st,
                       m.mb64, m.N, n2, a);
    const unsigned nb = (unsigned)(n2 / kSortLocal);
    hipLaunchKernelGGL(k_sort_local, dim3(nb), dim3(kSortThreads), 0, st, a, (int64_t)0);
    for (int64_t k = 2 * kSortLocal; k <= n2; k <<= 1) {
        for (int64_t j = k >> 1; j >= kSortLocal; j >>= 1)
            hipLaunchKernelGGL(k_sort_global, dim3((unsigned)(n2 / 2 / 256)), dim3(256), 0, st,
                               a, k, j);
        hipLaunchKernelGGL(k_sort_local, dim3(nb), dim3(kSortThreads), 0, st, a, k);
    }
    hipLaunchKernelGGL(k_greedy_unplace, dim3((unsigned)((m.N + 255) / 256)), dim3(256), 0, st,
                       m, p, a, l0);
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if (greedy_lds_map_bytes(m) <= (size_t)max_lds)
        hipLaunchKernelGGL(k_greedy_walk<true>, dim3(1), dim3(kGT), greedy_lds_map_bytes(m), st,
                           m, p, l0, l1, max_pass, out);
    else
        hipLaunchKernelGGL(k_greedy_walk<false>, dim3(1), dim3(kGT), greedy_lds_bytes(m), st, m,
                           p, l0, l1, max_pass, out);
    return hipGetLastError();
}

}  // namespace mps
