// batch.hip -- many models with uneven move lists evaluated by persistent
// workgroups, ending with each model's exact top k (the candidate evaluation
// of Alg. 5 applied to a population of schedules at once, the shape of work
// the metaheuristic of Alg. 2 produces: one schedule per individual, each with
// its own candidate list).
//
// Persistent launches over queues of work items (largest model first), taken
// by resident workgroups from an atomic counter, and small launches of one
// workgroup per model:
//   1. block items (model i, item j): the per-block quantities of the list
//      pass (c_b, removal term, precedence window) for tiles [j*tpi, j*tpi+tpi)
//      of 64 blocks, written to the model's block workspace;
//   2. move items (model i, item j): moves [j*mpi, j*mpi+mpi) of model i
//      scored and flagged, with the top 12 bits of their top-k keys counted
//      into the model's level-0 histogram;
//   3. the exact top k of every model (the key and order of mps_topk), by a
//      radix select whose passes over the moves are again move items:
//      a. per model, the level-0 boundary digit from that histogram;
//      b. move items of models whose boundary digit holds more than kSegCap
//         keys: keys above it are selected, the next 11 bits of the keys on
//         it are counted;
//      c. per model, the level-1 boundary digit;
//      d. move items: the remaining selected keys and the boundary keys
//         (at most kSegCap) are gathered;
//      e. per model: the boundary refined on chip, the k keys sorted.
//      A model with more than kSegCap keys sharing its top 23 key bits is
//      walked by one workgroup instead (e).
// The launch boundaries order the phases; no workgroup ever waits on another.
//
// Per-model tuning (from the autotuner, or defaults): tiles per block item,
// moves per move item, and the number of v rows each lane has in flight
// (8, 16 or 32; a template argument of the tile code).
#include "batch.h"
#include "eval_dev.h"
#include "topk_dev.h"

namespace mps {

constexpr int kBT = kNT;                 // threads per persistent workgroup
constexpr int kSegLevels = 6;
__constant__ int c_seg_shift[kSegLevels] = {52, 41, 30, 19, 8, 0};
__constant__ int c_seg_bits[kSegLevels] = {12, 11, 11, 11, 11, 8};

// LDS of the segmented top-k: histogram, part/res scratch, counters, the
// selected keys and two candidate buffers.
struct SegLds {
    uint32_t *h;      // [kSegBins]
    uint32_t *part;   // [4]
    int32_t *res;     // [4]
    int32_t *cnt;     // [4]: selected, candidates (two buffers), spare
    uint64_t *sel;    // [MPS_MAX_BATCH_TOPK]
    uint64_t *cand[2];// [kSegCap] each
};

__host__ __device__ inline size_t seg_lds_layout(char *base, SegLds *L) {
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t o = off;
        off = a16(off + bytes);
        return o;
    };
    const size_t o_h = put(sizeof(uint32_t) * kSegBins);
    const size_t o_p = put(sizeof(uint32_t) * 4);
    const size_t o_r = put(sizeof(int32_t) * 4);
    const size_t o_c = put(sizeof(int32_t) * 4);
    const size_t o_s = put(sizeof(uint64_t) * MPS_MAX_BATCH_TOPK);
    const size_t o_c0 = put(sizeof(uint64_t) * kSegCap);
    const size_t o_c1 = put(sizeof(uint64_t) * kSegCap);
    if (L) {
        L->h = (uint32_t *)(base + o_h);
        L->part = (uint32_t *)(base + o_p);
        L->res = (int32_t *)(base + o_r);
        L->cnt = (int32_t *)(base + o_c);
        L->sel = (uint64_t *)(base + o_s);
        L->cand[0] = (uint64_t *)(base + o_c0);
        L->cand[1] = (uint64_t *)(base + o_c1);
    }
    return off;
}

size_t batch_lds_bytes(const DevModel &m) {
    const size_t tile = tile_lds_layout(m, nullptr, nullptr);
    const size_t moves = tile + sizeof(uint32_t) * kSegBins;
    const size_t seg = seg_lds_layout(nullptr, nullptr);
    return moves > seg ? moves : seg;
}

// Clears the queue heads, histograms and per-model states.
__global__ void k_batch_init(uint32_t *ctl, int64_t nwords) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords;
         i += (int64_t)gridDim.x * blockDim.x)
        ctl[i] = 0u;
}

// ---- phase 1: per-block quantities of tiles [t0, t1) ------------------------
template <int KCH>
__device__ void batch_blocks(const DevModel &m, char *lds, int32_t t0, int32_t t1) {
    TileLds L;
    tile_lds_layout(m, lds, &L);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const TablePrefetch tp = issue_tables(m);
    const TabView tv = commit_tables(m, L, tp);   // barrier inside
    int32_t s0, s1;
    wave_range(m, wave, s0, s1);
    for (int32_t tile = t0; tile < t1; ++tile) {
        const int64_t b = (int64_t)tile * 64 + lane;
        const bool valid = b < m.N;
        float x[KCH];
        issue_rows(m, b, valid, s0, s1, x);
        BlockInfo bi{};
        if (valid && wave == 0) bi = load_block(m, b);
        for (int32_t w = wave; w < m.W; w += kNW)
            L.ore[w * 64 + lane] = valid ? gld(m.ore + (int64_t)w * m.N + b) : 0u;
        L.cpart[wave * 64 + lane] = wave_dot(m, m.e32, b, valid, s0, s1, x);
        __syncthreads();
        const float c = tile_c(L, lane, m.S);
        if (wave == 0 && valid) {
            auto ow = [&](int32_t w) { return L.ore[w * 64 + lane]; };
            put_list_rec(m, b, c, removal_term(m, tv, bi.pb, bi.ton32, ow), bi, ow);
        }
        __syncthreads();   // cpart and ore are rewritten by the next tile
    }
}

// ---- phase 2: moves [i0, i1) of one model ------------------------------------
__device__ void batch_moves(const DevModel &m, const BatchInst &I, char *lds, int64_t i0,
                            int64_t i1, uint32_t *ghist, uint8_t req, uint8_t forbid) {
    TileLds L;
    tile_lds_layout(m, lds, &L);
    uint32_t *h = (uint32_t *)L.end;
    const int tid = threadIdx.x;
    const TablePrefetch tp = issue_tables(m);
    for (int j = tid; j < kSegBins; j += kBT) h[j] = 0u;
    const TabView tv = commit_tables(m, L, tp);   // barrier inside
    // moves in block order (perm), results and keys at their own positions
    for (int64_t i = i0 + tid; i < i1; i += kBT) {
        const int64_t p = gld(I.perm + i);
        const MoveOut o = list_move(m, tv, L, gld(I.blk + p), (int32_t)gld(I.per + p));
        gst(I.score + p, o.score);
        gst(I.flags + p, o.flags);
        uint64_t key;
        if (key_from(o.score, o.flags, p, req, forbid, key))
            atomicAdd(&h[(int)(key >> 52)], 1u);
    }
    __syncthreads();
    for (int j = tid; j < kSegBins; j += kBT) {
        const uint32_t c = h[j];
        if (c) atomicAdd(&ghist[j], c);
    }
}

// Bitonic sort of n (a power of two, <= MPS_MAX_BATCH_TOPK) keys in LDS,
// descending.
__device__ void sort_desc(uint64_t *s, int n) {
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < (n >> 1); i += kBT) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool desc = (lo & size) == 0;
                const uint64_t a = s[lo], b = s[hi];
                if ((a < b) == desc) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

// ---- phase 3: exact top k of one model --------------------------------------
// Radix select on the 64-bit keys from the top digit down.  Level 0's
// histogram was filled by the phase-2 items.  While the keys on the boundary
// digit are too many for LDS, one pass over the model's moves appends the keys
// above the boundary to the selection and counts the next digit of the keys on
// it; once they fit, one pass collects them and the remaining levels run on
// chip.  Keys are unique, so the boundary narrows to exactly the keys needed.
// Calls fn(qualifies, key) for every move of a model: 32 moves per thread
// per step, their loads all issued before the first is used (one workgroup
// walks a whole model, so the passes are bound by load latency).  Every
// thread makes the same number of calls.
template <class F>
__device__ __forceinline__ void for_keys(const BatchInst &I, uint8_t req, uint8_t forbid, F fn) {
    constexpr int U = 32;
    const int64_t n = I.n;
    for (int64_t i0 = 0; i0 < n; i0 += (int64_t)U * kBT) {
        float sc[U];
        uint8_t fl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * kBT + threadIdx.x;
            sc[u] = i < n ? gld(I.score + i) : 0.0f;
            fl[u] = i < n ? gld(I.flags + i) : (uint8_t)0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * kBT + threadIdx.x;
            uint64_t key = 0;
            const bool q = i < n && key_from(sc[u], fl[u], i, req, forbid, key);
            fn(q, key);
        }
    }
}

// On-chip refinement of the boundary keys L.cand[0][0, L.cnt[1]), whose
// digits down to `level` equal the boundary's, until exactly `need` of them
// are selected: the keys above each level's boundary digit join L.sel.
// Returns the number of keys in L.sel.  Called by every thread.
__device__ int32_t refine_chip(const SegLds &L, int level, int32_t need) {
    const int tid = threadIdx.x;
    int cb = 0;
    while (need < L.cnt[1 + cb] && level + 1 < kSegLevels) {
        const int nb = 1 << c_seg_bits[level + 1];
        const int sh1 = c_seg_shift[level + 1];
        const uint64_t mask1 = (1ull << c_seg_bits[level + 1]) - 1ull;
        const int32_t nc = L.cnt[1 + cb];
        const uint64_t *src = cb ? L.cand[1] : L.cand[0];
        uint64_t *dst = cb ? L.cand[0] : L.cand[1];
        for (int j = tid; j < nb; j += kBT) L.h[j] = 0u;
        if (tid == 0) L.cnt[2 - cb] = 0;
        __syncthreads();
        for (int j = tid; j < nc; j += kBT)
            atomicAdd(&L.h[(int)((src[j] >> sh1) & mask1)], 1u);
        __syncthreads();
        select_digit(L.h, nb, need, L.part, L.res);
        const uint64_t dsel = (uint64_t)L.res[0];
        need -= L.res[1];
        for (int j0 = 0; j0 < nc; j0 += kBT) {
            const int j = j0 + tid;
            const uint64_t key = j < nc ? src[j] : 0ull;
            const uint64_t d = (key >> sh1) & mask1;
            wave_append(j < nc && d > dsel, key, L.sel, &L.cnt[0]);
            wave_append(j < nc && d == dsel, key, dst, &L.cnt[2 - cb]);
        }
        __syncthreads();
        cb = 1 - cb;
        ++level;
    }
    // the remaining boundary keys are exactly the ones still needed
    const int32_t nc = L.cnt[1 + cb];
    const int32_t ns = L.cnt[0];
    const uint64_t *last = cb ? L.cand[1] : L.cand[0];
    for (int j = tid; j < nc; j += kBT) L.sel[ns + j] = last[j];
    __syncthreads();
    return ns + nc;
}

// Sorts L.sel[0, n_sel_final) descending and writes the model's top k.
__device__ void write_topk(const BatchInst &I, const SegLds &L, int32_t n_sel_final, int32_t k) {
    const int tid = threadIdx.x;
    int P = 2;
    while (P < n_sel_final) P <<= 1;
    for (int j = n_sel_final + tid; j < P; j += kBT) L.sel[j] = 0ull;
    __syncthreads();
    sort_desc(L.sel, P);
    for (int j = tid; j < k; j += kBT) {
        if (j < n_sel_final) {
            const uint64_t key = L.sel[j];
            gst(I.top_idx + j, (int64_t)(0xffffffffu - (uint32_t)(key & 0xffffffffu)));
            if (I.top_score) gst(I.top_score + j, unord_f32((uint32_t)(key >> 32)));
        } else {
            gst(I.top_idx + j, (int64_t)-1);
            if (I.top_score) gst(I.top_score + j, -INFINITY);
        }
    }
    if (tid == 0) gst(I.top_count, n_sel_final);
}

__device__ void batch_topk(const BatchInst &I, char *lds, const uint32_t *ghist, int32_t k,
                           uint8_t req, uint8_t forbid) {
    SegLds L;
    seg_lds_layout(lds, &L);
    const int tid = threadIdx.x;
    const int64_t n = I.n;
    for (int j = tid; j < kSegBins; j += kBT) L.h[j] = ghist[j];
    if (tid < 4) L.cnt[tid] = 0;
    __syncthreads();
    select_digit(L.h, kSegBins, k, L.part, L.res);   // barriers inside
    const int32_t total = L.res[2];
    int32_t n_sel_final;
    if (total <= k) {
        // every qualifying move is selected
        for_keys(I, req, forbid,
                 [&](bool q, uint64_t key) { wave_append(q, key, L.sel, &L.cnt[0]); });
        __syncthreads();
        n_sel_final = L.cnt[0];
    } else {
        int level = 0;
        int32_t need = k - L.res[1];
        uint64_t pfx = (uint64_t)L.res[0];   // key >> shift[level] of the boundary
        uint32_t n_eq = L.h[L.res[0]];
        // global passes while the boundary keys do not fit on chip
        while (n_eq > (uint32_t)kSegCap && level + 1 < kSegLevels) {
            const int nb = 1 << c_seg_bits[level + 1];
            __syncthreads();
            for (int j = tid; j < nb; j += kBT) L.h[j] = 0u;
            __syncthreads();
            const int sh = c_seg_shift[level], sh1 = c_seg_shift[level + 1];
            const int shp = level > 0 ? c_seg_shift[level - 1] : 64;
            const uint64_t pfx_prev = pfx >> (shp - sh);   // unused at level 0
            const uint64_t mask1 = (1ull << c_seg_bits[level + 1]) - 1ull;
            for_keys(I, req, forbid, [&](bool q, uint64_t key) {
                bool above = false;
                if (q) {
                    const uint64_t top = key >> sh;
                    const bool in_prev = level == 0 || (key >> shp) == pfx_prev;
                    above = in_prev && top > pfx;
                    if (top == pfx) atomicAdd(&L.h[(int)((key >> sh1) & mask1)], 1u);
                }
                wave_append(above, key, L.sel, &L.cnt[0]);
            });
            __syncthreads();
            select_digit(L.h, nb, need, L.part, L.res);
            need -= L.res[1];
            n_eq = L.h[L.res[0]];
            pfx = (pfx << c_seg_bits[level + 1]) | (uint64_t)L.res[0];
            ++level;
        }
        // collect the keys above the boundary (within the previous prefix)
        // and the boundary keys themselves
        {
            const int sh = c_seg_shift[level];
            const int shp = level > 0 ? c_seg_shift[level - 1] : 64;
            const uint64_t pfx_prev = level > 0 ? pfx >> (shp - sh) : 0ull;
            for_keys(I, req, forbid, [&](bool q, uint64_t key) {
                const uint64_t top = key >> sh;
                const bool in_prev = level == 0 || (key >> shp) == pfx_prev;
                wave_append(q && in_prev && top > pfx, key, L.sel, &L.cnt[0]);
                wave_append(q && top == pfx, key, L.cand[0], &L.cnt[1]);
            });
            __syncthreads();
        }
        n_sel_final = refine_chip(L, level, need);
    }
    write_topk(I, L, n_sel_final, k);
}

// Take the next item of a queue: one atomic per workgroup, broadcast in LDS.
__device__ __forceinline__ int32_t next_item(uint32_t *head, int32_t *slot) {
    if (threadIdx.x == 0) *slot = (int32_t)atomicAdd(head, 1u);
    __syncthreads();
    const int32_t q = *slot;
    __syncthreads();
    return q;
}

__global__ void __launch_bounds__(kBT) k_batch_blocks(const BatchInst *insts, const int2 *items,
                                                      int32_t n_items, uint32_t *head) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int32_t s_item;
    for (;;) {
        const int32_t q = next_item(head, &s_item);
        if (q >= n_items) break;
        const int2 it = items[q];
        const BatchInst &I = insts[it.x];
        const int32_t t0 = it.y * I.tiles_per_item;
        const int32_t t1 = min(I.n_tiles, t0 + I.tiles_per_item);
        if (I.rows <= 8)
            batch_blocks<8>(I.m, lds, t0, t1);
        else if (I.rows <= 16)
            batch_blocks<16>(I.m, lds, t0, t1);
        else
            batch_blocks<32>(I.m, lds, t0, t1);
    }
}

__global__ void __launch_bounds__(kBT) k_batch_moves(const BatchInst *insts, const int2 *items,
                                                     int32_t n_items, uint32_t *head,
                                                     uint32_t *ghist_all, uint8_t req,
                                                     uint8_t forbid) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int32_t s_item;
    for (;;) {
        const int32_t q = next_item(head, &s_item);
        if (q >= n_items) break;
        const int2 it = items[q];
        const BatchInst &I = insts[it.x];
        const int64_t i0 = (int64_t)it.y * I.moves_per_item;
        const int64_t i1 = min(I.n, i0 + I.moves_per_item);
        batch_moves(I.m, I, lds, i0, i1, ghist_all + (size_t)it.x * kSegBins, req, forbid);
        __syncthreads();   // LDS is reused by the next item
    }
}

// ---- phase 3 with the passes as move items ----------------------------------
// Calls fn(qualifies, key) for every move of [i0, i1) of a model, eight moves
// per thread per step with their loads issued first.  Every thread of the
// workgroup makes the same number of calls.
template <class F>
__device__ __forceinline__ void for_keys_range(const BatchInst &I, int64_t i0, int64_t i1,
                                               uint8_t req, uint8_t forbid, F fn) {
    constexpr int U = 8;
    for (int64_t j0 = i0; j0 < i1; j0 += (int64_t)U * kBT) {
        float sc[U];
        uint8_t fl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = j0 + (int64_t)u * kBT + threadIdx.x;
            sc[u] = i < i1 ? gld(I.score + i) : 0.0f;
            fl[u] = i < i1 ? gld(I.flags + i) : (uint8_t)0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = j0 + (int64_t)u * kBT + threadIdx.x;
            uint64_t key = 0;
            const bool q = i < i1 && key_from(sc[u], fl[u], i, req, forbid, key);
            fn(q, key);
        }
    }
}

// wave_append into a global buffer of cap entries (a count past cap, which
// the histograms rule out, writes nothing).
__device__ __forceinline__ void wave_append_global(bool pred, uint64_t key, uint64_t *buf,
                                                   int32_t *cnt, int32_t cap) {
    const uint64_t mask = __ballot(pred);
    if (mask == 0) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (int32_t)__popcll(mask));
    base = __builtin_amdgcn_readlane(base, leader);
    if (pred) {
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        const int32_t j = base + (int32_t)__popcll(mask & below);
        if (j < cap) gst(buf + j, key);
    }
}

// a. level-0 boundary digit of model blockIdx.x
__global__ void __launch_bounds__(kBT) k_bt_select0(BatchCtl c, int32_t k) {
    __shared__ uint32_t h[kSegBins];
    __shared__ uint32_t part[4];
    __shared__ int32_t res[4];
    const int32_t i = blockIdx.x;
    const uint32_t *g = c.hist0 + (int64_t)i * kSegBins;
    for (int j = threadIdx.x; j < kSegBins; j += kBT) h[j] = g[j];
    __syncthreads();
    select_digit(h, kSegBins, k, part, res);   // barriers inside
    if (threadIdx.x == 0) {
        BtState &s = c.state[i];
        if (res[2] <= k) {
            s.mode = kBtTakeAll;
            s.need = 0;
        } else {
            const int32_t d0 = res[0];
            s.d0 = (uint32_t)d0;
            s.need = k - res[1];
            s.mode = h[d0] <= (uint32_t)kSegCap ? kBtCollect0 : kBtPass1;
        }
    }
}

// Take the next claim of g consecutive items of a queue.
__device__ __forceinline__ int32_t next_claim(uint32_t *head, int32_t g, int32_t *slot) {
    if (threadIdx.x == 0) *slot = (int32_t)atomicAdd(head, (uint32_t)g);
    __syncthreads();
    const int32_t q = *slot;
    __syncthreads();
    return q;
}

// Calls fn(model, i0, i1) for the claimed items [q0, q1), with consecutive
// items of one model merged into one range of its moves (uniform).
template <class F>
__device__ __forceinline__ void for_runs(const BatchInst *insts, const int2 *items, int32_t q0,
                                         int32_t q1, F fn) {
    int32_t model = -1;
    int64_t i0 = 0, i1 = 0;
    for (int32_t q = q0; q < q1; ++q) {
        const int2 it = items[q];
        const BatchInst &I = insts[it.x];
        const int64_t a = (int64_t)it.y * I.moves_per_item;
        const int64_t b = min(I.n, a + I.moves_per_item);
        if (it.x == model && a == i1) {
            i1 = b;
            continue;
        }
        if (model >= 0) fn(model, i0, i1);
        model = it.x;
        i0 = a;
        i1 = b;
    }
    if (model >= 0) fn(model, i0, i1);
}

// b. move items of models in kBtPass1: keys above the level-0 boundary are
// selected, the next 11 bits of the keys on it counted.  A claim takes g
// consecutive items; the LDS histogram is flushed when the model changes.
__global__ void __launch_bounds__(kBT) k_bt_pass1(const BatchInst *insts, const int2 *items,
                                                  int32_t n_items, int32_t g, BatchCtl c,
                                                  uint8_t req, uint8_t forbid) {
    __shared__ uint32_t h[kSegBins1];
    __shared__ int32_t s_item;
    auto flush = [&](int32_t model) {
        __syncthreads();
        uint32_t *gh = c.hist1 + (int64_t)model * kSegBins1;
        for (int j = threadIdx.x; j < kSegBins1; j += kBT) {
            const uint32_t v = h[j];
            if (v) atomicAdd(gh + j, v);
            h[j] = 0u;
        }
        __syncthreads();
    };
    for (int j = threadIdx.x; j < kSegBins1; j += kBT) h[j] = 0u;
    for (;;) {
        const int32_t q0 = next_claim(c.head + 2, g, &s_item);
        if (q0 >= n_items) break;
        for_runs(insts, items, q0, min(n_items, q0 + g), [&](int32_t model, int64_t i0, int64_t i1) {
            BtState &st = c.state[model];
            if (gld(&st.mode) != kBtPass1) return;   // uniform
            const BatchInst &I = insts[model];
            const uint64_t d0 = gld(&st.d0);
            uint64_t *sel = c.sel + (int64_t)model * MPS_MAX_BATCH_TOPK;
            for_keys_range(I, i0, i1, req, forbid, [&](bool qk, uint64_t key) {
                const uint64_t top = key >> 52;
                wave_append_global(qk && top > d0, key, sel, &st.n_sel, MPS_MAX_BATCH_TOPK);
                if (qk && top == d0) atomicAdd(&h[(int)((key >> 41) & (kSegBins1 - 1))], 1u);
            });
            flush(model);
        });
    }
}

// c. level-1 boundary digit of model blockIdx.x (models in kBtPass1)
__global__ void __launch_bounds__(kBT) k_bt_select1(BatchCtl c) {
    __shared__ uint32_t h[kSegBins1];
    __shared__ uint32_t part[4];
    __shared__ int32_t res[4];
    const int32_t i = blockIdx.x;
    BtState &s = c.state[i];
    if (gld(&s.mode) != kBtPass1) return;   // uniform
    const int32_t need = gld(&s.need);
    const uint32_t *g = c.hist1 + (int64_t)i * kSegBins1;
    for (int j = threadIdx.x; j < kSegBins1; j += kBT) h[j] = g[j];
    __syncthreads();
    select_digit(h, kSegBins1, need, part, res);   // barriers inside
    if (threadIdx.x == 0) {
        const int32_t d1 = res[0];
        s.d1 = (uint32_t)d1;
        s.need = need - res[1];
        s.mode = h[d1] <= (uint32_t)kSegCap ? kBtCollect1 : kBtFallback;
    }
}

// d. move items: the keys still to select and the boundary keys
__global__ void __launch_bounds__(kBT) k_bt_collect(const BatchInst *insts, const int2 *items,
                                                    int32_t n_items, int32_t g, BatchCtl c,
                                                    uint8_t req, uint8_t forbid) {
    __shared__ int32_t s_item;
    for (;;) {
        const int32_t q0 = next_claim(c.head + 3, g, &s_item);
        if (q0 >= n_items) break;
        for_runs(insts, items, q0, min(n_items, q0 + g), [&](int32_t model, int64_t i0, int64_t i1) {
        BtState &st = c.state[model];
        const int32_t mode = gld(&st.mode);
        if (mode != kBtTakeAll && mode != kBtCollect0 && mode != kBtCollect1) return;
        const BatchInst &I = insts[model];
        const uint64_t d0 = gld(&st.d0), d1 = gld(&st.d1);
        uint64_t *sel = c.sel + (int64_t)model * MPS_MAX_BATCH_TOPK;
        uint64_t *cand = c.cand + (int64_t)model * kSegCap;
        for_keys_range(I, i0, i1, req, forbid, [&](bool qk, uint64_t key) {
            const uint64_t top = key >> 52, mid = (key >> 41) & (kSegBins1 - 1);
            bool s_, c_;
            if (mode == kBtTakeAll) {
                s_ = qk;
                c_ = false;
            } else if (mode == kBtCollect0) {
                s_ = qk && top > d0;
                c_ = qk && top == d0;
            } else {
                s_ = qk && top == d0 && mid > d1;
                c_ = qk && top == d0 && mid == d1;
            }
            wave_append_global(s_, key, sel, &st.n_sel, MPS_MAX_BATCH_TOPK);
            wave_append_global(c_, key, cand, &st.n_cand, kSegCap);
        });
        });
    }
}

// e. one workgroup per model, largest model first: the boundary refined on
// chip and the k keys sorted; a model in kBtFallback is walked whole.
__global__ void __launch_bounds__(kBT) k_bt_final(const BatchInst *insts, const int32_t *order,
                                                  BatchCtl c, int32_t k, uint8_t req,
                                                  uint8_t forbid) {
    extern __shared__ __align__(16) char lds[];
    const int32_t i = order[blockIdx.x];
    const BatchInst &I = insts[i];
    const BtState st = c.state[i];
    if (st.mode == kBtFallback) {
        batch_topk(I, lds, c.hist0 + (int64_t)i * kSegBins, k, req, forbid);
        return;
    }
    SegLds L;
    seg_lds_layout(lds, &L);
    const int tid = threadIdx.x;
    const int32_t ns = min(st.n_sel, (int32_t)MPS_MAX_BATCH_TOPK);
    const int32_t nc = min(st.n_cand, (int32_t)kSegCap);
    const uint64_t *sel = c.sel + (int64_t)i * MPS_MAX_BATCH_TOPK;
    const uint64_t *cand = c.cand + (int64_t)i * kSegCap;
    for (int j = tid; j < ns; j += kBT) L.sel[j] = gld(sel + j);
    for (int j = tid; j < nc; j += kBT) L.cand[0][j] = gld(cand + j);
    if (tid == 0) {
        L.cnt[0] = ns;
        L.cnt[1] = nc;
        L.cnt[2] = 0;
        L.cnt[3] = 0;
    }
    __syncthreads();
    int32_t n_sel_final = ns;
    if (st.mode == kBtCollect0)
        n_sel_final = refine_chip(L, 0, st.need);
    else if (st.mode == kBtCollect1)
        n_sel_final = refine_chip(L, 1, st.need);
    write_topk(I, L, n_sel_final, k);
}

hipError_t launch_batch(const BatchLaunch &bl, hipStream_t st) {
    const BatchCtl c = batch_ctl(bl.ctl, bl.n_inst);
    const int64_t nwords = batch_ctl_clear_words(bl.n_inst);
    int64_t g = (nwords + 255) / 256;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_batch_init, dim3((unsigned)g), dim3(256), 0, st, bl.ctl, nwords);
    if (bl.n_items1 > 0)
        hipLaunchKernelGGL(k_batch_blocks, dim3((unsigned)bl.grid1), dim3(kBT), bl.lds_bytes, st,
                           bl.insts, bl.items1, bl.n_items1, c.head);
    if (bl.n_items2 > 0)
        hipLaunchKernelGGL(k_batch_moves, dim3((unsigned)bl.grid2), dim3(kBT), bl.lds_bytes, st,
                           bl.insts, bl.items2, bl.n_items2, c.head + 1, c.hist0, bl.req,
                           bl.forbid);
    const dim3 per_model((unsigned)bl.n_inst);
    hipLaunchKernelGGL(k_bt_select0, per_model, dim3(kBT), 0, st, c, bl.k);
    if (bl.n_items2 > 0)
        hipLaunchKernelGGL(k_bt_pass1, dim3((unsigned)bl.grid2), dim3(kBT), 0, st, bl.insts,
                           bl.items2, bl.n_items2, bl.claim, c, bl.req, bl.forbid);
    hipLaunchKernelGGL(k_bt_select1, per_model, dim3(kBT), 0, st, c);
    if (bl.n_items2 > 0)
        hipLaunchKernelGGL(k_bt_collect, dim3((unsigned)bl.grid2), dim3(kBT), 0, st, bl.insts,
                           bl.items2, bl.n_items2, bl.claim, c, bl.req, bl.forbid);
    hipLaunchKernelGGL(k_bt_final, per_model, dim3(kBT), bl.lds_bytes, st, bl.insts, bl.order, c,
                       bl.k, bl.req, bl.forbid);
    return hipGetLastError();
}

hipError_t batch_occupancy(size_t lds_bytes, int *per_cu) {
    int a = 0, b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_batch_blocks, kBT, lds_bytes);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_batch_moves, kBT, lds_bytes);
    *per_cu = a < b ? a : b;
    return e;
}

}  // namespace mps
