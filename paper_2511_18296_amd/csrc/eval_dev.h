// eval_dev.h -- device helpers of move evaluation shared by the single-model
// kernels (eval.hip) and the batched persistent kernel (batch.hip): the risk,
// penalty and flag arithmetic of one move, the per-block loads, the LDS
// staging of the penalty tables and the scenario-split dot product.
#pragma once
#include <float.h>

#include "internal.h"

namespace mps {

constexpr int kListCap = 256;   // partial-list entries staged in LDS per kind
constexpr int kNW = 8;          // waves per 64-block tile
constexpr int kNT = 64 * kNW;   // threads per tile
constexpr int kCH = 32;         // v rows in flight per lane

struct MoveOut {
    float score, dr, dpp, dpm;
    uint8_t flags;
};

// View of the penalty tables (LDS copies; long lists stay in HBM).
struct TabView {
    const uint32_t *full_add, *full_rem;   // [T][W]
    const int32_t *rng;                    // [4][T] list ranges
    const AddEntry *add_l, *add_g;         // list entries: LDS copy / in HBM
    const RemEntry *rem_l, *rem_g;
    bool small;                            // the lists fit their LDS copies
    bool add_small;                        // ... and the added-tonnage one was made
};

// Risk, penalty and flag arithmetic of one move, given the block quantities.
// ore_word(w) returns ore word w of block b.
template <class OreWord>
__device__ __forceinline__ MoveOut score_move(const DevModel &m, const TabView &tv,
                                              const double *d64, const double *Ms, int32_t t,
                                              int32_t pb, int32_t lo, int32_t hi, float c,
                                              float remv, float ton32, double ton64, float mb,
                                              float Vb, float var32, float sig32, float lam,
                                              float pps, OreWord ore_word) {
    const int32_t T = m.T;
    MoveOut o;
    const bool noop = (t == pb);
    const float dd = (float)(d64[t] - d64[pb]);
    const float dvar = fmaf(2.0f * dd, c, dd * dd * Vb);
    const float vp = fmaxf(var32 + dvar, 0.0f);
    const float den = sqrtf(vp) + sig32;
    const float dsig = den > 0.0f ? dvar / den : 0.0f;
    const float dr = fmaf(dd, mb, -lam * dsig);

    float addv = 0.0f;
    bool viol = false;
    if (t < T && !noop) {
        int32_t cnt = 0;
        const uint32_t *fa = tv.full_add + (int64_t)t * m.W;
        for (int32_t w = 0; w < m.W; ++w) cnt += __popc(ore_word(w) & fa[w]);
        addv = (float)cnt * ton32;
        viol = cnt != 0;
        const int32_t j0 = tv.rng[t], j1 = tv.rng[T + t];
        auto entry = [&](const AddEntry &e) {
            if ((ore_word(e.s >> 5) >> (e.s & 31)) & 1u) {
                addv += fmaxf(ton32 - e.d, 0.0f);
                if (ton64 >= e.tau) viol = true;
            }
        };
        // one loop per memory: LDS copy, or the lists in HBM
        if (tv.add_small)
            for (int32_t j = j0; j < j1; ++j) entry(tv.add_l[j]);
        else
            for (int32_t j = j0; j < j1; ++j) entry(gld(tv.add_g + j));
    }
    double am = 0.0;
    bool mine_ok = true;
    if (!noop) {
        if (t < T) {
            const double Mt = Ms[t];
            am += hinge64(Mt + ton64, m.mcap) - hinge64(Mt, m.mcap);
            mine_ok = Mt + ton64 <= m.mcap;
        }
        if (pb < T) {
            const double Mp = Ms[pb];
            am += hinge64(Mp - ton64, m.mcap) - hinge64(Mp, m.mcap);
        }
    }
    const float dpp = noop ? 0.0f : pps * (addv - remv);
    const float dpm = (float)(m.pen_mine * am);
    uint8_t f = 0;
    if (lo <= t && t <= hi) f |= MPS_PREC_OK;
    if (noop || t == T || mine_ok) f |= MPS_MINE_OK;
    if (noop || t == T || !viol) f |= MPS_PROC_OK;
    if (noop) f |= MPS_NOOP;
    o.flags = f;
    o.dr = noop ? 0.0f : dr;
    o.dpp = dpp;
    o.dpm = noop ? 0.0f : dpm;
    o.score = noop ? 0.0f : (dr - dpp) - dpm;
    return o;
}

// Removal term of block b from its current period pb:
// sum_s ore[s][b] * clamp(O[pb][s] - cap, 0, ton_b)  (0 when pb = T).
template <class OreWord>
__device__ __forceinline__ float removal_term(const DevModel &m, const TabView &tv, int32_t pb,
                                              float ton32, OreWord ore_word) {
    const int32_t T = m.T;
    if (pb >= T) return 0.0f;
    int32_t cnt = 0;
    const uint32_t *fr = tv.full_rem + (int64_t)pb * m.W;
    for (int32_t w = 0; w < m.W; ++w) cnt += __popc(ore_word(w) & fr[w]);
    float r = (float)cnt * ton32;
    const int32_t j0 = tv.rng[2 * T + pb], j1 = tv.rng[3 * T + pb];
    auto entry = [&](const RemEntry &e) {
        if ((ore_word(e.s >> 5) >> (e.s & 31)) & 1u) r += fminf(e.a, ton32);
    };
    if (tv.small)
        for (int32_t j = j0; j < j1; ++j) entry(tv.rem_l[j]);
    else
        for (int32_t j = j0; j < j1; ++j) entry(gld(tv.rem_g + j));
    return r;
}

// Per-lane block quantities used by every destination.
struct BlockInfo {
    int32_t pb, lo, hi;
    float ton32, mb, Vb;
    double ton64;
};

// The per-block quantities every destination of a block uses, computed once
// per block of a tile (by one wave) and shared with the tile's other waves
// through LDS: the block's data, its processing-capacity removal term, d(p_b)
// and the mining excess removed from p_b.
struct BlockShare {
    int32_t pb, lo, hi, pad;
    float ton32, mb, Vb, remv;
    double ton64, dpb, am_rem;
};

// Loads of block b's data; the precedence window (lo = max p over
// predecessors or 0, hi = min p over successors or T) comes from ten loads
// issued unconditionally (invalid neighbours read b itself and are masked).
__device__ __forceinline__ BlockInfo load_block(const DevModel &m, int64_t b) {
    BlockInfo bi;
    if (m.csr) {   // explicit lists: the window from the lists (uniform branch)
        bi.pb = gld(m.p + b);
        bi.ton32 = gld(m.ton32 + b);
        bi.ton64 = gld(m.ton64 + b);
        bi.mb = gld(m.mb32 + b);
        bi.Vb = gld(m.Vb32 + b);
        bi.lo = 0;
        bi.hi = m.T;
        const int32_t j0 = gld(m.pred_ptr + b), j1 = gld(m.pred_ptr + b + 1);
        for (int32_t j = j0; j < j1; ++j) bi.lo = max(bi.lo, (int32_t)gld(m.p + gld(m.pred_idx + j)));
        const int32_t k0 = gld(m.succ_ptr + b), k1 = gld(m.succ_ptr + b + 1);
        for (int32_t j = k0; j < k1; ++j) bi.hi = min(bi.hi, (int32_t)gld(m.p + gld(m.succ_idx + j)));
        return bi;
    }
    int32_t x, y, z;
    grid_coords(m, (int32_t)b, x, y, z);
    const int64_t nxy = (int64_t)m.nx * m.ny;
    const bool up = z > 0, dn = z + 1 < m.nz;
    const bool in[5] = {true, x > 0, x + 1 < m.nx, y > 0, y + 1 < m.ny};
    const int64_t off[5] = {0, -1, 1, -(int64_t)m.nx, (int64_t)m.nx};
    int32_t pu[5], pd[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        pu[k] = gld(m.p + ((up && in[k]) ? b - nxy + off[k] : b));
        pd[k] = gld(m.p + ((dn && in[k]) ? b + nxy + off[k] : b));
    }
    bi.pb = gld(m.p + b);
    bi.ton32 = gld(m.ton32 + b);
    bi.ton64 = gld(m.ton64 + b);
    bi.mb = gld(m.mb32 + b);
    bi.Vb = gld(m.Vb32 + b);
    bi.lo = 0;
    bi.hi = m.T;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        if (up && in[k]) bi.lo = max(bi.lo, pu[k]);
        if (dn && in[k]) bi.hi = min(bi.hi, pd[k]);
    }
    return bi;
}

struct TileLds {
    double *d64;      // [T+1]
    double *Ms;       // [T]
    float *cpart;     // [kNW][64]
    uint32_t *ore;    // [W][64]
    uint32_t *fa;     // [T][W]
    uint32_t *fr;     // [T][W]
    int32_t *rng;     // [4][T]
    AddEntry *al;     // [kListCap]
    RemEntry *rl;     // [kListCap]
    BlockShare *bs;   // [64]
    char *end;
};

__host__ __device__ inline size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t tile_lds_layout(const DevModel &m, char *base, TileLds *L) {
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t o = off;
        off = a16(off + bytes);
        return o;
    };
    const size_t o_d = put(sizeof(double) * (m.T + 1));
    const size_t o_M = put(sizeof(double) * m.T);
    const size_t o_c = put(sizeof(float) * 64 * kNW);
    const size_t o_o = put(sizeof(uint32_t) * 64 * m.W);
    const size_t o_fa = put(sizeof(uint32_t) * m.T * m.W);
    const size_t o_fr = put(sizeof(uint32_t) * m.T * m.W);
    const size_t o_rg = put(sizeof(int32_t) * 4 * m.T);
    const size_t o_al = put(sizeof(AddEntry) * kListCap);
    const size_t o_rl = put(sizeof(RemEntry) * kListCap);
    const size_t o_bs = put(sizeof(BlockShare) * 64);
    if (L) {
        L->d64 = (double *)(base + o_d);
        L->Ms = (double *)(base + o_M);
        L->cpart = (float *)(base + o_c);
        L->ore = (uint32_t *)(base + o_o);
        L->fa = (uint32_t *)(base + o_fa);
        L->fr = (uint32_t *)(base + o_fr);
        L->rng = (int32_t *)(base + o_rg);
        L->al = (AddEntry *)(base + o_al);
        L->rl = (RemEntry *)(base + o_rl);
        L->bs = (BlockShare *)(base + o_bs);
        L->end = base + off;
    }
    return off;
}

// Table staging in two halves: issue (loads into registers) and commit (LDS
// stores), so that the loads travel together with the tile's v stream.
struct TablePrefetch {
    double d, M;
    uint32_t fa, fr;
    int32_t rg;
    AddEntry ae;
    RemEntry re;
};

// kLists = false leaves the near-capacity list of the added tonnage in HBM
// (its LDS copy is not made), for kernels that read it with scalar loads; the
// list of the removed tonnage is always staged.
template <bool kLists = true>
__device__ __forceinline__ TablePrefetch issue_tables(const DevModel &m) {
    const int tid = threadIdx.x;
    const int32_t T = m.T, TW = m.T * m.W;
    TablePrefetch f;
    f.d = tid <= T ? gld(m.d64 + tid) : 0.0;
    f.M = tid < T ? gld(m.M + tid) : 0.0;
    f.fa = tid < TW ? gld(m.tab.full_add + tid) : 0u;
    f.fr = tid < TW ? gld(m.tab.full_rem + tid) : 0u;
    f.rg = tid < 4 * T ? gld(m.tab.rng + tid) : 0;
    // the packed lists hold T*S entries each: lanes past that load nothing
    // (their LDS slots are never read, the list ranges end before them)
    const bool in_list = tid < kListCap && tid < T * m.S;
    f.ae = AddEntry{0.0, 0.0f, 0};
    f.re = RemEntry{0.0f, 0};
    if (kLists && in_list) f.ae = gld(m.tab.add_packed + tid);
    if (in_list) f.re = gld(m.tab.rem_packed + tid);
    return f;
}

// Commit the prefetched tables to LDS (plus any remainder of large tables),
// then barrier.  Lists longer than kListCap in total are read in place.
template <bool kLists = true>
__device__ __forceinline__ TabView commit_tables(const DevModel &m, const TileLds &L,
                                                 const TablePrefetch &f) {
    const int tid = threadIdx.x;
    const int32_t T = m.T, TW = m.T * m.W;
    if (tid <= T) L.d64[tid] = f.d;
    if (tid < T) L.Ms[tid] = f.M;
    if (tid < TW) {
        L.fa[tid] = f.fa;
        L.fr[tid] = f.fr;
    }
    if (tid < 4 * T) L.rng[tid] = f.rg;
    for (int i = tid + kNT; i < TW; i += kNT) {   // tables beyond one word per thread
        L.fa[i] = gld(m.tab.full_add + i);
        L.fr[i] = gld(m.tab.full_rem + i);
    }
    if (tid < kListCap) {
        if (kLists) L.al[tid] = f.ae;
        L.rl[tid] = f.re;
    }
    __syncthreads();
    TabView tv;
    tv.full_add = L.fa;
    tv.full_rem = L.fr;
    tv.rng = L.rng;
    const bool small = L.rng[2 * T - 1] <= kListCap && L.rng[4 * T - 1] <= kListCap;
    tv.small = small;
    tv.add_small = kLists && small;
    tv.add_l = L.al;
    tv.add_g = m.tab.add_packed;
    tv.rem_l = L.rl;
    tv.rem_g = m.tab.rem_packed;
    return tv;
}

// This wave's share [s0, s1) of the scenarios (wave-uniform).
__device__ __forceinline__ void wave_range(const DevModel &m, int wave, int32_t &s0,
                                           int32_t &s1) {
    const int32_t Sw = (m.S + kNW - 1) / kNW;
    s0 = wave * Sw;
    s1 = min(m.S, s0 + Sw);
}

// Issue the loads of one chunk of kCH rows of v (all before any FMA).
// Branch-free: a row past the wave's share re-reads row min(s + k, S - 1)
// and gets weight 0 in fma_rows; a lane past the last block reads block 0.
template <int KCH>
__device__ __forceinline__ void issue_rows(const DevModel &m, int64_t b, bool valid, int32_t s,
                                           int32_t s1, float (&x)[KCH]) {
    const float *vp = m.v + (valid ? b : 0);
#pragma unroll
    for (int k = 0; k < KCH; ++k) x[k] = gld_nt(vp + (int64_t)min(s + k, m.S - 1) * m.vld);
}

// e: the scenario weights in global memory, padded by 64 entries past S, so
// that the KCH reads at s.. are in bounds; the wave-uniform reads are scalar
// loads, the entries past the wave's share are replaced by 0 before use.
template <int KCH>
__device__ __forceinline__ float fma_rows(const float *e, int32_t s, int32_t s1,
                                          const float (&x)[KCH], float acc) {
    if (s1 - s >= KCH) {   // the whole chunk is the wave's (uniform)
#pragma unroll
        for (int k = 0; k < KCH; ++k) acc = fmaf(gld(e + s + k), x[k], acc);
        return acc;
    }
#pragma unroll
    for (int k = 0; k < KCH; ++k) {
        // adding 0 * x leaves acc unchanged (v is finite)
        const float ek = gld(e + s + k);
        acc = fmaf(s + k < s1 ? ek : 0.0f, x[k], acc);
    }
    return acc;
}

// Dot product of this wave's share: the first KCH rows were issued by the
// caller before the table round trip; rows beyond them (S > kNW*KCH) follow
// eight at a time.
template <int KCH>
__device__ __forceinline__ float wave_dot(const DevModel &m, const float *e, int64_t b,
                                          bool valid, int32_t s0, int32_t s1, float (&x)[KCH]) {
    float acc = fma_rows(e, s0, s1, x, 0.0f);
    if (valid) {
        const float *vp = m.v + b;
        for (int32_t s = s0 + KCH; s < s1; s += 8) {
            float y[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                y[k] = s + k < s1 ? gld_nt(vp + (int64_t)(s + k) * m.vld) : 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (s + k < s1) acc = fmaf(gld(e + s + k), y[k], acc);
        }
    }
    return acc;
}

// c_b from the per-wave partials (fixed order).
__device__ __forceinline__ float tile_c(const TileLds &L, int lane, int32_t S) {
    float c = L.cpart[lane];
#pragma unroll
    for (int w = 1; w < kNW; ++w) c += L.cpart[w * 64 + lane];
    return c / (float)S;
}

// The shared quantities of the lane's block (ore words staged in L.ore,
// tables committed).
__device__ __forceinline__ BlockShare share_block(const DevModel &m, const TabView &tv,
                                                  const TileLds &L, int lane,
                                                  const BlockInfo &bi) {
    auto ow = [&](int32_t w) { return L.ore[w * 64 + lane]; };
    BlockShare s;
    s.pb = bi.pb;
    s.lo = bi.lo;
    s.hi = bi.hi;
    s.pad = 0;
    s.ton32 = bi.ton32;
    s.mb = bi.mb;
    s.Vb = bi.Vb;
    s.remv = removal_term(m, tv, bi.pb, bi.ton32, ow);
    s.ton64 = bi.ton64;
    s.dpb = L.d64[bi.pb];
    // mining excess removed from the old period: -clamp(M[p_b] - cap, 0, ton)
    s.am_rem = bi.pb < m.T ? -fmin(fmax(L.Ms[bi.pb] - m.mcap, 0.0), bi.ton64) : 0.0;
    return s;
}

// The moves of one lane's block are scored in two halves around the dot
// product: everything but the risk term does not depend on c_b, so it runs
// while the block's v rows are still in flight.  The halves meet in LDS.
struct MoveStage {
    float *dd;     // [64][D] d(t) - d(p_b)
    float *dpp;    // [64][D] processing penalty change; the score replaces it
    float *dpm;    // [64][D] mining penalty change
    uint8_t *f;    // [64][D] flags
};

// Every destination t = wave, wave + kNW, ... of one lane's block, for
// models with at most 8 ore words (S <= 256): the flags and the two penalty
// changes.  The block's invariants come shared (share_block) and its ore
// words sit in registers; each destination's table entries (d(t), M[t], the
// full-add words, the near-capacity list) are the same for every lane of the
// wave, so they are read once per wave (scalar loads).  Same definitions as
// score_move.
__device__ __forceinline__ void score_block_pre(const DevModel &m, const TileLds &L, int wave,
                                                int lane, const BlockShare &bi, int32_t D,
                                                float pps, const MoveStage &st) {
    const int32_t T = m.T, W = m.W;
    uint32_t orw[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) orw[w] = w < W ? L.ore[w * 64 + lane] : 0u;
    auto ow = [&](int32_t w) { return L.ore[w * 64 + lane]; };
    const int32_t pb = bi.pb;
    const float remv = bi.remv;
    const double dpb = bi.dpb;
    const double mcap = m.mcap, ton = bi.ton64;
    const double am_rem = bi.am_rem;
    for (int32_t t = wave; t < D; t += kNW) {
        const bool noop = t == pb;
        const float dd = (float)(gld(m.d64 + t) - dpb);
        float addv = 0.0f;
        bool viol = false, mine_ok = true;
        double am = am_rem;
        if (t < T) {
            // eight words read unconditionally (one scalar load): words past
            // W meet zero ore words, and the state arena continues after
            // full_add (full_rem, then the lists), so the reads stay inside it
            const uint32_t *fa = m.tab.full_add + (int64_t)t * W;
            int32_t cnt = 0;
#pragma unroll
            for (int w = 0; w < 8; ++w) cnt += __popc(orw[w] & gld(fa + w));
            addv = (float)cnt * bi.ton32;
            viol = cnt != 0;
            const int32_t j1 = gld(m.tab.rng + T + t);
            for (int32_t j = gld(m.tab.rng + t); j < j1; ++j) {
                const AddEntry e = gld(m.tab.add_packed + j);
                if ((ow(e.s >> 5) >> (e.s & 31)) & 1u) {
                    addv += fmaxf(bi.ton32 - e.d, 0.0f);
                    if (ton >= e.tau) viol = true;
                }
            }
            // mining excess added to the new period: clamp(M[t] + ton - cap, 0, ton)
            const double x = gld(m.M + t) + ton;
            mine_ok = x <= mcap;
            am += fmin(fmax(x - mcap, 0.0), ton);
        }
        uint8_t f = 0;
        if (bi.lo <= t && t <= bi.hi) f |= MPS_PREC_OK;
        if (noop || t == T || mine_ok) f |= MPS_MINE_OK;
        if (noop || t == T || !viol) f |= MPS_PROC_OK;
        if (noop) f |= MPS_NOOP;
        const int32_t i = lane * D + t;
        st.dd[i] = dd;
        st.dpp[i] = noop ? 0.0f : pps * (addv - remv);
        st.dpm[i] = noop ? 0.0f : (float)(m.pen_mine * am);
        st.f[i] = f;
    }
}

// The second half, once c_b is known: the risk term (hardware square root and
// reciprocal) and the score.  emit(t, out) receives each move.
template <class Emit>
__device__ __forceinline__ void score_block_post(int wave, int lane, const BlockShare &bi,
                                                 float c, int32_t D, float var32, float sig32,
                                                 float lam, const MoveStage &st, Emit emit) {
    for (int32_t t = wave; t < D; t += kNW) {
        const int32_t i = lane * D + t;
        const float dd = st.dd[i];
        const uint8_t f = st.f[i];
        const bool noop = (f & MPS_NOOP) != 0;
        const float dvar = fmaf(2.0f * dd, c, dd * dd * bi.Vb);
        const float vp = fmaxf(var32 + dvar, 0.0f);
        const float den = __builtin_amdgcn_sqrtf(vp) + sig32;
        const float dsig = den > 0.0f ? dvar * __builtin_amdgcn_rcpf(den) : 0.0f;
        const float dr = fmaf(dd, bi.mb, -lam * dsig);
        const float dpp = st.dpp[i], dpm = st.dpm[i];
        MoveOut o;
        o.flags = f;
        o.dr = noop ? 0.0f : dr;
        o.dpp = dpp;
        o.dpm = dpm;
        o.score = noop ? 0.0f : (dr - dpp) - dpm;
        emit(t, o);
    }
}

// Writes block b's record (one lane per block; four 16-byte stores).
template <class OreWord>
__device__ __forceinline__ void put_list_rec(const DevModel &m, int64_t b, float c, float rem,
                                             const BlockInfo &bi, OreWord ore_word) {
    ListRec r;
    r.c = c;
    r.rem = rem;
    r.info = bi.pb | (bi.lo << 8) | (bi.hi << 16);
    r.ton32 = bi.ton32;
    r.mb = bi.mb;
    r.Vb = bi.Vb;
    r.ton64 = bi.ton64;
#pragma unroll
    for (int w = 0; w < 8; ++w) r.ore[w] = w < m.W ? ore_word(w) : 0u;
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const u4 *src = (const u4 *)&r;
    u4 *dst = (u4 *)(m.blk_rec + b);
#pragma unroll
    for (int k = 0; k < 4; ++k) gst(dst + k, src[k]);
}

// One listed move (b, t) from the record the list pass wrote; a move out of
// range is BAD with score -FLT_MAX.
__device__ __forceinline__ MoveOut list_move(const DevModel &m, const TabView &tv,
                                             const TileLds &L, int32_t b, int32_t t) {
    if (b < 0 || (int64_t)b >= m.N || t < 0 || t > m.T) {
        MoveOut o;
        o.score = -FLT_MAX;
        o.flags = MPS_BAD;
        o.dr = o.dpp = o.dpm = 0.0f;
        return o;
    }
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const u4 *rp = (const u4 *)(m.blk_rec + b);
    const u4 q0 = gld(rp), q1 = gld(rp + 1);
    u4 q2 = {0u, 0u, 0u, 0u}, q3 = q2;
    if (m.W <= 8) {   // uniform
        q2 = gld(rp + 2);
        q3 = gld(rp + 3);
    }
    const float c = __uint_as_float(q0.x), rem = __uint_as_float(q0.y);
    const int32_t info = (int32_t)q0.z;
    const float ton32 = __uint_as_float(q0.w), mb = __uint_as_float(q1.x),
                Vb = __uint_as_float(q1.y);
    const double ton64 = __hiloint2double((int)q1.w, (int)q1.z);
    const int32_t pb = info & 0xff, lo = (info >> 8) & 0xff, hi = (info >> 16) & 0xff;
    const uint32_t ow8[8] = {q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
    auto ow = [&](int32_t w) {
        return m.W <= 8 ? ow8[w & 7] : gld(m.ore + (int64_t)w * m.N + b);
    };
    return score_move(m, tv, L.d64, L.Ms, t, pb, lo, hi, c, rem, ton32, ton64, mb, Vb,
                      gld(&m.sc->var32), gld(&m.sc->sigma32), (float)m.lambda,
                      (float)(m.pen_proc / m.S), ow);
}

}  // namespace mps
