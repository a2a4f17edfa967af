// eval.hip -- candidate-move evaluation (the per-candidate precedence,
// capacity and value check of Alg. 5, exact, for every destination period).
//
// For a move (b, t') with dd = d(t') - d(p_b) the per-scenario NPV changes by
// dd*v[s][b].  With m_b, V_b the scenario mean and variance of v[.][b] and
// c_b = (1/S) sum_s (N_s - mu) v[s][b], the new mean and variance are
//   mu' = mu + dd*m_b,   var' = var + 2 dd c_b + dd^2 V_b
// (algebra on the definition), so dR = dd*m_b - lambda*(sigma' - sigma) with
// sigma' - sigma = (var' - var)/(sigma' + sigma).  Streaming v once to form
// c_b is the only O(S) work per block; every destination is then O(1) for the
// risk term.  The processing penalty uses the per-period tables built from the
// FP64 tonnages (state.hip): scenarios always over capacity are counted with
// popcount on whole ore words, the few scenarios near the capacity come from
// short per-period lists, and the capacity flag is decided exactly as its
// FP64 definition states it.
//
// Layout: one workgroup = 512 threads = 8 waves per tile of 64 consecutive
// blocks; lane l owns block b0 + l.  The eight waves stream disjoint eighths
// of the scenario-major v[s][b] (each wave instruction reads 256 contiguous
// bytes) and then take every eighth destination period.  Every global load of
// a tile (its rows of v, block data, ore words, tables) is issued before
// the first wait, so a tile costs one memory round trip.  Scores and flags of
// the tile are staged in LDS and written as one contiguous, coalesced range.
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
    const AddEntry *add;
    const RemEntry *rem;
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
        const int32_t j1 = tv.rng[T + t];
        for (int32_t j = tv.rng[t]; j < j1; ++j) {
            const AddEntry e = tv.add[j];
            if ((ore_word(e.s >> 5) >> (e.s & 31)) & 1u) {
                addv += fmaxf(ton32 - e.d, 0.0f);
                if (ton64 >= e.tau) viol = true;
            }
        }
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
    const int32_t j1 = tv.rng[3 * T + pb];
    for (int32_t j = tv.rng[2 * T + pb]; j < j1; ++j) {
        const RemEntry e = tv.rem[j];
        if ((ore_word(e.s >> 5) >> (e.s & 31)) & 1u) r += fminf(e.a, ton32);
    }
    return r;
}

// Per-lane block quantities used by every destination.
struct BlockInfo {
    int32_t pb, lo, hi;
    float ton32, mb, Vb;
    double ton64;
};

// Loads of block b's data; the precedence window (lo = max p over
// predecessors or 0, hi = min p over successors or T) comes from ten loads
// issued unconditionally (invalid neighbours read b itself and are masked).
__device__ __forceinline__ BlockInfo load_block(const DevModel &m, int64_t b) {
    BlockInfo bi;
    int32_t x, y, z;
    grid_coords(m, (int32_t)b, x, y, z);
    const int64_t nxy = (int64_t)m.nx * m.ny;
    const bool up = z > 0, dn = z + 1 < m.nz;
    const bool in[5] = {true, x > 0, x + 1 < m.nx, y > 0, y + 1 < m.ny};
    const int64_t off[5] = {0, -1, 1, -(int64_t)m.nx, (int64_t)m.nx};
    int32_t pu[5], pd[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        pu[k] = m.p[(up && in[k]) ? b - nxy + off[k] : b];
        pd[k] = m.p[(dn && in[k]) ? b + nxy + off[k] : b];
    }
    bi.pb = m.p[b];
    bi.ton32 = m.ton32[b];
    bi.ton64 = m.ton64[b];
    bi.mb = m.mb32[b];
    bi.Vb = m.Vb32[b];
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
    float *e;         // [S] scenario weights N_s - mu
    uint32_t *ore;    // [W][64]
    uint32_t *fa;     // [T][W]
    uint32_t *fr;     // [T][W]
    int32_t *rng;     // [4][T]
    AddEntry *al;     // [kListCap]
    RemEntry *rl;     // [kListCap]
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
    const size_t o_e = put(sizeof(float) * m.S);
    const size_t o_o = put(sizeof(uint32_t) * 64 * m.W);
    const size_t o_fa = put(sizeof(uint32_t) * m.T * m.W);
    const size_t o_fr = put(sizeof(uint32_t) * m.T * m.W);
    const size_t o_rg = put(sizeof(int32_t) * 4 * m.T);
    const size_t o_al = put(sizeof(AddEntry) * kListCap);
    const size_t o_rl = put(sizeof(RemEntry) * kListCap);
    if (L) {
        L->d64 = (double *)(base + o_d);
        L->Ms = (double *)(base + o_M);
        L->cpart = (float *)(base + o_c);
        L->e = (float *)(base + o_e);
        L->ore = (uint32_t *)(base + o_o);
        L->fa = (uint32_t *)(base + o_fa);
        L->fr = (uint32_t *)(base + o_fr);
        L->rng = (int32_t *)(base + o_rg);
        L->al = (AddEntry *)(base + o_al);
        L->rl = (RemEntry *)(base + o_rl);
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
    float e;
    AddEntry ae;
    RemEntry re;
};

__device__ __forceinline__ TablePrefetch issue_tables(const DevModel &m) {
    const int tid = threadIdx.x;
    const int32_t T = m.T, TW = m.T * m.W;
    TablePrefetch f;
    f.d = tid <= T ? m.d64[tid] : 0.0;
    f.M = tid < T ? m.M[tid] : 0.0;
    f.fa = tid < TW ? m.tab.full_add[tid] : 0u;
    f.fr = tid < TW ? m.tab.full_rem[tid] : 0u;
    f.rg = tid < 4 * T ? m.tab.rng[tid] : 0;
    f.e = tid < m.S ? m.e32[tid] : 0.0f;
    f.ae = m.tab.add_packed[min(tid, kListCap - 1)];
    f.re = m.tab.rem_packed[min(tid, kListCap - 1)];
    return f;
}

// Commit the prefetched tables to LDS (plus any remainder of large tables),
// then barrier.  Lists longer than kListCap in total are read in place.
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
    if (tid < m.S) L.e[tid] = f.e;
    for (int i = tid + kNT; i < TW; i += kNT) {   // tables beyond one word per thread
        L.fa[i] = m.tab.full_add[i];
        L.fr[i] = m.tab.full_rem[i];
    }
    for (int i = tid + kNT; i < m.S; i += kNT) L.e[i] = m.e32[i];
    if (tid < kListCap) {
        L.al[tid] = f.ae;
        L.rl[tid] = f.re;
    }
    __syncthreads();
    TabView tv;
    tv.full_add = L.fa;
    tv.full_rem = L.fr;
    tv.rng = L.rng;
    const bool small = L.rng[2 * T - 1] <= kListCap && L.rng[4 * T - 1] <= kListCap;
    tv.add = small ? L.al : m.tab.add_packed;
    tv.rem = small ? L.rl : m.tab.rem_packed;
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
__device__ __forceinline__ void issue_rows(const DevModel &m, int64_t b, bool valid, int32_t s,
                                           int32_t s1, float (&x)[kCH]) {
    const float *vp = m.v + b;
#pragma unroll
    for (int k = 0; k < kCH; ++k) {
        x[k] = 0.0f;
        if (valid && s + k < s1) x[k] = __builtin_nontemporal_load(vp + (int64_t)(s + k) * m.N);
    }
}

__device__ __forceinline__ float fma_rows(const float *e, int32_t s, int32_t s1,
                                          const float (&x)[kCH], float acc) {
#pragma unroll
    for (int k = 0; k < kCH; ++k)
        if (s + k < s1) acc = fmaf(e[s + k], x[k], acc);
    return acc;
}

// Dot product of this wave's share: the first kCH rows were issued by the
// caller before the table round trip; rows beyond them (S > kNW*kCH) follow
// eight at a time.
__device__ __forceinline__ float wave_dot(const DevModel &m, const float *e, int64_t b,
                                          bool valid, int32_t s0, int32_t s1, float (&x)[kCH]) {
    float acc = fma_rows(e, s0, s1, x, 0.0f);
    if (valid) {
        const float *vp = m.v + b;
        for (int32_t s = s0 + kCH; s < s1; s += 8) {
            float y[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                y[k] = s + k < s1 ? __builtin_nontemporal_load(vp + (int64_t)(s + k) * m.N) : 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (s + k < s1) acc = fmaf(e[s + k], y[k], acc);
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

// ---- exhaustive: one tile of 64 blocks, all D destinations ------------------
template <bool COMP>
__global__ void __launch_bounds__(kNT) k_eval_exh(DevModel m, int32_t D, float *score,
                                                  uint8_t *flags, float *dR, float *dPp,
                                                  float *dPm) {
    extern __shared__ __align__(16) char lds[];
    TileLds L;
    tile_lds_layout(m, lds, &L);
    float *stage_s = (float *)L.end;
    uint8_t *stage_f = (uint8_t *)(L.end + a16(sizeof(float) * 64 * D));

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t b0 = (int64_t)blockIdx.x * 64;
    const int64_t b = b0 + lane;
    const bool valid = b < m.N;

    // one round trip: the wave's rows of v, tables, block data, ore words
    int32_t s0, s1;
    wave_range(m, wave, s0, s1);
    float x[kCH];
    issue_rows(m, b, valid, s0, s1, x);
    const TablePrefetch tp = issue_tables(m);
    BlockInfo bi{};
    if (valid) bi = load_block(m, b);
    uint32_t ow0 = 0;
    if (valid && wave < m.W) ow0 = m.ore[(int64_t)wave * m.N + b];
    const float var32 = m.sc->var32, sig32 = m.sc->sigma32;
    if (wave < m.W) L.ore[wave * 64 + lane] = ow0;
    for (int32_t w = wave + kNW; w < m.W; w += kNW)
        L.ore[w * 64 + lane] = valid ? m.ore[(int64_t)w * m.N + b] : 0u;
    const TabView tv = commit_tables(m, L, tp);   // barrier inside
    L.cpart[wave * 64 + lane] = wave_dot(m, L.e, b, valid, s0, s1, x);
    __syncthreads();
    const float c = tile_c(L, lane, m.S);

    const float lam = (float)m.lambda, pps = (float)(m.pen_proc / m.S);
    if (valid) {
        auto ow = [&](int32_t w) { return L.ore[w * 64 + lane]; };
        const float remv = removal_term(m, tv, bi.pb, bi.ton32, ow);
        for (int32_t t = wave; t < D; t += kNW) {
            const MoveOut o = score_move(m, tv, L.d64, L.Ms, t, bi.pb, bi.lo, bi.hi, c, remv,
                                         bi.ton32, bi.ton64, bi.mb, bi.Vb, var32, sig32, lam,
                                         pps, ow);
            stage_s[lane * D + t] = o.score;
            stage_f[lane * D + t] = o.flags;
            if (COMP) {
                const int64_t i = b * D + t;
                dR[i] = o.dr;
                dPp[i] = o.dpp;
                dPm[i] = o.dpm;
            }
        }
    }
    __syncthreads();
    const int64_t nb = min((int64_t)64, m.N - b0);
    const int64_t n_out = nb * D;
    const int64_t base = b0 * D;
    float *so = score + base;
    uint8_t *fo = flags + base;
    if ((((uintptr_t)so) & 15) == 0) {
        const int64_t n4 = n_out >> 2;
        for (int64_t i = tid; i < n4; i += kNT) ((float4 *)so)[i] = ((const float4 *)stage_s)[i];
        for (int64_t i = (n4 << 2) + tid; i < n_out; i += kNT) so[i] = stage_s[i];
    } else {
        for (int64_t i = tid; i < n_out; i += kNT) so[i] = stage_s[i];
    }
    if ((((uintptr_t)fo) & 3) == 0) {
        const int64_t n4 = n_out >> 2;
        for (int64_t i = tid; i < n4; i += kNT) ((uint32_t *)fo)[i] = ((const uint32_t *)stage_f)[i];
        for (int64_t i = (n4 << 2) + tid; i < n_out; i += kNT) fo[i] = stage_f[i];
    } else {
        for (int64_t i = tid; i < n_out; i += kNT) fo[i] = stage_f[i];
    }
}

// ---- list mode: per-block quantities, then one thread per move --------------
__global__ void __launch_bounds__(kNT) k_block_prep(DevModel m) {
    extern __shared__ __align__(16) char lds[];
    TileLds L;
    tile_lds_layout(m, lds, &L);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t b = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = b < m.N;
    int32_t s0, s1;
    wave_range(m, wave, s0, s1);
    float x[kCH];
    issue_rows(m, b, valid, s0, s1, x);
    const TablePrefetch tp = issue_tables(m);
    BlockInfo bi{};
    if (valid && wave == 0) bi = load_block(m, b);
    for (int32_t w = wave; w < m.W; w += kNW)
        L.ore[w * 64 + lane] = valid ? m.ore[(int64_t)w * m.N + b] : 0u;
    const TabView tv = commit_tables(m, L, tp);
    L.cpart[wave * 64 + lane] = wave_dot(m, L.e, b, valid, s0, s1, x);
    __syncthreads();
    const float c = tile_c(L, lane, m.S);
    if (wave == 0 && valid) {
        auto ow = [&](int32_t w) { return L.ore[w * 64 + lane]; };
        m.blk_c[b] = c;
        m.blk_rem[b] = removal_term(m, tv, bi.pb, bi.ton32, ow);
        m.blk_info[b] = bi.pb | (bi.lo << 8) | (bi.hi << 16);
    }
}

template <bool COMP>
__global__ void __launch_bounds__(kNT) k_eval_list(DevModel m, int64_t n, const int32_t *blk,
                                                   const int8_t *per, float *score,
                                                   uint8_t *flags, float *dR, float *dPp,
                                                   float *dPm) {
    extern __shared__ __align__(16) char lds[];
    TileLds L;
    tile_lds_layout(m, lds, &L);
    const TablePrefetch tp = issue_tables(m);
    const TabView tv = commit_tables(m, L, tp);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = blk[i];
    const int32_t t = per[i];
    if (b < 0 || (int64_t)b >= m.N || t < 0 || t > m.T) {
        score[i] = -FLT_MAX;
        flags[i] = MPS_BAD;
        if (COMP) {
            dR[i] = 0.0f;
            dPp[i] = 0.0f;
            dPm[i] = 0.0f;
        }
        return;
    }
    const int32_t info = m.blk_info[b];
    const int32_t pb = info & 0xff, lo = (info >> 8) & 0xff, hi = (info >> 16) & 0xff;
    auto ow = [&](int32_t w) { return m.ore[(int64_t)w * m.N + b]; };
    const MoveOut o = score_move(m, tv, L.d64, L.Ms, t, pb, lo, hi, m.blk_c[b], m.blk_rem[b],
                                 m.ton32[b], m.ton64[b], m.mb32[b], m.Vb32[b], m.sc->var32,
                                 m.sc->sigma32, (float)m.lambda, (float)(m.pen_proc / m.S), ow);
    score[i] = o.score;
    flags[i] = o.flags;
    if (COMP) {
        dR[i] = o.dr;
        dPp[i] = o.dpp;
        dPm[i] = o.dpm;
    }
}

hipError_t launch_eval(const DevModel &m, const mps_moves &mv, float *score, uint8_t *flags,
                       float *dR, float *dPp, float *dPm, hipStream_t st) {
    const bool comp = dR != nullptr;
    const unsigned tiles = (unsigned)((m.N + 63) / 64);
    const size_t base = tile_lds_layout(m, nullptr, nullptr);
    if (mv.exhaustive) {
        const int32_t D = mv.include_never ? m.T + 1 : m.T;
        const size_t lds = base + a16(sizeof(float) * 64 * D) + a16((size_t)64 * D);
        if (comp)
            hipLaunchKernelGGL(k_eval_exh<true>, dim3(tiles), dim3(kNT), lds, st, m, D, score,
                               flags, dR, dPp, dPm);
        else
            hipLaunchKernelGGL(k_eval_exh<false>, dim3(tiles), dim3(kNT), lds, st, m, D, score,
                               flags, dR, dPp, dPm);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_block_prep, dim3(tiles), dim3(kNT), base, st, m);
    if (mv.n > 0) {
        const unsigned g = (unsigned)((mv.n + kNT - 1) / kNT);
        if (comp)
            hipLaunchKernelGGL(k_eval_list<true>, dim3(g), dim3(kNT), base, st, m, mv.n,
                               mv.block, mv.period, score, flags, dR, dPp, dPm);
        else
            hipLaunchKernelGGL(k_eval_list<false>, dim3(g), dim3(kNT), base, st, m, mv.n,
                               mv.block, mv.period, score, flags, dR, dPp, dPm);
    }
    return hipGetLastError();
}

}  // namespace mps
