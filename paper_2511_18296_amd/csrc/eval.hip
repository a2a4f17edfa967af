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
// a tile is issued before the first wait: first the small ones (block data,
// ore words, tables), then the rows of v.  With at most 8 ore words
// (S <= 256) everything of a move but its risk term is computed while the
// rows are still in flight (score_block_pre), and only the risk term waits
// for c_b (score_block_post).  Scores and flags of the tile are staged in LDS
// and written as one contiguous, coalesced range.
#include <float.h>

#include "eval_dev.h"

namespace mps {

// ---- exhaustive: one tile of 64 blocks, all D destinations ------------------
// KCH = rows of v each lane keeps in flight: the smallest of the instantiated
// sizes that covers a wave's share of S.  Up to 25 rows the kernel fits in 64
// VGPRs, eight waves per SIMD: four workgroups per CU, so that the 844 tiles
// of a 54,000-block model are all resident at once (at six waves per SIMD,
// 768 are, and the rest run as a second round).
template <bool COMP, int KCH>
__global__ void __launch_bounds__(kNT, KCH <= 25 ? 8 : 1) k_eval_exh(DevModel m, int32_t D, float *score,
                                                  uint8_t *flags, float *dR, float *dPp,
                                                  float *dPm) {
    extern __shared__ __align__(16) char lds[];
    TileLds L;
    tile_lds_layout(m, lds, &L);
    // the tile's moves in LDS: d(t) - d(p_b), the two penalty changes (the
    // processing one replaced by the score), flags
    const size_t sf = a16(sizeof(float) * 64 * D);
    MoveStage st;
    st.dpp = (float *)L.end;
    st.dd = (float *)(L.end + sf);
    st.dpm = (float *)(L.end + 2 * sf);
    st.f = (uint8_t *)(L.end + 3 * sf);
    float *stage_s = st.dpp;
    uint8_t *stage_f = st.f;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t b0 = (int64_t)blockIdx.x * 64;
    const int64_t b = b0 + lane;
    const bool valid = b < m.N;

    // one round trip.  The small loads go first (block data, which one wave
    // loads for the tile and the others take from LDS; tables; ore words), so
    // that waiting for them does not wait for the rows of v.
    BlockInfo bi{};
    if (wave == 0 && valid) bi = load_block(m, b);
    const TablePrefetch tp = issue_tables<false>(m);
    uint32_t ow0 = 0;
    if (valid && wave < m.W) ow0 = m.ore[(int64_t)wave * m.N + b];
    const float var32 = gld(&m.sc->var32), sig32 = gld(&m.sc->sigma32);
    int32_t s0, s1;
    wave_range(m, wave, s0, s1);
    float x[KCH];
    issue_rows(m, b, valid, s0, s1, x);
    if (wave < m.W) L.ore[wave * 64 + lane] = ow0;
    for (int32_t w = wave + kNW; w < m.W; w += kNW)
        L.ore[w * 64 + lane] = valid ? m.ore[(int64_t)w * m.N + b] : 0u;
    const TabView tv = commit_tables<false>(m, L, tp);   // barrier inside (LDS only)
    if (wave == 0 && valid) L.bs[lane] = share_block(m, tv, L, lane, bi);
    __syncthreads();
    const float lam = (float)m.lambda, pps = (float)(m.pen_proc / m.S);
    // the block's shared quantities are read from LDS where used
    const BlockShare &bs = L.bs[lane];
    // while the rows travel: the moves' flags and penalty changes
    if (valid && m.W <= 8) score_block_pre(m, L, wave, lane, bs, D, pps, st);
    L.cpart[wave * 64 + lane] = wave_dot(m, m.e32, b, valid, s0, s1, x);
    __syncthreads();
    const float c = tile_c(L, lane, m.S);

    if (valid) {
        auto emit = [&](int32_t t, const MoveOut &o) {
            stage_s[lane * D + t] = o.score;
            stage_f[lane * D + t] = o.flags;
            if (COMP) {
                const int64_t i = b * D + t;
                dR[i] = o.dr;
                dPp[i] = o.dpp;
                dPm[i] = o.dpm;
            }
        };
        if (m.W <= 8) {
            score_block_post(wave, lane, bs, c, D, var32, sig32, lam, st, emit);
        } else {
            auto ow = [&](int32_t w) { return L.ore[w * 64 + lane]; };
            for (int32_t t = wave; t < D; t += kNW)
                emit(t, score_move(m, tv, L.d64, L.Ms, t, bs.pb, bs.lo, bs.hi, c, bs.remv,
                                   bs.ton32, bs.ton64, bs.mb, bs.Vb, var32, sig32, lam, pps,
                                   ow));
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
// A short list touches few of the 64-block tiles: it marks them first, and the
// block pass skips every unmarked tile (clearing each mark it consumes, so the
// marks are zero again between calls).  A long list touches nearly every tile
// (a tile escapes n uniform moves with probability about exp(-n/tiles)), and
// the pass covers all of them without marks.
__global__ void k_mark_tiles(int64_t n, int64_t N, const int32_t *blk, uint32_t *mark) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = blk[i];
    if (b >= 0 && b < N) mark[b >> 6] = 1u;
}

__global__ void __launch_bounds__(kNT) k_block_prep(DevModel m, uint32_t *mark) {
    if (mark != nullptr && mark[blockIdx.x] == 0u) return;   // uniform over the workgroup
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
    L.cpart[wave * 64 + lane] = wave_dot(m, m.e32, b, valid, s0, s1, x);
    __syncthreads();   // every thread has read the mark
    if (mark != nullptr && tid == 0) mark[blockIdx.x] = 0u;
    const float c = tile_c(L, lane, m.S);
    if (wave == 0 && valid) {
        auto ow = [&](int32_t w) { return L.ore[w * 64 + lane]; };
        put_list_rec(m, b, c, removal_term(m, tv, bi.pb, bi.ton32, ow), bi, ow);
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
    const MoveOut o = list_move(m, tv, L, blk[i], per[i]);
    score[i] = o.score;
    flags[i] = o.flags;
    if (COMP) {
        dR[i] = o.dr;
        dPp[i] = o.dpp;
        dPm[i] = o.dpm;
    }
}

size_t eval_lds_bytes(const DevModel &m, const mps_moves &mv) {
    const size_t base = tile_lds_layout(m, nullptr, nullptr);
    if (!mv.exhaustive) return base;
    const int32_t D = mv.include_never ? m.T + 1 : m.T;
    return base + 3 * a16(sizeof(float) * 64 * D) + a16((size_t)64 * D);
}

hipError_t launch_eval(const DevModel &m, const mps_moves &mv, float *score, uint8_t *flags,
                       float *dR, float *dPp, float *dPm, hipStream_t st) {
    if (has_variant(m)) return launch_eval_var(m, mv, score, flags, dR, dPp, dPm, st);
    const bool comp = dR != nullptr;
    const unsigned tiles = (unsigned)((m.N + 63) / 64);
    const size_t base = tile_lds_layout(m, nullptr, nullptr);
    if (mv.exhaustive) {
        const int32_t D = mv.include_never ? m.T + 1 : m.T;
        const size_t lds = eval_lds_bytes(m, mv);
        // rows per wave: up to 16 -> 16, 17..25 -> 25, more -> 32 (and a loop)
        const int32_t rows = (m.S + kNW - 1) / kNW;
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(tiles), dim3(kNT), lds, st, m, D, score, flags, dR, dPp,
                               dPm);
        };
        if (comp)
            go(k_eval_exh<true, kCH>);
        else if (rows <= 16)
            go(k_eval_exh<false, 16>);
        else if (rows <= 25)
            go(k_eval_exh<false, 25>);
        else
            go(k_eval_exh<false, kCH>);
        return hipGetLastError();
    }
    if (mv.n == 0) return hipGetLastError();
    uint32_t *mark = nullptr;
    if (mv.n < 8 * (int64_t)tiles) {
        mark = m.tmark;
        hipLaunchKernelGGL(k_mark_tiles, dim3((unsigned)((mv.n + 255) / 256)), dim3(256), 0, st,
                           mv.n, m.N, mv.block, mark);
    }
    hipLaunchKernelGGL(k_block_prep, dim3(tiles), dim3(kNT), base, st, m, mark);
    {
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
