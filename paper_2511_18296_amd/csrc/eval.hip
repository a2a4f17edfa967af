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
// FP64 tonnages (state.hip): whole words of "always over capacity" scenarios
// are counted with popcount, the few scenarios near the capacity are
// evaluated in FP64, and the capacity flag is decided in FP64 exactly as the
// definition states it.
#include <float.h>

#include "internal.h"

namespace mps {

struct MoveOut {
    float score, dr, dpp, dpm;
    uint8_t flags;
};

// Risk, penalty and flag arithmetic of one move, given the block quantities.
// ore_word(w) returns ore word w of block b.
template <class OreWord>
__device__ __forceinline__ MoveOut score_move(const DevModel &m, const double *d64,
                                              const double *Ms, int32_t t, int32_t pb,
                                              int32_t lo, int32_t hi, float c,
                                              float remv, float ton32, double ton64,
                                              float mb, float Vb, float var32,
                                              float sig32, float lam, float pps,
                                              OreWord ore_word) {
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
        const uint32_t *fa = m.tab.full_add + (int64_t)t * m.W;
        for (int32_t w = 0; w < m.W; ++w) cnt += __popc(ore_word(w) & fa[w]);
        addv = (float)cnt * ton32;
        viol = cnt != 0;
        const int32_t np = m.tab.n_part_add[t];
        const int32_t *ps = m.tab.part_add_s + (int64_t)t * m.S;
        const double *pO = m.tab.part_add_O + (int64_t)t * m.S;
        for (int32_t j = 0; j < np; ++j) {
            const int32_t s = ps[j];
            if ((ore_word(s >> 5) >> (s & 31)) & 1u) {
                const double O = pO[j];
                const double nw = O + ton64;
                if (nw > m.pcap) viol = true;
                addv += (float)(hinge64(nw, m.pcap) - hinge64(O, m.pcap));
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

// Removal term of block b from its current period pb < T:
// sum_s ore[s][b] * clamp(O[pb][s] - cap, 0, ton_b).
template <class OreWord>
__device__ __forceinline__ float removal_term(const DevModel &m, int32_t pb, float ton32,
                                              OreWord ore_word) {
    if (pb >= m.T) return 0.0f;
    int32_t cnt = 0;
    const uint32_t *fr = m.tab.full_rem + (int64_t)pb * m.W;
    for (int32_t w = 0; w < m.W; ++w) cnt += __popc(ore_word(w) & fr[w]);
    float r = (float)cnt * ton32;
    const int32_t np = m.tab.n_part_rem[pb];
    const int32_t *ps = m.tab.part_rem_s + (int64_t)pb * m.S;
    const float *pa = m.tab.part_rem_a + (int64_t)pb * m.S;
    for (int32_t j = 0; j < np; ++j) {
        const int32_t s = ps[j];
        if ((ore_word(s >> 5) >> (s & 31)) & 1u) r += fminf(pa[j], ton32);
    }
    return r;
}

// Partial dot product sum_{s in quarter(wave)} e_s v[s][b] of one lane's block;
// the four quarters are added in a fixed order by the caller.
__device__ __forceinline__ float dot_quarter(const DevModel &m, int64_t b, bool valid,
                                             int wave) {
    const int32_t S = m.S;
    const int32_t Sq = (S + 3) >> 2;
    const int32_t s0 = wave * Sq;
    const int32_t s1 = min(S, s0 + Sq);
    float acc = 0.0f;
    if (!valid) return acc;
    const float *vp = m.v + b;
    const int64_t N = m.N;
    int32_t s = s0;
    for (; s + 8 <= s1; s += 8) {
        float x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = __builtin_nontemporal_load(vp + (int64_t)(s + k) * N);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc = fmaf(m.e32[s + k], x[k], acc);
    }
    for (; s < s1; ++s) acc = fmaf(m.e32[s], __builtin_nontemporal_load(vp + (int64_t)s * N), acc);
    return acc;
}

struct TileLds {
    double *d64;      // [T+1]
    double *Ms;       // [T]
    float *cpart;     // [4][64]
    uint32_t *ore;    // [W][64]
};

__device__ __forceinline__ size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__device__ __forceinline__ TileLds carve(char *lds, const DevModel &m) {
    TileLds L;
    size_t off = 0;
    L.d64 = (double *)(lds + off);
    off = align16(off + sizeof(double) * (m.T + 1));
    L.Ms = (double *)(lds + off);
    off = align16(off + sizeof(double) * m.T);
    L.cpart = (float *)(lds + off);
    off = align16(off + sizeof(float) * 256);
    L.ore = (uint32_t *)(lds + off);
    return L;
}

__host__ __device__ static size_t tile_lds_bytes(const DevModel &m) {
    auto a16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
    size_t off = a16(sizeof(double) * (m.T + 1));
    off = a16(off + sizeof(double) * m.T);
    off = a16(off + sizeof(float) * 256);
    off = a16(off + sizeof(uint32_t) * 64 * m.W);
    return off;
}

// Phase A of a 64-block tile (256 threads = 4 waves): tables to LDS, quarter
// dot products, ore words.  Returns c_b for the lane's block.
__device__ __forceinline__ float tile_phase_a(const DevModel &m, const TileLds &L,
                                              int64_t b, bool valid) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i <= m.T; i += 256) L.d64[i] = m.d64[i];
    for (int i = tid; i < m.T; i += 256) L.Ms[i] = m.M[i];
    float acc = dot_quarter(m, b, valid, wave);
    L.cpart[wave * 64 + lane] = acc;
    for (int32_t w = wave; w < m.W; w += 4)
        L.ore[w * 64 + lane] = valid ? m.ore[(int64_t)w * m.N + b] : 0u;
    __syncthreads();
    float c = ((L.cpart[lane] + L.cpart[64 + lane]) + L.cpart[128 + lane]) + L.cpart[192 + lane];
    return c / (float)m.S;
}

// ---- exhaustive: one tile of 64 blocks, all D destinations ------------------
template <bool COMP>
__global__ void __launch_bounds__(256) k_eval_exh(DevModel m, int32_t D, float *score,
                                                  uint8_t *flags, float *dR, float *dPp,
                                                  float *dPm) {
    extern __shared__ __align__(16) char lds[];
    const TileLds L = carve(lds, m);
    const size_t base_off = tile_lds_bytes(m);
    float *stage_s = (float *)(lds + base_off);
    uint8_t *stage_f = (uint8_t *)(lds + base_off + align16(sizeof(float) * 64 * D));

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * 64;
    const int64_t b = b0 + lane;
    const bool valid = b < m.N;
    const float c = tile_phase_a(m, L, b, valid);

    const float var32 = m.sc->var32, sig32 = m.sc->sigma32;
    const float lam = (float)m.lambda, pps = (float)(m.pen_proc / m.S);
    if (valid) {
        const int32_t pb = m.p[b];
        int32_t lo, hi;
        prec_window(m, m.p, (int32_t)b, lo, hi);
        const float ton32 = m.ton32[b];
        const double ton64 = m.ton64[b];
        const float mb = m.mb32[b], Vb = m.Vb32[b];
        auto ow = [&](int32_t w) { return L.ore[w * 64 + lane]; };
        const float remv = removal_term(m, pb, ton32, ow);
        for (int32_t t = wave; t < D; t += 4) {
            MoveOut o = score_move(m, L.d64, L.Ms, t, pb, lo, hi, c, remv, ton32, ton64,
                                   mb, Vb, var32, sig32, lam, pps, ow);
            stage_s[lane * D + t] = o.score;
            stage_f[lane * D + t] = o.flags;
            if (COMP) {
                int64_t i = b * D + t;
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
        for (int64_t i = tid; i < n4; i += 256)
            ((float4 *)so)[i] = ((const float4 *)stage_s)[i];
        for (int64_t i = (n4 << 2) + tid; i < n_out; i += 256) so[i] = stage_s[i];
    } else {
        for (int64_t i = tid; i < n_out; i += 256) so[i] = stage_s[i];
    }
    if ((((uintptr_t)fo) & 3) == 0) {
        const int64_t n4 = n_out >> 2;
        for (int64_t i = tid; i < n4; i += 256)
            ((uint32_t *)fo)[i] = ((const uint32_t *)stage_f)[i];
        for (int64_t i = (n4 << 2) + tid; i < n_out; i += 256) fo[i] = stage_f[i];
    } else {
        for (int64_t i = tid; i < n_out; i += 256) fo[i] = stage_f[i];
    }
}

// ---- list mode: per-block quantities, then one thread per move --------------
__global__ void __launch_bounds__(256) k_block_prep(DevModel m) {
    extern __shared__ __align__(16) char lds[];
    const TileLds L = carve(lds, m);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t b = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = b < m.N;
    const float c = tile_phase_a(m, L, b, valid);
    if (wave == 0 && valid) {
        const int32_t pb = m.p[b];
        int32_t lo, hi;
        prec_window(m, m.p, (int32_t)b, lo, hi);
        auto ow = [&](int32_t w) { return L.ore[w * 64 + lane]; };
        m.blk_c[b] = c;
        m.blk_rem[b] = removal_term(m, pb, m.ton32[b], ow);
        m.blk_info[b] = pb | (lo << 8) | (hi << 16);
    }
}

template <bool COMP>
__global__ void __launch_bounds__(256) k_eval_list(DevModel m, int64_t n, const int32_t *blk,
                                                   const int8_t *per, float *score,
                                                   uint8_t *flags, float *dR, float *dPp,
                                                   float *dPm) {
    __shared__ double d64[MPS_MAX_PERIODS + 1];
    __shared__ double Ms[MPS_MAX_PERIODS];
    for (int i = threadIdx.x; i <= m.T; i += blockDim.x) d64[i] = m.d64[i];
    for (int i = threadIdx.x; i < m.T; i += blockDim.x) Ms[i] = m.M[i];
    __syncthreads();
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
    const float ton32 = m.ton32[b];
    const double ton64 = m.ton64[b];
    auto ow = [&](int32_t w) { return m.ore[(int64_t)w * m.N + b]; };
    MoveOut o = score_move(m, d64, Ms, t, pb, lo, hi, m.blk_c[b], m.blk_rem[b], ton32, ton64,
                           m.mb32[b], m.Vb32[b], m.sc->var32, m.sc->sigma32,
                           (float)m.lambda, (float)(m.pen_proc / m.S), ow);
    score[i] = o.score;
    flags[i] = o.flags;
    if (COMP) {
        dR[i] = o.dr;
        dPp[i] = o.dpp;
        dPm[i] = o.dpm;
    }
}

hipError_t launch_eval(const DevModel &m, const mps_moves &mv, float *score,
                       uint8_t *flags, float *dR, float *dPp, float *dPm,
                       hipStream_t st) {
    const bool comp = dR != nullptr;
    const unsigned tiles = (unsigned)((m.N + 63) / 64);
    if (mv.exhaustive) {
        const int32_t D = mv.include_never ? m.T + 1 : m.T;
        size_t lds = tile_lds_bytes(m) + ((sizeof(float) * 64 * D + 15) & ~(size_t)15) +
                     ((size_t)64 * D + 15);
        if (comp)
            hipLaunchKernelGGL(k_eval_exh<true>, dim3(tiles), dim3(256), lds, st, m, D, score,
                               flags, dR, dPp, dPm);
        else
            hipLaunchKernelGGL(k_eval_exh<false>, dim3(tiles), dim3(256), lds, st, m, D, score,
                               flags, dR, dPp, dPm);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_block_prep, dim3(tiles), dim3(256), tile_lds_bytes(m), st, m);
    if (mv.n > 0) {
        const unsigned g = (unsigned)((mv.n + 255) / 256);
        if (comp)
            hipLaunchKernelGGL(k_eval_list<true>, dim3(g), dim3(256), 0, st, m, mv.n, mv.block,
                               mv.period, score, flags, dR, dPp, dPm);
        else
            hipLaunchKernelGGL(k_eval_list<false>, dim3(g), dim3(256), 0, st, m, mv.n, mv.block,
                               mv.period, score, flags, dR, dPp, dPm);
    }
    return hipGetLastError();
}

}  // namespace mps
