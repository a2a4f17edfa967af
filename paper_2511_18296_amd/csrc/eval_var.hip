// eval_var.hip -- move evaluation under the objective variants: the value
// multiplier sigma(s,t) of Eq. 12 and the CVaR risk measure.
//
// With a multiplier the change of scenario s's NPV for a move (b, t') is
//   D_s = v[s][b] (w[s][t'] - w[s][p_b]),   w[s][t] = d(t) sigma(s,t), w[s][T] = 0,
// no longer one factor times v[s][b], so the rank-1 form of the base kernel
// does not apply: every move sweeps its S scenarios.
//   std measure:  dmu = mean_s D_s,
//                 dvar = (2/S) sum_s e_s D_s + (1/S) sum_s D_s^2 - dmu^2,
//                 dR = dmu - lambda (sigma' - sigma), sigma' = sqrt(var + dvar)
//                 (taken as dvar / (sigma' + sigma));
//   CVaR measure: R = mu - lambda (mu - CVaR_alpha(N)), and with e'_s = e_s + D_s
//                 dR = (1 - lambda) dmu + lambda (CVaR_alpha(e') - (CVaR_alpha(N) - mu)),
//                 CVaR_alpha(e') the lower-tail mean: the k = ceil(alpha S)
//                 smallest e'_s, the k-th with weight alpha S - k + 1, over alpha S;
// the capacity terms and flags are the base definitions, in FP64 against the
// period tonnages:
//   dPp = pen_proc/S sum_s ore[s][b] [hinge(O[t'][s] + ton) - hinge(O[t'][s])
//                                     + hinge(O[p_b][s] - ton) - hinge(O[p_b][s])],
//   PROC_OK iff no ore scenario has O[t'][s] + ton > proc_cap.
//
// Execution: one wave per block (exhaustive) or per listed move, lanes over
// scenarios (each lane keeps its scenarios' v and ore bits in registers and
// loops over the block's destinations).  A workgroup of four waves stages the
// period tonnages (FP64), the discounted multipliers (FP32) and e_s in LDS and
// then takes 64 blocks (or 64 listed moves); what a block's destinations
// share (its period, tonnage, precedence window, the mining term of leaving
// its period) is formed once per block, and the four sums of a move are
// reduced over the wave together.  The k-th smallest e'_s is found by a radix
// select on the order-preserving integer image of the FP32 values: 16 rounds
// of two bits, each counting the keys below three candidate prefixes with
// ballots.
#include <float.h>

#include <type_traits>

#include "internal.h"

namespace mps {

constexpr int kVT = 256;         // threads per workgroup
constexpr int kVW = kVT / 64;
constexpr int kVItems = 64;      // blocks (or listed moves) per workgroup
constexpr int kVQ = 16;          // scenarios per lane: S <= 1024

struct MoveOutVar {
    float score, dr, dpp, dpm;
    uint8_t flags;
};

struct VarLds {
    double *O;     // [T][S]
    double *M;     // [T]
    double *d;     // [T+1]
    float *w;      // [S][T+1] discounted multipliers (d(t) when there is none)
    float *e;      // [S]
};

__host__ __device__ inline size_t var_layout(int32_t S, int32_t T, char *base, VarLds *L) {
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 15) & ~(size_t)15;
        return o;
    };
    const size_t oO = put(8 * (size_t)T * S), oM = put(8 * (size_t)T), od = put(8 * (size_t)(T + 1)),
                 ow = put(4 * (size_t)S * (T + 1)), oe = put(4 * (size_t)S);
    if (L) {
        L->O = (double *)(base + oO);
        L->M = (double *)(base + oM);
        L->d = (double *)(base + od);
        L->w = (float *)(base + ow);
        L->e = (float *)(base + oe);
    }
    return off;
}

__device__ __forceinline__ float wsum_f(float x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
__device__ __forceinline__ double wsum_d(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
__device__ __forceinline__ int32_t wsum_i(int32_t x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
// Four sums over the wave at once: the four butterfly chains are independent,
// so their shuffle latencies overlap.
__device__ __forceinline__ void wsum4(float &a, float &b, float &c, double &d) {
    for (int o = 32; o > 0; o >>= 1) {
        const float ya = __shfl_xor(a, o), yb = __shfl_xor(b, o), yc = __shfl_xor(c, o);
        const double yd = __shfl_xor(d, o);
        a += ya;
        b += yb;
        c += yc;
        d += yd;
    }
}
__device__ __forceinline__ uint32_t ord32(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u >> 31) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ double hinge_v(double x, double cap) { return x > cap ? x - cap : 0.0; }

// What every destination of a block shares: its period, tonnage, precedence
// window and the mining term of leaving its period.
struct VarBlock {
    int32_t pb, lo, hi;
    double ton, am_rem;
    float var32, sig32, cvar_e;   // the state's scalars (read once per workgroup)
};
__device__ __forceinline__ VarBlock var_block(const DevModel &m, const VarLds &L, int32_t b,
                                              const float (&scal)[3]) {
    VarBlock k;
    k.var32 = scal[0];
    k.sig32 = scal[1];
    k.cvar_e = scal[2];
    k.pb = m.p[b];
    k.ton = m.ton64[b];
    prec_window(m, m.p, b, k.lo, k.hi);
    k.am_rem = k.pb < m.T ? hinge_v(L.M[k.pb] - k.ton, m.mcap) - hinge_v(L.M[k.pb], m.mcap) : 0.0;
    return k;
}

// Score and flags of the move (b, t) for the wave; v[q], ob (ore bit) of
// this lane's scenarios s = lane + 64 q (q < NQ <= Q); kb the block's shared
// quantities.
template <int Q>
__device__ __forceinline__ MoveOutVar score_var(const DevModel &m, const VarLds &L,
                                                const VarBlock &kb, int32_t t,
                                                const float (&v)[Q], const bool (&ob)[Q],
                                                int32_t NQ) {
    const int lane = threadIdx.x & 63;
    const int32_t S = m.S, T = m.T, T1 = m.T + 1;
    MoveOutVar o;
    const int32_t pb = kb.pb;
    const double ton = kb.ton;
    float sd = 0.0f, sed = 0.0f, sdd = 0.0f;
    float ep[Q];
    double pacc = 0.0;
    bool viol = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        ep[q] = 0.0f;
        if (q >= NQ) break;
        const int32_t s = lane + 64 * q;
        if (s >= S) break;
        const float dw = L.w[(size_t)s * T1 + t] - L.w[(size_t)s * T1 + pb];
        const float D = v[q] * dw;
        const float es = L.e[s];
        sd += D;
        sed = fmaf(es, D, sed);
        sdd = fmaf(D, D, sdd);
        ep[q] = es + D;
        if (ob[q]) {
            if (t < T) {
                const double ot = L.O[(size_t)t * S + s];
                pacc += hinge_v(ot + ton, m.pcap) - hinge_v(ot, m.pcap);
                viol = viol || (ot + ton > m.pcap);
            }
            if (pb < T) {
                const double op = L.O[(size_t)pb * S + s];
                pacc += hinge_v(op - ton, m.pcap) - hinge_v(op, m.pcap);
            }
        }
    }
    wsum4(sd, sed, sdd, pacc);
    viol = __ballot(viol) != 0ull;
    const float dmu = sd / S;
    float dr;
    if (m.risk == 1) {
        // k-th smallest e'_s (0-based k - 1) by a radix select on its key
        const double aS = m.alpha * S;
        int32_t k = (int32_t)ceil(aS);
        k = k < 1 ? 1 : (k > S ? S : k);
        uint32_t key[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int32_t s = lane + 64 * q;
            key[q] = (q < NQ && s < S) ? ord32(ep[q]) : 0xffffffffu;
        }
        // two bits per round: the counts of keys below the three candidate
        // prefixes pre | 01, pre | 10, pre | 11 of the round's bit pair
        uint32_t pre = 0u;
        for (int bit = 30; bit >= 0; bit -= 2) {
            const uint32_t c1 = pre | (1u << bit), c2 = pre | (2u << bit), c3 = pre | (3u << bit);
            // counts over the wave by ballot: no cross-lane round trip
            int32_t n1 = 0, n2 = 0, n3 = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (q < NQ) {
                    const bool in = lane + 64 * q < S;
                    n1 += __popcll(__ballot(in && key[q] < c1));
                    n2 += __popcll(__ballot(in && key[q] < c2));
                    n3 += __popcll(__ballot(in && key[q] < c3));
                }
            // the largest candidate with at most k - 1 keys below it
            pre = n3 <= k - 1 ? c3 : n2 <= k - 1 ? c2 : n1 <= k - 1 ? c1 : pre;
        }
        // pre is the key of the k-th smallest value
        float xk = 0.0f, below = 0.0f;
        int32_t nb = 0;
        bool hk = false;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (q >= NQ || lane + 64 * q >= S) continue;
            if (key[q] < pre) {
                below += ep[q];
                ++nb;
            } else if (key[q] == pre) {
                xk = ep[q];
                hk = true;
            }
        }
        below = wsum_f(below);
        nb = wsum_i(nb);
        // every lane holding the k-th key holds the same value
        const uint64_t has = __ballot(hk);
        xk = __shfl(xk, __ffsll((unsigned long long)has) - 1);
        const float cv = (below + (float)(k - 1 - nb) * xk + (float)(aS - (k - 1)) * xk) / (float)aS;
        dr = (1.0f - (float)m.lambda) * dmu + (float)m.lambda * (cv - kb.cvar_e);
    } else {
        const float var32 = kb.var32, sig32 = kb.sig32;
        const float dvar = 2.0f * sed / S + sdd / S - dmu * dmu;
        const float vp = fmaxf(var32 + dvar, 0.0f);
        const float den = sqrtf(vp) + sig32;
        const float dsig = den > 0.0f ? dvar / den : 0.0f;
        dr = dmu - (float)m.lambda * dsig;
    }
    double am = 0.0;
    bool mine_ok = true;
    if (t < T) {
        const double Mt = L.M[t];
        am += hinge_v(Mt + ton, m.mcap) - hinge_v(Mt, m.mcap);
        mine_ok = Mt + ton <= m.mcap;
    }
    am += kb.am_rem;
    const int32_t lo = kb.lo, hi = kb.hi;
    const bool noop = t == pb;
    uint8_t f = 0;
    if (lo <= t && t <= hi) f |= MPS_PREC_OK;
    if (noop || t == T || mine_ok) f |= MPS_MINE_OK;
    if (noop || t == T || !viol) f |= MPS_PROC_OK;
    if (noop) f |= MPS_NOOP;
    o.flags = f;
    const float dpp = (float)(m.pen_proc * pacc / S);
    const float dpm = (float)(m.pen_mine * am);
    o.dr = noop ? 0.0f : dr;
    o.dpp = noop ? 0.0f : dpp;
    o.dpm = noop ? 0.0f : dpm;
    o.score = noop ? 0.0f : (dr - dpp) - dpm;
    return o;
}

__device__ __forceinline__ void var_stage(const DevModel &m, const VarLds &L) {
    const int tid = threadIdx.x;
    const int32_t S = m.S, T = m.T, T1 = m.T + 1;
    for (int64_t i = tid; i < (int64_t)T * S; i += kVT) L.O[i] = m.O[i];
    for (int i = tid; i < T; i += kVT) L.M[i] = m.M[i];
    for (int i = tid; i <= T; i += kVT) L.d[i] = m.d64[i];
    for (int64_t i = tid; i < (int64_t)S * T1; i += kVT) {
        const int32_t t = (int32_t)(i % T1);
        L.w[i] = m.wmult32 ? m.wmult32[i] : (float)m.d64[t];
    }
    for (int i = tid; i < S; i += kVT) L.e[i] = m.e32[i];
    __syncthreads();
}

template <int Q>
__device__ __forceinline__ void var_column(const DevModel &m, int32_t b, int32_t NQ,
                                           float (&v)[Q], bool (&ob)[Q]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        v[q] = 0.0f;
        ob[q] = false;
        if (q >= NQ) continue;
        const int32_t s = lane + 64 * q;
        if (s >= m.S) continue;
        v[q] = m.v[(int64_t)s * m.vld + b];
        ob[q] = (m.ore[(int64_t)(s >> 5) * m.N + b] >> (s & 31)) & 1u;
    }
}

template <int Q>
__global__ void __launch_bounds__(kVT) k_eval_var_exh(DevModel m, int32_t D, float *score,
                                                      uint8_t *flags, float *dR, float *dPp,
                                                      float *dPm) {
    extern __shared__ char lds_raw[];
    VarLds L;
    var_layout(m.S, m.T, lds_raw, &L);
    var_stage(m, L);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t NQ = (m.S + 63) / 64;
    const float scal[3] = {gld(&m.sc->var32), gld(&m.sc->sigma32), (float)gld(&m.sc->cvar_e)};
    const int64_t b0 = (int64_t)blockIdx.x * kVItems;
    for (int i = wave; i < kVItems; i += kVW) {
        const int64_t b = b0 + i;
        if (b >= m.N) break;
        float v[Q];
        bool ob[Q];
        var_column<Q>(m, (int32_t)b, NQ, v, ob);
        const VarBlock kb = var_block(m, L, (int32_t)b, scal);
        for (int32_t t = 0; t < D; ++t) {
            const MoveOutVar o = score_var<Q>(m, L, kb, t, v, ob, NQ);
            if (lane == 0) {
                const int64_t j = b * D + t;
                score[j] = o.score;
                flags[j] = o.flags;
                if (dR) {
                    dR[j] = o.dr;
                    dPp[j] = o.dpp;
                    dPm[j] = o.dpm;
                }
            }
        }
    }
}

template <int Q>
__global__ void __launch_bounds__(kVT) k_eval_var_list(DevModel m, int64_t n, const int32_t *blk,
                                                       const int8_t *per, float *score,
                                                       uint8_t *flags, float *dR, float *dPp,
                                                       float *dPm) {
    extern __shared__ char lds_raw[];
    VarLds L;
    var_layout(m.S, m.T, lds_raw, &L);
    var_stage(m, L);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t NQ = (m.S + 63) / 64;
    const float scal[3] = {gld(&m.sc->var32), gld(&m.sc->sigma32), (float)gld(&m.sc->cvar_e)};
    const int64_t i0 = (int64_t)blockIdx.x * kVItems;
    for (int i = wave; i < kVItems; i += kVW) {
        const int64_t j = i0 + i;
        if (j >= n) break;
        const int32_t b = blk[j], t = per[j];
        MoveOutVar o;
        if (b < 0 || b >= m.N || t < 0 || t > m.T) {
            o.score = -FLT_MAX;
            o.flags = MPS_BAD;
            o.dr = o.dpp = o.dpm = 0.0f;
        } else {
            float v[Q];
            bool ob[Q];
            var_column<Q>(m, b, NQ, v, ob);
            o = score_var<Q>(m, L, var_block(m, L, b, scal), t, v, ob, NQ);
        }
        if (lane == 0) {
            score[j] = o.score;
            flags[j] = o.flags;
            if (dR) {
                dR[j] = o.dr;
                dPp[j] = o.dpp;
                dPm[j] = o.dpm;
            }
        }
    }
}

size_t eval_var_lds_bytes(const DevModel &m) { return var_layout(m.S, m.T, nullptr, nullptr); }

hipError_t launch_eval_var(const DevModel &m, const mps_moves &mv, float *score, uint8_t *flags,
                           float *dR, float *dPp, float *dPm, hipStream_t st) {
    const size_t lds = eval_var_lds_bytes(m);
    // registers for the scenarios a lane holds: 64, 128, 256, 512 or 1024 per wave
    const int32_t nq = (m.S + 63) / 64;
    auto go = [&](auto qtag) {
        constexpr int Q = decltype(qtag)::value;
        if (mv.exhaustive) {
            const int32_t D = mv.include_never ? m.T + 1 : m.T;
            const unsigned g = (unsigned)((m.N + kVItems - 1) / kVItems);
            hipLaunchKernelGGL(k_eval_var_exh<Q>, dim3(g), dim3(kVT), lds, st, m, D, score, flags,
                               dR, dPp, dPm);
        } else if (mv.n > 0) {
            const unsigned g = (unsigned)((mv.n + kVItems - 1) / kVItems);
            hipLaunchKernelGGL(k_eval_var_list<Q>, dim3(g), dim3(kVT), lds, st, m, mv.n,
                               mv.block, mv.period, score, flags, dR, dPp, dPm);
        }
    };
    if (nq <= 1) go(std::integral_constant<int, 1>());
    else if (nq <= 2) go(std::integral_constant<int, 2>());
    else if (nq <= 4) go(std::integral_constant<int, 4>());
    else if (nq <= 8) go(std::integral_constant<int, 8>());
    else go(std::integral_constant<int, kVQ>());
    return hipGetLastError();
}

}  // namespace mps
