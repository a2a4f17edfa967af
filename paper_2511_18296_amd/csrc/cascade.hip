// cascade.hip -- cascading repair (Alg. 4 with its fallback): the greedy
// repair walk, where a candidate (b, t') that precedence (Eq. 15) forbids is
// taken together with the blocks that forbid it.
//
// Moving b earlier (t' < p_b) takes along every ancestor reached through
// predecessors mined after t'; moving it later takes along every descendant
// reached through successors mined before t'.  The set moves to t' as one
// composite move, scored exactly against the current state in FP64:
//   N'_s = N_s + sum_{x in set} v[s][x] (d(t') - d(p_x)), mu', sigma' two-pass,
//   dR = (mu' - lambda sigma') - (mu - lambda sigma),
//   the processing hinge terms of every period the set leaves or enters,
//   sum_s [hinge(O'[u][s]) - hinge(O[u][s])], and the mining hinge terms.
// It is applied iff the set has at most max_set blocks, none was moved
// earlier in this call, Eq. 15 holds at every moved block of the result,
// (hard mode) period t' stays within both capacities, and the score is > 0.
//
// Execution: one workgroup walks the candidates in order.  The per-scenario
// NPV and the period tonnages live in LDS (FP64, updated in place on every
// accept, each O'[u][s] formed with the additions in the set's order, so each
// capacity decision is the sequential one bit for bit).  The set is formed by
// one wave breadth-first (neighbours in list order: the 1-5 stencil's
// predecessors up, x-1, x+1, y-1, y+1 and successors by increasing index, or
// the explicit lists in their order),
// with membership tested against the set in LDS; the checks and the scoring
// spread over the workgroup.  After the walk the state is re-derived from the
// schedule.
#include <float.h>

#include "internal.h"

namespace mps {

constexpr int kCT = 256;              // threads of the walk
constexpr int kCW = kCT / 64;
constexpr int kCMaxSet = kCascadeMaxSet;   // largest set a call may allow

__device__ __forceinline__ double hinge_c(double x, double cap) { return x > cap ? x - cap : 0.0; }

// Sum over the workgroup (every thread gets it); red is kCW doubles of LDS.
__device__ __forceinline__ double cascade_sum(double x, double *red) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kCW; ++w) s += red[w];
    return s;
}

struct CascadeShared {
    int32_t b, t, pb, skip, n, too_big, ok_flag;
    int32_t set[kCMaxSet];
    int32_t setp[kCMaxSet];
    double setton[kCMaxSet];
    uint64_t touched[2];
    double red[kCW];
};

__global__ void __launch_bounds__(kCT) k_cascade_clear(uint8_t *mark, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        mark[i] = 0;
}

__global__ void __launch_bounds__(kCT) k_cascade_walk(DevModel m, mps_moves mv, int32_t D,
                                                      const int64_t *idx, const int32_t *count,
                                                      int32_t max_cand, int32_t hard,
                                                      int32_t max_set, uint8_t *mark,
                                                      int32_t *applied_out) {
    extern __shared__ double lds[];
    const int32_t S = m.S, T = m.T;
    double *O = lds;                        // [T][S]
    double *Ml = O + (size_t)T * S;         // [T]
    double *Ns = Ml + T;                    // [S]
    double *Np = Ns + S;                    // [S]
    double *dl = Np + S;                    // [T+1]
    __shared__ CascadeShared sh;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t i = tid; i < (int64_t)T * S; i += kCT) O[i] = m.O[i];
    for (int i = tid; i < T; i += kCT) Ml[i] = m.M[i];
    for (int i = tid; i < S; i += kCT) Ns[i] = m.Ns[i];
    for (int i = tid; i <= T; i += kCT) dl[i] = m.d64[i];
    int32_t n_cand = min(*count, max_cand);
    int32_t applied = 0;
    __syncthreads();
    for (int32_t c = 0; c < n_cand; ++c) {
        // every thread has read the previous candidate's shared fields
        __syncthreads();
        if (tid == 0) {
            const int64_t id = idx[c];
            int32_t b = -1, t = -1;
            if (id >= 0) {
                if (mv.exhaustive) {
                    if (id < m.N * D) {
                        b = (int32_t)(id / D);
                        t = (int32_t)(id % D);
                    }
                } else if (id < mv.n) {
                    b = mv.block[id];
                    t = mv.period[id];
                }
            }
            int32_t skip = (b < 0 || b >= m.N || t < 0 || t > T) ? 1 : 0;
            int32_t pb = 0;
            if (!skip) {
                pb = m.p[b];
                if (mark[b] || pb == t) skip = 1;
            }
            sh.b = b;
            sh.t = t;
            sh.pb = pb;
            sh.skip = skip;
            sh.n = 1;
            sh.too_big = 0;
            sh.ok_flag = 1;
            sh.set[0] = b;
            sh.setp[0] = pb;
            sh.setton[0] = skip ? 0.0 : m.ton64[b];
        }
        __syncthreads();
        if (sh.skip) continue;
        const int32_t t = sh.t;
        // ---- the set, breadth-first, by wave 0 ----
        if (wave == 0) {
            const bool earlier = t < sh.pb;
            int32_t n = 1;
            bool big = false;
            for (int32_t q = 0; q < n && !big; ++q) {
                const int64_t a = lane < MPS_MAX_DEGREE ? nbr(m, sh.set[q], lane, earlier) : -1;
                int32_t pa = 0;
                bool want = false;
                if (a >= 0) {
                    pa = m.p[a];
                    want = earlier ? pa > t : pa < t;
                    for (int32_t j = 0; j < n && want; ++j)
                        if (sh.set[j] == (int32_t)a) want = false;
                }
                const uint64_t bal = __ballot(want);
                const int32_t add = __popcll(bal);
                if (n + add > max_set) {
                    big = true;
                    break;
                }
                if (want) {
                    const int32_t pos = n + __popcll(bal & ((1ull << lane) - 1ull));
                    sh.set[pos] = (int32_t)a;
                    sh.setp[pos] = pa;
                    sh.setton[pos] = m.ton64[a];
                }
                n += add;
                // this wave's LDS writes land before its next reads of the set
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            }
            if (lane == 0) {
                sh.n = n;
                sh.too_big = big ? 1 : 0;
            }
        }
        __syncthreads();
        if (sh.too_big) continue;
        const int32_t n = sh.n;
        // ---- moved marks and Eq. 15 at every moved block of the result ----
        bool ok = true;
        constexpr int kD = MPS_MAX_DEGREE;
        for (int32_t i = tid; i < n * 2 * kD; i += kCT) {
            const int32_t q = i / (2 * kD), k = i % (2 * kD);
            const int32_t x = sh.set[q];
            if (k == 0 && mark[x]) ok = false;
            const bool pred = k < kD;
            const int64_t a = nbr(m, x, pred ? k : k - kD, pred);
            if (a < 0) continue;
            int32_t pa = m.p[a];
            for (int32_t j = 0; j < n; ++j)
                if (sh.set[j] == (int32_t)a) pa = t;
            if (pred ? pa > t : t > pa) ok = false;
        }
        if (!__syncthreads_and(ok)) continue;
        // ---- exact score ----
        double s1 = 0.0;
        for (int32_t s = tid; s < S; s += kCT) {
            double acc = Ns[s];
            for (int32_t q = 0; q < n; ++q)
                acc += (double)m.v[(int64_t)s * m.vld + sh.set[q]] * (dl[t] - dl[sh.setp[q]]);
            Np[s] = acc;
            s1 += acc;
        }
        double s0 = 0.0;
        for (int32_t s = tid; s < S; s += kCT) s0 += Ns[s];
        const double mu2 = cascade_sum(s1, sh.red) / S;
        const double mu = cascade_sum(s0, sh.red) / S;
        double q1 = 0.0, q0 = 0.0;
        for (int32_t s = tid; s < S; s += kCT) {
            q1 += (Np[s] - mu2) * (Np[s] - mu2);
            q0 += (Ns[s] - mu) * (Ns[s] - mu);
        }
        const double sd2 = sqrt(cascade_sum(q1, sh.red) / S);
        const double sd = sqrt(cascade_sum(q0, sh.red) / S);
        const double dR = (mu2 - m.lambda * sd2) - (mu - m.lambda * sd);
        if (tid == 0) {
            uint64_t tw[2] = {0ull, 0ull};
            if (t < T) tw[t >> 6] |= 1ull << (t & 63);
            for (int32_t q = 0; q < n; ++q) {
                const int32_t u = sh.setp[q];
                if (u < T) tw[u >> 6] |= 1ull << (u & 63);
            }
            sh.touched[0] = tw[0];
            sh.touched[1] = tw[1];
        }
        __syncthreads();
        // O' of a touched period u in scenario s, additions in the set's order
        auto o_after = [&](int32_t u, int32_t s) {
            double o = O[(size_t)u * S + s];
            for (int32_t q = 0; q < n; ++q) {
                const int32_t x = sh.set[q];
                if (!((m.ore[(int64_t)(s >> 5) * m.N + x] >> (s & 31)) & 1u)) continue;
                if (sh.setp[q] == u) o -= sh.setton[q];
                if (t == u) o += sh.setton[q];
            }
            return o;
        };
        auto m_after = [&](int32_t u) {
            double o = Ml[u];
            for (int32_t q = 0; q < n; ++q) {
                if (sh.setp[q] == u) o -= sh.setton[q];
                if (t == u) o += sh.setton[q];
            }
            return o;
        };
        double pacc = 0.0;
        bool hard_ok = true;
        for (int32_t u = 0; u < T; ++u) {
            if (!((sh.touched[u >> 6] >> (u & 63)) & 1ull)) continue;
            for (int32_t s = tid; s < S; s += kCT) {
                const double op = o_after(u, s);
                pacc += hinge_c(op, m.pcap) - hinge_c(O[(size_t)u * S + s], m.pcap);
                if (hard && u == t && !(op <= m.pcap)) hard_ok = false;
            }
        }
        const double pp = cascade_sum(pacc, sh.red);
        double am = 0.0;
        for (int32_t u = 0; u < T; ++u)
            if ((sh.touched[u >> 6] >> (u & 63)) & 1ull)
                am += hinge_c(m_after(u), m.mcap) - hinge_c(Ml[u], m.mcap);
        if (hard && t < T && !(m_after(t) <= m.mcap)) hard_ok = false;
        const double score = dR - m.pen_proc * pp / S - m.pen_mine * am;
        const bool accept = __syncthreads_and(hard_ok) && score > 0.0;
        if (!accept) continue;
        // ---- apply ----
        // each thread owns scenario s of every touched row: no other thread
        // reads O[u][s] before the barrier below
        for (int32_t s = tid; s < S; s += kCT)
            for (int32_t u = 0; u < T; ++u)
                if ((sh.touched[u >> 6] >> (u & 63)) & 1ull) O[(size_t)u * S + s] = o_after(u, s);
        __syncthreads();
        if (tid == 0)
            for (int32_t u = 0; u < T; ++u)
                if ((sh.touched[u >> 6] >> (u & 63)) & 1ull) Ml[u] = m_after(u);
        for (int32_t s = tid; s < S; s += kCT) Ns[s] = Np[s];
        for (int32_t q = tid; q < n; q += kCT) {
            m.p[sh.set[q]] = (int8_t)t;
            mark[sh.set[q]] = 1;
        }
        ++applied;
        __syncthreads();
    }
    if (tid == 0 && applied_out) *applied_out = applied;
}

size_t cascade_lds_bytes(const DevModel &m) {
    return 8 * ((size_t)m.T * m.S + m.T + 2 * (size_t)m.S + m.T + 1) + sizeof(CascadeShared);
}

hipError_t launch_cascade(const DevModel &m, const mps_moves &mv, const int64_t *idx,
                          const int32_t *count, int32_t max_cand, int32_t hard, int32_t max_set,
                          int32_t *applied, uint8_t *mark, double *partial, int chunks,
                          hipStream_t st) {
    const int32_t D = mv.include_never ? m.T + 1 : m.T;
    hipLaunchKernelGGL(k_cascade_clear, dim3(256), dim3(kCT), 0, st, mark, m.N);
    hipLaunchKernelGGL(k_cascade_walk, dim3(1), dim3(kCT),
                       cascade_lds_bytes(m) - sizeof(CascadeShared), st, m, mv, D, idx, count,
                       max_cand, hard, max_set, mark, applied);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_set_schedule(m, m.p, partial, chunks, st);
}

}  // namespace mps
