// repair.hip -- greedy repair over an ordered candidate list (Alg. 4, with
// the per-iteration GPU evaluation amortised over a top-k list).
//
// The walk is strictly sequential: every applied move changes the schedule,
// the per-scenario NPVs and the period tonnages seen by the next candidate.
// One wave (64 lanes) runs it.  Lane l owns scenarios l, l+64, ...; the
// state (N_s, O[t][s], M[t]) lives in LDS, so every step is a handful of
// LDS accesses and two FP64 wave reductions.  Re-scoring is FP64:
//   c = (1/S) sum_s (N_s - mu) v[s][b],  var' = var + 2 dd c + dd^2 V_b,
//   dR = dd m_b - lambda (sigma' - sigma),
// and the penalty differences are the hinge differences of the two touched
// periods, term by term as defined.  Blocks moved in this call are kept in
// an LDS hash map (block -> new period); every other block's period is read
// from the schedule in HBM, which only this kernel writes meanwhile and only
// for blocks that are in the map.
#include <float.h>

#include "internal.h"

namespace mps {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ uint32_t hslot(int32_t b, int hbits) {
    return ((uint32_t)b * 0x9E3779B1u) >> (32 - hbits);
}

struct RepairLds {
    double *O;      // [T][S]
    double *Ns;     // [S]
    double *M;      // [T]
    double *d;      // [T+1]
    int32_t *hkey;  // [H]
    int8_t *hval;   // [H]
};

static size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

static int hash_bits(int32_t max_cand) {
    int h = 6;
    while ((1 << h) < 2 * max_cand) ++h;
    return h;
}

size_t repair_lds_bytes(const DevModel &m, int32_t max_cand) {
    size_t H = (size_t)1 << hash_bits(max_cand);
    return a16(sizeof(double) * (size_t)m.T * m.S) + a16(sizeof(double) * m.S) +
           a16(sizeof(double) * m.T) + a16(sizeof(double) * (m.T + 1)) +
           a16(sizeof(int32_t) * H) + a16(H);
}

__device__ __forceinline__ RepairLds carve_repair(char *lds, const DevModel &m, int hbits) {
    RepairLds L;
    size_t off = 0;
    auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
    L.O = (double *)(lds + off);
    off += al(sizeof(double) * (size_t)m.T * m.S);
    L.Ns = (double *)(lds + off);
    off += al(sizeof(double) * m.S);
    L.M = (double *)(lds + off);
    off += al(sizeof(double) * m.T);
    L.d = (double *)(lds + off);
    off += al(sizeof(double) * (m.T + 1));
    L.hkey = (int32_t *)(lds + off);
    off += al(sizeof(int32_t) * ((size_t)1 << hbits));
    L.hval = (int8_t *)(lds + off);
    return L;
}

__global__ void __launch_bounds__(64) k_repair(DevModel m, mps_moves mv, int32_t D,
                                               const int64_t *idx, const int32_t *count,
                                               int32_t max_cand, int32_t hard,
                                               int32_t *applied_out, int hbits) {
    extern __shared__ __align__(16) char lds[];
    const RepairLds L = carve_repair(lds, m, hbits);
    const int lane = threadIdx.x;
    const int32_t S = m.S, T = m.T;
    const int64_t N = m.N;
    const int32_t H = 1 << hbits;
    for (int64_t i = lane; i < (int64_t)T * S; i += 64) L.O[i] = m.O[i];
    for (int32_t i = lane; i < S; i += 64) L.Ns[i] = m.Ns[i];
    for (int32_t i = lane; i < T; i += 64) L.M[i] = m.M[i];
    for (int32_t i = lane; i <= T; i += 64) L.d[i] = m.d64[i];
    for (int32_t i = lane; i < H; i += 64) L.hkey[i] = -1;
    __syncthreads();

    auto stats = [&](double &mu, double &var) {
        double s = 0.0;
        for (int32_t j = lane; j < S; j += 64) s += L.Ns[j];
        mu = wave_sum(s) / S;
        double q = 0.0;
        for (int32_t j = lane; j < S; j += 64) {
            double e = L.Ns[j] - mu;
            q += e * e;
        }
        var = wave_sum(q) / S;
    };
    double mu, var;
    stats(mu, var);
    double sigma = sqrt(var);

    int32_t n = *count;
    if (n > max_cand) n = max_cand;
    if (n < 0) n = 0;
    int32_t applied = 0;
    const int32_t nx = m.nx, nxy = m.nx * m.ny;

    for (int32_t i = 0; i < n; ++i) {
        const int64_t id = idx[i];
        int32_t b, t;
        if (mv.exhaustive) {
            if (id < 0 || id >= N * (int64_t)D) continue;
            b = (int32_t)(id / D);
            t = (int32_t)(id % D);
        } else {
            if (id < 0 || id >= mv.n) continue;
            b = mv.block[id];
            t = mv.period[id];
            if (b < 0 || (int64_t)b >= N || t < 0 || t > T) continue;
        }
        // lane 0: the block itself; lanes 1..5 predecessors; 6..10 successors
        int32_t x, y, z;
        grid_coords(m, b, x, y, z);
        int32_t key = -1;
        if (lane == 0) {
            key = b;
        } else if (lane <= 5 && z > 0) {
            const int k = lane - 1;
            const int dx = (k == 1) ? -1 : (k == 2) ? 1 : 0;
            const int dy = (k == 3) ? -1 : (k == 4) ? 1 : 0;
            if (x + dx >= 0 && x + dx < nx && y + dy >= 0 && y + dy < m.ny)
                key = b - nxy + dx + dy * nx;
        } else if (lane >= 6 && lane <= 10 && z + 1 < m.nz) {
            const int k = lane - 6;
            const int dx = (k == 1) ? -1 : (k == 2) ? 1 : 0;
            const int dy = (k == 3) ? -1 : (k == 4) ? 1 : 0;
            if (x + dx >= 0 && x + dx < nx && y + dy >= 0 && y + dy < m.ny)
                key = b + nxy + dx + dy * nx;
        }
        int32_t cur = 0;
        bool found = false;
        if (key >= 0) {
            uint32_t h = hslot(key, hbits);
            for (int32_t probe = 0; probe < H; ++probe) {
                const int32_t k = L.hkey[h];
                if (k == key) {
                    found = true;
                    cur = L.hval[h];
                    break;
                }
                if (k < 0) break;
                h = (h + 1) & (uint32_t)(H - 1);
            }
            if (!found) cur = m.p[key];
        }
        if (__ballot(lane == 0 && found)) continue;   // block already moved
        const int32_t pb = __shfl(cur, 0);
        const bool bad = key >= 0 && ((lane >= 1 && lane <= 5 && cur > t) ||
                                      (lane >= 6 && lane <= 10 && t > cur));
        if (__ballot(bad)) continue;                  // precedence fails
        if (t == pb) continue;                        // no-op

        const double ton = m.ton64[b];
        const double dd = L.d[t] - L.d[pb];
        double cp = 0.0, pen = 0.0;
        bool viol = false;
        for (int32_t s = lane; s < S; s += 64) {
            const double vs = (double)m.v[(int64_t)s * N + b];
            cp += (L.Ns[s] - mu) * vs;
            if ((m.ore[(int64_t)(s >> 5) * N + b] >> (s & 31)) & 1u) {
                if (t < T) {
                    const double o = L.O[(int64_t)t * S + s];
                    pen += hinge64(o + ton, m.pcap) - hinge64(o, m.pcap);
                    if (o + ton > m.pcap) viol = true;
                }
                if (pb < T) {
                    const double o = L.O[(int64_t)pb * S + s];
                    pen += hinge64(o - ton, m.pcap) - hinge64(o, m.pcap);
                }
            }
        }
        const double c = wave_sum(cp) / S;
        pen = wave_sum(pen);
        const bool any_viol = __ballot(viol) != 0ull;
        const double dvar = 2.0 * dd * c + dd * dd * m.Vb64[b];
        const double sp = sqrt(fmax(var + dvar, 0.0));
        const double den = sp + sigma;
        const double dsig = den > 0.0 ? dvar / den : 0.0;
        const double dR = dd * m.mb64[b] - m.lambda * dsig;
        const double dPp = m.pen_proc * pen / S;
        double am = 0.0;
        bool mine_ok = true;
        if (t < T) {
            am += hinge64(L.M[t] + ton, m.mcap) - hinge64(L.M[t], m.mcap);
            mine_ok = L.M[t] + ton <= m.mcap;
        }
        if (pb < T) am += hinge64(L.M[pb] - ton, m.mcap) - hinge64(L.M[pb], m.mcap);
        const double score = dR - dPp - m.pen_mine * am;
        bool ok = score > 0.0;
        if (hard) ok = ok && mine_ok && !any_viol;
        if (!ok) continue;

        // apply the move
        for (int32_t s = lane; s < S; s += 64) {
            const double vs = (double)m.v[(int64_t)s * N + b];
            L.Ns[s] += vs * dd;
            if ((m.ore[(int64_t)(s >> 5) * N + b] >> (s & 31)) & 1u) {
                if (pb < T) L.O[(int64_t)pb * S + s] -= ton;
                if (t < T) L.O[(int64_t)t * S + s] += ton;
            }
        }
        if (lane == 0) {
            if (pb < T) L.M[pb] -= ton;
            if (t < T) L.M[t] += ton;
            m.p[b] = (int8_t)t;
            uint32_t h = hslot(b, hbits);
            while (L.hkey[h] >= 0) h = (h + 1) & (uint32_t)(H - 1);
            L.hkey[h] = b;
            L.hval[h] = (int8_t)t;
        }
        ++applied;
        __syncthreads();
        stats(mu, var);
        sigma = sqrt(var);
    }
    __syncthreads();
    for (int64_t i = lane; i < (int64_t)T * S; i += 64) m.O[i] = L.O[i];
    for (int32_t i = lane; i < S; i += 64) m.Ns[i] = L.Ns[i];
    for (int32_t i = lane; i < T; i += 64) m.M[i] = L.M[i];
    if (lane == 0 && applied_out) *applied_out = applied;
}

hipError_t launch_repair(const DevModel &m, const mps_moves &mv, const int64_t *idx,
                         const int32_t *count, int32_t max_cand, int32_t hard,
                         int32_t *applied, hipStream_t st) {
    const int hb = hash_bits(max_cand);
    const int32_t D = mv.include_never ? m.T + 1 : m.T;
    hipLaunchKernelGGL(k_repair, dim3(1), dim3(64), repair_lds_bytes(m, max_cand), st, m, mv, D,
                       idx, count, max_cand, hard, applied, hb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_prep(m, st);
}

}  // namespace mps
