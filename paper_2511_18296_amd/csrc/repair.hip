// repair.hip -- greedy repair over an ordered candidate list (Alg. 4, with
// the per-iteration GPU evaluation amortised over a top-k list).
//
// Sequential definition: walk the candidates in order; skip a block already
// moved in this call; re-check precedence and re-score the move exactly
// against the current schedule and state; apply it iff it is feasible and its
// score is positive.
//
// Execution: one workgroup of kWaves waves.  In each round wave w scores
// candidate pos + w against the SAME state.  All candidates before the first
// accepted one were scored against exactly the state the sequential walk
// would see (nothing was applied in between), so their rejections stand; the
// first accepted candidate is applied, the later ones are discarded and
// re-scored in the next round.  The result is the sequential walk's, decision
// for decision.  Scoring is FP64 on an S-wide split over the wave's lanes:
//   c = (1/S) sum_s (N_s - mu) v[s][b],  var' = var + 2 dd c + dd^2 V_b,
//   dR = dd m_b - lambda (sigma' - sigma),
// plus the hinge differences of the two touched periods, term by term.
// State (N_s, O[t][s], M[t], mu, var) lives in LDS.  A parallel gather first
// writes one contiguous record per candidate (header, v column, ore words);
// the walk copies the records batch by batch into LDS, loading the next
// batch while it walks the current one, so the walk itself waits on no
// global load.  Blocks moved in this call are kept in an LDS hash map
// (block -> new period) that overrides the periods recorded by the gather.
#include <float.h>

#include "internal.h"

namespace mps {

constexpr int kWaves = 8;   // candidates scored per round (a multiple of 8)
constexpr int kThreads = 64 * kWaves;
constexpr int kNbr = 11;   // the block, 5 predecessors, 5 successors
constexpr size_t kBatchBytes = 32768;   // candidate records per LDS batch buffer
constexpr int kPf = (int)(kBatchBytes / (16 * kThreads));   // float4 per thread per batch
static_assert(kWaves % 8 == 0 && kPf >= 1, "repair launch shape");

// DPP move of a double (both 32-bit halves); lanes whose source is outside
// the row or masked out read 0 (bound_ctrl) or keep `old` (row_mask).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wave, returned to every lane: inclusive scans
// inside each row of 16 lanes (row_shr 1, 2, 4, 8), then the row totals are
// carried across rows (row_bcast 15 into rows 1 and 3, row_bcast 31 into rows
// 2 and 3), so lane 63 holds the total, which is read back as a scalar.  The
// order of the additions is fixed, so every call sums identically.
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_f64<0x111, 0xf>(x);   // row_shr:1
    x += dpp_f64<0x112, 0xf>(x);   // row_shr:2
    x += dpp_f64<0x114, 0xf>(x);   // row_shr:4
    x += dpp_f64<0x118, 0xf>(x);   // row_shr:8
    x += dpp_f64<0x142, 0xa>(x);   // row_bcast:15 -> rows 1, 3
    x += dpp_f64<0x143, 0xc>(x);   // row_bcast:31 -> rows 2, 3
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// wave_sum of two values at once: the two DPP chains are independent, so
// their latencies overlap.  Same order of additions as wave_sum.
__device__ __forceinline__ void wave_sum2(double &x, double &y) {
    x += dpp_f64<0x111, 0xf>(x);
    y += dpp_f64<0x111, 0xf>(y);
    x += dpp_f64<0x112, 0xf>(x);
    y += dpp_f64<0x112, 0xf>(y);
    x += dpp_f64<0x114, 0xf>(x);
    y += dpp_f64<0x114, 0xf>(y);
    x += dpp_f64<0x118, 0xf>(x);
    y += dpp_f64<0x118, 0xf>(y);
    x += dpp_f64<0x142, 0xa>(x);
    y += dpp_f64<0x142, 0xa>(y);
    x += dpp_f64<0x143, 0xc>(x);
    y += dpp_f64<0x143, 0xc>(y);
    const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
    const int xl = __builtin_amdgcn_readlane((int)(bx & 0xffffffff), 63);
    const int xh = __builtin_amdgcn_readlane((int)(bx >> 32), 63);
    const int yl = __builtin_amdgcn_readlane((int)(by & 0xffffffff), 63);
    const int yh = __builtin_amdgcn_readlane((int)(by >> 32), 63);
    x = __longlong_as_double(((long long)xh << 32) | (unsigned)xl);
    y = __longlong_as_double(((long long)yh << 32) | (unsigned)yl);
}

__device__ __forceinline__ uint32_t hslot(int32_t b, int hbits) {
    return ((uint32_t)b * 0x9E3779B1u) >> (32 - hbits);
}

static int hash_bits(int32_t max_cand) {
    int h = 6;
    while ((1 << h) < 2 * max_cand) ++h;
    return h;
}

__host__ __device__ inline size_t ra16(size_t x) { return (x + 15) & ~(size_t)15; }

// One candidate record: header, v column, ore words.
struct CandHdr {
    int32_t b, t;          // b < 0: invalid entry
    int32_t key[kNbr];     // block ids (index 0 the block itself), -1 = none
    int8_t p0[kNbr];       // their periods before the walk (hash overrides)
    int8_t pad[5];
    double mb, Vb, ton;
};

__host__ __device__ inline size_t rec_bytes(int32_t S, int32_t W) {
    return ra16(sizeof(CandHdr) + sizeof(float) * (size_t)S + sizeof(uint32_t) * (size_t)W);
}

struct RepairLayout {
    size_t O, Ns, M, d, hkey, hval, buf[2], res, total;
    int B;   // candidates per batch
};

__host__ __device__ inline RepairLayout repair_layout(int32_t S, int32_t T, int32_t W,
                                                      int hbits) {
    RepairLayout L;
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t o = off;
        off = ra16(off + bytes);
        return o;
    };
    const size_t H = (size_t)1 << hbits;
    const size_t rb = rec_bytes(S, W);
    int B = (int)(kBatchBytes / rb);
    if (B > 64) B = 64;
    if (B < 1) B = 1;
    L.O = put(sizeof(double) * (size_t)T * S);
    L.Ns = put(sizeof(double) * S);
    L.M = put(sizeof(double) * T);
    L.d = put(sizeof(double) * (T + 1));
    L.hkey = put(sizeof(int32_t) * H);
    L.hval = put(H);
    L.buf[0] = put(rb * B);
    L.buf[1] = put(rb * B);
    L.res = put(sizeof(double) * (3 * kWaves + 3) + sizeof(int32_t) * kWaves + kWaves + 16);
    L.total = off;
    L.B = B;
    return L;
}

size_t repair_lds_bytes(const DevModel &m, int32_t max_cand) {
    return repair_layout(m.S, m.T, m.W, hash_bits(max_cand)).total;
}

size_t repair_gather_bytes(int32_t S, int32_t W) {
    return rec_bytes(S, W) * (size_t)MPS_MAX_TOPK;
}

// Decode candidate id into (b, t) of the move set; false if out of range.
__device__ __forceinline__ bool decode(const DevModel &m, const mps_moves &mv, int32_t D,
                                       int64_t id, int32_t &b, int32_t &t) {
    if (mv.exhaustive) {
        if (id < 0 || id >= m.N * (int64_t)D) return false;
        b = (int32_t)(id / D);
        t = (int32_t)(id % D);
        return true;
    }
    if (id < 0 || id >= mv.n) return false;
    b = mv.block[id];
    t = mv.period[id];
    return b >= 0 && (int64_t)b < m.N && t >= 0 && t <= m.T;
}

// Neighbour k of block b: 0 = b, 1..5 predecessors, 6..10 successors; -1
// outside the grid.
__device__ __forceinline__ int32_t neighbour(const DevModel &m, int32_t b, int k) {
    if (k == 0) return b;
    int32_t x, y, z;
    grid_coords(m, b, x, y, z);
    const int j = (k - 1) % 5;
    const int dz = k <= 5 ? -1 : 1;
    const int dx = j == 1 ? -1 : j == 2 ? 1 : 0;
    const int dy = j == 3 ? -1 : j == 4 ? 1 : 0;
    if (z + dz < 0 || z + dz >= m.nz || x + dx < 0 || x + dx >= m.nx || y + dy < 0 ||
        y + dy >= m.ny)
        return -1;
    return b + dz * m.nx * m.ny + dy * m.nx + dx;
}

// Gather the records of candidates 0 .. min(*count, max_cand) - 1: one
// 64-thread workgroup per candidate.
__global__ void __launch_bounds__(64) k_repair_gather(DevModel m, mps_moves mv, int32_t D,
                                                      const int64_t *idx, const int32_t *count,
                                                      int32_t max_cand, char *rec) {
    const int32_t c = blockIdx.x;
    int32_t n = *count;
    if (n > max_cand) n = max_cand;
    if (c >= n) return;
    const int lane = threadIdx.x;
    const int32_t S = m.S, W = m.W;
    char *r = rec + (size_t)c * rec_bytes(S, W);
    CandHdr *h = (CandHdr *)r;
    float *v = (float *)(r + sizeof(CandHdr));
    uint32_t *ore = (uint32_t *)(v + S);
    int32_t b = -1, t = 0;
    if (!decode(m, mv, D, idx[c], b, t)) b = -1;
    if (lane == 0) {
        h->b = b;
        h->t = t;
        h->mb = b >= 0 ? m.mb64[b] : 0.0;
        h->Vb = b >= 0 ? m.Vb64[b] : 0.0;
        h->ton = b >= 0 ? m.ton64[b] : 0.0;
    }
    if (lane < kNbr) {
        const int32_t key = b >= 0 ? neighbour(m, b, lane) : -1;
        h->key[lane] = key;
        h->p0[lane] = key >= 0 ? m.p[key] : 0;
    }
    for (int32_t s = lane; s < S; s += 64) v[s] = b >= 0 ? m.v[(int64_t)s * m.N + b] : 0.0f;
    for (int32_t w = lane; w < W; w += 64) ore[w] = b >= 0 ? m.ore[(int64_t)w * m.N + b] : 0u;
}

__global__ void __launch_bounds__(kThreads) k_repair(DevModel m, int32_t n_max,
                                                     const int32_t *count, int32_t hard,
                                                     int32_t *applied_out, int hbits,
                                                     const char *rec) {
    extern __shared__ __align__(16) char lds[];
    const int32_t S = m.S, T = m.T, W = m.W;
    const RepairLayout Lo = repair_layout(S, T, W, hbits);
    const int B = Lo.B;
    const size_t rb = rec_bytes(S, W);
    double *O = (double *)(lds + Lo.O);
    double *Ns = (double *)(lds + Lo.Ns);
    double *Ml = (double *)(lds + Lo.M);
    double *dl = (double *)(lds + Lo.d);
    int32_t *hkey = (int32_t *)(lds + Lo.hkey);
    int8_t *hval = (int8_t *)(lds + Lo.hval);
    // the two batch buffers; selected by offset so that every access stays
    // an LDS access
    const size_t boff0 = Lo.buf[0], boff1 = Lo.buf[1];
    // per wave: mu, var, sigma after its candidate's move; then mu, var,
    // sigma of the current state; then the wave's current period of the
    // block and one accept byte per wave
    double *res = (double *)(lds + Lo.res);
    double *stat = res + 3 * kWaves;
    int32_t *ipb = (int32_t *)(stat + 3);
    uint8_t *acc = (uint8_t *)(ipb + kWaves);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int32_t H = 1 << hbits;
    const double inv_S = 1.0 / S, pen_per_S = m.pen_proc / S;

    int32_t n = *count;
    if (n > n_max) n = n_max;
    if (n < 0) n = 0;

    // batch j = candidates [j*B, j*B + B) = bytes [j*B*rb, ...) of rec
    auto issue = [&](int32_t c0, float4 (&pf)[kPf]) {
        const int32_t c1 = min(n, c0 + B);
        const size_t bytes = (size_t)(c1 - c0) * rb;
        const float4 *src = (const float4 *)(rec + (size_t)c0 * rb);
#pragma unroll
        for (int k = 0; k < kPf; ++k) {
            const size_t i = (size_t)tid + (size_t)k * kThreads;
            pf[k] = i * 16 < bytes ? src[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto commit = [&](int buf, const float4 (&pf)[kPf]) {
        float4 *dst = (float4 *)(lds + (buf ? boff1 : boff0));
        const size_t cap = (size_t)B * rb;
#pragma unroll
        for (int k = 0; k < kPf; ++k) {
            const size_t i = (size_t)tid + (size_t)k * kThreads;
            if (i * 16 < cap) dst[i] = pf[k];
        }
    };

    float4 pf[kPf];
    if (n > 0) issue(0, pf);
    for (int64_t i = tid; i < (int64_t)T * S; i += kThreads) O[i] = m.O[i];
    for (int32_t i = tid; i < S; i += kThreads) Ns[i] = m.Ns[i];
    for (int32_t i = tid; i < T; i += kThreads) Ml[i] = m.M[i];
    for (int32_t i = tid; i <= T; i += kThreads) dl[i] = m.d64[i];
    for (int32_t i = tid; i < H; i += kThreads) hkey[i] = -1;
    if (n > 0) commit(0, pf);
    __syncthreads();
    // mu and var from N_s (two passes); the walk keeps them current in
    // closed form
    if (wave == 0) {
        double s = 0.0;
        for (int32_t j = lane; j < S; j += 64) s += Ns[j];
        const double mu = wave_sum(s) / S;
        double q = 0.0;
        for (int32_t j = lane; j < S; j += 64) {
            const double e = Ns[j] - mu;
            q += e * e;
        }
        const double var = wave_sum(q) / S;
        if (lane == 0) {
            stat[0] = mu;
            stat[1] = var;
            stat[2] = sqrt(var);
        }
    }
    __syncthreads();

    int32_t applied = 0;
    int buf = 0;
    for (int32_t c0 = 0; c0 < n; c0 += B) {
        const int32_t c1 = min(n, c0 + B);
        if (c1 < n) issue(c1, pf);   // next batch travels while this one is walked
        const char *bb = lds + (buf ? boff1 : boff0);
        int32_t pos = c0;
        while (pos < c1) {
            const int32_t ne = min(kWaves, c1 - pos);
            // ---- wave w scores candidate pos + w against the current state
            if (wave < ne) {
                const char *rp = bb + (size_t)(pos + wave - c0) * rb;
                const CandHdr &e = *(const CandHdr *)rp;
                const float *vb = (const float *)(rp + sizeof(CandHdr));
                const uint32_t *ob = (const uint32_t *)(vb + S);
                int32_t cur = 0;
                bool found = false;
                const int32_t key = lane < kNbr ? e.key[lane] : -1;
                const int32_t p0 = lane < kNbr ? e.p0[lane] : 0;
                if (key >= 0) {
                    uint32_t hs = hslot(key, hbits);
                    for (int32_t probe = 0; probe < H; ++probe) {
                        const int32_t kk = hkey[hs];
                        if (kk == key) {
                            found = true;
                            cur = hval[hs];
                            break;
                        }
                        if (kk < 0) break;
                        hs = (hs + 1) & (uint32_t)(H - 1);
                    }
                    if (!found) cur = p0;
                }
                const int32_t t = e.t;
                const int32_t pb = __shfl(cur, 0);
                const bool moved = __ballot(lane == 0 && found) != 0ull;
                const bool bad_prec =
                    __ballot(key >= 0 && ((lane >= 1 && lane <= 5 && cur > t) ||
                                          (lane >= 6 && lane <= 10 && t > cur))) != 0ull;
                bool eligible = e.b >= 0 && !moved && !bad_prec && t != pb;
                double score = -1.0, mu1 = 0.0, var1 = 0.0, sig1 = 0.0;
                if (eligible) {
                    const double mu = stat[0], var = stat[1], sigma = stat[2];
                    const double ton = e.ton;
                    const double dd = dl[t] - dl[pb];
                    double cp = 0.0, pen = 0.0;
                    bool viol = false;
                    // rows of the two touched periods (a valid row when the
                    // period is "never"; its terms are then masked off)
                    const bool tin = t < T, pin = pb < T;
                    const double *Ot = O + (int64_t)(tin ? t : 0) * S;
                    const double *Op = O + (int64_t)(pin ? pb : 0) * S;
                    const double cap = m.pcap;
                    // four scenarios per lane per step: every LDS read of
                    // the step is issued before the arithmetic, which is
                    // branch-free
                    for (int32_t s0 = 0; s0 < S; s0 += 256) {
                        float vs[4];
                        double ns[4], ot[4], op[4];
                        uint32_t ow[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int32_t sj = s0 + lane + 64 * j;
                            const int32_t sc = sj < S ? sj : 0;
                            vs[j] = vb[sc];
                            ns[j] = Ns[sc];
                            ot[j] = Ot[sc];
                            op[j] = Op[sc];
                            ow[j] = ob[sc >> 5];
                        }
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int32_t sj = s0 + lane + 64 * j;
                            const bool ok = sj < S;
                            const bool in = ok && ((ow[j] >> (sj & 31)) & 1u);
                            cp += ok ? (ns[j] - mu) * (double)vs[j] : 0.0;
                            // max(0, o + ton - cap) - max(0, o - cap) is the
                            // excess added, clamp(o + ton - cap, 0, ton); the
                            // removal from the old period likewise
                            const double xa = ot[j] + ton - cap;
                            const double a = fmin(fmax(xa, 0.0), ton);
                            const double r = fmin(fmax(op[j] - cap, 0.0), ton);
                            pen += (in && tin ? a : 0.0) - (in && pin ? r : 0.0);
                            viol |= in && tin && xa > 0.0;
                        }
                    }
                    wave_sum2(cp, pen);
                    const double c = cp * inv_S;
                    viol = __ballot(viol) != 0ull;
                    const double dvar = 2.0 * dd * c + dd * dd * e.Vb;
                    var1 = fmax(var + dvar, 0.0);
                    const double sp = sqrt(var1);
                    sig1 = sp;
                    mu1 = mu + dd * e.mb;
                    const double den = sp + sigma;
                    const double dsig = den > 0.0 ? dvar / den : 0.0;
                    const double dR = dd * e.mb - m.lambda * dsig;
                    const double dPp = pen * pen_per_S;
                    double am = 0.0;
                    bool mine_ok = true;
                    if (t < T) {
                        am += hinge64(Ml[t] + ton, m.mcap) - hinge64(Ml[t], m.mcap);
                        mine_ok = Ml[t] + ton <= m.mcap;
                    }
                    if (pb < T) am += hinge64(Ml[pb] - ton, m.mcap) - hinge64(Ml[pb], m.mcap);
                    score = dR - dPp - m.pen_mine * am;
                    if (hard && !(mine_ok && !viol)) eligible = false;
                }
                if (lane == 0) {
                    acc[wave] = (eligible && score > 0.0) ? 1 : 0;
                    ipb[wave] = pb;
                    res[3 * wave] = mu1;
                    res[3 * wave + 1] = var1;
                    res[3 * wave + 2] = sig1;
                }
            } else if (lane == 0) {
                acc[wave] = 0;
            }
            __syncthreads();
            // ---- the first accepted candidate of the round, if any: one
            // byte per wave, read as 64-bit words (eight waves each)
            int32_t r = ne;
#pragma unroll
            for (int q = kWaves / 8 - 1; q >= 0; --q) {
                const uint64_t am = ((const uint64_t *)acc)[q] & 0x0101010101010101ull;
                if (am) r = q * 8 + (__builtin_ctzll(am) >> 3);
            }
            if (r < ne) {
                const char *rp = bb + (size_t)(pos + r - c0) * rb;
                const CandHdr &e = *(const CandHdr *)rp;
                const float *vb = (const float *)(rp + sizeof(CandHdr));
                const uint32_t *ob = (const uint32_t *)(vb + S);
                const int32_t t = e.t, pb = ipb[r];
                const double dd = dl[t] - dl[pb];
                const double ton = e.ton;
                for (int32_t s = tid; s < S; s += kThreads) {
                    Ns[s] += (double)vb[s] * dd;
                    if ((ob[s >> 5] >> (s & 31)) & 1u) {
                        if (pb < T) O[(int64_t)pb * S + s] -= ton;
                        if (t < T) O[(int64_t)t * S + s] += ton;
                    }
                }
                if (tid == 0) {
                    if (pb < T) Ml[pb] -= ton;
                    if (t < T) Ml[t] += ton;
                    m.p[e.b] = (int8_t)t;
                    uint32_t hs = hslot(e.b, hbits);
                    while (hkey[hs] >= 0) hs = (hs + 1) & (uint32_t)(H - 1);
                    hkey[hs] = e.b;
                    hval[hs] = (int8_t)t;
                }
                if (tid >= 64 && tid < 67) stat[tid - 64] = res[3 * r + tid - 64];
                ++applied;
                pos += r + 1;
            } else {
                pos += ne;
            }
            __syncthreads();
        }
        if (c1 < n) {
            buf ^= 1;
            commit(buf, pf);   // the other buffer is free: its batch is done
            __syncthreads();
        }
    }
    __syncthreads();
    for (int64_t i = tid; i < (int64_t)T * S; i += kThreads) m.O[i] = O[i];
    for (int32_t i = tid; i < S; i += kThreads) m.Ns[i] = Ns[i];
    for (int32_t i = tid; i < T; i += kThreads) m.M[i] = Ml[i];
    if (tid == 0 && applied_out) *applied_out = applied;
}

hipError_t launch_repair(const DevModel &m, const mps_moves &mv, const int64_t *idx,
                         const int32_t *count, int32_t max_cand, int32_t hard,
                         int32_t *applied, void *gather, hipStream_t st) {
    const int hb = hash_bits(max_cand);
    const int32_t D = mv.include_never ? m.T + 1 : m.T;
    const RepairLayout L = repair_layout(m.S, m.T, m.W, hb);
    if (max_cand > 0)
        hipLaunchKernelGGL(k_repair_gather, dim3(max_cand), dim3(64), 0, st, m, mv, D, idx, count,
                           max_cand, (char *)gather);
    hipLaunchKernelGGL(k_repair, dim3(1), dim3(kThreads), L.total, st, m, max_cand, count, hard,
                       applied, hb, (const char *)gather);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_prep(m, st);
}

}  // namespace mps
