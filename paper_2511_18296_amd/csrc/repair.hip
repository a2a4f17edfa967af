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
// for decision.  Scoring is FP64, each lane taking four adjacent scenarios of
// every 256:
//   c = (1/S) sum_s (N_s - mu) v[s][b],  var' = var + 2 dd c + dd^2 V_b,
//   dR = dd m_b - lambda (sigma' - sigma),
// plus the hinge differences of the two touched periods, term by term.
//
// Where the state lives: O[t][s], M[t] and a period map in LDS; N_s in
// registers, the same copy in every wave (every wave reads all of it every
// round); mu, var and sigma in registers.  A parallel gather first writes one
// contiguous record per candidate (header, v column, ore words), and the walk
// copies the records batch by batch into LDS, loading the next batch while it
// walks the current one, so a round waits on no global load.
//
// The period map: only candidate blocks can move during a walk, so the map
// has one entry per candidate, and a block's entry is that of its FIRST
// candidate.  A marking pass stores, per block, the index of its first
// candidate (atomic min); the gather writes that index into the record for
// the block and for each of its precedence neighbours, so the walk finds the
// current period of any of them with one LDS read.  The marks are cleared at
// the end of the walk.
//
// The accept test: with B = dd m_b - dPp - pen_mine dPm, the score is
// B - lambda (sigma' - sigma), and for lambda > 0 it is positive iff
// A = B / lambda + sigma satisfies A > 0 and A^2 > var' (both sides of
// sigma' < A squared); lambda < 0 flips the comparison, lambda = 0 leaves
// B > 0.  The square root is then taken once per applied move, not once per
// scored candidate.  The wave whose candidate is applied writes the two
// changed O rows and the M entries from the values it scored with.
#include <float.h>

#include "repair.h"

namespace mps {

constexpr int kWaves = 8;   // candidates scored per round
constexpr int kThreads = 64 * kWaves;
constexpr int kDeg = MPS_MAX_DEGREE;
constexpr int kNbr = 1 + 2 * kDeg;   // the block, its predecessors, its successors
constexpr size_t kBatchBytes = 40960;   // candidate records per LDS batch buffer
constexpr int kPf = (int)(kBatchBytes / (16 * kThreads));   // float4 per thread per batch
static_assert((kWaves == 4 || kWaves == 8) && kPf >= 1,
              "one 64-bit word holds the accept bytes of a round");
constexpr uint64_t kAccMask = kWaves == 8 ? 0x0101010101010101ull : 0x01010101ull;
static_assert(kBatchBytes % (16 * kThreads) == 0, "a batch is whole float4 per thread");

// DPP move of a double (both 32-bit halves); lanes whose source is outside
// the row or masked out read 0 (bound_ctrl) or keep `old` (row_mask).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double lane63(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wave, returned to every lane: inclusive scans
// inside each row of 16 lanes (row_shr 1, 2, 4, 8), then the row totals are
// carried across rows (row_bcast 15 into rows 1 and 3, row_bcast 31 into rows
// 2 and 3), so lane 63 holds the total, which is read back as a scalar.  The
// order of the additions is fixed, so every wave sums identically.
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_f64<0x111, 0xf>(x);   // row_shr:1
    x += dpp_f64<0x112, 0xf>(x);   // row_shr:2
    x += dpp_f64<0x114, 0xf>(x);   // row_shr:4
    x += dpp_f64<0x118, 0xf>(x);   // row_shr:8
    x += dpp_f64<0x142, 0xa>(x);   // row_bcast:15 -> rows 1, 3
    x += dpp_f64<0x143, 0xc>(x);   // row_bcast:31 -> rows 2, 3
    return lane63(x);
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
    x = lane63(x);
    y = lane63(y);
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, not for its global loads in flight (the next batch of records
// travels across many rounds).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0); vmcnt, expcnt untouched
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Keeps a wave-uniform constant in a vector register: the walk holds more
// uniform values than the scalar register file has room for.  (Applied to a
// value loaded from LDS it would force an early wait for the load.)
template <class T>
__device__ __forceinline__ T in_vgpr(T x) {
    asm volatile("" : "+v"(x));
    return x;
}

__host__ __device__ inline size_t ra16(size_t x) { return (x + 15) & ~(size_t)15; }
__host__ __device__ inline int32_t pad4(int32_t S) { return (S + 3) & ~3; }

// Neighbour word of a record: bits 25..31 = the candidate's destination
// period t, bit 24 = the neighbour exists, bits 16..23 = its period before
// the walk, bits 0..15 = 1 + its period-map entry, or 0 when it is no
// candidate's block (its period then cannot change).  Word 0 is the block
// itself; an invalid candidate has word 0 = 0.
constexpr uint32_t kNbPresent = 1u << 24;
constexpr int kNbTShift = 25;
static_assert(MPS_MAX_PERIODS < 128, "t fits in seven bits");
constexpr uint16_t kMoved = 0x100;   // period-map flag: moved in this call
// O row and M entry of the destination "never": every capacity term of a
// move to or from it is 0 (finite, so that sums stay finite)
constexpr double kNever = -1e300;

// One candidate record: header, v column (S rounded up to 4, zero-padded),
// ore words.
struct CandHdr {
    int32_t b, t;           // b < 0: invalid entry
    uint32_t nb[kNbr];      // index 0 the block itself, 1..kDeg predecessors, then successors
    int32_t pad;
    double mb, Vb, ton;
};
static_assert(sizeof(CandHdr) % 16 == 0, "v column 16-byte aligned");
static_assert((sizeof(CandHdr) + 4 * kRepairMaxScen + 4 * ((kRepairMaxScen + 31) / 32) + 15) / 16 *
                      16 * kWaves <=
                  kBatchBytes,
              "a batch holds at least one window of records");

// Per candidate, for the set-up and the end of the walk.
struct CandInfo {
    int32_t b;    // block, -1 if the entry is invalid
    int32_t p0;   // its period before the walk
};

__host__ __device__ inline size_t rec_bytes(int32_t S, int32_t W) {
    return ra16(sizeof(CandHdr) + sizeof(float) * (size_t)pad4(S) + sizeof(uint32_t) * (size_t)W);
}

struct WalkLayout {
    size_t O, M, d, map, buf[2], res, total;
    int B;   // candidates per batch
};

__host__ __device__ inline WalkLayout walk_layout(int32_t S, int32_t T, int32_t W,
                                                  int32_t max_cand) {
    WalkLayout L;
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t o = off;
        off = ra16(off + bytes);
        return o;
    };
    // whole windows of kWaves candidates per batch (S <= kRepairMaxScen
    // keeps kWaves records within kBatchBytes)
    const size_t rb = rec_bytes(S, W);
    int B = (int)(kBatchBytes / rb);
    if (B > 64) B = 64;
    B -= B % kWaves;
    if (B < kWaves) B = kWaves;
    L.O = put(sizeof(double) * (size_t)(T + 1) * pad4(S));
    L.M = put(sizeof(double) * (T + 1));
    L.d = put(sizeof(double) * (T + 1));
    L.map = put(sizeof(uint16_t) * (size_t)(max_cand > 0 ? max_cand : 1));
    L.buf[0] = put(rb * B);
    L.buf[1] = put(rb * B);
    L.res = put(sizeof(double) * 3 * kWaves + 16);
    L.total = off;
    L.B = B;
    return L;
}

size_t repair_lds_bytes(const DevModel &m, int32_t max_cand) {
    return walk_layout(m.S, m.T, m.W, max_cand).total;
}

size_t repair_gather_bytes(int32_t S, int32_t W) {
    return (rec_bytes(S, W) + sizeof(CandInfo)) * (size_t)MPS_MAX_TOPK;
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

// Neighbour k of block b: 0 = b, 1..kDeg predecessors, kDeg+1..2 kDeg
// successors; -1 where b has fewer.
__device__ __forceinline__ int32_t neighbour(const DevModel &m, int32_t b, int k) {
    if (k == 0) return b;
    return k <= kDeg ? nbr(m, b, k - 1, true) : nbr(m, b, k - 1 - kDeg, false);
}

__device__ __forceinline__ int32_t cand_count(const int32_t *count, int32_t max_cand) {
    int32_t n = *count;
    return n > max_cand ? max_cand : n < 0 ? 0 : n;
}

// first[b] = the smallest candidate index whose block is b.
__global__ void __launch_bounds__(256) k_repair_mark(DevModel m, mps_moves mv, int32_t D,
                                                     const int64_t *idx, const int32_t *count,
                                                     int32_t max_cand, int32_t *first) {
    const int32_t c = blockIdx.x * 256 + threadIdx.x;
    if (c >= cand_count(count, max_cand)) return;
    int32_t b, t;
    if (decode(m, mv, D, idx[c], b, t)) atomicMin(&first[b], c);
}

// Gather the records of candidates 0 .. min(*count, max_cand) - 1: one
// 64-thread workgroup per candidate.
__global__ void __launch_bounds__(64) k_repair_gather(DevModel m, mps_moves mv, int32_t D,
                                                      const int64_t *idx, const int32_t *count,
                                                      int32_t max_cand, const int32_t *first,
                                                      char *rec, CandInfo *info) {
    const int32_t c = blockIdx.x;
    const int32_t n = cand_count(count, max_cand);
    if (c >= n) return;
    const int lane = threadIdx.x;
    const int32_t S = m.S, W = m.W, Sp = pad4(S);
    char *r = rec + (size_t)c * rec_bytes(S, W);
    CandHdr *h = (CandHdr *)r;
    float *v = (float *)(r + sizeof(CandHdr));
    uint32_t *ore = (uint32_t *)(v + Sp);
    int32_t b = -1, t = 0;
    if (!decode(m, mv, D, idx[c], b, t)) {
        b = -1;
        t = 0;
    }
    if (lane == 0) {
        h->b = b;
        h->t = t;
        h->pad = 0;
        h->mb = b >= 0 ? m.mb64[b] : 0.0;
        h->Vb = b >= 0 ? m.Vb64[b] : 0.0;
        h->ton = b >= 0 ? m.ton64[b] : 0.0;
        info[c].b = b;
        info[c].p0 = b >= 0 ? m.p[b] : 0;
    }
    if (lane < kNbr) {
        const int32_t key = b >= 0 ? neighbour(m, b, lane) : -1;
        uint32_t w = 0;
        if (key >= 0) {
            const int32_t f = first[key];
            w = ((uint32_t)t << kNbTShift) | kNbPresent | ((uint32_t)(uint8_t)m.p[key] << 16) |
                (f < n ? (uint32_t)(f + 1) : 0u);
        }
        h->nb[lane] = w;
    }
    for (int32_t s = lane; s < Sp; s += 64)
        v[s] = (b >= 0 && s < S) ? m.v[(int64_t)s * m.vld + b] : 0.0f;
    // ore bits of scenarios >= S cleared
    for (int32_t w = lane; w < W; w += 64) {
        const int32_t left = S - 32 * w;
        const uint32_t keep = left >= 32 ? 0xffffffffu : (1u << left) - 1u;
        ore[w] = b >= 0 ? m.ore[(int64_t)w * m.N + b] & keep : 0u;
    }
}

// The walk.  NQ = chunks of 256 scenarios (S <= 256 * NQ).
//
// Candidates are taken in windows of kWaves, wave w holding candidate
// pos + w, and a window is finished before the next one starts:
//   1. At the window start every wave reads, in one LDS trip, the O rows of
//      its destination t and of its block's period p0 before the walk, M and
//      the discount factors at both, and the period-map entries of its block
//      and neighbours.  (A block moved in this call is skipped, so an
//      eligible candidate's current period is always p0.)
//   2. The undecided waves score their candidates and publish accept bytes.
//      The first accepted candidate r is applied: every wave folds the move
//      into its N_s, mu, var and sigma; wave r writes its two O rows, M and
//      its map entry to LDS; waves after r fold the move into the O values,
//      M values and map entries they hold and score again (step 2) against
//      the new state, without reading LDS state.  Waves up to r are done.
//   3. When no undecided candidate is accepted, the window is done.
// Each scoring of a wave thus sees exactly the state the sequential walk
// would see at that candidate.  The next window's records are loaded into
// registers while the current window is walked.
template <int NQ>
__global__ void __launch_bounds__(kThreads) k_repair_walk(DevModel m, int32_t n_max,
                                                          const int32_t *count, int32_t hard,
                                                          int32_t *applied_out, const char *rec,
                                                          const CandInfo *info, int32_t *first) {
    extern __shared__ __align__(16) char lds[];
    const int32_t S = m.S, T = m.T, W = m.W, Sp = pad4(S);
    const WalkLayout Lo = walk_layout(S, T, W, n_max);
    const int B = Lo.B;
    const size_t rb = rec_bytes(S, W);
    double *O = (double *)(lds + Lo.O);   // [T + 1][Sp]; row T ("never") holds kNever
    double *Ml = (double *)(lds + Lo.M);  // [T + 1]; entry T holds kNever
    double *dl = (double *)(lds + Lo.d);  // [T + 1]
    uint16_t *pmap = (uint16_t *)(lds + Lo.map);
    // the two batch buffers; selected by offset so that every access stays
    // an LDS access
    const size_t boff0 = Lo.buf[0], boff1 = Lo.buf[1];
    // per wave: mu and var after its candidate's move and its dd; then two
    // sets (alternating by decision) of one accept byte per wave
    double *res = (double *)(lds + Lo.res);
    uint8_t *acc = (uint8_t *)(res + 3 * kWaves);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double inv_S = in_vgpr(1.0 / S), pen_per_S = in_vgpr(m.pen_proc / S);
    const double lambda = m.lambda;
    const double inv_lambda = in_vgpr(lambda != 0.0 ? 1.0 / lambda : 0.0);
    const double pcap = in_vgpr(m.pcap), mcap = in_vgpr(m.mcap), pen_mine = in_vgpr(m.pen_mine);
    const int32_t n = cand_count(count, n_max);

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
    // global -> LDS copies with eight loads in flight per thread
    auto stage = [&](int32_t cnt, auto ld, auto st) {
        for (int32_t base = tid; base < cnt; base += 8 * kThreads) {
            decltype(ld(0)) x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int32_t i = base + k * kThreads;
                if (i < cnt) x[k] = ld(i);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int32_t i = base + k * kThreads;
                if (i < cnt) st(i, x[k]);
            }
        }
    };

    float4 pf[kPf];
    if (n > 0) issue(0, pf);
    stage(
        (T + 1) * Sp,
        [&](int32_t i) {
            const int32_t t = i / Sp, s = i - t * Sp;
            return t == T ? kNever : s < S ? m.O[(int64_t)t * S + s] : 0.0;
        },
        [&](int32_t i, double x) { O[i] = x; });
    stage(
        2 * T + 2, [&](int32_t i) { return i < T ? m.M[i] : i == T ? kNever : m.d64[i - T - 1]; },
        [&](int32_t i, double x) {
            if (i <= T)
                Ml[i] = x;
            else
                dl[i - T - 1] = x;
        });
    stage(
        n, [&](int32_t c) { return info[c].p0; },
        [&](int32_t c, int32_t p0) { pmap[c] = (uint16_t)p0; });

    // With up to two chunks, N_s - mu and, per window, v and the ore bits
    // as doubles are kept in registers; with more they are formed when used.
    constexpr bool kRich = NQ <= 2;
    // N_s: lane holds s = 256 q + 4 lane + j; padding scenarios hold 0
    double ns[NQ][4], ev[NQ][4];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t s = 256 * q + 4 * lane + j;
            ns[q][j] = s < S ? m.Ns[s] : 0.0;
        }
    // mu and var from N_s (two passes); the walk keeps them current in
    // closed form.  Every wave computes the same values.
    double mu, var, sigma;
    {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) a += ns[q][j];
        mu = wave_sum(a) / S;
        double e2 = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int32_t s = 256 * q + 4 * lane + j;
                const double e = ns[q][j] - mu;
                e2 += s < S ? e * e : 0.0;
            }
        var = wave_sum(e2) / S;
        sigma = sqrt(var);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) ev[q][j] = ns[q][j] - mu;
    if (n > 0) commit(0, pf);
    __syncthreads();

    // ---- candidate registers: the record part of a candidate
    struct Cand {
        uint32_t nb;     // this lane's neighbour word
        float4 v[NQ];    // v column, this lane's scenarios
        uint32_t ow[NQ]; // their ore bits (the whole word until the window
                         // start shifts this lane's four to the bottom)
        double mb, Vb, ton;
    };
    auto load_rec = [&](size_t bo, int32_t i, Cand &c) {
        const char *rp = lds + bo + (size_t)i * rb;
        const CandHdr &e = *(const CandHdr *)rp;
        const float *vb = (const float *)(rp + sizeof(CandHdr));
        const uint32_t *ob = (const uint32_t *)(vb + Sp);
        c.nb = lane < kNbr ? e.nb[lane] : 0u;
        c.mb = e.mb;
        c.Vb = e.Vb;
        c.ton = e.ton;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int32_t s0 = 256 * q + 4 * lane;
            if (s0 < S) {
                c.v[q] = *(const float4 *)(vb + s0);
                c.ow[q] = ob[s0 >> 5];   // shifted at use: no wait here
            } else {
                c.v[q] = make_float4(0.f, 0.f, 0.f, 0.f);
                c.ow[q] = 0;
            }
        }
    };

    constexpr bool kPrefetch = kRich;
    int32_t applied = 0;
    int buf = 0, it = 0;
    for (int32_t c0 = 0; c0 < n; c0 += B) {
        const int32_t c1 = min(n, c0 + B);
        if (c1 < n) issue(c1, pf);   // next batch travels while this one is walked
        const size_t bo = buf ? boff1 : boff0;
        Cand C, N;
        if (wave < min(kWaves, c1 - c0)) load_rec(bo, wave, C);
        for (int32_t pos = c0; pos < c1; pos += kWaves) {
            const int32_t ne = min(kWaves, c1 - pos);
            bool undecided = wave < ne;
            // ---- step 1: this candidate's view of the state
            const uint32_t nb0 = __builtin_amdgcn_readlane(C.nb, 0);
            const bool valid = undecided && (nb0 & kNbPresent);
            const int32_t t = valid ? (int32_t)(nb0 >> kNbTShift) : 0;
            const int32_t p0 = valid ? (int32_t)((nb0 >> 16) & 0xffu) : 0;
            const uint32_t slot0 = (nb0 & 0xffffu) - 1;
#pragma unroll
            for (int q = 0; q < NQ; ++q) C.ow[q] >>= (4 * lane) & 31;
            double ot[NQ][4], op[NQ][4];
            double mlt = 0.0, mlp = 0.0, dd = 0.0;
            uint32_t cur = 0;
            if (valid) {
                const double *Ot = O + (size_t)t * Sp;
                const double *Op = O + (size_t)p0 * Sp;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int32_t s0 = 256 * q + 4 * lane;
                    if (s0 < S) {
                        const double2 x0 = *(const double2 *)(Ot + s0);
                        const double2 x1 = *(const double2 *)(Ot + s0 + 2);
                        const double2 y0 = *(const double2 *)(Op + s0);
                        const double2 y1 = *(const double2 *)(Op + s0 + 2);
                        ot[q][0] = x0.x;
                        ot[q][1] = x0.y;
                        ot[q][2] = x1.x;
                        ot[q][3] = x1.y;
                        op[q][0] = y0.x;
                        op[q][1] = y0.y;
                        op[q][2] = y1.x;
                        op[q][3] = y1.y;
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) ot[q][j] = op[q][j] = 0.0;
                    }
                }
                mlt = Ml[t];
                mlp = Ml[p0];
                dd = dl[t] - dl[p0];
                const uint32_t sl = C.nb & 0xffffu;
                cur = sl ? (uint32_t)pmap[sl - 1] : (C.nb >> 16) & 0xffu;
            }
            // v and the ore bits as doubles, for the whole window
            double vd[NQ][4], inb[NQ][4];
            if constexpr (kRich) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const float x[4] = {C.v[q].x, C.v[q].y, C.v[q].z, C.v[q].w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        vd[q][j] = (double)x[j];
                        inb[q][j] = ((C.ow[q] >> j) & 1u) ? 1.0 : 0.0;
                    }
                }
            }
            // the next window's record (same batch) travels meanwhile; with
            // more than two chunks there are not registers enough for that.
            // The LDS reads of this window are waited for first (free after
            // the state rows' wait), so that no later wait for this window's
            // record also waits for these reads.
            if constexpr (kPrefetch) {
                __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
                if (pos + kWaves + wave < c1) load_rec(bo, pos + kWaves + wave - c0, N);
            }
            // ---- step 2, as long as some candidate of the window is open
            while (true) {
                bool accept = false;
                if (valid && undecided) {
                    const uint32_t own = __builtin_amdgcn_readlane(cur, 0);
                    const int32_t pk = (int32_t)(cur & 0xffu);
                    const bool bad_prec =
                        __ballot((C.nb & kNbPresent) && ((lane >= 1 && lane <= kDeg && pk > t) ||
                                                         (lane > kDeg && lane < kNbr && t > pk))) !=
                        0ull;
                    if (!(own & kMoved) && !bad_prec && t != p0) {
                        const double ton = C.ton, tmc = ton - pcap;
                        // what does not need the sums: the mining-capacity
                        // term (Ml[T] = kNever gives 0); dvar = k1 * cp + k2
                        // with k1 = 2 dd / S, k2 = dd^2 V_b;
                        // Bs = B0 - pen * pen_proc / S
                        const double am = (hinge64(mlt + ton, mcap) - hinge64(mlt, mcap)) +
                                          (hinge64(mlp - ton, mcap) - hinge64(mlp, mcap));
                        const bool mine_ok = mlt + ton <= mcap;
                        const double k1 = 2.0 * dd * inv_S, k2 = dd * dd * C.Vb;
                        const double B0 = dd * C.mb - pen_mine * am;
                        const double mu1 = mu + dd * C.mb;
                        // max(0, o + ton - cap) - max(0, o - cap) is the
                        // excess added, clamp(o + ton - cap, 0, ton); the
                        // removal from the old period likewise.  The "never"
                        // row makes both 0.
                        double cp = 0.0, pen = 0.0;
                        bool viol = false;
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            const float vj[4] = {C.v[q].x, C.v[q].y, C.v[q].z, C.v[q].w};
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const double xa = ot[q][j] + tmc;
                                const double a = fmin(fmax(xa, 0.0), ton);
                                const double r = fmin(fmax(op[q][j] - pcap, 0.0), ton);
                                if constexpr (kRich) {
                                    cp = fma(ev[q][j], vd[q][j], cp);
                                    pen = fma(a - r, inb[q][j], pen);   // exact for 0 and 1
                                } else {
                                    cp = fma(ns[q][j] - mu, (double)vj[j], cp);
                                    pen += ((C.ow[q] >> j) & 1u) ? a - r : 0.0;
                                }
                            }
                        }
                        if (hard) {
#pragma unroll
                            for (int q = 0; q < NQ; ++q)
#pragma unroll
                                for (int j = 0; j < 4; ++j)
                                    viol |= ((C.ow[q] >> j) & 1u) && ot[q][j] + tmc > 0.0;
                        }
                        wave_sum2(cp, pen);
                        viol = __ballot(viol) != 0ull;
                        const double dvar = fma(k1, cp, k2);
                        const double var1 = fmax(var + dvar, 0.0);
                        // score = Bs - lambda (sqrt(var1) - sigma)
                        const double Bs = B0 - pen * pen_per_S;
                        if (lambda > 0.0) {
                            const double A = Bs * inv_lambda + sigma;
                            accept = A > 0.0 && A * A > var1;
                        } else if (lambda < 0.0) {
                            const double A = Bs * inv_lambda + sigma;
                            accept = A < 0.0 || A * A < var1;
                        } else {
                            accept = Bs > 0.0;
                        }
                        if (hard && !(mine_ok && !viol)) accept = false;
                        if (lane == 0 && accept) {
                            res[3 * wave] = mu1;
                            res[3 * wave + 1] = var1;
                            res[3 * wave + 2] = dd;
                        }
                    }
                }
                uint8_t *ab = acc + (it & 1) * 8;
                if (lane == 0) ab[wave] = accept ? 1 : 0;
                lds_barrier();
                ++it;
                const uint64_t am = *(const uint64_t *)ab & kAccMask;
                if (!am) break;   // every open candidate rejected: window done
                const int r = __builtin_ctzll(am) >> 3;
                // ---- apply candidate r
                const char *rr = lds + bo + (size_t)(pos + r - c0) * rb;
                const CandHdr &er = *(const CandHdr *)rr;
                const float *vr = (const float *)(rr + sizeof(CandHdr));
                const uint32_t *orr = (const uint32_t *)(vr + Sp);
                // every read of the applied candidate in one LDS trip: the
                // column reads are unconditional (lanes past S read the
                // record's first entries) and their values masked after
                float4 wv[NQ];
                uint32_t wo[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int32_t s0 = 256 * q + 4 * lane;
                    const int32_t sc = s0 < S ? s0 : 0;
                    wv[q] = *(const float4 *)(vr + sc);
                    wo[q] = orr[sc >> 5];
                }
                const uint32_t wnb0 = er.nb[0];
                const double w_ton = er.ton;
                const double ddr = res[3 * r + 2];
                mu = res[3 * r];
                var = res[3 * r + 1];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const int32_t s0 = 256 * q + 4 * lane;
                    if (s0 >= S) wv[q] = make_float4(0.f, 0.f, 0.f, 0.f);
                    wo[q] = s0 < S ? wo[q] >> (s0 & 31) : 0u;
                }
                const int32_t w_t = (int32_t)(wnb0 >> kNbTShift);
                const int32_t w_p0 = (int32_t)((wnb0 >> 16) & 0xffu);
                const uint32_t w_slot0 = (wnb0 & 0xffffu) - 1;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const float x[4] = {wv[q].x, wv[q].y, wv[q].z, wv[q].w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        ns[q][j] += (double)x[j] * ddr;
                        ev[q][j] = ns[q][j] - mu;
                    }
                }
                sigma = sqrt(var);
                ++applied;
                if (wave == r) {
                    // the applied move's O rows, M entries and map entry
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        const int32_t s0 = 256 * q + 4 * lane;
                        if (s0 < S) {
                            double nt[4], np[4];
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const bool in = (C.ow[q] >> j) & 1u;
                                nt[j] = in ? ot[q][j] + C.ton : ot[q][j];
                                np[j] = in ? op[q][j] - C.ton : op[q][j];
                            }
                            if (t < T) {
                                double *Ot = O + (size_t)t * Sp;
                                *(double2 *)(Ot + s0) = make_double2(nt[0], nt[1]);
                                *(double2 *)(Ot + s0 + 2) = make_double2(nt[2], nt[3]);
                            }
                            if (p0 < T) {
                                double *Op = O + (size_t)p0 * Sp;
                                *(double2 *)(Op + s0) = make_double2(np[0], np[1]);
                                *(double2 *)(Op + s0 + 2) = make_double2(np[2], np[3]);
                            }
                        }
                    }
                    if (lane == 0) {
                        if (t < T) Ml[t] = mlt + C.ton;
                        if (p0 < T) Ml[p0] = mlp - C.ton;
                        pmap[slot0] = (uint16_t)(t | kMoved);
                    }
                }
                if (wave <= r) undecided = false;
                if (undecided && valid) {
                    // fold the move into the state this wave holds
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const bool in = (wo[q] >> j) & 1u;
                            if (w_t < T && t == w_t) ot[q][j] = in ? ot[q][j] + w_ton : ot[q][j];
                            if (w_p0 < T && t == w_p0) ot[q][j] = in ? ot[q][j] - w_ton : ot[q][j];
                            if (w_t < T && p0 == w_t) op[q][j] = in ? op[q][j] + w_ton : op[q][j];
                            if (w_p0 < T && p0 == w_p0) op[q][j] = in ? op[q][j] - w_ton : op[q][j];
                        }
                    if (w_t < T && t == w_t) mlt += w_ton;
                    if (w_p0 < T && t == w_p0) mlt -= w_ton;
                    if (w_t < T && p0 == w_t) mlp += w_ton;
                    if (w_p0 < T && p0 == w_p0) mlp -= w_ton;
                    const uint32_t sl = C.nb & 0xffffu;
                    if (sl != 0 && sl - 1 == w_slot0) cur = (uint32_t)w_t | kMoved;
                }
                if (r == ne - 1) {
                    lds_barrier();   // the last applying wave's writes land
                    break;
                }
            }
            if (kPrefetch)
                C = N;
            else if (pos + kWaves + wave < c1)
                load_rec(bo, pos + kWaves + wave - c0, C);
        }
        if (c1 < n) {
            buf ^= 1;
            commit(buf, pf);   // the other buffer is free: its batch is done
            lds_barrier();
        }
    }
    __syncthreads();
    for (int32_t i = tid; i < T * Sp; i += kThreads) {
        const int32_t t = i / Sp, s = i - t * Sp;
        if (s < S) m.O[(int64_t)t * S + s] = O[i];
    }
    if (wave == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int32_t s = 256 * q + 4 * lane + j;
                if (s < S) m.Ns[s] = ns[q][j];
            }
    }
    for (int32_t i = tid; i < T; i += kThreads) m.M[i] = Ml[i];
    // the schedule, and the marks cleared for the next call
    stage(
        n, [&](int32_t c) { return info[c].b; },
        [&](int32_t c, int32_t b) {
            if (b < 0) return;
            const uint16_t e = pmap[c];
            if (e & kMoved) m.p[b] = (int8_t)(e & 0xffu);
            first[b] = INT32_MAX;
        });
    if (tid == 0 && applied_out) *applied_out = applied;
}

hipError_t launch_repair(const DevModel &m, const mps_moves &mv, const int64_t *idx,
                         const int32_t *count, int32_t max_cand, int32_t hard,
                         int32_t *applied, void *gather, int32_t *first, hipStream_t st) {
    if (m.S > kRepairMaxScen) return hipErrorInvalidValue;
    const int32_t D = mv.include_never ? m.T + 1 : m.T;
    const WalkLayout L = walk_layout(m.S, m.T, m.W, max_cand);
    char *rec = (char *)gather;
    CandInfo *info = (CandInfo *)(rec + rec_bytes(m.S, m.W) * (size_t)MPS_MAX_TOPK);
    if (max_cand > 0) {
        hipLaunchKernelGGL(k_repair_mark, dim3((max_cand + 255) / 256), dim3(256), 0, st, m, mv,
                           D, idx, count, max_cand, first);
        hipLaunchKernelGGL(k_repair_gather, dim3(max_cand), dim3(64), 0, st, m, mv, D, idx, count,
                           max_cand, (const int32_t *)first, rec, info);
    }
    const int nq = (m.S + 255) / 256;
    if (nq <= 1)
        hipLaunchKernelGGL(k_repair_walk<1>, dim3(1), dim3(kThreads), L.total, st, m, max_cand,
                           count, hard, applied, (const char *)rec, (const CandInfo *)info, first);
    else if (nq == 2)
        hipLaunchKernelGGL(k_repair_walk<2>, dim3(1), dim3(kThreads), L.total, st, m, max_cand,
                           count, hard, applied, (const char *)rec, (const CandInfo *)info, first);
    else
        hipLaunchKernelGGL(k_repair_walk<4>, dim3(1), dim3(kThreads), L.total, st, m, max_cand,
                           count, hard, applied, (const char *)rec, (const CandInfo *)info, first);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_prep(m, st);
}

}  // namespace mps
