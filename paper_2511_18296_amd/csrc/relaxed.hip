// relaxed.hip -- relaxed (differentiable) schedule objective, its
// hand-written adjoint, and gradient ranking of all moves.
//
// x[b,t] in [0,1] is the cumulative fraction of block b mined by the end of
// period t, y[b,t] = x[b,t] - x[b,t-1] (x[b,-1] = 0).  The forward pass forms
//   NPV_s   = sum_b v[s,b] D_b,          D_b = sum_t d(t) y[b,t]
//   Ot[s,t] = sum_b ore[s,b] ton_b y[b,t],  Mt[t] = sum_b ton_b y[b,t]
//   J = mu - lambda sigma - (mu_proc/S) sum max(0, Ot - Pcap)^2
//       - mu_mine sum max(0, Mt - Mcap)^2
//       - mu_prec sum_b sum_{a in Pred(b)} sum_t max(0, x[b,t] - x[a,t])^2
// (the risk-adjusted expectation of Eq. 14 on a relaxed plan, with quadratic
// versions of the capacity and precedence constraints, Eq. 15-16).  The
// adjoint is the exact derivative: with w_s = 1/S - lambda (NPV_s - mu)/(S sigma),
//   dJ/dy[b,t] = d(t) sum_s w_s v[s,b]
//              - ton_b [ (2 mu_proc/S) sum_s ore[s,b] E[s,t] + 2 mu_mine Em[t] ]
// E = max(0, Ot - Pcap), Em = max(0, Mt - Mcap); dJ/dx = dJ/dy[t] - dJ/dy[t+1]
// plus the precedence terms.
//
// Forward.  The blocks are cut into chunks and the scenarios, with one extra
// row whose ore bits are all 1 (it sums to Mt), into groups; a workgroup of
// eight waves takes one (chunk, group) pair.  Its four work waves stage x,
// the group's ore words and ton_b in LDS and form D_b and ton_b y[b,t], the
// latter as three bf16 parts that add up to it exactly (each part keeps the
// top eight significant bits of what is left).  Ot over the chunk is then a
// dense contraction of the 0/1 ore matrix with those parts: 16x16x32 bf16
// MFMA, fp32 accumulation, products exact; the same waves then sum the
// precedence penalty of the chunk.  Its four stream waves load the rows of v
// from the moment the staged operands are in (lanes over blocks, 14 rows in
// flight per wave) and dot them with D_b as soon as it is there.  A second kernel adds the chunk partials
// in chunk order, and one workgroup forms the scalars and w_s.
//
// Backward.  128-block tiles: u_b = sum_s w_s v[s,b] streams v the same way,
// and G[b,t] = sum_s ore[s,b] E[s,t] is the same MFMA contraction with the
// scenarios as the inner dimension and E split into bf16 parts by the forward
// pass.
#include <float.h>
#include <math.h>

#include "internal.h"

namespace mps {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

constexpr int kRT = 512;      // threads of the chunk and tile kernels (eight waves)
constexpr int kRB = 6;        // rows of v per register batch; two batches in flight
constexpr int kStage = 16;    // staged loads of x values and ore words per thread

__host__ __device__ static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
__host__ __device__ static inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }

// ---- division by a run-time constant: q = (umulhi(n, m) + n) >> s with
// s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1 (Granlund and
// Montgomery's round-up method; exact for every 32-bit n).
struct DivU32 {
    uint32_t m, s;
};
static DivU32 make_div(uint32_t d) {
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    const uint64_t mm = ((((uint64_t)1 << s) - d) << 32) / d + 1;
    return DivU32{(uint32_t)mm, s};
}
__device__ __forceinline__ uint32_t divu(uint32_t n, DivU32 q) {
    const uint32_t t = __umulhi(n, q.m);
    return (uint32_t)(((uint64_t)t + n) >> q.s);
}

// y == h + m + l exactly: each part takes the top eight significant bits of
// what the previous parts left (truncation), and a float has 24.
__device__ __forceinline__ void split3(float y, uint16_t &h, uint16_t &md, uint16_t &l) {
    const uint32_t hu = __float_as_uint(y) & 0xffff0000u;
    const float r = y - __uint_as_float(hu);
    const uint32_t mu = __float_as_uint(r) & 0xffff0000u;
    const float r2 = r - __uint_as_float(mu);
    h = (uint16_t)(hu >> 16);
    md = (uint16_t)(mu >> 16);
    l = (uint16_t)(__float_as_uint(r2) >> 16);
}

// bf16 1.0 is 0x3F80: a sign-extended bit masked with it is 1.0 or 0.0.
__device__ __forceinline__ uint32_t bf16_pair(uint32_t w0, uint32_t p0, uint32_t w1, uint32_t p1) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_sbfe((int)w0, p0, 1) & 0x3F80u;
    const uint32_t hi = (uint32_t)__builtin_amdgcn_sbfe((int)w1, p1, 1) & 0x3F800000u;
    return lo | hi;
}

// The element at a 32-bit offset of off 4-byte words from base (off < 2^30):
// a wave-uniform base plus one 32-bit register per lane, the same registers
// for every row.
template <typename V>
__device__ __forceinline__ V ld_off(const V *base, uint32_t off) {
    return *(const V *)((const char *)base + (off << 2));
}

__device__ __forceinline__ f32x4 mfma_bf16(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Sum over the 64 lanes of a wave (inclusive scans inside rows of 16 lanes,
// then the row totals carried across rows; lane 63 holds the total).  The
// order of the additions is fixed.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float x) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true));
}
__device__ __forceinline__ float wave_sum_f32(float x) {
    x += dpp_f32<0x111, 0xf>(x);   // row_shr:1
    x += dpp_f32<0x112, 0xf>(x);   // row_shr:2
    x += dpp_f32<0x114, 0xf>(x);   // row_shr:4
    x += dpp_f32<0x118, 0xf>(x);   // row_shr:8
    x += dpp_f32<0x142, 0xa>(x);   // row_bcast:15 -> rows 1, 3
    x += dpp_f32<0x143, 0xc>(x);   // row_bcast:31 -> rows 2, 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_f64(double x) {   // same order as wave_sum_f32
    x += dpp_f64<0x111, 0xf>(x);
    x += dpp_f64<0x112, 0xf>(x);
    x += dpp_f64<0x114, 0xf>(x);
    x += dpp_f64<0x118, 0xf>(x);
    x += dpp_f64<0x142, 0xa>(x);
    x += dpp_f64<0x143, 0xc>(x);
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ---- saved-state layout ------------------------------------------------------
struct SavedView {
    double *scal;   // [8]: J, mu, sigma, Pproc, Pmine, Pprec, spare, spare
    double *npv;    // [S]
    float *w;       // [S]
    float *E;       // [S][T]
    float *Em;      // [T]
    uint16_t *Es;   // [T][3][Sp] bf16 parts of E, scenarios padded with zeros to Sp
};

__host__ __device__ static inline int32_t pad_scen(int32_t S) { return (S + 31) & ~31; }

__host__ __device__ static inline size_t saved_bytes(int32_t S, int32_t T) {
    return al256(8 * 8) + al256(8 * (size_t)S) + al256(4 * (size_t)S) +
           al256(4 * (size_t)S * T) + al256(4 * (size_t)T) +
           al256(2 * 3 * (size_t)T * pad_scen(S));
}

__host__ __device__ static inline SavedView saved_view(void *p, int32_t S, int32_t T) {
    char *c = (char *)p;
    SavedView v;
    v.scal = (double *)c;
    c += al256(8 * 8);
    v.npv = (double *)c;
    c += al256(8 * (size_t)S);
    v.w = (float *)c;
    c += al256(4 * (size_t)S);
    v.E = (float *)c;
    c += al256(4 * (size_t)S * T);
    v.Em = (float *)c;
    c += al256(4 * (size_t)T);
    v.Es = (uint16_t *)c;
    return v;
}

size_t relaxed_saved_bytes(const DevModel &m) { return saved_bytes(m.S, m.T); }

struct RelaxK {
    double lambda, mu_proc, mu_mine, mu_prec, pcap, mcap;
};

// ---- forward geometry ----------------------------------------------------------
// The forward workgroup has two kinds of waves: waves 0-3 stream the rows of
// v, waves 4-7 stage the operands and run the contraction and the
// precedence sum.
constexpr int kSW = 4;        // stream waves
// Rows of v per register batch of a stream wave (two batches in flight):
// 2 x 7 rows of four loads stay below the 63 a wave can have outstanding.
constexpr int kRBs = 7;
constexpr int kStX = 20;      // staged x entries per work thread (CB T <= 5120)
constexpr int kStO = 16;      // staged ore rows per work thread (SG <= 512)
constexpr int kPR = 8;        // precedence entries per work thread in flight

struct FwdGeom {
    int32_t CB;      // blocks per staged piece (multiple of 32, <= 256)
    int32_t nsub;    // pieces per workgroup
    int32_t G;       // chunks (= partials)
    int32_t SG;      // scenario rows per group (multiple of 32)
    int32_t OG;      // groups
    int32_t ntt;     // 16-period tiles
    int32_t TT;      // period tiles per work wave, padded to 1, 2, 4 or 8
    int32_t SL;      // s-tiles per work wave (8 / TT)
    int32_t Q;       // loads per row of v and lane (ceil(CB / 64))
    int64_t ncols;   // (S + 1) T + S partial columns
    int64_t Cp;      // padded
    int32_t nred;    // reduce workgroups (16 columns each)
    size_t lds;
};

static size_t fwd_lds(int32_t CB, int32_t T, int32_t SG) {
    return al16(4 * (size_t)CB * T) + al16(6 * (size_t)CB * (T + 1)) +
           al16(4 * (size_t)(SG / 32 + 1) * CB) + al16(4 * (size_t)CB) * 3 + al16(4 * (size_t)SG) +
           al16(4 * (size_t)T) + 8 * 4;
}

static FwdGeom fwd_geom(const DevModel &m) {
    FwdGeom g{};
    const int32_t T = m.T, S = m.S;
    const int64_t N = m.N;
    g.ntt = (T + 15) / 16;
    g.TT = g.ntt <= 1 ? 1 : g.ntt <= 2 ? 2 : g.ntt <= 4 ? 4 : 8;
    g.SL = 8 / g.TT;
    // s-tiles per group: each of the four work waves takes at most SL
    const int32_t st_max = 4 * g.SL;
    const int32_t rows = S + 1;                   // the Mt row is scenario S
    int32_t st_need = (rows + 15) / 16;
    st_need = (st_need + 1) & ~1;
    g.SG = 16 * (st_need < st_max ? st_need : st_max);
    g.OG = (rows + g.SG - 1) / g.SG;
    // blocks per piece: the LDS budget and the staged loads bound it
    int32_t lim = 256;
    while (lim > 32 &&
           (fwd_lds(lim, T, g.SG) > 65536 || (int64_t)lim * T > (int64_t)kStX * (kRT - 64 * kSW)))
        lim -= 32;
    const int32_t target = 256 / g.OG > 1 ? 256 / g.OG : 1;   // chunks wanted
    const int64_t want = 32 * ((N + 32LL * target - 1) / (32LL * target));
    if (want <= lim) {
        g.CB = (int32_t)want;
        g.nsub = 1;
    } else {
        g.CB = lim;
        g.nsub = (int32_t)((want + lim - 1) / lim);
    }
    g.G = (int32_t)((N + (int64_t)g.CB * g.nsub - 1) / ((int64_t)g.CB * g.nsub));
    g.Q = (g.CB + 63) / 64;
    g.ncols = (int64_t)(S + 1) * T + S;
    g.Cp = (g.ncols + 63) & ~(int64_t)63;
    g.nred = (int32_t)((g.ncols + 15) / 16);
    g.lds = fwd_lds(g.CB, T, g.SG);
    return g;
}

// ---- backward geometry ---------------------------------------------------------
constexpr int kStE = 6;       // staged 16-byte pieces of the E parts per thread
struct BwdGeom {
    int32_t TB;     // blocks per tile (128, or 64 for T > 64)
    int32_t Q;      // TB / 64
    int32_t KC;     // scenarios staged per pass (multiple of 32)
    int32_t MT;     // most tiles per wave (2, 4 or 8)
    size_t lds;
};

static size_t bwd_lds(int32_t TB, int32_t KC, int32_t T, int32_t S) {
    return al16(6 * (size_t)(T + 1) * KC) + al16(4 * (size_t)(KC / 32) * TB) +
           al16(4 * (size_t)TB * (T + 1)) + al16(4 * 8 * (size_t)TB) + 2 * al16(4 * (size_t)TB) +
           2 * al16(4 * (size_t)T) + al16(4 * (size_t)S);
}

static BwdGeom bwd_geom(const DevModel &m) {
    BwdGeom g{};
    const int32_t T = m.T, ntt = (T + 15) / 16;
    g.TB = ntt <= 4 ? 128 : 64;
    g.Q = g.TB / 64;
    const int32_t twv = 8 / (g.TB / 16);                 // waves per 16-block row tile
    const int32_t tiles = (ntt + twv - 1) / twv;          // period tiles per wave
    g.MT = tiles <= 2 ? 2 : tiles <= 4 ? 4 : 8;
    int32_t kc = pad_scen(m.S);
    if (kc > 1024) kc = 1024;
    while (kc > 32 && (bwd_lds(g.TB, kc, T, m.S) > 65536 || 3LL * T * (kc / 8) > (int64_t)kStE * kRT))
        kc -= 32;
    g.KC = kc;
    g.lds = bwd_lds(g.TB, kc, T, m.S);
    return g;
}

// ---- workspace -------------------------------------------------------------------
struct RelaxWs {
    uint16_t *nmask;   // [N] neighbour bits: 0-4 predecessors, 5-9 successors
    float *P;          // [G][Cp] chunk partials: Ot rows 0..S (row S = Mt), then NPV
    double *pq;        // [nred] sums of E^2 per reduce workgroup
    double *pmq;       // [nred] sums of Em^2
    double *prq;       // [G] precedence sums per chunk
};

size_t relaxed_ws_bytes(const DevModel &m) {
    const FwdGeom g = fwd_geom(m);
    return al256(2 * (size_t)m.N) + al256(4 * (size_t)g.G * g.Cp) + 2 * al256(8 * (size_t)g.nred) +
           al256(8 * (size_t)g.G);
}

static RelaxWs relax_ws(void *ws, const DevModel &m, const FwdGeom &g) {
    char *c = (char *)ws;
    RelaxWs r;
    r.nmask = (uint16_t *)c;
    c += al256(2 * (size_t)m.N);
    r.P = (float *)c;
    c += al256(4 * (size_t)g.G * g.Cp);
    r.pq = (double *)c;
    c += al256(8 * (size_t)g.nred);
    r.pmq = (double *)c;
    c += al256(8 * (size_t)g.nred);
    r.prq = (double *)c;
    return r;
}

// The 1-5 precedence stencil (Eq. 15) of every block as ten bits: the block
// below and its four horizontal neighbours (predecessors), the same above
// (successors).  Built once per model.
__global__ void k_relax_init(DevModel m, uint16_t *nmask) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m.N) return;
    if (m.csr) {   // explicit lists: the precedence terms come from k_relax_prec_*_csr
        nmask[b] = 0;
        return;
    }
    int32_t xx, yy, zz;
    grid_coords(m, (int32_t)b, xx, yy, zz);
    const uint32_t nb = (xx > 0 ? 2u : 0u) | (xx + 1 < m.nx ? 4u : 0u) | (yy > 0 ? 8u : 0u) |
                        (yy + 1 < m.ny ? 16u : 0u) | 1u;
    uint32_t bits = 0;
    if (zz > 0) bits |= nb;
    if (zz + 1 < m.nz) bits |= nb << 5;
    nmask[b] = (uint16_t)bits;
}

hipError_t launch_relaxed_init(const DevModel &m, void *ws, hipStream_t st) {
    const FwdGeom g = fwd_geom(m);
    const RelaxWs r = relax_ws(ws, m, g);
    hipLaunchKernelGGL(k_relax_init, dim3((unsigned)((m.N + 255) / 256)), dim3(256), 0, st, m,
                       r.nmask);
    return hipGetLastError();
}

// ---- forward: one (chunk, scenario group) per workgroup --------------------------
struct FwdArgs {
    const float *x;
    float *P;
    double *prq;
    const uint16_t *nmask;
    int64_t Cp;
    int32_t CB, nsub, SG, ntt;
    DivU32 divT;
};

// MULTI: more than one staged piece per workgroup (very large models); with
// one piece the loop over pieces disappears and nothing is kept across it.
template <int SL, int TT, bool MULTI>
__global__ void __launch_bounds__(kRT, 2) k_relax_fwd_chunk(DevModel m, FwdArgs a) {
    constexpr int Q = 4;                               // blocks of a row per lane
    extern __shared__ __align__(16) char lds[];
    const int32_t T = m.T, S = m.S, CB = a.CB, SG = a.SG, nwm = a.SG / 32;
    const int64_t N = m.N;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool streamer = wave < kSW;
    const int ww = wave - kSW;                         // work wave index
    const int32_t s_lo = (int32_t)blockIdx.y * SG;     // first scenario row of the group
    const int32_t w_lo = s_lo >> 5;
    const int32_t nwr = max(0, min(nwm, m.W - w_lo));  // real ore words of the group
    const int32_t s_hi = min(S + 1, s_lo + SG);        // rows [s_lo, s_hi), row S = Mt
    const int32_t nst = (s_hi - s_lo + 15) >> 4;        // s-tiles of the group
    const int32_t sv_hi = min(S, s_lo + SG);            // rows of v in the group
    // stream wave w takes rows s_lo + w + 4 i; work wave ww the s-tiles ww + 4 sl
    const int32_t nrow = streamer && sv_hi > s_lo + wave ? (sv_hi - s_lo - wave + kSW - 1) / kSW : 0;
    const int32_t nslw = !streamer && nst > ww ? (nst - ww + 3) / 4 : 0;
    const bool do_prec = blockIdx.y == 0;               // the first group sums the precedence term

    char *c = lds;
    float *xs = (float *)c;                       // [CB*T] x of the piece
    c += al16(4 * (size_t)CB * T);
    uint16_t *Ys = (uint16_t *)c;                 // [T+1][3][CB] parts of ton*y; row T = 0
    c += al16(6 * (size_t)CB * (T + 1));
    uint32_t *orl = (uint32_t *)c;                // [nwm + 1][CB]; row nwm is the Mt row
    c += al16(4 * (size_t)(nwm + 1) * CB);
    float *Dl = (float *)c;                       // [CB]
    c += al16(4 * (size_t)CB);
    float *tonl = (float *)c;                     // [CB]
    c += al16(4 * (size_t)CB);
    uint32_t *nml = (uint32_t *)c;                // [CB] precedence-stencil bits
    c += al16(4 * (size_t)CB);
    float *npl = (float *)c;                      // [SG] NPV partials of the group's rows
    c += al16(4 * (size_t)SG);
    float *dl = (float *)c;                       // [T] d(t)
    c += al16(4 * (size_t)T);
    double *redp = (double *)c;                   // [4] precedence sums of the work waves

    f32x4 acc[SL][TT];
#pragma unroll
    for (int i = 0; i < SL; ++i)
#pragma unroll
        for (int j = 0; j < TT; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    double prec = 0.0;
    for (int32_t i = tid; i < SG; i += kRT) npl[i] = 0.0f;
    for (int32_t i = tid; i < 3 * CB; i += kRT) Ys[(size_t)T * 3 * CB + i] = 0;
    const int64_t NT = N * T, nxy = (int64_t)m.nx * m.ny;
    const int64_t poff[5] = {-nxy * T, (-nxy - 1) * T, (-nxy + 1) * T, (-nxy - m.nx) * T,
                             (-nxy + m.nx) * T};

    // Every load of v is issued unconditionally (rows and blocks past the end
    // are clamped to valid addresses and never used), so that each wait
    // names exactly the batch it needs.
    // lane blocks: ln + 64 q
    auto issue = [&](float (&buf)[kRBs][Q], int64_t bc, int32_t nb, int32_t i0, uint32_t ln) {
#pragma unroll
        for (int r = 0; r < kRBs; ++r) {
            const int32_t i = min(i0 + r, max(nrow - 1, 0));
            const int32_t s = min(s_lo + wave + kSW * i, S - 1);
            const float *row = m.v + (int64_t)s * m.vld + bc;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                buf[r][q] = ld_off(row, min(ln + 64u * q, (uint32_t)(nb - 1)));
        }
    };
    const int32_t g8 = 8 * (lane >> 4);
    const int64_t b_beg = (int64_t)blockIdx.x * a.nsub * CB;
    const int32_t npc = MULTI ? a.nsub : 1;
    for (int32_t pc = 0; pc < npc; ++pc) {
        const int64_t bc = b_beg + (int64_t)pc * CB;
        if (bc >= N) break;
        const int32_t nb = (int32_t)min((int64_t)CB, N - bc);
        const int32_t nbT = nb * T;
        // The two roles pass the same three barriers per piece (after the
        // staged operands, after D_b and the parts, at the end of the piece),
        // each inside its own branch, so that the registers of the rows in
        // flight and those of the contraction are never live together.
        if (streamer) {
            // the lane index passes through an empty asm, so that nothing of
            // this role is computed before the branch (and kept live across
            // the other role's code)
            uint32_t ln = (uint32_t)lane;
            asm volatile("" : "+v"(ln));
            float va[kRBs][Q], vb[kRBs][Q];
            // ---- the first rows of v (lane blocks j = lane + 64 q), issued once
            // the staged operands are in, so that they do not delay them
            __syncthreads();
            issue(va, bc, nb, 0, ln);
            issue(vb, bc, nb, kRBs, ln);
            __syncthreads();
            // ---- NPV of the piece: rows of v against D_b; one batch is
            // consumed while the other is in flight
            float dq[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int32_t j = lane + 64 * q;
                dq[q] = j < nb ? Dl[j] : 0.0f;
            }
            auto consume = [&](float (&buf)[kRBs][Q], int32_t i0) {
#pragma unroll
                for (int r = 0; r < kRBs; ++r) {
                    if (i0 + r < nrow) {
                        float p = 0.0f;
#pragma unroll
                        for (int q = 0; q < Q; ++q) p = fmaf(buf[r][q], dq[q], p);
                        p = wave_sum_f32(p);
                        if (lane == 0) npl[wave + kSW * (i0 + r)] += p;
                    }
                }
            };
            // (the scheduling barriers keep each batch's new loads after its
            // consumption: issued earlier they would need a second set of
            // registers)
            for (int32_t i0 = 0; i0 < nrow; i0 += 2 * kRBs) {
                consume(va, i0);
                __builtin_amdgcn_sched_barrier(0);
                issue(va, bc, nb, i0 + 2 * kRBs, ln);
                __builtin_amdgcn_sched_barrier(0);
                consume(vb, i0 + kRBs);
                __builtin_amdgcn_sched_barrier(0);
                issue(vb, bc, nb, i0 + 3 * kRBs, ln);
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
        } else {
            int wt = tid - 64 * kSW;   // work thread index, opaque as above
            asm volatile("" : "+v"(wt));
            // ---- staged operands
            float xr[kStX];
            const float *xc0 = a.x + bc * T;
#pragma unroll
            for (int k = 0; k < kStX; ++k)
                if (k * 256 < CB * T) xr[k] = ld_off(xc0, (uint32_t)min(wt + k * 256, nbT - 1));
            const uint32_t jc = (uint32_t)min(wt, nb - 1);
            uint32_t orr[kStO];
#pragma unroll
            for (int k = 0; k < kStO; ++k)
                if (k < nwr) orr[k] = ld_off(m.ore + (int64_t)(w_lo + k) * N + bc, jc);
            const float tv = m.ton32[bc + jc];
            const uint32_t nmv = a.nmask[bc + jc];
            const double dv = m.d64[min(wt, T - 1)];
#pragma unroll
            for (int k = 0; k < kStX; ++k) {
                const int32_t e = wt + k * 256;
                if (k * 256 < CB * T && e < CB * T) xs[e] = e < nbT ? xr[k] : 0.0f;
            }
            if (wt < CB) {
#pragma unroll
                for (int k = 0; k < kStO; ++k)
                    if (k < nwr) orl[k * CB + wt] = wt < nb ? orr[k] : 0u;
                orl[nwm * CB + wt] = wt < nb ? 1u : 0u;
                tonl[wt] = wt < nb ? tv : 0.0f;
                nml[wt] = wt < nb ? nmv : 0u;
            }
            if (wt < T) dl[wt] = (float)dv;
            __syncthreads();
            // ---- per block: D_b and the three parts of ton_b y[b,t]
            if (wt < CB) {
                const int32_t j = wt;
                const float tj = tonl[j];
                float prev = 0.0f, dsum = 0.0f;
                for (int32_t t = 0; t < T; ++t) {
                    const float xc = xs[j * T + t];
                    const float y = xc - prev;
                    prev = xc;
                    dsum = fmaf(dl[t], y, dsum);
                    uint16_t h, md, l;
                    split3(tj * y, h, md, l);
                    Ys[(t * 3 + 0) * CB + j] = h;
                    Ys[(t * 3 + 1) * CB + j] = md;
                    Ys[(t * 3 + 2) * CB + j] = l;
                }
                Dl[j] = dsum;
            }
            __syncthreads();
            // ---- Ot (and Mt) of the piece on the matrix cores: the 0/1
            // fragments of the wave's s-tiles are built once per step of 32
            // blocks, each part of ton*y is loaded once per period tile and
            // serves them all; periods past T read the zero row
            const int32_t nkb = (nb + 31) & ~31;
            for (int32_t kb = 0; kb < nkb; kb += 32) {
                u32x4 A[SL];
#pragma unroll
                for (int sl = 0; sl < SL; ++sl) {
                    if (sl < nslw) {
                        const int32_t s = s_lo + 16 * (ww + 4 * sl) + (lane & 15);
                        const int32_t orow = s < S ? (s - s_lo) >> 5 : nwm;
                        const uint32_t bp = s < S ? (uint32_t)(s & 31) : (s == S ? 0u : 1u);
                        const uint32_t *ow = orl + orow * CB + kb + g8;
                        const u32x4 w0 = *(const u32x4 *)ow;
                        const u32x4 w1 = *(const u32x4 *)(ow + 4);
                        A[sl].x = bf16_pair(w0.x, bp, w0.y, bp);
                        A[sl].y = bf16_pair(w0.z, bp, w0.w, bp);
                        A[sl].z = bf16_pair(w1.x, bp, w1.y, bp);
                        A[sl].w = bf16_pair(w1.z, bp, w1.w, bp);
                    }
                }
#pragma unroll
                for (int tt = 0; tt < TT; ++tt) {
                    if (tt < a.ntt) {
                        const int32_t t = min(16 * tt + (lane & 15), T);
                        const uint16_t *yb = Ys + (size_t)t * 3 * CB + kb + g8;
                        const u32x4 B0 = *(const u32x4 *)yb;
                        const u32x4 B1 = *(const u32x4 *)(yb + CB);
                        const u32x4 B2 = *(const u32x4 *)(yb + 2 * CB);
#pragma unroll
                        for (int sl = 0; sl < SL; ++sl) {
                            if (sl < nslw) {
                                acc[sl][tt] = mfma_bf16(A[sl], B0, acc[sl][tt]);
                                acc[sl][tt] = mfma_bf16(A[sl], B1, acc[sl][tt]);
                                acc[sl][tt] = mfma_bf16(A[sl], B2, acc[sl][tt]);
                            }
                        }
                    }
                }
            }
            // ---- precedence penalty of the piece: max(0, x[b,t] - x[a,t])^2
            // over the (up to) five predecessors a; loads at clamped offsets,
            // masked with the stencil bits
            if (do_prec) {
                for (int32_t e0 = wt; e0 < nbT; e0 += kPR * 256) {
                    float px[kPR][5];
#pragma unroll
                    for (int u = 0; u < kPR; ++u) {
                        const int64_t eg = bc * T + min(e0 + u * 256, nbT - 1);
#pragma unroll
                        for (int k = 0; k < 5; ++k)
                            px[u][k] = a.x[(uint32_t)min(max(eg + poff[k], (int64_t)0), NT - 1)];
                    }
#pragma unroll
                    for (int u = 0; u < kPR; ++u) {
                        const int32_t e = e0 + u * 256;
                        if (e < nbT) {
                            const uint32_t nm = nml[divu((uint32_t)e, a.divT)];
                            const float xc = xs[e];
#pragma unroll
                            for (int k = 0; k < 5; ++k) {
                                const float d = xc - px[u][k];
                                if (((nm >> k) & 1u) && d > 0.0f) prec += (double)d * (double)d;
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    // ---- partials of the chunk
    float *P = a.P + (int64_t)blockIdx.x * a.Cp;
    if (!streamer) {
#pragma unroll
        for (int sl = 0; sl < SL; ++sl) {
#pragma unroll
            for (int tt = 0; tt < TT; ++tt) {
                const int32_t t = 16 * tt + (lane & 15);
                const int32_t s0 = s_lo + 16 * (ww + 4 * sl) + 4 * (lane >> 4);
                if (sl < nslw && tt < a.ntt && t < T) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (s0 + q <= S) P[(int64_t)(s0 + q) * T + t] = acc[sl][tt][q];
                }
            }
        }
        if (do_prec) {
            const double w = wave_sum_f64(prec);
            if (lane == 0) redp[ww] = w;
        }
    }
    for (int32_t r = tid; r < sv_hi - s_lo; r += kRT) P[(int64_t)(S + 1) * T + s_lo + r] = npl[r];
    if (do_prec) {
        __syncthreads();
        if (tid == 0) a.prq[blockIdx.x] = ((redp[0] + redp[1]) + redp[2]) + redp[3];
    }
}

// ---- chunk partials in chunk order -------------------------------------------------
struct RedArgs {
    const float *P;
    int64_t Cp, ncols;
    int32_t G, nred, Sp;
    double *pq, *pmq;
    const double *prq;
    DivU32 divT;
};

__global__ void __launch_bounds__(256) k_relax_fwd_reduce(DevModel m, RedArgs a, RelaxK rk,
                                                          SavedView sv) {
    __shared__ double red[256];
    __shared__ double rq[2][16];
    const int tid = threadIdx.x;
    const int32_t S = m.S, T = m.T;
    // 16 columns per workgroup, the chunks split in 16 ranges
    const int col = tid & 15, part = tid >> 4;
    const int64_t cidx = (int64_t)blockIdx.x * 16 + col;
    const bool cok = cidx < a.ncols;
    const int32_t per = (a.G + 15) / 16;
    const int32_t g0 = part * per, g1 = min(a.G, g0 + per);
    double s = 0.0;
    // loads at clamped (valid) positions, all in flight before the first add
    const float *pc = a.P + min(cidx, a.ncols - 1);
    for (int32_t gg = g0; gg < g1; gg += 16) {
        float buf[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) buf[i] = pc[(int64_t)min(gg + i, a.G - 1) * a.Cp];
#pragma unroll
        for (int i = 0; i < 16; ++i) s += (cok && gg + i < g1) ? (double)buf[i] : 0.0;
    }
    red[tid] = s;
    __syncthreads();
    if (part == 0) {
        double tot = 0.0;
        for (int p = 0; p < 16; ++p) tot += red[p * 16 + col];
        double q = 0.0, qm = 0.0;
        if (cok) {
            if (cidx < (int64_t)S * T) {
                const uint32_t sc = divu((uint32_t)cidx, a.divT);
                const int32_t t = (int32_t)(cidx - (int64_t)sc * T);
                const double e = hinge64(tot, rk.pcap);
                const float ef = (float)e;
                sv.E[cidx] = ef;
                uint16_t h, md, l;
                split3(ef, h, md, l);
                uint16_t *er = sv.Es + (size_t)t * 3 * a.Sp + sc;
                er[0] = h;
                er[a.Sp] = md;
                er[2 * a.Sp] = l;
                q = e * e;
            } else if (cidx < (int64_t)(S + 1) * T) {
                const int32_t t = (int32_t)(cidx - (int64_t)S * T);
                const double e = hinge64(tot, rk.mcap);
                sv.Em[t] = (float)e;
                qm = e * e;
            } else {
                sv.npv[cidx - (int64_t)(S + 1) * T] = tot;
            }
        }
        rq[0][col] = q;
        rq[1][col] = qm;
    }
    __syncthreads();
    if (tid == 0) {
        double q = 0.0, qm = 0.0;
        for (int i = 0; i < 16; ++i) {
            q += rq[0][i];
            qm += rq[1][i];
        }
        a.pq[blockIdx.x] = q;
        a.pmq[blockIdx.x] = qm;
    }
}

// Scalars: mu, sigma, penalties, J, w_s; zeros in the padding of the E parts.
// One workgroup of 16 waves; sums in a fixed order (thread, wave, waves in
// order).
__global__ void __launch_bounds__(1024) k_relax_fwd_final(DevModel m, RelaxK rk, SavedView sv,
                                                          RedArgs a, double *J_out) {
    __shared__ double part[16][4];
    __shared__ double tot[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t S = m.S, T = m.T;
    constexpr int kNV = MPS_MAX_SCENARIOS / 1024;
    double nv[kNV];
    double sn = 0.0, pp = 0.0, pm = 0.0, pr = 0.0;
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
        const int32_t s = tid + 1024 * k;
        nv[k] = s < S ? sv.npv[s] : 0.0;
    }
    for (int32_t i = tid; i < a.nred; i += 1024) {
        pp += a.pq[i];
        pm += a.pmq[i];
    }
    for (int32_t i = tid; i < a.G; i += 1024) pr += a.prq[i];
#pragma unroll
    for (int k = 0; k < kNV; ++k) sn += nv[k];
    sn = wave_sum_f64(sn);
    pp = wave_sum_f64(pp);
    pm = wave_sum_f64(pm);
    pr = wave_sum_f64(pr);
    if (lane == 0) {
        part[wave][0] = sn;
        part[wave][1] = pp;
        part[wave][2] = pm;
        part[wave][3] = pr;
    }
    __syncthreads();
    if (tid < 4) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += part[w][tid];
        tot[tid] = t;
    }
    __syncthreads();
    const double mu = tot[0] / S;
    double q = 0.0;
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
        const double e = nv[k] - mu;
        if (tid + 1024 * k < S) q += e * e;
    }
    q = wave_sum_f64(q);
    __syncthreads();
    if (lane == 0) part[wave][0] = q;
    __syncthreads();
    double qq = 0.0;
    for (int w = 0; w < 16; ++w) qq += part[w][0];
    const double sigma = sqrt(qq / S);
    const bool degenerate = !(sigma > 1e-12 * fmax(1.0, fabs(mu)));
#pragma unroll
    for (int k = 0; k < kNV; ++k) {
        const int32_t s = tid + 1024 * k;
        if (s < S)
            sv.w[s] = (float)(degenerate ? 1.0 / S : 1.0 / S - rk.lambda * (nv[k] - mu) / (S * sigma));
    }
    const int32_t padn = a.Sp - S;
    if (padn > 0)
        for (int32_t i = tid; i < 3 * T * padn; i += 1024) {
            const int32_t row = i / padn, k = i - row * padn;
            sv.Es[(size_t)row * a.Sp + S + k] = 0;
        }
    if (tid == 0) {
        const double Pp = rk.mu_proc * tot[1] / S;
        const double Pm = rk.mu_mine * tot[2];
        const double Pr = rk.mu_prec * tot[3];
        const double J = mu - rk.lambda * sigma - Pp - Pm - Pr;
        sv.scal[0] = J;
        sv.scal[1] = mu;
        sv.scal[2] = sigma;
        sv.scal[3] = Pp;
        sv.scal[4] = Pm;
        sv.scal[5] = Pr;
        if (J_out) {
            J_out[0] = J;
            J_out[1] = mu;
            J_out[2] = sigma;
            J_out[3] = Pp;
            J_out[4] = Pm;
            J_out[5] = Pr;
        }
    }
}

// ---- backward, per tile of TB blocks ---------------------------------------------
struct BwdArgs {
    const float *x;
    const uint16_t *nmask;
    float *grad;
    const double *dJ;
    int32_t TB, KC, Sp;
    DivU32 divT, divKC8;
};

template <int Q, int MT>
__global__ void __launch_bounds__(kRT, MT <= 2 ? 4 : 2) k_relax_bwd_tile(DevModel m, BwdArgs a, RelaxK rk,
                                                           SavedView sv) {
    extern __shared__ __align__(16) char lds[];
    const int32_t T = m.T, S = m.S, TB = a.TB, KC = a.KC;
    const int64_t N = m.N;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t b0 = (int64_t)blockIdx.x * TB;
    const int32_t nb = (int32_t)min((int64_t)TB, N - b0);
    const int32_t ntt = (T + 15) >> 4;
    // this wave's tiles: one 16-block row tile, period tiles tt0 + twv k
    const int32_t nrt = TB >> 4, twv = 8 / nrt;
    const int32_t rt = wave % nrt, tt0 = wave / nrt;
    const int32_t Kp = a.Sp;                         // scenarios padded to whole words
    const int32_t nrow = S > wave ? (S - wave + 7) >> 3 : 0;

    char *c = lds;
    uint16_t *Esl = (uint16_t *)c;                   // [T+1][3][KC] staged parts of E; row T = 0
    c += al16(6 * (size_t)(T + 1) * KC);
    uint32_t *orl = (uint32_t *)c;                   // [KC/32][TB] ore words
    c += al16(4 * (size_t)(KC / 32) * TB);
    float *gy = (float *)c;                          // [TB][T+1]
    c += al16(4 * (size_t)TB * (T + 1));
    float *up = (float *)c;                          // [8][TB] u_b partials per wave
    c += al16(4 * 8 * (size_t)TB);
    float *tonl = (float *)c;                        // [TB]
    c += al16(4 * (size_t)TB);
    float *dl = (float *)c;                          // [T] d(t)
    c += al16(4 * (size_t)T);
    float *eml = (float *)c;                         // [T] Em[t]
    c += al16(4 * (size_t)T);
    uint32_t *nml = (uint32_t *)c;                   // [TB] precedence-stencil bits
    c += al16(4 * (size_t)TB);
    float *wl = (float *)c;                          // [S] w_s

    f32x4 acc[MT];
#pragma unroll
    for (int k = 0; k < MT; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float u[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) u[q] = 0.0f;
    for (int32_t i = tid; i < 3 * KC; i += kRT) Esl[(size_t)T * 3 * KC + i] = 0;

    // every load of v is issued unconditionally (clamped rows and blocks are
    // never used), so that each wait names exactly the batch it needs
    auto issue = [&](float (&buf)[kRB][Q], int32_t i0) {
#pragma unroll
        for (int r = 0; r < kRB; ++r) {
            const int32_t i = min(i0 + r, max(nrow - 1, 0));
            const int32_t s = min(wave + 8 * i, S - 1);
            const float *row = m.v + (int64_t)s * m.vld + b0;
#pragma unroll
            for (int q = 0; q < Q; ++q) buf[r][q] = ld_off(row, (uint32_t)min(lane + 64 * q, nb - 1));
        }
    };
    auto consume = [&](float (&buf)[kRB][Q], int32_t i0) {
#pragma unroll
        for (int r = 0; r < kRB; ++r) {
            if (i0 + r < nrow) {
                const float w = wl[wave + 8 * (i0 + r)];
#pragma unroll
                for (int q = 0; q < Q; ++q) u[q] = fmaf(w, buf[r][q], u[q]);
            }
        }
    };

    const int32_t rstep = kRT / TB;                  // ore rows staged per pass of the threads
    const int32_t jj = tid & (TB - 1), rq0 = wave / (TB / 64);
    const uint32_t jc = (uint32_t)min(jj, nb - 1);
    const int32_t kc8 = KC / 8;
    // staged operands of the scenarios [kc0, kc0 + KC): parts of E and ore words
    auto stage = [&](int32_t kc0, auto &&after_loads) {
        const int32_t kcn = min(KC, Kp - kc0);
        const int32_t nw = kcn / 32;
        u32x4 er[kStE];
#pragma unroll
        for (int k = 0; k < kStE; ++k) {
            if (k * kRT < 3 * T * kc8) {
                const uint32_t e = min((uint32_t)(tid + k * kRT), (uint32_t)(3 * T * kc8 - 1));
                const uint32_t row = divu(e, a.divKC8);
                const uint32_t q8 = min(e - row * kc8, (uint32_t)(kcn / 8 - 1));
                er[k] = *(const u32x4 *)(sv.Es + kc0 + (row * (uint32_t)Kp + 8 * q8));
            }
        }
        uint32_t orr[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k * rstep < nw) {
                const int32_t r = min(rq0 + k * rstep, nw - 1);
                orr[k] = ld_off(m.ore + (int64_t)(kc0 / 32 + r) * N + b0, jc);
            }
        }
        after_loads();
#pragma unroll
        for (int k = 0; k < kStE; ++k) {
            const uint32_t e = tid + k * kRT;
            if (k * kRT < 3 * T * kc8 && e < (uint32_t)(3 * T * kc8)) {
                const uint32_t row = divu(e, a.divKC8), q8 = e - row * kc8;
                if (q8 < (uint32_t)(kcn / 8)) *(u32x4 *)(Esl + (size_t)row * KC + 8 * q8) = er[k];
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t r = rq0 + k * rstep;
            if (k * rstep < nw && r < nw) orl[r * TB + jj] = jj < nb ? orr[k] : 0u;
        }
    };
    // G[b,t] += sum over the staged scenarios of ore[s,b] E[s,t].  The 0/1
    // fragment of the row tile is built once per word and serves the wave's
    // period tiles; periods past T read the zero row.
    auto contract = [&](int32_t kc0) {
        const int32_t nw = min(KC, Kp - kc0) / 32;
        const int32_t j = 16 * rt + (lane & 15);
        const uint32_t p0 = 8 * (lane >> 4);
        for (int32_t ks = 0; ks < nw; ++ks) {
            const uint32_t w = orl[ks * TB + j];
            u32x4 A;
            A.x = bf16_pair(w, p0 + 0, w, p0 + 1);
            A.y = bf16_pair(w, p0 + 2, w, p0 + 3);
            A.z = bf16_pair(w, p0 + 4, w, p0 + 5);
            A.w = bf16_pair(w, p0 + 6, w, p0 + 7);
#pragma unroll
            for (int k = 0; k < MT; ++k) {
                const int32_t tt = tt0 + twv * k;
                if (tt < ntt) {
                    const int32_t t = min(16 * tt + (lane & 15), T);
                    const uint16_t *eb = Esl + (size_t)t * 3 * KC + 32 * ks + p0;
#pragma unroll
                    for (int sp = 0; sp < 3; ++sp)
                        acc[k] = mfma_bf16(A, *(const u32x4 *)(eb + sp * KC), acc[k]);
                }
            }
        }
    };

    // ---- first pass: the staged operands, the first rows of v, then batch b
    // in flight during the contraction
    const float tv = m.ton32[b0 + min(tid, nb - 1)];
    const uint32_t nmv = a.nmask[b0 + min(tid, nb - 1)];
    const double dv = m.d64[min(tid, T - 1)];
    const float emv = sv.Em[min(tid, T - 1)];
    float va[kRB][Q], vb[kRB][Q];
    stage(0, [&] { issue(va, 0); });
    for (int32_t s = tid; s < S; s += kRT) wl[s] = sv.w[s];
    if (tid < TB) {
        tonl[tid] = tid < nb ? tv : 0.0f;
        nml[tid] = tid < nb ? nmv : 0u;
    }
    if (tid < T) {
        dl[tid] = (float)dv;
        eml[tid] = emv;
    }
    issue(vb, kRB);
    __syncthreads();
    contract(0);
    // ---- u_b = sum_s w_s v[s,b] over this wave's rows
    // software pipeline: one batch is consumed while the other is in flight
    for (int32_t i0 = 0; i0 < nrow; i0 += 2 * kRB) {
        consume(va, i0);
        issue(va, i0 + 2 * kRB);
        consume(vb, i0 + kRB);
        issue(vb, i0 + 3 * kRB);
    }
    // ---- further scenario passes (S above the staged width)
    for (int32_t kc0 = KC; kc0 < Kp; kc0 += KC) {
        __syncthreads();
        stage(kc0, [] {});
        __syncthreads();
        contract(kc0);
    }
    // ---- dJ/dx entries of the tile: x[b,t] and its (up to) ten neighbours
    // are loaded for every entry at clamped (valid) offsets and masked
    // afterwards; the first round is issued here, so that it travels while
    // u_b is reduced
    const float scale = a.dJ ? (float)a.dJ[0] : 1.0f;
    const float cprec = (float)(2.0 * rk.mu_prec);
    const int64_t nxy = (int64_t)m.nx * m.ny;
    const int64_t offs[5] = {0, -1, 1, -(int64_t)m.nx, (int64_t)m.nx};
    const int64_t NT = N * T;
    constexpr int kEB = 5;   // entries per thread in flight
    float xb[kEB], xn[kEB][10];
    auto load_round = [&](int32_t e0) {
#pragma unroll
        for (int u = 0; u < kEB; ++u) {
            const int64_t eg = b0 * T + min(e0 + u * kRT, nb * T - 1);
            xb[u] = a.x[(uint32_t)eg];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int64_t ep = eg + (offs[k] - nxy) * T, es = eg + (offs[k] + nxy) * T;
                xn[u][k] = a.x[(uint32_t)min(max(ep, (int64_t)0), NT - 1)];
                xn[u][5 + k] = a.x[(uint32_t)min(max(es, (int64_t)0), NT - 1)];
            }
        }
    };
    // cprec (pp - ps) of the round's entries: pp over the predecessors a of
    // max(0, x[b,t] - x[a,t]), ps over the successors c of max(0, x[c,t] - x[b,t])
    float pr[kEB];
    auto prec_round = [&](int32_t e0) {
#pragma unroll
        for (int u = 0; u < kEB; ++u) {
            const int32_t e = min(e0 + u * kRT, nb * T - 1);
            const uint32_t nm = nml[divu((uint32_t)e, a.divT)];
            float pp = 0.0f, ps = 0.0f;
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if ((nm >> k) & 1u) pp += fmaxf(xb[u] - xn[u][k], 0.0f);
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if ((nm >> (5 + k)) & 1u) ps += fmaxf(xn[u][5 + k] - xb[u], 0.0f);
            pr[u] = cprec * (pp - ps);
        }
    };
    load_round(tid);
    // ---- u_b over the waves, in wave order
#pragma unroll
    for (int q = 0; q < Q; ++q) up[wave * TB + lane + 64 * q] = u[q];
    __syncthreads();
    if (tid < TB) {
        float ub = up[tid];
        for (int w = 1; w < 8; ++w) ub += up[w * TB + tid];
        up[tid] = ub;
        gy[tid * (T + 1) + T] = 0.0f;
    }
    __syncthreads();
    prec_round(tid);
    // ---- dJ/dy = d(t) u_b - ton_b (cproc G + cmine Em[t]) from the accumulators
    const float cproc = (float)(2.0 * rk.mu_proc / S), cmine = (float)(2.0 * rk.mu_mine);
#pragma unroll
    for (int k = 0; k < MT; ++k) {
        const int32_t tt = tt0 + twv * k;
        const int32_t t = 16 * tt + (lane & 15);
        if (tt < ntt && t < T) {
            const int32_t j0 = 16 * rt + 4 * (lane >> 4);
            const float dt = dl[t], me = cmine * eml[t];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                gy[(j0 + q) * (T + 1) + t] = dt * up[j0 + q] - tonl[j0 + q] * fmaf(cproc, acc[k][q], me);
        }
    }
    __syncthreads();
    // ---- dJ/dx = dJ/dy[t] - dJ/dy[t+1] with the precedence terms; coalesced
    // writes of the tile
    for (int32_t e0 = tid; e0 < nb * T; e0 += kEB * kRT) {
        if (e0 != tid) {
            load_round(e0);
            prec_round(e0);
        }
#pragma unroll
        for (int u = 0; u < kEB; ++u) {
            const int32_t e = e0 + u * kRT;
            if (e < nb * T) {
                const int32_t j = (int32_t)divu((uint32_t)e, a.divT), t = e - j * T;
                const float g = gy[j * (T + 1) + t] - gy[j * (T + 1) + t + 1] - pr[u];
                a.grad[b0 * T + e] = scale * g;
            }
        }
    }
}

template <int SL, int TT>
static void go_fwd(const DevModel &m, const FwdGeom &g, const FwdArgs &a, hipStream_t st) {
    if (g.nsub > 1)
        hipLaunchKernelGGL((k_relax_fwd_chunk<SL, TT, true>), dim3(g.G, g.OG), dim3(kRT), g.lds, st,
                           m, a);
    else
        hipLaunchKernelGGL((k_relax_fwd_chunk<SL, TT, false>), dim3(g.G, g.OG), dim3(kRT), g.lds,
                           st, m, a);
}

// Precedence penalty under explicit lists, for the blocks of chunk g:
// sum over b, a in Pred(b), t of max(0, x[b,t] - x[a,t])^2, added to the
// chunk's precedence sum (the stencil part is 0 for such models).
__global__ void __launch_bounds__(256) k_relax_prec_fwd_csr(DevModel m, const float *x,
                                                            double *prq, int32_t G) {
    __shared__ double red[4];
    const int64_t per = (m.N + G - 1) / G;
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(m.N, b0 + per);
    const int32_t T = m.T;
    double acc = 0.0;
    for (int64_t i = b0 * T + threadIdx.x; i < b1 * T; i += 256) {
        const int64_t b = i / T;
        const int32_t t = (int32_t)(i - b * T);
        const float xb = x[i];
        for (int32_t j = m.pred_ptr[b]; j < m.pred_ptr[b + 1]; ++j) {
            const float e = xb - x[(int64_t)m.pred_idx[j] * T + t];
            if (e > 0.0f) acc += (double)e * (double)e;
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) prq[blockIdx.x] += ((red[0] + red[1]) + red[2]) + red[3];
}

// Its derivative, added to grad (scaled by dJ): -2 mu_prec (sum over
// predecessors a of max(0, x[b,t] - x[a,t]) - sum over successors c of
// max(0, x[c,t] - x[b,t])).
__global__ void __launch_bounds__(256) k_relax_prec_bwd_csr(DevModel m, const float *x,
                                                            const double *dJ, double mu_prec,
                                                            float *grad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int32_t T = m.T;
    if (i >= m.N * T) return;
    const int64_t b = i / T;
    const int32_t t = (int32_t)(i - b * T);
    const float xb = x[i];
    float pp = 0.0f, ps = 0.0f;
    for (int32_t j = m.pred_ptr[b]; j < m.pred_ptr[b + 1]; ++j)
        pp += fmaxf(xb - x[(int64_t)m.pred_idx[j] * T + t], 0.0f);
    for (int32_t j = m.succ_ptr[b]; j < m.succ_ptr[b + 1]; ++j)
        ps += fmaxf(x[(int64_t)m.succ_idx[j] * T + t] - xb, 0.0f);
    const float scale = dJ ? (float)dJ[0] : 1.0f;
    grad[i] -= scale * (float)(2.0 * mu_prec) * (pp - ps);
}

hipError_t launch_relaxed_fwd(const DevModel &m, const float *x, const mps_relax_params &rp,
                              double *J_out, void *saved, void *ws, hipStream_t st) {
    const RelaxK rk{m.lambda, rp.mu_proc, rp.mu_mine, rp.mu_prec, m.pcap, m.mcap};
    const FwdGeom g = fwd_geom(m);
    const RelaxWs r = relax_ws(ws, m, g);
    const SavedView sv = saved_view(saved, m.S, m.T);
    const FwdArgs fa{x, r.P, r.prq, r.nmask, g.Cp, g.CB, g.nsub, g.SG, g.ntt,
                     make_div((uint32_t)m.T)};
    switch (g.TT) {
        case 1: go_fwd<8, 1>(m, g, fa, st); break;
        case 2: go_fwd<4, 2>(m, g, fa, st); break;
        case 4: go_fwd<2, 4>(m, g, fa, st); break;
        default: go_fwd<1, 8>(m, g, fa, st); break;
    }
    if (m.csr)
        hipLaunchKernelGGL(k_relax_prec_fwd_csr, dim3((unsigned)g.G), dim3(256), 0, st, m, x,
                           r.prq, g.G);
    const RedArgs ra{r.P, g.Cp, g.ncols, g.G, g.nred, pad_scen(m.S), r.pq, r.pmq, r.prq,
                     make_div((uint32_t)m.T)};
    hipLaunchKernelGGL(k_relax_fwd_reduce, dim3((unsigned)g.nred), dim3(256), 0, st, m, ra, rk,
                       sv);
    hipLaunchKernelGGL(k_relax_fwd_final, dim3(1), dim3(1024), 0, st, m, rk, sv, ra, J_out);
    return hipGetLastError();
}

template <int Q, int MT>
static void go_bwd(const DevModel &m, const BwdGeom &g, const BwdArgs &a, const RelaxK &rk,
                   const SavedView &sv, hipStream_t st) {
    const unsigned tiles = (unsigned)((m.N + g.TB - 1) / g.TB);
    hipLaunchKernelGGL((k_relax_bwd_tile<Q, MT>), dim3(tiles), dim3(kRT), g.lds, st, m, a, rk, sv);
}

hipError_t launch_relaxed_bwd(const DevModel &m, const float *x, const mps_relax_params &rp,
                              const void *saved, const double *dJ, float *grad, void *ws,
                              hipStream_t st) {
    const RelaxK rk{m.lambda, rp.mu_proc, rp.mu_mine, rp.mu_prec, m.pcap, m.mcap};
    const FwdGeom fg = fwd_geom(m);
    const RelaxWs r = relax_ws(ws, m, fg);
    const BwdGeom g = bwd_geom(m);
    const SavedView sv = saved_view((void *)saved, m.S, m.T);
    const BwdArgs a{x,        r.nmask, grad, dJ, g.TB, g.KC, pad_scen(m.S), make_div((uint32_t)m.T),
                    make_div((uint32_t)(g.KC / 8))};
    if (g.Q == 2)
        g.MT == 2 ? go_bwd<2, 2>(m, g, a, rk, sv, st)
                  : (g.MT == 4 ? go_bwd<2, 4>(m, g, a, rk, sv, st) : go_bwd<2, 8>(m, g, a, rk, sv, st));
    else
        g.MT == 2 ? go_bwd<1, 2>(m, g, a, rk, sv, st)
                  : (g.MT == 4 ? go_bwd<1, 4>(m, g, a, rk, sv, st) : go_bwd<1, 8>(m, g, a, rk, sv, st));
    if (m.csr)
        hipLaunchKernelGGL(k_relax_prec_bwd_csr, dim3((unsigned)((m.N * m.T + 255) / 256)),
                           dim3(256), 0, st, m, x, dJ, rp.mu_prec, grad);
    return hipGetLastError();
}

// x(p)[b,t] = [t >= p_b]: the integer point of the current schedule.
__global__ void k_integer_x(DevModel m, float *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.N * m.T) return;
    const int64_t b = i / m.T;
    const int32_t t = (int32_t)(i - b * m.T);
    x[i] = t >= m.p[b] ? 1.0f : 0.0f;
}

hipError_t launch_integer_x(const DevModel &m, float *x, hipStream_t st) {
    const int64_t n = m.N * m.T;
    hipLaunchKernelGGL(k_integer_x, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m, x);
    return hipGetLastError();
}

}  // namespace mps
