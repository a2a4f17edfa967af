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
// Forward: each workgroup takes a chunk of blocks; its threads own scenarios
// (the per-period tonnages are an outer-product accumulation over blocks);
// chunk partials are reduced in a fixed order.  Backward: 64-block tiles,
// threads own blocks, the four waves split the scenarios as in evaluation.
#include <float.h>
#include <math.h>

#include "internal.h"

namespace mps {

constexpr int kTch = 32;         // periods per register chunk

__host__ __device__ static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// ---- saved-state layout ------------------------------------------------------
struct SavedView {
    double *scal;   // [8]: J, mu, sigma, Pproc, Pmine, Pprec, spare, spare
    double *npv;    // [S]
    float *w;       // [S]
    float *E;       // [S][T]
    float *Em;      // [T]
};

__host__ __device__ static inline size_t saved_bytes(int32_t S, int32_t T) {
    return al256(8 * 8) + al256(8 * (size_t)S) + al256(4 * (size_t)S) +
           al256(4 * (size_t)S * T) + al256(4 * (size_t)T);
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
    return v;
}

size_t relaxed_saved_bytes(const DevModel &m) { return saved_bytes(m.S, m.T); }

// LDS of one forward workgroup for a chunk of CB blocks.
static size_t fwd_lds_bytes(const DevModel &m, int CB) {
    return sizeof(float) * ((size_t)CB * m.T + CB) + sizeof(uint32_t) * (size_t)m.W * CB +
           16 + 256 * sizeof(double);
}

// Blocks per forward workgroup: 256, halved until the chunk fits 64 KB of LDS.
static int fwd_chunk(const DevModel &m) {
    int CB = 256;
    while (CB > 8 && fwd_lds_bytes(m, CB) > 65536) CB >>= 1;
    return CB;
}

static int fwd_groups(const DevModel &m) {
    const int CB = fwd_chunk(m);
    return (int)((m.N + CB - 1) / CB);
}

struct FwdWs {
    float *npv, *Ot, *Mt;
    double *prec;
    double *acc;   // [S*T + T + 1] squared excesses and the precedence sum
};

// chunk partials: [G][S] npv, [G][S][T] Ot, [G][T] Mt, [G] precedence
size_t relaxed_ws_bytes(const DevModel &m) {
    size_t G = (size_t)fwd_groups(m);
    return al256(4 * G * m.S) + al256(4 * G * m.S * m.T) + al256(4 * G * m.T) + al256(8 * G) +
           al256(8 * ((size_t)m.S * m.T + m.T + 1));
}

static FwdWs fwd_ws(void *ws, const DevModel &m) {
    size_t G = (size_t)fwd_groups(m);
    char *c = (char *)ws;
    FwdWs f;
    f.npv = (float *)c;
    c += al256(4 * G * m.S);
    f.Ot = (float *)c;
    c += al256(4 * G * m.S * m.T);
    f.Mt = (float *)c;
    c += al256(4 * G * m.T);
    f.prec = (double *)c;
    c += al256(8 * G);
    f.acc = (double *)c;
    return f;
}

struct RelaxK {
    double lambda, mu_proc, mu_mine, mu_prec, pcap, mcap;
};

// ---- forward, per chunk of CB blocks ---------------------------------------------
__global__ void __launch_bounds__(256) k_relax_fwd_chunk(DevModel m, const float *x, RelaxK rk,
                                                         FwdWs ws, int CB) {
    extern __shared__ __align__(16) char lds[];
    const int32_t T = m.T, S = m.S, W = m.W;
    const int tid = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * CB;
    const int32_t nb = (int32_t)min((int64_t)CB, m.N - b0);
    double *red = (double *)lds;                               // [256]
    float *Y = (float *)(red + 256);                           // [CB][T] ton * y
    float *Dl = Y + (size_t)CB * T;                            // [CB]
    uint32_t *orel = (uint32_t *)(Dl + CB);                    // [W][CB]

    for (int32_t i = tid; i < CB * T; i += 256) {
        const int32_t j = i / T, t = i - j * T;
        float yv = 0.0f;
        if (j < nb) {
            const int64_t b = b0 + j;
            const float xc = x[b * T + t];
            const float xp = t > 0 ? x[b * T + t - 1] : 0.0f;
            yv = m.ton32[b] * (xc - xp);
        }
        Y[i] = yv;
    }
    for (int32_t i = tid; i < W * CB; i += 256) {
        const int32_t w = i / CB, j = i - w * CB;
        orel[i] = j < nb ? m.ore[(int64_t)w * m.N + b0 + j] : 0u;
    }
    // D_b = sum_t d(t) y[b,t], and the precedence penalty of the chunk
    double pr = 0.0;
    for (int32_t j = tid; j < CB; j += 256) {
        float dsum = 0.0f;
        if (j < nb) {
            const int64_t b = b0 + j;
            for (int32_t t = 0; t < T; ++t) {
                const float xc = x[b * T + t];
                const float xp = t > 0 ? x[b * T + t - 1] : 0.0f;
                dsum = fmaf((float)m.d64[t], xc - xp, dsum);
            }
            int32_t xx, yy, zz;
            grid_coords(m, (int32_t)b, xx, yy, zz);
            if (zz > 0) {
                const int32_t nxy = m.nx * m.ny;
                int64_t pa[5];
                int np = 0;
                pa[np++] = b - nxy;
                if (xx > 0) pa[np++] = b - nxy - 1;
                if (xx + 1 < m.nx) pa[np++] = b - nxy + 1;
                if (yy > 0) pa[np++] = b - nxy - m.nx;
                if (yy + 1 < m.ny) pa[np++] = b - nxy + m.nx;
                for (int k = 0; k < np; ++k)
                    for (int32_t t = 0; t < T; ++t) {
                        const float e = x[b * T + t] - x[pa[k] * T + t];
                        if (e > 0.0f) pr += (double)e * (double)e;
                    }
            }
        }
        Dl[j] = dsum;
    }
    red[tid] = pr;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) ws.prec[blockIdx.x] = red[0];
    // period tonnage totals of the chunk
    for (int32_t t = tid; t < T; t += 256) {
        float s = 0.0f;
        for (int32_t j = 0; j < nb; ++j) s += Y[j * T + t];
        ws.Mt[(size_t)blockIdx.x * T + t] = s;
    }
    // threads own scenarios: NPV and per-period ore tonnage partials
    for (int32_t s = tid; s < S; s += 256) {
        const uint32_t *orow = orel + (size_t)(s >> 5) * CB;
        const uint32_t bit = s & 31;
        const float *vrow = m.v + (int64_t)s * m.N + b0;
        for (int32_t tc = 0; tc < T; tc += kTch) {
            float acc[kTch];
#pragma unroll
            for (int k = 0; k < kTch; ++k) acc[k] = 0.0f;
            float an = 0.0f;
            for (int32_t j = 0; j < nb; ++j) {
                const float o = (float)((orow[j] >> bit) & 1u);
                const float *yr = Y + j * T + tc;
#pragma unroll
                for (int k = 0; k < kTch; ++k)
                    if (tc + k < T) acc[k] = fmaf(o, yr[k], acc[k]);
                if (tc == 0) an = fmaf(vrow[j], Dl[j], an);
            }
            float *op = ws.Ot + ((size_t)blockIdx.x * S + s) * T;
#pragma unroll
            for (int k = 0; k < kTch; ++k)
                if (tc + k < T) op[tc + k] = acc[k];
            if (tc == 0) ws.npv[(size_t)blockIdx.x * S + s] = an;
        }
    }
}

// Sum chunk partials in chunk order: NPV_s, E[s][t] = max(0, Ot - Pcap),
// Em[t] and the penalty sums (as doubles in scal[]).
__global__ void k_relax_fwd_reduce(DevModel m, FwdWs ws, int G, RelaxK rk, SavedView sv) {
    double *acc_out = ws.acc;
    const int32_t S = m.S, T = m.T;
    const int64_t n = (int64_t)S * T + S + T + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        if (i < (int64_t)S * T) {
            const int32_t sc = (int32_t)(i / T), t = (int32_t)(i % T);
            for (int g = 0; g < G; ++g) s += (double)ws.Ot[((size_t)g * S + sc) * T + t];
            const double e = hinge64(s, rk.pcap);
            sv.E[i] = (float)e;
            acc_out[i] = e * e;
        } else if (i < (int64_t)S * T + S) {
            const int32_t sc = (int32_t)(i - (int64_t)S * T);
            for (int g = 0; g < G; ++g) s += (double)ws.npv[(size_t)g * S + sc];
            sv.npv[sc] = s;
        } else if (i < (int64_t)S * T + S + T) {
            const int32_t t = (int32_t)(i - (int64_t)S * T - S);
            for (int g = 0; g < G; ++g) s += (double)ws.Mt[(size_t)g * T + t];
            const double e = hinge64(s, rk.mcap);
            sv.Em[t] = (float)e;
            acc_out[(int64_t)S * T + t] = e * e;
        } else {
            for (int g = 0; g < G; ++g) s += ws.prec[g];
            acc_out[(int64_t)S * T + T] = s;
        }
    }
}

__device__ double bsum256(double x, double *red) {
    const int tid = threadIdx.x;
    __syncthreads();
    red[tid] = x;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Scalars: mu, sigma, penalties, J, w_s.  One workgroup of 256 threads.
__global__ void __launch_bounds__(256) k_relax_fwd_final(DevModel m, RelaxK rk, SavedView sv,
                                                         const double *acc, double *J_out) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int32_t S = m.S, T = m.T;
    double a = 0.0;
    for (int32_t s = tid; s < S; s += 256) a += sv.npv[s];
    const double mu = bsum256(a, red) / S;
    double q = 0.0;
    for (int32_t s = tid; s < S; s += 256) {
        const double e = sv.npv[s] - mu;
        q += e * e;
    }
    const double sigma = sqrt(bsum256(q, red) / S);
    double pp = 0.0;
    for (int64_t i = tid; i < (int64_t)S * T; i += 256) pp += acc[i];
    pp = bsum256(pp, red);
    const bool degenerate = !(sigma > 1e-12 * fmax(1.0, fabs(mu)));
    for (int32_t s = tid; s < S; s += 256)
        sv.w[s] = (float)(degenerate ? 1.0 / S
                                     : 1.0 / S - rk.lambda * (sv.npv[s] - mu) / (S * sigma));
    if (tid == 0) {
        double pm = 0.0;
        for (int32_t t = 0; t < T; ++t) pm += acc[(int64_t)S * T + t];
        const double Pp = rk.mu_proc * pp / S;
        const double Pm = rk.mu_mine * pm;
        const double Pr = rk.mu_prec * acc[(int64_t)S * T + T];
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

// ---- backward, per 64-block tile -------------------------------------------------
__global__ void __launch_bounds__(256) k_relax_bwd_tile(DevModel m, const float *x, RelaxK rk,
                                                        SavedView sv, const double *dJ,
                                                        float *grad) {
    extern __shared__ __align__(16) char lds[];
    const int32_t T = m.T, S = m.S, W = m.W;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t b0 = (int64_t)blockIdx.x * 64;
    const int64_t b = b0 + lane;
    const bool valid = b < m.N;
    float *upart = (float *)lds;                    // [4][64]
    float *gpart = upart + 256;                     // [4][64][kTch]
    float *gy = gpart + 4 * 64 * kTch;              // [64][T+1]
    uint32_t *orel = (uint32_t *)(gy + 64 * (T + 1));  // [W][64]

    for (int32_t w = wave; w < W; w += 4) orel[w * 64 + lane] = valid ? m.ore[(int64_t)w * m.N + b] : 0u;
    // u_b partial over this wave's quarter of the scenarios
    const int32_t Sq = (S + 3) >> 2;
    const int32_t s0 = wave * Sq, s1 = min(S, s0 + Sq);
    float u = 0.0f;
    if (valid)
        for (int32_t s = s0; s < s1; ++s) u = fmaf(sv.w[s], m.v[(int64_t)s * m.N + b], u);
    upart[wave * 64 + lane] = u;
    __syncthreads();
    const float scale = dJ ? (float)dJ[0] : 1.0f;
    const float ub = ((upart[lane] + upart[64 + lane]) + upart[128 + lane]) + upart[192 + lane];
    const float ton = valid ? m.ton32[b] : 0.0f;
    const float cproc = (float)(2.0 * rk.mu_proc / S), cmine = (float)(2.0 * rk.mu_mine);
    for (int32_t tc = 0; tc < T; tc += kTch) {
        float acc[kTch];
#pragma unroll
        for (int k = 0; k < kTch; ++k) acc[k] = 0.0f;
        for (int32_t s = s0; s < s1; ++s) {
            const float o = (float)((orel[(s >> 5) * 64 + lane] >> (s & 31)) & 1u);
            const float *er = sv.E + (int64_t)s * T + tc;
#pragma unroll
            for (int k = 0; k < kTch; ++k)
                if (tc + k < T) acc[k] = fmaf(o, er[k], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < kTch; ++k) gpart[(wave * 64 + lane) * kTch + k] = acc[k];
        __syncthreads();
        // dJ/dy for this period chunk (wave 0 lanes own the blocks)
        for (int32_t i = tid; i < 64 * kTch; i += 256) {
            const int j = i / kTch, k = i - j * kTch;
            const int32_t t = tc + k;
            if (t >= T) continue;
            const float G = ((gpart[(0 * 64 + j) * kTch + k] + gpart[(1 * 64 + j) * kTch + k]) +
                             gpart[(2 * 64 + j) * kTch + k]) +
                            gpart[(3 * 64 + j) * kTch + k];
            // ub and ton belong to lane j: read them through LDS-free recompute
            gy[j * (T + 1) + t] = G;   // stash G; combined below by the owning lane
        }
        __syncthreads();
    }
    // the owning lane (wave 0) turns G into dJ/dy for its block
    if (wave == 0) {
        for (int32_t t = 0; t < T; ++t) {
            const float G = gy[lane * (T + 1) + t];
            gy[lane * (T + 1) + t] =
                (float)m.d64[t] * ub - ton * fmaf(cproc, G, cmine * sv.Em[t]);
        }
        gy[lane * (T + 1) + T] = 0.0f;
    }
    __syncthreads();
    // dJ/dx with the precedence terms; coalesced writes of the tile
    const int64_t nb = min((int64_t)64, m.N - b0);
    const float cprec = (float)(2.0 * rk.mu_prec);
    for (int64_t i = tid; i < nb * T; i += 256) {
        const int32_t j = (int32_t)(i / T), t = (int32_t)(i - (int64_t)j * T);
        const int64_t bb = b0 + j;
        float g = gy[j * (T + 1) + t] - gy[j * (T + 1) + t + 1];
        int32_t xx, yy, zz;
        grid_coords(m, (int32_t)bb, xx, yy, zz);
        const float xb = x[bb * T + t];
        const int32_t nxy = m.nx * m.ny;
        float pp = 0.0f, ps = 0.0f;
        if (zz > 0) {
            const int64_t a = bb - nxy;
            pp += fmaxf(xb - x[a * T + t], 0.0f);
            if (xx > 0) pp += fmaxf(xb - x[(a - 1) * T + t], 0.0f);
            if (xx + 1 < m.nx) pp += fmaxf(xb - x[(a + 1) * T + t], 0.0f);
            if (yy > 0) pp += fmaxf(xb - x[(a - m.nx) * T + t], 0.0f);
            if (yy + 1 < m.ny) pp += fmaxf(xb - x[(a + m.nx) * T + t], 0.0f);
        }
        if (zz + 1 < m.nz) {
            const int64_t c = bb + nxy;
            ps += fmaxf(x[c * T + t] - xb, 0.0f);
            if (xx > 0) ps += fmaxf(x[(c - 1) * T + t] - xb, 0.0f);
            if (xx + 1 < m.nx) ps += fmaxf(x[(c + 1) * T + t] - xb, 0.0f);
            if (yy > 0) ps += fmaxf(x[(c - m.nx) * T + t] - xb, 0.0f);
            if (yy + 1 < m.ny) ps += fmaxf(x[(c + m.nx) * T + t] - xb, 0.0f);
        }
        g -= cprec * (pp - ps);
        grad[b0 * T + i] = scale * g;
    }
}

hipError_t launch_relaxed_fwd(const DevModel &m, const float *x, const mps_relax_params &rp,
                              double *J_out, void *saved, void *ws, hipStream_t st) {
    RelaxK rk{m.lambda, rp.mu_proc, rp.mu_mine, rp.mu_prec, m.pcap, m.mcap};
    const int CB = fwd_chunk(m);
    const int G = fwd_groups(m);
    FwdWs f = fwd_ws(ws, m);
    SavedView sv = saved_view(saved, m.S, m.T);
    hipLaunchKernelGGL(k_relax_fwd_chunk, dim3(G), dim3(256), fwd_lds_bytes(m, CB), st, m, x, rk,
                       f, CB);
    const int64_t n = (int64_t)m.S * m.T + m.S + m.T + 1;
    hipLaunchKernelGGL(k_relax_fwd_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m,
                       f, G, rk, sv);
    hipLaunchKernelGGL(k_relax_fwd_final, dim3(1), dim3(256), 0, st, m, rk, sv, f.acc, J_out);
    return hipGetLastError();
}

hipError_t launch_relaxed_bwd(const DevModel &m, const float *x, const mps_relax_params &rp,
                              const void *saved, const double *dJ, float *grad, hipStream_t st) {
    RelaxK rk{m.lambda, rp.mu_proc, rp.mu_mine, rp.mu_prec, m.pcap, m.mcap};
    SavedView sv = saved_view((void *)saved, m.S, m.T);
    size_t lds = sizeof(float) * (256 + 4 * 64 * kTch + 64 * (m.T + 1)) +
                 sizeof(uint32_t) * 64 * m.W;
    const unsigned tiles = (unsigned)((m.N + 63) / 64);
    hipLaunchKernelGGL(k_relax_bwd_tile, dim3(tiles), dim3(256), lds, st, m, x, rk, sv, dJ, grad);
    return hipGetLastError();
}

// ---- gradient ranking ---------------------------------------------------------------
// gain(b,t') = Gc[b,p_b] - Gc[b,t'], Gc[b,t] = sum_{u<t} dJ/dx[b,u] (FP64 prefix
// sums): the first-order change of J for moving b from p_b to t'.  No-op moves
// get flag 0 so that the top-k (require 1) skips them.
__global__ void k_rank_gains(DevModel m, const float *grad, float *gain, uint8_t *fl) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m.N) return;
    const int32_t T = m.T, D = T + 1;
    const int32_t pb = m.p[b];
    double gpb = 0.0;
    {
        double run = 0.0;
        for (int32_t t = 0; t < D; ++t) {
            if (t == pb) gpb = run;
            if (t < T) run += (double)grad[b * T + t];
        }
    }
    // only moves that keep the schedule precedence-feasible (Eq. 15) rank:
    // the repair could never apply the others
    int32_t lo, hi;
    prec_window(m, m.p, (int32_t)b, lo, hi);
    double run = 0.0;
    for (int32_t t = 0; t < D; ++t) {
        gain[b * D + t] = (float)(gpb - run);
        fl[b * D + t] = (t != pb && lo <= t && t <= hi) ? 1 : 0;
        if (t < T) run += (double)grad[b * T + t];
    }
}

__global__ void k_rank_decode(int32_t D, const int64_t *idx, int32_t k, int32_t *blk, int8_t *per) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    const int64_t id = idx[i];
    blk[i] = id >= 0 ? (int32_t)(id / D) : -1;
    per[i] = id >= 0 ? (int8_t)(id % D) : (int8_t)-1;
}

size_t rank_ws_bytes(const DevModel &m, int32_t k) {
    const int64_t n = m.N * (m.T + 1);
    return al256(4 * (size_t)n) + al256((size_t)n) + al256(8 * (size_t)k) + topk_ws_bytes(n, k);
}

hipError_t launch_rank(const DevModel &m, const float *grad, int32_t k, int32_t *blk, int8_t *per,
                       float *gain_out, int32_t *count, void *ws, hipStream_t st) {
    const int64_t n = m.N * (m.T + 1);
    char *c = (char *)ws;
    float *gain = (float *)c;
    c += al256(4 * (size_t)n);
    uint8_t *fl = (uint8_t *)c;
    c += al256((size_t)n);
    int64_t *idx = (int64_t *)c;
    c += al256(8 * (size_t)k);
    hipLaunchKernelGGL(k_rank_gains, dim3((unsigned)((m.N + 255) / 256)), dim3(256), 0, st, m,
                       grad, gain, fl);
    hipError_t e = launch_topk(gain, fl, n, k, 1, 0, idx, gain_out, count, c, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_decode, dim3((k + 255) / 256), dim3(256), 0, st, m.T + 1, idx, k,
                       blk, per);
    return hipGetLastError();
}

}  // namespace mps

namespace mps {

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
