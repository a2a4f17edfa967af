// state.hip -- per-block statistics, schedule state and penalty tables.
//
// State of a schedule p (Sec. 5, Eq. 14 and 16):
//   N_s = sum_b v[s][b] d(p_b)           (FP64)
//   O[t][s] = sum_{b: p_b = t} ton_b ore[s][b],  M[t] = sum_{b: p_b=t} ton_b
// Every reduction has a fixed order (per-thread strided partial sums, then a
// fixed tree), so results are bit-reproducible run to run.
#include "internal.h"

namespace mps {

// ---- per-block mean and variance over scenarios (two-pass, FP64) ----------
__global__ void k_block_stats(DevModel m, float *mb32, float *Vb32, double *mb64,
                              double *Vb64) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m.N) return;
    double s1 = 0.0;
    for (int32_t s = 0; s < m.S; ++s) s1 += (double)m.v[(int64_t)s * m.vld + b];
    double mu = s1 / m.S;
    double s2 = 0.0;
    for (int32_t s = 0; s < m.S; ++s) {
        double e = (double)m.v[(int64_t)s * m.vld + b] - mu;
        s2 += e * e;
    }
    double var = s2 / m.S;
    mb64[b] = mu;
    Vb64[b] = var;
    mb32[b] = (float)mu;
    Vb32[b] = (float)var;
}

hipError_t launch_block_stats(const DevModel &m, float *mb32, float *Vb32,
                              double *mb64, double *Vb64, hipStream_t st) {
    int64_t grid = (m.N + 255) / 256;
    hipLaunchKernelGGL(k_block_stats, dim3((unsigned)grid), dim3(256), 0, st, m,
                       mb32, Vb32, mb64, Vb64);
    return hipGetLastError();
}

// ---- schedule state --------------------------------------------------------
// Copy p into the model, clamping values outside 0..T to T (never mined).
__global__ void k_copy_schedule(DevModel m, const int8_t *p_in) {
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m.N) return;
    int32_t t = p_in[b];
    m.p[b] = (int8_t)((t < 0 || t > m.T) ? m.T : t);
}

// Partial sums over one chunk of blocks.  Row r < S: N_s and O[.][s] for
// scenario s = r; row r == S: M[.], precedence violations and clamped
// entries.  64 threads; each keeps private per-period accumulators in LDS.
// Loads of eight blocks are issued before their accumulations so that the
// loop is not bound by memory latency.
// partial layout: [chunk][S+1][T+1]  (entry T of a scenario row holds N_s,
// entry T of the last row the violation count).
constexpr int kStU = 8;

__global__ void __launch_bounds__(64) k_state_partial(DevModel m, const int8_t *p_in,
                                                      double *partial, int chunks) {
    extern __shared__ double acc[];   // [T][64], then d[T+1]
    const int tid = threadIdx.x;
    const int ch = blockIdx.x;
    const int r = blockIdx.y;
    const int32_t T = m.T;
    double *dl = acc + (size_t)T * 64;
    for (int t = 0; t < T; ++t) acc[t * 64 + tid] = 0.0;
    // scenario rows discount with d(t) sigma(s,t) under a value multiplier
    const double *drow = (m.wmult && r < m.S) ? m.wmult + (size_t)r * (T + 1) : m.d64;
    for (int t = tid; t <= T; t += 64) dl[t] = drow[t];
    __syncthreads();
    const int64_t per = (m.N + chunks - 1) / chunks;
    const int64_t b0 = (int64_t)ch * per, b1 = min(m.N, b0 + per);
    double nacc = 0.0;
    if (r < m.S) {
        const int32_t s = r;
        const float *vrow = m.v + (int64_t)s * m.vld;
        const uint32_t *orow = m.ore + (int64_t)(s >> 5) * m.N;
        const uint32_t bit = 1u << (s & 31);
        for (int64_t bb = b0 + tid; bb < b1; bb += 64 * kStU) {
            int32_t tv[kStU];
            float vv[kStU];
            uint32_t ov[kStU];
            double tn[kStU];
#pragma unroll
            for (int u = 0; u < kStU; ++u) {
                const int64_t b = min(bb + 64 * u, b1 - 1);
                tv[u] = m.p[b];
                vv[u] = vrow[b];
                ov[u] = orow[b];
                tn[u] = m.ton64[b];
            }
#pragma unroll
            for (int u = 0; u < kStU; ++u) {
                if (bb + 64 * u >= b1) break;
                const int32_t t = tv[u];
                nacc += (double)vv[u] * dl[t];
                if (t < T && (ov[u] & bit)) acc[t * 64 + tid] += tn[u];
            }
        }
    } else {
        const int32_t nxy = m.nx * m.ny;
        for (int64_t b = b0 + tid; b < b1; b += 64) {
            const int32_t t0 = p_in[b];
            const bool bad = (t0 < 0 || t0 > T);
            const int32_t t = m.p[b];
            if (t < T) acc[t * 64 + tid] += m.ton64[b];
            // predecessor pairs with p[a] > p[b]
            if (m.csr) {
                double nv = bad ? 1.0 : 0.0;
                for (int32_t j = m.pred_ptr[b]; j < m.pred_ptr[b + 1]; ++j)
                    if (m.p[m.pred_idx[j]] > t) nv += 1.0;
                nacc += nv;
                continue;
            }
            int32_t x, y, z;
            grid_coords(m, (int32_t)b, x, y, z);
            const int64_t a = b - nxy;
            const int64_t ia[5] = {a, a - 1, a + 1, a - m.nx, a + m.nx};
            const bool va[5] = {z > 0, z > 0 && x > 0, z > 0 && x + 1 < m.nx, z > 0 && y > 0,
                                z > 0 && y + 1 < m.ny};
            double nv = bad ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int32_t pa = m.p[va[k] ? ia[k] : b];
                if (va[k] && pa > t) nv += 1.0;
            }
            nacc += nv;
        }
    }
    __syncthreads();
    double *out = partial + ((int64_t)ch * (m.S + 1) + r) * (T + 1);
    for (int t = tid; t < T; t += 64) {
        double sum = 0.0;
        for (int j = 0; j < 64; ++j) sum += acc[t * 64 + j];
        out[t] = sum;
    }
    // fixed-order tree over the 64 lanes for the scalar accumulator
    __syncthreads();
    acc[tid] = nacc;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (tid < w) acc[tid] += acc[tid + w];
        __syncthreads();
    }
    if (tid == 0) out[T] = acc[0];
}

// Sum the chunk partials in chunk order into N_s, O, M and the counts.
__global__ void k_state_finish(DevModel m, const double *partial, int chunks) {
    const int32_t S = m.S, T = m.T;
    int64_t n = (int64_t)(S + 1) * (T + 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * n + i];
        int32_t r = (int32_t)(i / (T + 1)), t = (int32_t)(i % (T + 1));
        if (r < S) {
            if (t < T) m.O[(int64_t)t * S + r] = s;
            else m.Ns[r] = s;
        } else {
            if (t < T) m.M[t] = s;
            else m.sc->n_prec_viol = s;
        }
    }
}

hipError_t launch_set_schedule(const DevModel &m, const int8_t *p_in,
                               double *partial, int chunks, hipStream_t st) {
    int64_t g = (m.N + 255) / 256;
    hipLaunchKernelGGL(k_copy_schedule, dim3((unsigned)g), dim3(256), 0, st, m, p_in);
    size_t lds = ((size_t)m.T * 64 + m.T + 1) * sizeof(double);
    if (lds < 64 * sizeof(double)) lds = 64 * sizeof(double);
    hipLaunchKernelGGL(k_state_partial, dim3(chunks, m.S + 1), dim3(64), lds, st, m,
                       p_in, partial, chunks);
    hipLaunchKernelGGL(k_state_finish, dim3(64), dim3(256), 0, st, m, partial, chunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_prep(m, st);
}

// ---- statistics and penalty tables from (N_s, O, M) ------------------------
// One launch of two workgroups of kPT threads.
//
// Workgroup 0, the scalars: mu, var, sigma, e_s and the objective terms.  N_s
// and the M entries are staged in LDS while the processing-excess terms are
// summed, so that all their loads are in flight together.  Every sum is a
// fixed-order tree whose leaves are the strided partial sums of threads
// 0..255; the other threads add zeros, which changes no partial sum.
//
// Workgroup 1, the penalty tables of every period.  The items (t, s), t < T,
// s < S, in period-major order; a packed list is the order-preserving
// compaction of the items by "partial add" (or "partial rem"), so each
// period's entries are contiguous and scenario-ascending, periods in order.
// The items are cut into jobs of 64 scenarios of one period, one job per wave
// at a time: a first pass counts each job's partial entries (and writes its
// words of the full-bit tables), a scan over the jobs gives each job's output
// offsets, and a second pass writes the entries and the period ranges.
constexpr int kPT = 1024;
constexpr int kPW = kPT / 64;

__device__ double block_sum_f64(double x, double *red) {
    // fixed-order tree over blockDim.x (power of two) threads
    const int tid = threadIdx.x;
    __syncthreads();
    red[tid] = x;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// Two such trees at once (red holds 2 * blockDim.x entries).
__device__ void block_sum2_f64(double &x, double &y, double *red) {
    const int tid = threadIdx.x, n = blockDim.x;
    __syncthreads();
    red[tid] = x;
    red[n + tid] = y;
    __syncthreads();
    for (int w = n / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[tid] += red[tid + w];
            red[n + tid] += red[n + tid + w];
        }
        __syncthreads();
    }
    x = red[0];
    y = red[n];
    __syncthreads();
}

// Smallest non-negative double x with O + x > cap in FP64 arithmetic (the sum
// is monotone in x, so a bisection over the bit patterns of non-negative
// doubles finds it); hi is known to exceed the threshold.  The bisection
// keeps lo below the threshold and hi above it; it starts from the bracket
// cap - O -/+ a few units in the last place of the larger of cap and O, where
// the threshold lies, whenever both ends check out (about a dozen halvings
// instead of some sixty), and from [0, hi] otherwise.
__device__ double min_exceeding(double O, double cap, double hi) {
    if (O + 0.0 > cap) return 0.0;
    if (!(O + hi > cap)) return hi;   // not a partial entry; never taken
    uint64_t lo_b = 0, hi_b = (uint64_t)__double_as_longlong(hi);
    const double x0 = cap - O;
    const double w = 0x1p-49 * fmax(fabs(cap), fabs(O)) + 0x1p-1000;
    const double a = fmax(x0 - w, 0.0), b = fmin(x0 + w, hi);
    if (!(O + a > cap)) lo_b = (uint64_t)__double_as_longlong(a);
    if (O + b > cap) hi_b = (uint64_t)__double_as_longlong(b);
    while (hi_b - lo_b > 1) {          // at most 64 halvings
        const uint64_t mid = lo_b + (hi_b - lo_b) / 2;
        if (O + __longlong_as_double((long long)mid) > cap) hi_b = mid;
        else lo_b = mid;
    }
    return __longlong_as_double((long long)hi_b);
}

__device__ void prep_scalars(const DevModel &m, double *red, double *nsl, double *ml) {
    const int tid = threadIdx.x;
    const int32_t S = m.S, T = m.T;
    const bool act = tid < 256;
    for (int32_t i = tid; i < S; i += kPT) nsl[i] = m.Ns[i];
    if (tid < T) ml[tid] = m.M[tid];   // T < kPT
    double pp = 0.0;
    if (act)
        for (int64_t i = tid; i < (int64_t)S * T; i += 256) pp += hinge64(m.O[i], m.pcap);
    __syncthreads();
    double s = 0.0;
    if (act)
        for (int32_t i = tid; i < S; i += 256) s += nsl[i];
    block_sum2_f64(s, pp, red);
    const double mu = s / S;
    double q = 0.0;
    if (act)
        for (int32_t i = tid; i < S; i += 256) {
            const double e = nsl[i] - mu;
            q += e * e;
        }
    const double var = block_sum_f64(q, red) / S;
    for (int32_t i = tid; i < S; i += kPT) m.e32[i] = (float)(nsl[i] - mu);
    // CVaR of the lower alpha tail: scenario i of rank r (value, then index)
    // weighs 1 below rank k-1, alpha*S - k + 1 at rank k-1
    double cv = 0.0;
    const double aS = m.alpha * S;
    int32_t kq = (int32_t)ceil(aS);
    kq = kq < 1 ? 1 : (kq > S ? S : kq);
    if (m.risk == 1) {
        double part = 0.0;
        if (act)
            for (int32_t i = tid; i < S; i += 256) {
                const double x = nsl[i];
                int32_t r = 0;
                for (int32_t j = 0; j < S; ++j) {
                    const double y = nsl[j];
                    r += (y < x || (y == x && j < i)) ? 1 : 0;
                }
                if (r < kq - 1) part += x;
                else if (r == kq - 1) part += (aS - (kq - 1)) * x;
            }
        cv = block_sum_f64(part, red) / aS;
    }
    if (tid == 0) {
        double pm = 0.0;
        for (int32_t u = 0; u < T; ++u) pm += hinge64(ml[u], m.mcap);
        double sigma = sqrt(var);
        DevScalars *sc = m.sc;
        sc->mu = mu;
        sc->var = var;
        sc->sigma = sigma;
        sc->sigma32 = (float)sigma;
        sc->var32 = (float)var;
        sc->cvar_e = m.risk == 1 ? cv - mu : 0.0;
        sc->R = m.risk == 1 ? mu - m.lambda * (mu - cv) : mu - m.lambda * sigma;
        sc->Pp = m.pen_proc * pp / S;
        sc->Pm = m.pen_mine * pm;
        sc->J = sc->R - sc->Pp - sc->Pm;
    }
}

struct PrepItem {
    double O;
    bool full_add, part_add, full_rem, part_rem;
};

__device__ __forceinline__ PrepItem prep_item(const DevModel &m, int32_t t, int32_t s) {
    PrepItem k;
    const bool in = s < m.S;
    k.O = in ? m.O[(int64_t)t * m.S + s] : 0.0;
    k.full_add = in && k.O >= m.pcap && k.O + m.ton_min > m.pcap;
    k.part_add = in && !k.full_add && k.O + m.ton_max > m.pcap;
    const double a = k.O - m.pcap;
    k.full_rem = in && a >= m.ton_max;
    k.part_rem = in && !k.full_rem && a > 0.0;
    return k;
}

__device__ void prep_tables(const DevModel &m, uint64_t *jc) {
    __shared__ uint64_t wt[kPW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t S = m.S, T = m.T, W = m.W;
    const int32_t nc = (S + 63) / 64, J = T * nc;
    // pass 1: per job, the counts (add in the low half, rem in the high half)
    for (int32_t j = wave; j < J; j += kPW) {
        const int32_t t = j / nc, c = j - t * nc;
        const PrepItem k = prep_item(m, t, 64 * c + lane);
        const uint64_t bfa = __ballot(k.full_add), bfr = __ballot(k.full_rem);
        const uint64_t bpa = __ballot(k.part_add), bpr = __ballot(k.part_rem);
        if (lane == 0) {
            const int32_t w0 = 2 * c;   // 64 scenarios = 2 words
            if (w0 < W) {
                m.tab.full_add[(int64_t)t * W + w0] = (uint32_t)bfa;
                m.tab.full_rem[(int64_t)t * W + w0] = (uint32_t)bfr;
            }
            if (w0 + 1 < W) {
                m.tab.full_add[(int64_t)t * W + w0 + 1] = (uint32_t)(bfa >> 32);
                m.tab.full_rem[(int64_t)t * W + w0 + 1] = (uint32_t)(bfr >> 32);
            }
            jc[j] = (uint64_t)__popcll(bpa) | ((uint64_t)__popcll(bpr) << 32);
        }
    }
    __syncthreads();
    // exclusive scan of the job counts: thread tid owns jobs [j0, j1); both
    // halves scan at once (each total is below 2^32, so no carry crosses)
    const int32_t E = (J + kPT - 1) / kPT;
    const int32_t j0 = min(J, tid * E), j1 = min(J, j0 + E);
    uint64_t own = 0;
    for (int32_t j = j0; j < j1; ++j) own += jc[j];
    uint64_t x = own;
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wt[wave] = x;
    __syncthreads();
    uint64_t run = x - own, tot = 0;
    for (int w = 0; w < kPW; ++w) {
        if (w < wave) run += wt[w];
        tot += wt[w];
    }
    for (int32_t j = j0; j < j1; ++j) {
        const uint64_t c = jc[j];
        jc[j] = run;
        run += c;
    }
    __syncthreads();
    // pass 2: the entries at their offsets, and the period ranges
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int32_t j = wave; j < J; j += kPW) {
        const int32_t t = j / nc, c = j - t * nc, s = 64 * c + lane;
        const PrepItem k = prep_item(m, t, s);
        const uint64_t bpa = __ballot(k.part_add), bpr = __ballot(k.part_rem);
        const uint64_t base = jc[j];
        const int32_t ba = (int32_t)(uint32_t)base, br = (int32_t)(base >> 32);
        if (k.part_add) {
            AddEntry e;
            e.tau = min_exceeding(k.O, m.pcap, 2.0 * m.ton_max);
            e.d = (float)(m.pcap - k.O);
            e.s = s;
            m.tab.add_packed[ba + (int32_t)__popcll(bpa & below)] = e;
        }
        if (k.part_rem) {
            RemEntry e;
            e.a = (float)(k.O - m.pcap);
            e.s = s;
            m.tab.rem_packed[br + (int32_t)__popcll(bpr & below)] = e;
        }
        if (c == 0 && lane == 0) {
            m.tab.rng[t] = ba;
            m.tab.rng[2 * T + t] = br;
            if (t > 0) {
                m.tab.rng[T + t - 1] = ba;
                m.tab.rng[3 * T + t - 1] = br;
            }
        }
    }
    if (tid == 0) {
        m.tab.rng[2 * T - 1] = (int32_t)(uint32_t)tot;
        m.tab.rng[4 * T - 1] = (int32_t)(tot >> 32);
    }
}

__global__ void __launch_bounds__(kPT) k_prep(DevModel m) {
    extern __shared__ __align__(16) char lds[];
    __shared__ double red[2 * kPT];
    if (blockIdx.x == 0)
        prep_scalars(m, red, (double *)lds, (double *)lds + m.S);
    else
        prep_tables(m, (uint64_t *)lds);
}

hipError_t launch_prep(const DevModel &m, hipStream_t st) {
    const size_t a = sizeof(double) * ((size_t)m.S + m.T);
    const size_t b = sizeof(uint64_t) * (size_t)m.T * ((m.S + 63) / 64);
    hipLaunchKernelGGL(k_prep, dim3(2), dim3(kPT), a > b ? a : b, st, m);
    return hipGetLastError();
}

__global__ void k_objective_copy(DevModel m, double *out) {
    if (threadIdx.x == 0) {
        const DevScalars *sc = m.sc;
        out[0] = sc->mu;
        out[1] = sc->sigma;
        out[2] = sc->R;
        out[3] = sc->Pp;
        out[4] = sc->Pm;
        out[5] = sc->J;
        out[6] = sc->n_prec_viol;
    }
}

hipError_t launch_objective_copy(const DevModel &m, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_objective_copy, dim3(1), dim3(64), 0, st, m, out);
    return hipGetLastError();
}

}  // namespace mps
