// rank.hip -- gradient ranking of every move: gain(b,t') = Gc[b,p_b] - Gc[b,t'],
// Gc[b,t] = sum_{u<t} dJ/dx[b,u] (FP64 prefix sums), the first-order change of
// J for moving b from p_b to t'.  Only moves that keep the schedule
// precedence-feasible (Eq. 15) rank (the repair could never apply the others),
// and no-op moves get flag 0, so that the top-k (require 1) skips both.
//
// One workgroup of 256 threads per 64 consecutive blocks.  The blocks' rows
// of dJ/dx are staged in LDS with coalesced loads; one thread per block forms
// its precedence window and the running FP64 prefix sums Gc[b,0..T] (in LDS);
// then all threads form the workgroup's contiguous range of outputs (b, t')
// from them and write it directly, coalesced.
#include "internal.h"

namespace mps {

constexpr int kRT = 256;   // threads per workgroup
constexpr int kRBk = 64;   // blocks per workgroup

__host__ __device__ static inline size_t ral256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t rank_lds_bytes(int32_t T) {
    return sizeof(double) * kRBk * (size_t)(T + 1) + sizeof(int32_t) * 3 * kRBk +
           sizeof(float) * kRBk * (size_t)T;
}

__global__ void __launch_bounds__(kRT) k_rank_gains(DevModel m, const float *grad, float *gain,
                                                    uint8_t *fl) {
    extern __shared__ __align__(16) char lds[];
    const int32_t T = m.T, D = T + 1;
    double *pre = (double *)lds;                      // [kRBk][D] prefix sums Gc
    int32_t *win = (int32_t *)(pre + (size_t)kRBk * D);   // [kRBk][3]: p_b, lo, hi
    float *gs = (float *)(win + 3 * kRBk);            // [kRBk][T] rows of dJ/dx
    const int tid = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kRBk;
    const int32_t nb = (int32_t)min((int64_t)kRBk, m.N - b0);
    const int32_t ng = nb * T, no = nb * D;
    const float *gsrc = grad + b0 * T;
    for (int32_t i = tid; i < ng; i += kRT) gs[i] = gsrc[i];
    int32_t lo = 0, hi = 0, pb = 0;
    if (tid < nb) {
        pb = m.p[b0 + tid];
        prec_window(m, m.p, (int32_t)(b0 + tid), lo, hi);
    }
    __syncthreads();
    if (tid < nb) {
        win[3 * tid] = pb;
        win[3 * tid + 1] = lo;
        win[3 * tid + 2] = hi;
        const float *g = gs + (size_t)tid * T;
        double *c = pre + (size_t)tid * D;
        double run = 0.0;
        c[0] = 0.0;
        for (int32_t u = 0; u < T; ++u) {
            run += (double)g[u];
            c[u + 1] = run;
        }
    }
    __syncthreads();
    float *gd = gain + b0 * D;
    uint8_t *fd = fl + b0 * D;
    for (int32_t i = tid; i < no; i += kRT) {
        const int32_t bl = i / D, t = i - bl * D;
        const int32_t p = win[3 * bl], l = win[3 * bl + 1], h = win[3 * bl + 2];
        const double *c = pre + (size_t)bl * D;
        gd[i] = (float)(c[p] - c[t]);
        fd[i] = (t != p && l <= t && t <= h) ? 1 : 0;
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
    return ral256(4 * (size_t)n) + ral256((size_t)n) + ral256(8 * (size_t)k) + topk_ws_bytes(n, k);
}

hipError_t launch_rank(const DevModel &m, const float *grad, int32_t k, int32_t *blk, int8_t *per,
                       float *gain_out, int32_t *count, void *ws, hipStream_t st) {
    const int64_t n = m.N * (m.T + 1);
    char *c = (char *)ws;
    float *gain = (float *)c;
    c += ral256(4 * (size_t)n);
    uint8_t *fl = (uint8_t *)c;
    c += ral256((size_t)n);
    int64_t *idx = (int64_t *)c;
    c += ral256(8 * (size_t)k);
    hipLaunchKernelGGL(k_rank_gains, dim3((unsigned)((m.N + kRBk - 1) / kRBk)), dim3(kRT),
                       rank_lds_bytes(m.T), st, m, grad, gain, fl);
    hipError_t e = launch_topk(gain, fl, n, k, 1, 0, idx, gain_out, count, c, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_decode, dim3((k + 255) / 256), dim3(256), 0, st, m.T + 1, idx, k,
                       blk, per);
    return hipGetLastError();
}

}  // namespace mps
