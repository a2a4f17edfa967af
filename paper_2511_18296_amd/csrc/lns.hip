// lns.hip -- device steps of the LNS + simulated-annealing driver (Alg. 2
// without its GA and RL parts): the destroy region of a neighbourhood and the
// list of its repair moves.  The driver loop itself (repair rounds, fitness,
// acceptance) is host code in api.hip around the evaluation, top-k and
// repair kernels.
//
// Region of the column tile [x0,x1) x [y0,y1): the tile's blocks on every
// bench and every descendant of them.  Under the 1-5 stencil a block's
// predecessors lie on the bench above, so one sweep bench by bench, top
// down, closes the region: block b on bench z joins if it is in the tile or
// one of its predecessors joined.  Explicit lists may point anywhere: the
// region grows in rounds until a round adds no block.
//
// The move list holds (b, t) for every region block b by increasing index and
// t = 0..T-1 in order, built by one workgroup with an ordered compaction
// (ballot prefix counts, chunk by chunk); the same pass sets every region
// block to "never" (the destroy).
#include "internal.h"

namespace mps {

constexpr int kLT = 1024;

__global__ void k_lns_region(DevModel m, int32_t z, int32_t x0, int32_t x1, int32_t y0,
                             int32_t y1, uint8_t *reg) {
    const int64_t nxy = (int64_t)m.nx * m.ny;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nxy) return;
    const int64_t b = (int64_t)z * nxy + i;
    const int32_t x = (int32_t)(i % m.nx), y = (int32_t)(i / m.nx);
    bool in = x >= x0 && x < x1 && y >= y0 && y < y1;
    if (!in && z > 0) {
        const int64_t up = b - nxy;
        in = reg[up] || (x > 0 && reg[up - 1]) || (x + 1 < m.nx && reg[up + 1]) ||
             (y > 0 && reg[up - m.nx]) || (y + 1 < m.ny && reg[up + m.nx]);
    }
    reg[b] = in ? 1 : 0;
}

// Explicit lists: tile membership, then rounds of "a block joins when one of
// its predecessors is in the region" until a round adds nothing (*changed
// stays 0).
__global__ void k_lns_tile_csr(DevModel m, int32_t x0, int32_t x1, int32_t y0, int32_t y1,
                               uint8_t *reg) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m.N) return;
    int32_t x, y, z;
    grid_coords(m, (int32_t)b, x, y, z);
    reg[b] = (x >= x0 && x < x1 && y >= y0 && y < y1) ? 1 : 0;
}

__global__ void k_lns_grow_csr(DevModel m, uint8_t *reg, int32_t *changed) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m.N || reg[b]) return;
    for (int32_t j = m.pred_ptr[b]; j < m.pred_ptr[b + 1]; ++j)
        if (reg[m.pred_idx[j]]) {
            reg[b] = 1;
            *changed = 1;
            return;
        }
}

__global__ void k_lns_flag_clear(int32_t *changed) { *changed = 0; }

__global__ void __launch_bounds__(kLT) k_lns_list(DevModel m, const uint8_t *reg, int32_t *lb,
                                                  int8_t *lt, int32_t *count) {
    __shared__ int32_t wc[kLT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t T = m.T;
    int32_t base = 0;
    for (int64_t c0 = 0; c0 < m.N; c0 += kLT) {
        const int64_t b = c0 + tid;
        const bool in = b < m.N && reg[b];
        const uint64_t bal = __ballot(in);
        if (lane == 0) wc[wave] = __popcll(bal);
        __syncthreads();
        int32_t before = base, tot = 0;
        for (int w = 0; w < kLT / 64; ++w) {
            if (w < wave) before += wc[w];
            tot += wc[w];
        }
        if (in) {
            const int32_t r = before + (int32_t)__popcll(bal & ((1ull << lane) - 1ull));
            for (int32_t t = 0; t < T; ++t) {
                lb[(int64_t)r * T + t] = (int32_t)b;
                lt[(int64_t)r * T + t] = (int8_t)t;
            }
            m.p[b] = (int8_t)T;
        }
        base += tot;
        __syncthreads();   // wc is rewritten by the next chunk
    }
    if (tid == 0) *count = base * T;
}

hipError_t launch_lns_destroy(const DevModel &m, int32_t x0, int32_t x1, int32_t y0, int32_t y1,
                              uint8_t *reg, int32_t *lb, int8_t *lt, int32_t *count,
                              hipStream_t st) {
    if (m.csr) {
        // count[1] serves as the round's change flag (read back by the host)
        const unsigned gn = (unsigned)((m.N + 255) / 256);
        hipLaunchKernelGGL(k_lns_tile_csr, dim3(gn), dim3(256), 0, st, m, x0, x1, y0, y1, reg);
        for (int64_t round = 0; round <= m.N; ++round) {
            hipLaunchKernelGGL(k_lns_flag_clear, dim3(1), dim3(1), 0, st, count + 1);
            hipLaunchKernelGGL(k_lns_grow_csr, dim3(gn), dim3(256), 0, st, m, reg, count + 1);
            int32_t changed = 0;
            hipError_t e = hipMemcpyAsync(&changed, count + 1, sizeof(int32_t),
                                          hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return e;
            if (!changed) break;
        }
    } else {
        const int64_t nxy = (int64_t)m.nx * m.ny;
        const unsigned g = (unsigned)((nxy + 255) / 256);
        for (int32_t z = 0; z < m.nz; ++z)
            hipLaunchKernelGGL(k_lns_region, dim3(g), dim3(256), 0, st, m, z, x0, x1, y0, y1,
                               reg);
    }
    hipLaunchKernelGGL(k_lns_list, dim3(1), dim3(kLT), 0, st, m, (const uint8_t *)reg, lb, lt,
                       count);
    return hipGetLastError();
}

}  // namespace mps
