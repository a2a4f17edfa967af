// batch_sort.hip -- the block order of a batch's move lists, computed once
// when the batch is built or retuned: within each move item's range of
// moves, the positions sorted by moved block (a stable segmented radix sort, so
// equal blocks keep their list order).  The move items then score their
// moves in that order, and neighbouring lanes read neighbouring blocks' data.
#include <hipcub/hipcub.hpp>

#include "batch.h"

namespace mps {

__global__ void k_iota_segments(int64_t n, int32_t len, int32_t nseg, int32_t *pos,
                                int32_t *beg, int32_t *end) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pos[i] = (int32_t)i;
    if (i < nseg) {
        beg[i] = (int32_t)(i * len);
        end[i] = (int32_t)min(n, (i + 1) * (int64_t)len);
    }
}

hipError_t batch_sort_moves(const int32_t *blk, int64_t n, int32_t len, int32_t *perm,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int32_t nseg = (int32_t)((n + len - 1) / len);
    int32_t *pos = nullptr, *keys = nullptr, *beg = nullptr, *end = nullptr;
    void *tmp = nullptr;
    size_t tb = 0;
    hipError_t e = hipMalloc((void **)&pos, sizeof(int32_t) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void **)&keys, sizeof(int32_t) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void **)&beg, sizeof(int32_t) * (size_t)nseg);
    if (e == hipSuccess) e = hipMalloc((void **)&end, sizeof(int32_t) * (size_t)nseg);
    if (e == hipSuccess) {
        const int64_t cnt = n > nseg ? n : nseg;
        hipLaunchKernelGGL(k_iota_segments, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
                           n, len, nseg, pos, beg, end);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, tb, blk, keys, pos, perm, (int)n,
                                                        nseg, beg, end, 0, 32, st);
    if (e == hipSuccess) e = hipMalloc(&tmp, tb > 0 ? tb : 1);
    if (e == hipSuccess)
        e = hipcub::DeviceSegmentedRadixSort::SortPairs(tmp, tb, blk, keys, pos, perm, (int)n, nseg,
                                                        beg, end, 0, 32, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(tmp);
    hipFree(end);
    hipFree(beg);
    hipFree(keys);
    hipFree(pos);
    return e;
}

}  // namespace mps
