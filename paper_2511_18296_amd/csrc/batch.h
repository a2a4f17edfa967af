// batch.h -- descriptors of the batched persistent evaluation (batch.hip),
// shared with the entry points that build them (api.hip).
#pragma once
#include "internal.h"

namespace mps {

constexpr int kSegBins = 4096;   // level-0 histogram bins per model

// One model of a batch: its device view, its move list and outputs, and the
// work split chosen for it.
struct BatchInst {
    DevModel m;
    const int32_t *blk;
    const int8_t *per;
    int64_t n;
    float *score;
    uint8_t *flags;
    int64_t *top_idx;
    float *top_score;
    int32_t *top_count;
    int32_t n_tiles;          // 64-block tiles of the model
    int32_t tiles_per_item;   // tiles per block item
    int32_t n1, n2;           // block items and move items
    int32_t moves_per_item;   // moves per move item
    int32_t rows;             // v rows in flight per lane (8, 16, 32)
};

struct BatchLaunch {
    const BatchInst *insts;
    const int2 *items1;       // block items (model, item) in queue order
    const int2 *items2;       // move items
    const int32_t *order;     // models, largest first
    int32_t n_items1, n_items2, n_inst;
    uint32_t *ctl;            // head1, head2, hist[n][kSegBins]
    int32_t k;
    uint8_t req, forbid;
    int grid1, grid2;
    size_t lds_bytes;
};

inline int64_t batch_ctl_words(int32_t n_inst) {
    return 2 + (int64_t)kSegBins * n_inst;
}

size_t batch_lds_bytes(const DevModel &m);
hipError_t launch_batch(const BatchLaunch &bl, hipStream_t st);
hipError_t batch_occupancy(size_t lds_bytes, int *per_cu);

}  // namespace mps
