// batch.h -- descriptors of the batched persistent evaluation (batch.hip),
// shared with the entry points that build them (api.hip).
#pragma once
#include "internal.h"

namespace mps {

constexpr int kSegBins = 4096;   // level-0 histogram bins per model (top 12 key bits)
constexpr int kSegBins1 = 2048;  // level-1 histogram bins per model (next 11 bits)
constexpr int kSegCap = 1024;    // boundary keys refined on chip

// Per-model state of the top-k phases (8 words).
struct BtState {
    int32_t mode;     // kBt* below
    int32_t need;     // keys still to take from the boundary digit
    uint32_t d0, d1;  // boundary digits at levels 0 and 1
    int32_t n_sel;    // keys in sel (all above the boundary)
    int32_t n_cand;   // keys in cand (on the boundary)
    int32_t pad[2];
};
static_assert(sizeof(BtState) == 32, "state is 8 words");
enum : int32_t {
    kBtTakeAll = 1,   // at most k qualify: all are selected
    kBtCollect0 = 2,  // level-0 boundary digit fits on chip
    kBtPass1 = 3,     // a pass counts level 1 of the boundary digit
    kBtCollect1 = 4,  // level-1 boundary digit fits on chip
    kBtFallback = 5   // more than kSegCap keys share 23 key bits: one workgroup walks the model
};

// The control area of a batch (32-bit words): four queue heads, the level-0
// and level-1 histograms and the state of every model (cleared by each
// launch), then the selected and boundary keys of every model (64-bit).
struct BatchCtl {
    uint32_t *head;        // [4]: block items, move items, level-1 pass, collection
    uint32_t *hist0;       // [n][kSegBins]
    uint32_t *hist1;       // [n][kSegBins1]
    BtState *state;        // [n]
    uint64_t *sel;         // [n][MPS_MAX_BATCH_TOPK]
    uint64_t *cand;        // [n][kSegCap]
};
__host__ __device__ inline int64_t batch_ctl_clear_words(int32_t n_inst) {
    return 4 + (int64_t)(kSegBins + kSegBins1 + 8) * n_inst;
}
__host__ __device__ inline int64_t batch_ctl_words(int32_t n_inst) {
    return batch_ctl_clear_words(n_inst) + 2 * (int64_t)(MPS_MAX_BATCH_TOPK + kSegCap) * n_inst;
}
__host__ __device__ inline BatchCtl batch_ctl(uint32_t *ctl, int32_t n_inst) {
    BatchCtl c;
    c.head = ctl;
    c.hist0 = ctl + 4;
    c.hist1 = c.hist0 + (int64_t)kSegBins * n_inst;
    c.state = (BtState *)(c.hist1 + (int64_t)kSegBins1 * n_inst);
    c.sel = (uint64_t *)(ctl + batch_ctl_clear_words(n_inst));
    c.cand = c.sel + (int64_t)MPS_MAX_BATCH_TOPK * n_inst;
    return c;
}

// One model of a batch: its device view, its move list and outputs, and the
// work split chosen for it.
struct BatchInst {
    DevModel m;
    const int32_t *blk;
    const int8_t *per;
    // positions 0 .. n-1 ordered by moved block (stable) within each range
    // of moves_per_item: a move item scores its moves in this order, so that
    // neighbouring lanes read neighbouring blocks' data
    const int32_t *perm;
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
    uint32_t *ctl;            // the control area (BatchCtl)
    int32_t k;
    uint8_t req, forbid;
    int grid1, grid2;
    int32_t claim;            // move items per claim in the top-k passes
    size_t lds_bytes;
};


size_t batch_lds_bytes(const DevModel &m);
hipError_t launch_batch(const BatchLaunch &bl, hipStream_t st);
hipError_t batch_occupancy(size_t lds_bytes, int *per_cu);

// perm[0 .. n) = the positions of blk[0 .. n) ordered by block, stably,
// within each range [j*len, (j+1)*len).  Allocates its temporary buffers;
// synchronises the stream.
hipError_t batch_sort_moves(const int32_t *blk, int64_t n, int32_t len, int32_t *perm,
                            hipStream_t st);

}  // namespace mps
