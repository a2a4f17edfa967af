// repair.h -- launch interface of the greedy repair walk (repair.hip), used
// by the entry points (api.hip).
#pragma once
#include "internal.h"

namespace mps {

// Largest S the walk supports: each lane keeps four scenarios per 256 of
// N_s in registers, up to four such chunks.
constexpr int32_t kRepairMaxScen = MPS_MAX_REPAIR_SCENARIOS;

// LDS bytes of one walk over at most max_cand candidates.
size_t repair_lds_bytes(const DevModel &m, int32_t max_cand);
// Device workspace of the candidate records (any count up to MPS_MAX_TOPK).
size_t repair_gather_bytes(int32_t S, int32_t W);
// `first` is a device int32[N] that holds INT32_MAX in every entry between
// calls (the walk restores what the call changed).
hipError_t launch_repair(const DevModel &m, const mps_moves &mv, const int64_t *idx,
                         const int32_t *count, int32_t max_cand, int32_t hard,
                         int32_t *applied, void *gather, int32_t *first, hipStream_t st);

}  // namespace mps
