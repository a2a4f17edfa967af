// internal.h -- device-side layout of a model and the launch helpers shared
// by the HIP translation units of libmps.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mps.h"

namespace mps {

constexpr int kWave = 64;

// Scalars derived from the per-scenario NPV vector; written by the state
// kernels, read by every evaluation.
struct DevScalars {
    double mu, var, sigma;
    double R, Pp, Pm, J;
    double n_prec_viol;      // as double so the objective is one double[7]
    double cvar_e;           // CVaR risk: CVaR_alpha(N) - mu (0 for the std measure)
    float sigma32, var32;
    int32_t n_bad_periods;   // schedule entries outside 0..T (clamped)
    int32_t pad;
};

// Per-period tables of the processing-capacity penalty.  For period t and
// scenario s with O = O[t][s] (FP64):
//   add term (block b moved INTO t):  hinge(O + ton_b) - hinge(O)
//     full add    : O >= cap and O + ton_min > cap -> value ton_b and a
//                   capacity violation for every block (bit in full_add)
//     partial add : otherwise, if O + ton_max > cap -> list entry with
//                   d = cap - O (value max(0, ton_b - d)) and the exact FP64
//                   threshold tau = min{x >= 0 : O + x > cap} (violation iff
//                   ton_b >= tau, the same decision as evaluating O + ton_b > cap)
//     neither     : O + ton_max <= cap               -> 0, never a violation
//   removal term (block b moved OUT of t): hinge(O - ton_b) - hinge(O)
//     = -clamp(O - cap, 0, ton_b)
//     full rem    : O - cap >= ton_max               -> -ton_b (bit in full_rem)
//     partial rem : 0 < O - cap < ton_max            -> list entry a = O - cap,
//                   value -min(a, ton_b)
// Lists are per period and scenario-ascending, concatenated over the periods
// in order; rng gives each period's range.
struct AddEntry {
    double tau;
    float d;
    int32_t s;
};
struct RemEntry {
    float a;
    int32_t s;
};
struct PeriodTables {
    uint32_t *full_add;   // [T][W] bit s%32 of word s/32
    uint32_t *full_rem;   // [T][W]
    int32_t *rng;         // [4][T]: packed add begin/end, rem begin/end
    AddEntry *add_packed; // [T*S] concatenated lists
    RemEntry *rem_packed; // [T*S]
};

// The list pass's record of one block: everything a listed move of the block
// reads, in one 64-byte line (the ore words too when S <= 256), so that a
// move costs one line instead of a load from each of eight arrays.
struct alignas(16) ListRec {
    float c;           // (1/S) sum_s e_s v[s][b]
    float rem;         // removal term of the block's current period
    int32_t info;      // p | maxPred << 8 | minSucc << 16
    float ton32, mb, Vb;
    double ton64;
    uint32_t ore[8];   // ore words 0..7 (S <= 256); larger S reads them from m.ore
};
static_assert(sizeof(ListRec) == 64, "one line per block");

struct DevModel {
    int64_t N;
    int32_t S, T, W, nx, ny, nz;
    double lambda, pen_proc, pen_mine, pcap, mcap;
    double ton_min, ton_max;
    const float *v;        // [S][vld]: row s holds v[s][0 .. N), zero-padded
    int64_t vld;           // row stride of v: N rounded up to 32 (128-byte rows)
    const uint32_t *ore;   // [W][N]
    const double *ton64;   // [N]
    const float *ton32;    // [N]
    const double *mb64;    // [N] mean_s v[s][b]
    const double *Vb64;    // [N] population variance_s v[s][b]
    const float *mb32;
    const float *Vb32;
    int8_t *p;             // [N] current schedule
    double *Ns;            // [S] per-scenario NPV
    double *O;             // [T][S] ore tonnage per period and scenario
    double *M;             // [T] tonnage per period
    float *e32;            // [S] N_s - mu (the allocation has 64 more entries)
    DevScalars *sc;
    const double *d64;     // [T+1] discount factors, d[T] = 0
    PeriodTables tab;
    // precedence: csr = 0 the 1-5 stencil of the grid; csr = 1 the lists
    // (predecessors of b: pred_idx[pred_ptr[b] .. pred_ptr[b+1]), successors
    // likewise), at most MPS_MAX_DEGREE each
    int32_t csr;
    const int32_t *pred_ptr, *pred_idx, *succ_ptr, *succ_idx;
    // objective variants: wmult [S][T+1] = d(t) sigma(s,t) (FP64; d(T) = 0),
    // wmult32 the same in FP32; both NULL without a value multiplier.
    // risk 0: mu - lambda sigma; risk 1: mu - lambda (mu - CVaR_alpha).
    const double *wmult;
    const float *wmult32;
    int32_t risk;
    double alpha;
    // list-mode per-block workspace
    ListRec *blk_rec;      // [N] per-block record of the list pass
    uint32_t *tmark;       // [ceil(N/64)] tiles a move list touches; zero between calls
};

// Sets the thread-local text mps_last_error() returns; returns st.
mps_status report_error(mps_status st, const char *msg);

// Launch wrappers (each returns the hipError_t of its launches).
hipError_t launch_block_stats(const DevModel &m, float *mb32, float *Vb32,
                              double *mb64, double *Vb64, hipStream_t st);
hipError_t launch_set_schedule(const DevModel &m, const int8_t *p_in,
                               double *partial, int chunks, hipStream_t st);
hipError_t launch_prep(const DevModel &m, hipStream_t st);
hipError_t launch_objective_copy(const DevModel &m, double *out, hipStream_t st);
// LDS bytes per workgroup of the evaluation kernels for these moves: the
// period bit tables and block data of one 64-block tile, plus the per-move
// staging of the exhaustive form.
size_t eval_lds_bytes(const DevModel &m, const mps_moves &mv);
hipError_t launch_eval(const DevModel &m, const mps_moves &mv, float *score,
                       uint8_t *flags, float *dR, float *dPp, float *dPm,
                       hipStream_t st);
size_t topk_ws_bytes(int64_t n, int32_t k);
// Leading bytes of a top-k workspace that must be zero when a call starts
// (every call leaves them zero).
size_t topk_ws_zero_bytes();
hipError_t launch_topk(const float *score, const uint8_t *flags, int64_t n,
                       int32_t k, uint8_t req, uint8_t forbid, int64_t *idx,
                       float *top_score, int32_t *count, void *ws,
                       hipStream_t st);

size_t relaxed_saved_bytes(const DevModel &m);
size_t relaxed_ws_bytes(const DevModel &m);
hipError_t launch_relaxed_fwd(const DevModel &m, const float *x, const mps_relax_params &rp,
                              double *J_out, void *saved, void *ws, hipStream_t st);
hipError_t launch_relaxed_bwd(const DevModel &m, const float *x, const mps_relax_params &rp,
                              const void *saved, const double *dJ, float *grad, void *ws,
                              hipStream_t st);
// Once per model: the precedence-stencil bits kept in the relaxed workspace.
hipError_t launch_relaxed_init(const DevModel &m, void *ws, hipStream_t st);
size_t rank_ws_bytes(const DevModel &m, int32_t k);
hipError_t launch_rank(const DevModel &m, const float *grad, int32_t k, int32_t *blk,
                       int8_t *per, float *gain_out, int32_t *count, void *ws, hipStream_t st);
hipError_t launch_integer_x(const DevModel &m, float *x, hipStream_t st);
// Move evaluation under an objective variant (value multiplier and/or CVaR
// risk); LDS bytes of its workgroup.
constexpr int32_t kVariantMaxScen = 1024;
size_t eval_var_lds_bytes(const DevModel &m);
hipError_t launch_eval_var(const DevModel &m, const mps_moves &mv, float *score, uint8_t *flags,
                           float *dR, float *dPp, float *dPm, hipStream_t st);
__host__ __device__ inline bool has_variant(const DevModel &m) {
    return m.wmult != nullptr || m.risk != 0;
}
// Cascading repair walk; mark is a device uint8 [N] workspace.  Re-derives
// the state from the schedule afterwards (partial/chunks as for
// launch_set_schedule).
constexpr int32_t kCascadeMaxSet = 256;
size_t cascade_lds_bytes(const DevModel &m);
hipError_t launch_cascade(const DevModel &m, const mps_moves &mv, const int64_t *idx,
                          const int32_t *count, int32_t max_cand, int32_t hard, int32_t max_set,
                          int32_t *applied, uint8_t *mark, double *partial, int chunks,
                          hipStream_t st);
// LNS destroy step: region of the column tile [x0,x1) x [y0,y1) and its
// descendants into reg (uint8 [N]), every region block set to never in the
// model's schedule, and the repair move list (b, t < T) by increasing b into
// lb/lt with its length in *count (device).
hipError_t launch_lns_destroy(const DevModel &m, int32_t x0, int32_t x1, int32_t y0, int32_t y1,
                              uint8_t *reg, int32_t *lb, int8_t *lt, int32_t *count,
                              hipStream_t st);
// Greedy initializer: writes the schedule into p (device int8 [N]) and
// {passes, placed} into out (device int32 [2]).
size_t greedy_ws_bytes(const DevModel &m);
size_t greedy_lds_bytes(const DevModel &m);
hipError_t launch_greedy(const DevModel &m, int8_t *p, int32_t max_pass, void *ws,
                         int32_t *out, hipStream_t st);

// Global-memory access through an explicitly global pointer.  Pointers held
// in device-memory descriptors (not kernel arguments) are otherwise generic,
// and generic (flat) accesses also count against the LDS wait counter.
template <class T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ T gld_nt(const T *p) {
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T *)p);
}
template <class T>
__device__ __forceinline__ void gst(T *p, const T &v) {
    *(__attribute__((address_space(1))) T *)p = v;
}
__device__ __forceinline__ AddEntry gld(const AddEntry *p) {
    AddEntry e;
    e.tau = gld(&p->tau);
    e.d = gld(&p->d);
    e.s = gld(&p->s);
    return e;
}
__device__ __forceinline__ RemEntry gld(const RemEntry *p) {
    RemEntry e;
    e.a = gld(&p->a);
    e.s = gld(&p->s);
    return e;
}

// Precedence neighbours under the 1-5 stencil; shared by the kernels.
__device__ __forceinline__ void grid_coords(const DevModel &m, int32_t b,
                                            int32_t &x, int32_t &y, int32_t &z) {
    int32_t nxy = m.nx * m.ny;
    z = b / nxy;
    int32_t r = b - z * nxy;
    y = r / m.nx;
    x = r - y * m.nx;
}

// Neighbour k of b: predecessor k (pred = true) or successor k, -1 when b
// has fewer.  Stencil predecessors in the order up, x-1, x+1, y-1, y+1 (the
// block on the bench above and its face neighbours); stencil successors by
// increasing index; list neighbours in list order.  k < MPS_MAX_DEGREE.
__device__ __forceinline__ int32_t nbr(const DevModel &m, int32_t b, int k, bool pred) {
    if (m.csr) {
        const int32_t *ptr = pred ? m.pred_ptr : m.succ_ptr;
        const int32_t *ix = pred ? m.pred_idx : m.succ_idx;
        const int32_t j = ptr[b] + k;
        return j < ptr[b + 1] ? ix[j] : -1;
    }
    int32_t x, y, z;
    grid_coords(m, b, x, y, z);
    const int32_t nxy = m.nx * m.ny;
    if (pred) {
        if (z == 0) return -1;
        const int32_t up = b - nxy;
        switch (k) {
            case 0: return up;
            case 1: return x > 0 ? up - 1 : -1;
            case 2: return x + 1 < m.nx ? up + 1 : -1;
            case 3: return y > 0 ? up - m.nx : -1;
            case 4: return y + 1 < m.ny ? up + m.nx : -1;
            default: return -1;
        }
    }
    if (z + 1 >= m.nz) return -1;
    const int32_t dn = b + nxy;
    switch (k) {
        case 0: return y > 0 ? dn - m.nx : -1;
        case 1: return x > 0 ? dn - 1 : -1;
        case 2: return dn;
        case 3: return x + 1 < m.nx ? dn + 1 : -1;
        case 4: return y + 1 < m.ny ? dn + m.nx : -1;
        default: return -1;
    }
}

// max over predecessors of p (0 if none) and min over successors (T if none),
// the two numbers that decide PREC_OK for every destination of b.
__device__ __forceinline__ void prec_window(const DevModel &m, const int8_t *p,
                                            int32_t b, int32_t &lo, int32_t &hi) {
    if (m.csr) {
        const int32_t T = m.T;
        lo = 0;
        hi = T;
        auto rd = [&](int32_t a) {
            int32_t v = p[a];
            return (v < 0 || v > T) ? T : v;
        };
        for (int32_t j = m.pred_ptr[b]; j < m.pred_ptr[b + 1]; ++j) lo = max(lo, rd(m.pred_idx[j]));
        for (int32_t j = m.succ_ptr[b]; j < m.succ_ptr[b + 1]; ++j) hi = min(hi, rd(m.succ_idx[j]));
        return;
    }
    int32_t x, y, z;
    grid_coords(m, b, x, y, z);
    const int32_t nx = m.nx, nxy = m.nx * m.ny, T = m.T;
    lo = 0;
    hi = T;
    auto rd = [&](int32_t a) {
        int32_t v = p[a];
        return (v < 0 || v > T) ? T : v;
    };
    if (z > 0) {
        int32_t a = b - nxy;
        lo = max(lo, rd(a));
        if (x > 0) lo = max(lo, rd(a - 1));
        if (x + 1 < nx) lo = max(lo, rd(a + 1));
        if (y > 0) lo = max(lo, rd(a - nx));
        if (y + 1 < m.ny) lo = max(lo, rd(a + nx));
    }
    if (z + 1 < m.nz) {
        int32_t c = b + nxy;
        hi = min(hi, rd(c));
        if (x > 0) hi = min(hi, rd(c - 1));
        if (x + 1 < nx) hi = min(hi, rd(c + 1));
        if (y > 0) hi = min(hi, rd(c - nx));
        if (y + 1 < m.ny) hi = min(hi, rd(c + nx));
    }
}

__device__ __forceinline__ double hinge64(double x, double cap) {
    return x > cap ? x - cap : 0.0;
}

}  // namespace mps
