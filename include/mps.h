/* mps.h -- C ABI of the MI355X candidate-move evaluation engine.
 *
 * Problem statement (paper Sec. 5, Eq. 14-16):
 *   N = nx*ny*nz blocks, block index b = x + nx*(y + ny*z), z = 0 the top bench;
 *   a schedule p[b] in {0..T-1} is the period in which block b is mined, and
 *   p[b] = T means "never mined";
 *   precedence (Eq. 15): p[a] <= p[b] for each predecessor a of b; by default
 *   the 1-5 slope stencil (the block right above b and the four blocks
 *   sharing a face with that block, bench z-1, clipped at the grid edges),
 *   or explicit predecessor lists (MPS_PREC_CSR);
 *   S geological scenarios give block values v[s][b] ($) and ore indicators
 *   ore[s][b] (block processed in scenario s); ton[b] is the block tonnage.
 *
 * Objective of a schedule (the expectation of Eq. 14, risk-adjusted, with the
 * capacity constraints of Eq. 16 and of the processing plant as penalties):
 *   d(t) = (1+rate)^-t for t < T, d(T) = 0       (Alg. 5 discounts by 1.08^-t)
 *   N_s  = sum_b v[s][b] d(p_b),  mu = mean_s N_s,  sigma = population std
 *   O[s][t] = sum_{b: p_b=t} ton_b ore[s][b],  M[t] = sum_{b: p_b=t} ton_b
 *   J = mu - lambda*sigma - pen_proc/S * sum_{s,t<T} max(0, O[s][t] - proc_cap)
 *                         - pen_mine   * sum_{t<T}   max(0, M[t]    - mine_cap)
 *
 * A move (b, t') sets p[b] = t'.  Its score is J(p') - J(p); its flags are
 *   MPS_PREC_OK  every predecessor a has p[a] <= t', every successor c has t' <= p[c]
 *   MPS_MINE_OK  t' == T or t' == p[b] or M[t'] + ton_b <= mine_cap
 *   MPS_PROC_OK  t' == T or t' == p[b] or, for every s with ore[s][b],
 *                O[s][t'] + ton_b <= proc_cap
 *   MPS_NOOP     t' == p[b]               (score exactly 0)
 *   MPS_BAD      b outside [0,N) or t' outside [0,T] (score = -FLT_MAX)
 * This is the per-candidate precedence / capacity / value evaluation of the
 * paper's Alg. 5, made exact and extended to every destination period.
 *
 * Conventions.  Every call returns an mps_status; nothing throws across the
 * ABI.  On a non-OK status mps_last_error() returns a thread-local message.
 * Array arguments are DEVICE pointers owned by the caller unless stated
 * otherwise; scalars and structs are host memory.  Calls taking a `stream`
 * (a hipStream_t; NULL = the default stream) enqueue asynchronously and
 * neither allocate nor synchronise, unless their comment says otherwise.
 * Host-detectable argument errors return MPS_E_INVALID_ARG before any work
 * is enqueued.  Data errors found on the device never abort: they are
 * reported in outputs (BAD flags, violation counts). */
#ifndef MPS_H
#define MPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPS_OK = 0,
    MPS_E_INVALID_ARG = 1,
    MPS_E_OUT_OF_MEMORY = 2,
    MPS_E_DEVICE = 3,
    MPS_E_INFEASIBLE = 4,
    MPS_E_NOT_CAPTURABLE = 5,
    MPS_E_INTERNAL = 6
} mps_status;

enum {
    MPS_PREC_OK = 1,
    MPS_MINE_OK = 2,
    MPS_PROC_OK = 4,
    MPS_NOOP = 8,
    MPS_BAD = 16
};

/* Limits enforced by the host checks. */
#define MPS_MAX_PERIODS 126          /* T; periods are int8 with T = never */
#define MPS_MAX_SCENARIOS 4096       /* S */
#define MPS_MAX_TOPK 8192            /* k of mps_topk / mps_rank_moves */
#define MPS_MAX_BATCH_TOPK 1024      /* k of a batch (per model) */
#define MPS_MAX_BATCH 4096           /* models in one batch */
#define MPS_MAX_REPAIR_SCENARIOS 1024 /* S of mps_repair and mps_search */

typedef struct mps_model mps_model;

/* Precedence of a model (Eq. 15's predecessor sets):
 *   MPS_PREC_GRID_1_5  the 1-5 slope stencil of the grid (the default);
 *   MPS_PREC_CSR       explicit predecessor lists given to mps_build_model:
 *                      the predecessors of b are pred_idx[pred_ptr[b] ..
 *                      pred_ptr[b+1]), at most MPS_MAX_DEGREE of them, and no
 *                      block has more than MPS_MAX_DEGREE successors. */
#define MPS_PREC_GRID_1_5 0
#define MPS_PREC_CSR 1
#define MPS_MAX_DEGREE 9

typedef struct {
    int32_t nx, ny, nz;      /* grid; N = nx*ny*nz >= 1 */
    int32_t n_scen;          /* S, 1..MPS_MAX_SCENARIOS */
    int32_t n_periods;       /* T, 1..MPS_MAX_PERIODS; destination T = never */
    int32_t precedence;      /* MPS_PREC_GRID_1_5 or MPS_PREC_CSR */
    double discount_rate;    /* per period, > -1 (0.08 in the paper) */
    double lambda;           /* weight of the std, finite */
    double pen_proc;         /* $ per tonne of processing excess, >= 0 */
    double pen_mine;         /* $ per tonne of mining excess, >= 0 */
    double proc_cap;         /* tonnes per period */
    double mine_cap;         /* tonnes per period */
} mps_params;

typedef struct {
    double mu, sigma, R, Pp, Pm, J;  /* R = mu - lambda*sigma, J = R - Pp - Pm */
    int64_t n_prec_viol;             /* predecessor pairs with p[a] > p[b] */
} mps_objective;

/* A set of moves.  exhaustive != 0: move i is (i / D, i % D) for
 * i in [0, N*D), D = T+1 if include_never else T (block, period ignored).
 * Otherwise the n moves (block[i], period[i]) given as device arrays. */
typedef struct {
    int32_t exhaustive;
    int32_t include_never;
    int64_t n;
    const int32_t *block;
    const int8_t *period;
} mps_moves;

/* Penalty weights of the relaxed objective (see mps_relaxed_fwd). */
typedef struct {
    double mu_proc, mu_mine, mu_prec;
} mps_relax_params;

/* Thread-local text of the last error ("" if none). */
const char *mps_last_error(void);

/* ABI version (major*100 + minor). */
int32_t mps_version(void);

/* Number of visible GPUs; MPS_E_DEVICE (and *n = 0) when there is none. */
mps_status mps_device_count(int32_t *n);

/* Build a model from device arrays on the current device (Sec. 5 parameters):
 *   v        float [S][N]     block values, scenario-major;
 *   ore_bits uint32 [ceil(S/32)][N]; scenario s is bit s%32 of word s/32;
 *   ton      double [N]       tonnages, > 0;
 *   pred_ptr int32 [N+1], pred_idx int32 [pred_ptr[N]]: HOST arrays, the
 *            predecessor lists of MPS_PREC_CSR (Eq. 15's sets; each list
 *            without repeats or b itself, indices in [0,N)); NULL with
 *            MPS_PREC_GRID_1_5.  The successor lists are derived.
 * Invalid lists (bad pointers or indices, a repeat, a self loop, more than
 * MPS_MAX_DEGREE predecessors or successors) return MPS_E_INVALID_ARG.
 * The model copies what it keeps (the caller may free its arrays afterwards),
 * derives per-block statistics, allocates every buffer later calls need, and
 * starts with the schedule "everything in period 0".  Synchronises `stream`.
 * Not capturable. */
mps_status mps_build_model(const mps_params *prm, const float *v,
                           const uint32_t *ore_bits, const double *ton,
                           const int32_t *pred_ptr, const int32_t *pred_idx,
                           void *stream, mps_model **out);

/* Free a model and its device memory (synchronises the device). */
mps_status mps_destroy_model(mps_model *m);

/* Problem size of a model. */
mps_status mps_model_dims(const mps_model *m, int64_t *N, int32_t *S, int32_t *T);

/* Load schedule p (device int8 [N], values 0..T) and derive the state
 * (per-scenario NPV, period tonnages, penalty tables).  Values outside
 * 0..T are clamped to T and counted as violations in mps_get_objective. */
mps_status mps_set_schedule(mps_model *m, const int8_t *p, void *stream);

/* Copy the model's current schedule into p (device int8 [N]). */
mps_status mps_get_schedule(mps_model *m, int8_t *p, void *stream);

/* Objective of the current schedule into a HOST struct (synchronises). */
mps_status mps_get_objective(mps_model *m, mps_objective *out, void *stream);

/* Objective terms of the current schedule into DEVICE memory
 * (double[7]: mu, sigma, R, Pp, Pm, J, n_prec_viol); capturable. */
mps_status mps_objective_async(mps_model *m, double *out, void *stream);

/* Search state: the schedule and everything derived from it (per-scenario
 * NPV, period tonnages, objective terms, penalty tables) occupy one device
 * region of mps_state_bytes(m) bytes.  mps_state_save copies it into `buf`
 * (device, caller-owned), mps_state_restore copies such a buffer back: a
 * checkpoint of the search that is restored without re-reading the block
 * values.  A buffer restores only into the model it was saved from (or one
 * built from the same inputs).  Capturable (device-to-device copies). */
size_t mps_state_bytes(const mps_model *m);
mps_status mps_state_save(mps_model *m, void *buf, void *stream);
mps_status mps_state_restore(mps_model *m, const void *buf, void *stream);

/* Evaluate moves against the current schedule (Alg. 5, every destination):
 *   score  float [n_moves]  J(p') - J(p), FP32 arithmetic on FP64 state;
 *   flags  uint8 [n_moves]  MPS_* bits;
 *   d_risk, d_pen_proc, d_pen_mine  float [n_moves] or NULL: the change of
 *          mu - lambda*sigma and of the two penalty terms (score =
 *          d_risk - d_pen_proc - d_pen_mine).
 * n_moves = N*D (exhaustive) or moves->n.  Output index = move index.
 * One 64-block tile's period tables stay on chip, so S and T together are
 * bounded by the LDS of a workgroup: about 12.6 KB + 864*T + 256*W + 8*T*W
 * bytes with W = ceil(S/32) (exhaustive; a little less for lists).  On a
 * 160 KB device that allows S = 4096 with T <= 62, or T = 126 with
 * S <= 1056.  Beyond it: MPS_E_INVALID_ARG, before any device work. */
mps_status mps_eval_moves(mps_model *m, const mps_moves *moves, float *score,
                          uint8_t *flags, float *d_risk, float *d_pen_proc,
                          float *d_pen_mine, void *stream);

/* Workspace bytes mps_topk needs for n items and k selected. */
size_t mps_topk_ws_bytes(int64_t n, int32_t k);

/* Top-k selection (the argmax reduction of Alg. 5 generalised to k):
 * keep items i with (flags[i] & require) == require and (flags[i] & forbid)
 * == 0 (NaN scores never qualify); order by score descending, then index
 * ascending; write the first min(k, #kept) to idx (int64 [k]) and top_score
 * (float [k], may be NULL), and that count to *count (device int32).
 * Entries past the count are set to -1 / -inf.  1 <= k <= MPS_MAX_TOPK,
 * 0 <= n < 2^31.  ws: device workspace of mps_topk_ws_bytes(n, k) bytes,
 * zero-filled by the caller before its first use; every call leaves it ready
 * for the next (a workspace is reusable for any n and k it is large enough
 * for).  Calls that share a workspace must not overlap. */
mps_status mps_topk(const float *score, const uint8_t *flags, int64_t n,
                    int32_t k, uint8_t require, uint8_t forbid, int64_t *idx,
                    float *top_score, int32_t *count, void *ws,
                    size_t ws_bytes, void *stream);

/* mps_topk for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same selection and outputs, with the workspace in a device array the
 * library owns (33 MiB per device, held until the process ends)
 * instead of a caller buffer.  Limits: 0 <= n <= 2^21 (2,097,152 items),
 * 1 <= k <= MPS_MAX_TOPK; beyond them MPS_E_INVALID_ARG before any work.
 * Runs on the current device; allocates nothing.  Every call on one device
 * shares that device's array: calls that overlap in time on one device
 * (another stream, another thread) race and must be serialised by the
 * caller. */
mps_status mps_topk_noalloc(const float *score, const uint8_t *flags, int64_t n,
                            int32_t k, uint8_t require, uint8_t forbid, int64_t *idx,
                            float *top_score, int32_t *count, void *stream);

/* Greedy repair (Alg. 4 amortised over an ordered candidate list): walk the
 * candidates idx[0 .. *count) (device int32 count, at most max_cand) that
 * index into `moves`, in order; skip a block already moved in this call;
 * re-check precedence and re-score the move exactly (FP64) against the
 * current schedule and state; apply it iff PREC_OK (and MINE_OK and PROC_OK
 * when hard_capacity != 0) and its score is > 0, updating the schedule and
 * state in place.  *applied (device int32, may be NULL) receives the number
 * of applied moves.  The state is held on chip during the walk: the call
 * returns MPS_E_INVALID_ARG when S > MPS_MAX_REPAIR_SCENARIOS or when
 * 8*(T+1)*S rounded up to 4 (O rows) + 16*(T+1) + 2*max_cand (period map) +
 * two batches of candidate records (up to 40 KB each) exceed one workgroup's
 * LDS; max_cand <= MPS_MAX_TOPK.  Calls on one model must not overlap. */
mps_status mps_repair(mps_model *m, const mps_moves *moves,
                      const int64_t *idx, const int32_t *count,
                      int32_t max_cand, int32_t hard_capacity,
                      int32_t *applied, void *stream);

/* Cascading repair (Alg. 4 with its fallback): as mps_repair, except that a
 * candidate (b, t') precedence forbids is not skipped but moved together with
 * the blocks that forbid it -- for t' < p[b] every ancestor reached through
 * predecessors with p > t', for t' > p[b] every descendant reached through
 * successors with p < t' -- all set to t' as one composite move.  The
 * composite is scored exactly (FP64: every N'_s, mu', sigma' and the hinge
 * terms of every period the set leaves or enters) and applied iff the set
 * has at most max_set blocks (1..256), none of them was moved earlier in this
 * call, Eq. 15 holds at every moved block of the result, (hard_capacity) the
 * mining and processing tonnages of t' stay within their capacities, and the
 * score is > 0.  A candidate that needs no companions is the plain repair's
 * move.  *applied (device int32, may be NULL) receives the number of applied
 * (composite) moves; the state is re-derived from the schedule at the end.
 * The walk keeps 8*(T*S + 2S + 2T + 1) bytes of state in one workgroup's LDS,
 * else MPS_E_INVALID_ARG.  Capturable; calls on one model must not overlap. */
mps_status mps_repair_cascade(mps_model *m, const mps_moves *moves, const int64_t *idx,
                              const int32_t *count, int32_t max_cand, int32_t hard_capacity,
                              int32_t max_set, int32_t *applied, void *stream);

/* ---- relaxed, differentiable schedule ------------------------------------
 * x (device float [N][T]) is the cumulative fraction of each block mined by
 * the end of each period, y[b,t] = x[b,t] - x[b,t-1] (x[b,-1] = 0); the caller
 * keeps x in [0,1] and non-decreasing in t.  The relaxed objective is the
 * risk-adjusted expectation of Eq. 14 on the relaxed plan with quadratic
 * penalties for the capacities (Eq. 16 and the plant) and for precedence
 * (Eq. 15):
 *   NPV_s = sum_b v[s][b] sum_t d(t) y[b,t];  mu, sigma over s
 *   Ot[s,t] = sum_b ton_b ore[s][b] y[b,t],  Mt[t] = sum_b ton_b y[b,t]
 *   J = mu - lambda*sigma - (mu_proc/S) sum_{s,t} max(0, Ot - proc_cap)^2
 *       - mu_mine sum_t max(0, Mt - mine_cap)^2
 *       - mu_prec sum_b sum_{a in Pred(b)} sum_t max(0, x[b,t] - x[a,t])^2
 * At an integer point x[b,t] = [t >= p_b] of a feasible schedule with
 * mu_proc = mu_mine = 0, J equals mu - lambda*sigma of mps_get_objective. */

/* Device bytes of the state the forward pass saves for the backward pass. */
size_t mps_relaxed_saved_bytes(const mps_model *m);

/* Forward: J_out (device double[6] or NULL) = J, mu, sigma, proc penalty,
 * mining penalty, precedence penalty; `saved` (device, caller-owned,
 * mps_relaxed_saved_bytes) receives what the backward pass needs.  Uses the
 * model's workspace: calls on one model must not overlap. */
mps_status mps_relaxed_fwd(mps_model *m, const float *x, const mps_relax_params *rp,
                           double *J_out, void *saved, void *stream);

/* Adjoint: grad_x (device float [N][T]) = dJ * dJ/dx at x, from the state a
 * forward call at the same x saved.  dJ: device double scalar, or NULL for 1.
 * The derivative of sigma uses w_s = 1/S - lambda (NPV_s - mu)/(S sigma), and
 * 1/S when sigma <= 1e-12 * max(1, |mu|). */
mps_status mps_relaxed_bwd(mps_model *m, const float *x, const mps_relax_params *rp,
                           const void *saved, const double *dJ, float *grad_x,
                           void *stream);

/* Workspace bytes of mps_rank_moves for k moves. */
size_t mps_rank_ws_bytes(const mps_model *m, int32_t k);

/* Gradient ranking of every non-no-op move (b, t') that keeps the current
 * schedule precedence-feasible (Eq. 15; the others could never be applied):
 * gain = Gc[b][p_b] - Gc[b][t'] with Gc[b][t] = sum_{u<t} grad_x[b][u]
 * (the first-order change of J along x(p') - x(p)); returns the k best
 * (gain descending, move index b*(T+1)+t' ascending) as block (int32 [k]),
 * period (int8 [k]), gain (float [k], may be NULL) and *count (device int32);
 * entries past the count are -1.  1 <= k <= MPS_MAX_TOPK.  ws: device
 * workspace of mps_rank_ws_bytes(m, k) bytes, zero-filled by the caller
 * before its first use (every call leaves it ready for the next). */
mps_status mps_rank_moves(mps_model *m, const float *grad_x, int32_t k, int32_t *block,
                          int8_t *period, float *gain, int32_t *count, void *ws,
                          size_t ws_bytes, void *stream);

/* Search loops from the current schedule (the repair-driven local search the
 * paper's Alg. 2 and 4 run around the GPU evaluation):
 *   mode 0 (exhaustive): repeat { evaluate all N(T+1) moves, top k, repair }
 *     until a repair applies nothing;
 *   mode 1 (gradient-ranked): repeat { relaxed gradient at x(p), rank all
 *     moves, evaluate the top k exactly, top k, repair }; when a round applies
 *     nothing, one exhaustive round certifies (and the loop continues if it
 *     applied something).
 * ALLOCATES its buffers and SYNCHRONISES every round (not capturable).
 * S <= MPS_MAX_REPAIR_SCENARIOS, and S and T must fit the LDS bound of
 * mps_eval_moves; otherwise MPS_E_INVALID_ARG before any device work. */
typedef struct {
    int64_t iterations;    /* rounds run */
    int64_t evaluations;   /* moves evaluated exactly (eval calls) */
    int64_t applied;       /* moves applied */
    double J;              /* objective of the final schedule */
} mps_search_stats;

mps_status mps_search(mps_model *m, int32_t mode, int32_t k, const mps_relax_params *rp,
                      int32_t max_iter, mps_search_stats *out, void *stream);

/* ---- objective variants ---------------------------------------------------
 * Two variants of the objective, set per model:
 *   value multiplier (Eq. 12): a block mined in period t is worth
 *     sigma(s,t) * v[s][b] in scenario s, so N_s = sum_b v[s][b] sigma(s,p_b) d(p_b);
 *   risk measure: MPS_RISK_STD gives R = mu - lambda*sigma; MPS_RISK_CVAR gives
 *     R = mu - lambda*(mu - CVaR_alpha(N)), where CVaR_alpha is the mean of the
 *     lower alpha tail of the scenario NPVs: with them sorted ascending and
 *     k = ceil(alpha*S), (sum of the k-1 smallest + (alpha*S - k + 1) * the
 *     k-th smallest) / (alpha*S)  (alpha = 0.1 is the paper's CVaR10).
 * mult: HOST double [S][T] (read during the call) or NULL for sigma = 1.
 * The state of the current schedule is re-derived (synchronises; not
 * capturable).  mps_get_objective, mps_set_schedule and mps_eval_moves then
 * follow the variant (evaluation: S <= 1024 and 8*T*S + 4*S*(T+1) bytes of
 * tables in one workgroup's LDS, else MPS_E_INVALID_ARG); every call built
 * on the base objective's arithmetic (repair, cascading repair, search,
 * relaxed objective, ranking, greedy initializer, batches) returns
 * MPS_E_INVALID_ARG while a variant is set.  mult = NULL with MPS_RISK_STD
 * restores the base objective. */
#define MPS_RISK_STD 0
#define MPS_RISK_CVAR 1
mps_status mps_set_objective_variant(mps_model *m, const double *mult, int32_t risk,
                                     double cvar_alpha, void *stream);

/* Greedy initializer (Alg. 3 with every uncertainty factor equal to 1):
 * replaces the model's schedule by the one built greedily from "nothing
 * mined".  Blocks are taken in descending expected value mean_s v[s][b] (ties:
 * smaller index); each is placed in the earliest period t < T that keeps the
 * partial schedule precedence-feasible (every predecessor already placed in t
 * or earlier; an unplaced block counts as never mined) and both capacities
 * hard (M[t] + ton_b <= mine_cap; O[s][t] + ton_b <= proc_cap in every
 * scenario in which b is ore), or stays unplaced (period T).  Passes over the
 * unplaced blocks, in the same order, repeat until one places nothing or
 * max_pass passes ran.  *passes and *placed (host, may be NULL) receive the
 * pass count and the number of placed blocks; the model's state is derived
 * from the result.  ALLOCATES its workspace and SYNCHRONISES (not
 * capturable).  The period tonnages are kept on chip: 8*(T*S + T) bytes
 * must fit one workgroup's LDS, else MPS_E_INVALID_ARG. */
mps_status mps_greedy_init(mps_model *m, int32_t max_pass, int32_t *passes, int64_t *placed,
                           void *stream);

/* LNS + simulated-annealing driver (Alg. 2 without its GA and RL parts).
 * Neighbourhoods are the tile x tile block columns of the grid (every bench),
 * in row-major tile order; n_tiles = ceil(nx/tile) * ceil(ny/tile).  One step
 * on neighbourhood i of iteration it:
 *   destroy: the tile's blocks and every descendant of them go to "never";
 *   repair: up to max_rounds rounds of { evaluate every move (b, t < T) of the
 *     destroyed blocks (b ascending, then t), top k (PREC_OK required, NOOP
 *     and BAD forbidden), greedy repair (mps_repair) }, stopping after a round
 *     that applies nothing;
 *   eps-relaxed fitness: f = R - max(0, Pp + Pm - eps), eps = eps_max *
 *     (1 - it/n_iter) (linear; f = J at eps = 0);
 *   acceptance: the candidate becomes the current schedule iff
 *     f(cand) > f(cur) - u[it*n_tiles + i] * temp0 * cool^it.
 * u: HOST double [n_iter * n_tiles], the caller's uniform draws in [0,1).
 * traj: HOST double [n_iter * n_tiles][4] or NULL: J, R, Pp + Pm of each
 * candidate and 1/0 accepted.  The model ends at the best schedule by J seen
 * (the input included).  ALLOCATES and SYNCHRONISES every step (not
 * capturable).  Limits as mps_search. */
typedef struct {
    int32_t n_iter, tile, k, max_rounds;
    double eps_max, temp0, cool;
} mps_lns_params;

typedef struct {
    int64_t steps, accepted, evaluations, applied;
    double J_best;
} mps_lns_stats;

mps_status mps_lns_sa(mps_model *m, const mps_lns_params *prm, const double *u, double *traj,
                      mps_lns_stats *out, void *stream);

/* ---- batched evaluation ---------------------------------------------------
 * Many models (for instance, one schedule per individual of the population
 * the metaheuristic of Alg. 2 keeps), each with its own list of candidate
 * moves of any length, are evaluated by persistent workgroups and end with
 * every model's exact top k.  Three persistent launches each take work
 * items from an atomic counter, largest model first: per-block passes over
 * each model's block values, then chunks of each model's moves, then one
 * top-k selection per model.  Results equal those of mps_eval_moves on each
 * model's list followed by mps_topk with the same k, require and forbid.
 *
 * Tuning: how the work of one model is cut into items, set per model (the
 * autotuner sets it per class of models with the same S range). */
typedef struct {
    int32_t tiles_per_item;   /* 64-block tiles per block-pass item, 1..64 */
    int32_t moves_per_item;   /* moves per move item: a multiple of 512 in 512..65536 */
    int32_t rows;             /* block values each lane has in flight: 8, 16 or 32 */
    int32_t reserved;         /* must be 0 */
} mps_tuning;

/* One model's part of a batch (device pointers, caller-owned). */
typedef struct {
    const int32_t *block;     /* [n] moved block */
    const int8_t *period;     /* [n] destination period 0..T */
    int64_t n;                /* 0 <= n < 2^31 */
    float *score;             /* [n] out: as mps_eval_moves */
    uint8_t *flags;           /* [n] out */
    int64_t *top_idx;         /* [k] out: positions in this model's list, -1 past the count */
    float *top_score;         /* [k] out or NULL */
    int32_t *top_count;       /* out: device int32 */
} mps_batch_item;

typedef struct mps_batch mps_batch;

/* Build a batch over n_models models (all on one device; they must outlive
 * the batch) and their move lists.  Allocates the descriptor table, the work
 * queue, the counters and, per model, the order in which its moves are
 * scored (4 bytes per move: within each move item, the positions sorted by
 * moved block, so that neighbouring lanes read neighbouring blocks' data).
 * Every move is scored once and its results stay at its own position, so a
 * move list that changes after this call still gives exact results; only the
 * locality is lost until mps_batch_set_tuning recomputes the order.  The
 * tuning of each model comes from the process
 * tuning cache (filled by mps_batch_autotune) or from defaults.  Two batches
 * that share a model must not run at the same time (they share its block
 * workspace), nor may a batch run concurrently with mps_eval_moves in list
 * mode on one of its models.  Synchronises; not capturable.
 * 1 <= n_models <= MPS_MAX_BATCH, 1 <= k <= MPS_MAX_BATCH_TOPK. */
mps_status mps_batch_create(mps_model *const *models, const mps_batch_item *items,
                            int32_t n_models, int32_t k, uint8_t require, uint8_t forbid,
                            mps_batch **out);
mps_status mps_batch_destroy(mps_batch *b);

/* Set the tuning of model i (or of every model when i = -1), or read it.
 * Rebuilds the work queue (synchronises).  Invalid values: MPS_E_INVALID_ARG. */
mps_status mps_batch_set_tuning(mps_batch *b, int32_t i, const mps_tuning *t);
mps_status mps_batch_get_tuning(const mps_batch *b, int32_t i, mps_tuning *t);

/* Resident workgroups of the persistent launch: 0 = as many as fit on the
 * device at once (the default), otherwise 1 .. that number. */
mps_status mps_batch_set_workgroups(mps_batch *b, int32_t n);

/* Enqueue the batch on `stream`: one small clearing kernel (no memset) and
 * the three persistent launches.  Capturable.  Calls on one batch must not
 * overlap. */
mps_status mps_batch_run(mps_batch *b, void *stream);

/* The same work replayed as a HIP graph: the first call captures
 * mps_batch_run into a graph (on a stream of the batch's own) and
 * instantiates it; every call then launches that graph on `stream`.  A
 * tuning or workgroup change drops the graph.  Not capturable itself. */
mps_status mps_batch_graph_launch(mps_batch *b, void *stream);

/* Autotune: for each class of models (S <= 32, <= 64, <= 128, > 128) try
 * the candidate values of rows, tiles_per_item and moves_per_item in turn
 * (coordinate descent), then the workgroup count, timing `reps` runs of the
 * whole batch per candidate with HIP events (median); keep the fastest,
 * apply it and store it in the process tuning cache.  The batch's outputs
 * hold the results of its last timed run.  Synchronises; not capturable.
 * *best_us (may be NULL) receives the median time of the chosen tuning. */
mps_status mps_batch_autotune(mps_batch *b, int32_t reps, double *best_us, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MPS_H */
