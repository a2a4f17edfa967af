/* oracle.h -- plain FP64 CPU reference of the candidate-move evaluation
 * method.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU
 * baseline leg of the benchmark call it; the product library never does.
 * It shares no code, header or table with the HIP library.
 *
 * Problem statement followed (Sec. 5, Eq. 14-16):
 *   a schedule p[b] in {0..T-1} gives the period in which block b is mined;
 *   p[b] = T means "never mined" (contributes no value and no tonnage);
 *   precedence (Eq. 15): every predecessor a of b satisfies p[a] <= p[b];
 *   mining capacity (Eq. 16): tonnage mined per period <= Mcap.
 * The risk-adjusted objective (mean - lambda*std over scenarios of the
 * discounted NPV) and the capacity penalties are the readings documented in
 * the design notes; each function below restates what it computes. */
#ifndef MPS_ORACLE_H
#define MPS_ORACLE_H
#include <stdint.h>

#define OR_PREC_OK 1
#define OR_MINE_OK 2
#define OR_PROC_OK 4
#define OR_NOOP    8
#define OR_BAD     16

typedef struct {
    int32_t nx, ny, nz;   /* N = nx*ny*nz, b = x + nx*(y + ny*z), z = 0 top */
    int32_t S, T;         /* scenarios, periods (T = never) */
    double rate;          /* discount rate per period */
    double lambda;        /* risk weight on the std */
    double pen_proc;      /* $ per tonne of processing excess (scenario mean) */
    double pen_mine;      /* $ per tonne of mining excess */
    double pcap, mcap;    /* processing / mining capacity, tonnes per period */
    const float *v;       /* [S][N] block values */
    const uint8_t *ore;   /* [S][N] 0/1: processed in that scenario */
    const double *ton;    /* [N] tonnage */
    /* General precedence (the sets beta_b^Pred of Eq. 15 given explicitly):
     * the predecessors of b are pred_idx[pred_ptr[b] .. pred_ptr[b+1]), its
     * successors succ_idx[succ_ptr[b] .. succ_ptr[b+1]) (the transpose, from
     * or_successor_csr).  All four NULL: the 1-5 slope stencil of the grid.
     * At most OR_MAX_DEG of each per block. */
    const int32_t *pred_ptr, *pred_idx, *succ_ptr, *succ_idx;
    /* Objective variants.  mult [S][T] (NULL: all 1) multiplies the value of
     * a block mined in period t under scenario s (Eq. 12's sigma(s,t)).
     * risk 0: R = mu - lambda*sigma; risk 1: R = mu - lambda*(mu - CVaR),
     * CVaR the mean of the worst alpha share of the scenario NPVs (lower
     * tail, fractional weight on the boundary scenario). */
    const double *mult;
    int32_t risk;
    double alpha;
} or_inst;

#define OR_MAX_DEG 9

typedef struct {
    double mu, sigma, R, Pp, Pm, J;
    int64_t n_prec_viol;
} or_objective_t;

typedef struct {
    double mu_proc, mu_mine, mu_prec;  /* quadratic penalty weights */
} or_relax_t;

void or_discount(int32_t T, double rate, double *d /* [T+1] */);
int32_t or_predecessors(const or_inst *I, int32_t b, int32_t *out /* [OR_MAX_DEG] */);
int32_t or_successors(const or_inst *I, int32_t b, int32_t *out /* [OR_MAX_DEG] */);

/* Successor lists of a predecessor CSR: c is a successor of b iff b is a
 * predecessor of c; each list in increasing c.  succ_ptr [N+1], succ_idx
 * [pred_ptr[N]]. */
void or_successor_csr(int64_t N, const int32_t *pred_ptr, const int32_t *pred_idx,
                      int32_t *succ_ptr, int32_t *succ_idx);

/* CVaR of the lower alpha tail of x [n]: with x sorted ascending and
 * k = ceil(alpha*n), (sum_{i<k-1} x_(i) + (alpha*n - k + 1) x_(k-1)) / (alpha*n). */
double or_cvar(const double *x, int32_t n, double alpha);

/* Full objective of schedule p.  Ns [S], O [S][T], M [T] may be NULL. */
void or_objective(const or_inst *I, const int8_t *p, or_objective_t *out,
                  double *Ns, double *O, double *M);

/* Move evaluation.  exhaustive != 0: moves are b*D + t' for b in [0,N),
 * t' in [0,D), D = T+1 if include_never else T (block/period ignored);
 * otherwise the n listed moves.  Outputs have one entry per move; dR, dPp,
 * dPm may be NULL.  n_threads <= 0 means "all available". */
void or_eval_moves(const or_inst *I, const int8_t *p, int32_t exhaustive,
                   int32_t include_never, int64_t n, const int32_t *block,
                   const int8_t *period, double *score, uint8_t *flags,
                   double *dR, double *dPp, double *dPm, int32_t n_threads);

/* J(p') - J(p) by two full re-scorings (brute force). */
double or_eval_bruteforce(const or_inst *I, const int8_t *p, int32_t b, int32_t t);

/* Top-k: keep (flags & req) == req and (flags & forbid) == 0, order by
 * score descending then move index ascending, return the first k. */
int32_t or_topk(const double *score, const uint8_t *flags, int64_t n, int32_t k,
                uint8_t req, uint8_t forbid, int64_t *idx, double *top_score);

/* Greedy repair over an ordered candidate list; p is updated in place.
 * Returns the number of applied moves; J_out receives J of the result. */
int32_t or_repair(const or_inst *I, int8_t *p, int32_t n_cand,
                  const int32_t *cand_block, const int8_t *cand_period,
                  int32_t hard_capacity, double *J_out, uint8_t *accepted);

/* Cascading repair: as or_repair, but a candidate precedence forbids moves
 * together with the ancestors (moving earlier) or descendants (moving later)
 * that forbid it, as one composite move to the same period, scored exactly;
 * sets larger than max_set blocks are skipped.  set_size [n_cand] (may be
 * NULL) receives each candidate's set size (0: skipped before forming it,
 * -1: too large). */
int32_t or_repair_cascade(const or_inst *I, int8_t *p, int32_t n_cand,
                          const int32_t *cand_block, const int8_t *cand_period,
                          int32_t hard_capacity, int32_t max_set, double *J_out,
                          uint8_t *accepted, int32_t *set_size);

/* Relaxed objective of a cumulative schedule x [N][T]; grad (may be NULL)
 * receives dJ/dx [N][T]. */
double or_relaxed(const or_inst *I, const float *x, const or_relax_t *rp,
                  double *grad);
double or_relaxed_d(const or_inst *I, const double *x, const or_relax_t *rp,
                    double *grad);

/* Gradient ranking: first-order gain of every non-no-op move at schedule p
 * that keeps p precedence-feasible (Eq. 15: every predecessor a has
 * p[a] <= t', every successor c has t' <= p[c]), from the gradient at x(p);
 * returns the top k (gain desc, index asc). */
int32_t or_rank_moves(const or_inst *I, const int8_t *p, const double *grad,
                      int32_t k, int32_t *block, int8_t *period, double *gain);

/* Search loops.  mode 0: exhaustive, mode 1: gradient-ranked.  p is updated
 * in place; stats[0] = iterations, stats[1] = exact move evaluations,
 * stats[2] = applied moves.  Returns J of the final schedule. */
double or_search(const or_inst *I, int8_t *p, int32_t mode, int32_t k,
                 const or_relax_t *rp, int32_t max_iter, int64_t *stats,
                 int32_t n_threads);

/* Greedy initializer (Alg. 3, uncertainty factors 1): p [N] receives the
 * schedule built by placing blocks in descending expected value at their
 * earliest period that keeps precedence and both hard capacities, in passes
 * until a pass places nothing (at most max_pass).  Returns the number of
 * passes; *n_placed (may be NULL) the number of blocks placed. */
int32_t or_greedy_init(const or_inst *I, int8_t *p, int32_t max_pass, int64_t *n_placed);

/* LNS + simulated annealing driver (Alg. 2 without GA and RL): n_iter
 * iterations over the nb x nb column tiles; each step destroys a tile and its
 * descendants, repairs with up to max_rounds rounds of list evaluation, top k
 * and greedy repair, and accepts the candidate iff
 * f(cand) > f(cur) - u temp0 cool^it with f = R - max(0, Pp + Pm - eps),
 * eps = eps_max (1 - it/n_iter).  u [n_iter * tiles] are the uniform draws.
 * p receives the best schedule by J; returns its J.  traj [steps][4] (may be
 * NULL): J, R, P of each candidate and 1/0 accepted; stats [4]: steps,
 * accepted, moves evaluated, moves applied. */
double or_lns_sa(const or_inst *I, int8_t *p, int32_t n_iter, int32_t nb, int32_t k,
                 int32_t max_rounds, double eps_max, double temp0, double cool,
                 const double *u, double *traj, int64_t *stats, int32_t n_threads);

/* Exhaustive optimum over every precedence-feasible schedule (tiny grids).
 * Returns J*; p_best gets the lexicographically smallest maximiser;
 * *n_feasible the number of feasible schedules.  Every predecessor must have
 * a smaller index than its successor (true of the grid stencil); otherwise
 * NaN is returned. */
double or_optimum(const or_inst *I, int8_t *p_best, int64_t *n_feasible);

#endif
