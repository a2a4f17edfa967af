/* oracle.c -- plain FP64 CPU reference of the candidate-move evaluation
 * method.  TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the
 * benchmark); the product library never links or calls it.
 *
 * Everything is written as the literal definition: no rank-1 shortcuts, no
 * tiling, no reordering.  Each move re-derives every per-scenario NPV and the
 * mean and standard deviation from scratch; each penalty difference re-derives
 * the hinge terms it touches.  Citations are to the paper's sections,
 * equations and algorithms. */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t n_blocks(const or_inst *I) {
    return (int64_t)I->nx * I->ny * I->nz;
}

static double val(const or_inst *I, int32_t s, int32_t b) {
    return (double)I->v[(int64_t)s * n_blocks(I) + b];
}

static int ore(const or_inst *I, int32_t s, int32_t b) {
    return I->ore[(int64_t)s * n_blocks(I) + b] != 0;
}

/* Discount factor of each period (Alg. 5 discounts period t by 1/1.08^t; the
 * first period is undiscounted).  Built by repeated division so that no
 * library power function is involved; d(T) = 0 for "never mined". */
void or_discount(int32_t T, double rate, double *d) {
    d[0] = 1.0;
    for (int32_t t = 1; t < T; ++t) d[t] = d[t - 1] / (1.0 + rate);
    d[T] = 0.0;
}

/* Direct predecessors (the set beta_b^Pred of Eq. 15): the given lists when
 * the instance carries them, else the 1-5 slope stencil: the block right
 * above b and the four blocks sharing a face with that block, all on the
 * bench above, clipped at the grid edges. */
int32_t or_predecessors(const or_inst *I, int32_t b, int32_t *out) {
    if (I->pred_ptr) {
        int32_t n = 0;
        for (int32_t k = I->pred_ptr[b]; k < I->pred_ptr[b + 1]; ++k) out[n++] = I->pred_idx[k];
        return n;
    }
    int32_t nx = I->nx, ny = I->ny;
    int32_t x = b % nx, y = (b / nx) % ny, z = b / (nx * ny);
    if (z == 0) return 0;
    static const int dx[5] = {0, -1, 1, 0, 0};
    static const int dy[5] = {0, 0, 0, -1, 1};
    int32_t n = 0;
    for (int k = 0; k < 5; ++k) {
        int32_t xa = x + dx[k], ya = y + dy[k];
        if (xa < 0 || xa >= nx || ya < 0 || ya >= ny) continue;
        out[n++] = xa + nx * (ya + ny * (z - 1));
    }
    return n;
}

/* Successors: every block c with b among the predecessors of c (the
 * transposed lists when the instance carries them). */
int32_t or_successors(const or_inst *I, int32_t b, int32_t *out) {
    if (I->pred_ptr) {
        int32_t n = 0;
        for (int32_t k = I->succ_ptr[b]; k < I->succ_ptr[b + 1]; ++k) out[n++] = I->succ_idx[k];
        return n;
    }
    int32_t nx = I->nx, ny = I->ny, nz = I->nz;
    int32_t x = b % nx, y = (b / nx) % ny, z = b / (nx * ny);
    int32_t n = 0;
    if (z + 1 >= nz) return 0;
    for (int32_t yc = y - 1; yc <= y + 1; ++yc)
        for (int32_t xc = x - 1; xc <= x + 1; ++xc) {
            if (xc < 0 || xc >= nx || yc < 0 || yc >= ny) continue;
            int32_t c = xc + nx * (yc + ny * (z + 1));
            int32_t pr[OR_MAX_DEG];
            int32_t np = or_predecessors(I, c, pr);
            for (int32_t k = 0; k < np; ++k)
                if (pr[k] == b) out[n++] = c;
        }
    return n;
}

void or_successor_csr(int64_t N, const int32_t *pred_ptr, const int32_t *pred_idx,
                      int32_t *succ_ptr, int32_t *succ_idx) {
    for (int64_t b = 0; b <= N; ++b) succ_ptr[b] = 0;
    for (int64_t c = 0; c < N; ++c)
        for (int32_t k = pred_ptr[c]; k < pred_ptr[c + 1]; ++k) ++succ_ptr[pred_idx[k] + 1];
    for (int64_t b = 0; b < N; ++b) succ_ptr[b + 1] += succ_ptr[b];
    int32_t *fill = malloc(sizeof(int32_t) * (N > 0 ? N : 1));
    for (int64_t b = 0; b < N; ++b) fill[b] = succ_ptr[b];
    for (int64_t c = 0; c < N; ++c)   /* increasing c: each list comes out sorted */
        for (int32_t k = pred_ptr[c]; k < pred_ptr[c + 1]; ++k)
            succ_idx[fill[pred_idx[k]]++] = (int32_t)c;
    free(fill);
}

/* Discounted multiplier of scenario s in period t: d(t) sigma(s,t), and 0
 * for "never" (Eq. 12 with the paper's discounting; sigma = 1 without a
 * multiplier table). */
static double wdisc(const or_inst *I, const double *d, int32_t s, int32_t t) {
    if (t >= I->T) return 0.0;
    return I->mult ? d[t] * I->mult[(int64_t)s * I->T + t] : d[t];
}

static int cmp_dbl(const void *pa, const void *pb) {
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a > b) - (a < b);
}

double or_cvar(const double *x, int32_t n, double alpha) {
    double *y = malloc(sizeof(double) * n);
    memcpy(y, x, sizeof(double) * n);
    qsort(y, (size_t)n, sizeof(double), cmp_dbl);
    double an = alpha * n;
    int32_t k = (int32_t)ceil(an);
    if (k < 1) k = 1;
    if (k > n) k = n;
    double acc = 0.0;
    for (int32_t i = 0; i < k - 1; ++i) acc += y[i];
    acc += (an - (k - 1)) * y[k - 1];
    free(y);
    return acc / an;
}

static void mean_std(const double *x, int32_t n, double *mu, double *sd) {
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s += x[i];
    double m = s / n;
    double q = 0.0;
    for (int32_t i = 0; i < n; ++i) q += (x[i] - m) * (x[i] - m);
    *mu = m;
    *sd = sqrt(q / n);
}

static double hinge(double x, double cap) { return x > cap ? x - cap : 0.0; }

/* Risk-adjusted value of the scenario NPVs: mu - lambda*sigma, or with the
 * CVaR measure mu - lambda*(mu - CVaR_alpha). */
static double risk_value(const or_inst *I, const double *Ns, double mu, double sd) {
    if (I->risk == 1) return mu - I->lambda * (mu - or_cvar(Ns, I->S, I->alpha));
    return mu - I->lambda * sd;
}

/* Per-scenario NPV, period tonnages and the objective (Eq. 14 expectation,
 * extended by the risk term and the capacity penalties):
 *   N_s = sum_b v[s,b] d(p_b),  mu = mean_s N_s,  sigma = population std,
 *   R = mu - lambda sigma,
 *   O[s,t] = sum_{b: p_b = t} ton_b ore[s,b],  M[t] = sum_{b: p_b = t} ton_b,
 *   Pp = pen_proc (1/S) sum_s sum_{t<T} max(0, O[s,t] - Pcap),
 *   Pm = pen_mine sum_{t<T} max(0, M[t] - Mcap),
 *   J = R - Pp - Pm. */
void or_objective(const or_inst *I, const int8_t *p, or_objective_t *out,
                  double *Ns_out, double *O_out, double *M_out) {
    int64_t N = n_blocks(I);
    int32_t S = I->S, T = I->T;
    double *d = malloc(sizeof(double) * (T + 1));
    double *Ns = malloc(sizeof(double) * S);
    double *O = calloc((size_t)S * T, sizeof(double));
    double *M = calloc((size_t)T, sizeof(double));
    or_discount(T, I->rate, d);
    for (int32_t s = 0; s < S; ++s) {
        double acc = 0.0;
        for (int64_t b = 0; b < N; ++b) acc += val(I, s, (int32_t)b) * wdisc(I, d, s, p[b]);
        Ns[s] = acc;
    }
    for (int64_t b = 0; b < N; ++b) {
        int32_t t = p[b];
        if (t >= T) continue;
        M[t] += I->ton[b];
        for (int32_t s = 0; s < S; ++s)
            if (ore(I, s, (int32_t)b)) O[(int64_t)s * T + t] += I->ton[b];
    }
    double mu, sd;
    mean_std(Ns, S, &mu, &sd);
    double pp = 0.0, pm = 0.0;
    for (int32_t s = 0; s < S; ++s)
        for (int32_t t = 0; t < T; ++t) pp += hinge(O[(int64_t)s * T + t], I->pcap);
    pp = I->pen_proc * pp / S;
    for (int32_t t = 0; t < T; ++t) pm += hinge(M[t], I->mcap);
    pm = I->pen_mine * pm;
    int64_t nv = 0;
    for (int64_t b = 0; b < N; ++b) {
        int32_t pr[OR_MAX_DEG];
        int32_t np = or_predecessors(I, (int32_t)b, pr);
        for (int32_t k = 0; k < np; ++k)
            if (p[pr[k]] > p[b]) ++nv;
    }
    out->mu = mu;
    out->sigma = sd;
    out->R = risk_value(I, Ns, mu, sd);
    out->Pp = pp;
    out->Pm = pm;
    out->J = out->R - pp - pm;
    out->n_prec_viol = nv;
    if (Ns_out) memcpy(Ns_out, Ns, sizeof(double) * S);
    if (O_out) memcpy(O_out, O, sizeof(double) * S * T);
    if (M_out) memcpy(M_out, M, sizeof(double) * T);
    free(d); free(Ns); free(O); free(M);
}

/* One move (b -> t) against the state (Ns, O, M) of schedule p.
 * Flags follow Eq. 15 (both directions, same period allowed) and Eq. 16 /
 * the processing capacity; the score is R(p') - R(p) minus the change of
 * both penalties, every term re-derived from its definition. */
static void eval_one(const or_inst *I, const int8_t *p, const double *Ns,
                     const double *O, const double *M, const double *d,
                     double mu, double sd, int32_t b, int32_t t, double *Np,
                     double *score, uint8_t *flags, double *dR_out,
                     double *dPp_out, double *dPm_out) {
    int64_t N = n_blocks(I);
    int32_t S = I->S, T = I->T;
    if (b < 0 || b >= N || t < 0 || t > T) {
        *flags = OR_BAD;
        *score = -(double)FLT_MAX;
        if (dR_out) *dR_out = 0.0;
        if (dPp_out) *dPp_out = 0.0;
        if (dPm_out) *dPm_out = 0.0;
        return;
    }
    int32_t pb = p[b];
    double ton = I->ton[b];
    uint8_t f = 0;
    if (t == pb) f |= OR_NOOP;

    int prec_ok = 1;
    int32_t nb[OR_MAX_DEG];
    int32_t n = or_predecessors(I, b, nb);
    for (int32_t k = 0; k < n; ++k)
        if (p[nb[k]] > t) prec_ok = 0;
    n = or_successors(I, b, nb);
    for (int32_t k = 0; k < n; ++k)
        if (t > p[nb[k]]) prec_ok = 0;
    if (prec_ok) f |= OR_PREC_OK;

    if (t == T || t == pb || M[t] + ton <= I->mcap) f |= OR_MINE_OK;

    int proc_ok = 1;
    if (t != T && t != pb)
        for (int32_t s = 0; s < S; ++s)
            if (ore(I, s, b) && O[(int64_t)s * T + t] + ton > I->pcap) proc_ok = 0;
    if (proc_ok) f |= OR_PROC_OK;

    /* Risk-adjusted expected NPV of p' from scratch. */
    for (int32_t s = 0; s < S; ++s)
        Np[s] = Ns[s] + val(I, s, b) * (wdisc(I, d, s, t) - wdisc(I, d, s, pb));
    double mu2, sd2;
    mean_std(Np, S, &mu2, &sd2);
    double dR = risk_value(I, Np, mu2, sd2) - risk_value(I, Ns, mu, sd);

    double dPp = 0.0, dPm = 0.0;
    if (t != pb) {
        double acc = 0.0;
        for (int32_t s = 0; s < S; ++s) {
            if (!ore(I, s, b)) continue;
            if (t < T) {
                double o = O[(int64_t)s * T + t];
                acc += hinge(o + ton, I->pcap) - hinge(o, I->pcap);
            }
            if (pb < T) {
                double o = O[(int64_t)s * T + pb];
                acc += hinge(o - ton, I->pcap) - hinge(o, I->pcap);
            }
        }
        dPp = I->pen_proc * acc / S;
        double am = 0.0;
        if (t < T) am += hinge(M[t] + ton, I->mcap) - hinge(M[t], I->mcap);
        if (pb < T) am += hinge(M[pb] - ton, I->mcap) - hinge(M[pb], I->mcap);
        dPm = I->pen_mine * am;
    }
    *score = dR - dPp - dPm;
    *flags = f;
    if (dR_out) *dR_out = dR;
    if (dPp_out) *dPp_out = dPp;
    if (dPm_out) *dPm_out = dPm;
}

void or_eval_moves(const or_inst *I, const int8_t *p, int32_t exhaustive,
                   int32_t include_never, int64_t n, const int32_t *block,
                   const int8_t *period, double *score, uint8_t *flags,
                   double *dR, double *dPp, double *dPm, int32_t n_threads) {
    int64_t N = n_blocks(I);
    int32_t S = I->S, T = I->T;
    int32_t D = include_never ? T + 1 : T;
    double *d = malloc(sizeof(double) * (T + 1));
    double *Ns = malloc(sizeof(double) * S);
    double *O = malloc(sizeof(double) * S * T);
    double *M = malloc(sizeof(double) * T);
    or_discount(T, I->rate, d);
    or_objective_t obj;
    or_objective(I, p, &obj, Ns, O, M);
    int64_t nm = exhaustive ? N * D : n;
#ifdef _OPENMP
    int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
#endif
    {
        double *Np = malloc(sizeof(double) * S);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t i = 0; i < nm; ++i) {
            int32_t b, t;
            if (exhaustive) {
                b = (int32_t)(i / D);
                t = (int32_t)(i % D);
            } else {
                b = block[i];
                t = period[i];
            }
            eval_one(I, p, Ns, O, M, d, obj.mu, obj.sigma, b, t, Np, &score[i],
                     &flags[i], dR ? &dR[i] : NULL, dPp ? &dPp[i] : NULL,
                     dPm ? &dPm[i] : NULL);
        }
        free(Np);
    }
    (void)n_threads;
    free(d); free(Ns); free(O); free(M);
}

double or_eval_bruteforce(const or_inst *I, const int8_t *p, int32_t b, int32_t t) {
    int64_t N = n_blocks(I);
    int8_t *q = malloc((size_t)N);
    memcpy(q, p, (size_t)N);
    q[b] = (int8_t)t;
    or_objective_t a, c;
    or_objective(I, p, &a, NULL, NULL, NULL);
    or_objective(I, q, &c, NULL, NULL, NULL);
    free(q);
    return c.J - a.J;
}

/* ---- top-k: exact selection by sorting ---------------------------------- */
typedef struct { double s; int64_t i; } sidx_t;

static int cmp_sidx(const void *pa, const void *pb) {
    const sidx_t *a = pa, *b = pb;
    if (a->s > b->s) return -1;
    if (a->s < b->s) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

int32_t or_topk(const double *score, const uint8_t *flags, int64_t n, int32_t k,
                uint8_t req, uint8_t forbid, int64_t *idx, double *top_score) {
    sidx_t *a = malloc(sizeof(sidx_t) * (n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if ((flags[i] & req) == req && (flags[i] & forbid) == 0) {
            a[m].s = score[i];
            a[m].i = i;
            ++m;
        }
    qsort(a, (size_t)m, sizeof(sidx_t), cmp_sidx);
    int32_t c = (int32_t)(m < k ? m : k);
    for (int32_t j = 0; j < c; ++j) {
        idx[j] = a[j].i;
        if (top_score) top_score[j] = a[j].s;
    }
    free(a);
    return c;
}

/* ---- greedy repair (Alg. 4, amortised over an ordered candidate list) ----
 * Walk the list in order.  A block already moved in this call is skipped.
 * Otherwise the move is re-scored exactly against the current schedule and
 * state; it is applied iff precedence holds (and both capacities, in hard
 * mode) and its score is positive.  Applying updates p, N_s, O and M. */
int32_t or_repair(const or_inst *I, int8_t *p, int32_t n_cand,
                  const int32_t *cand_block, const int8_t *cand_period,
                  int32_t hard_capacity, double *J_out, uint8_t *accepted) {
    int64_t N = n_blocks(I);
    int32_t S = I->S, T = I->T;
    double *d = malloc(sizeof(double) * (T + 1));
    double *Ns = malloc(sizeof(double) * S);
    double *Np = malloc(sizeof(double) * S);
    double *O = malloc(sizeof(double) * S * T);
    double *M = malloc(sizeof(double) * T);
    uint8_t *moved = calloc((size_t)N, 1);
    or_discount(T, I->rate, d);
    or_objective_t obj;
    or_objective(I, p, &obj, Ns, O, M);
    int32_t applied = 0;
    for (int32_t i = 0; i < n_cand; ++i) {
        int32_t b = cand_block[i], t = cand_period[i];
        if (accepted) accepted[i] = 0;
        if (b < 0 || b >= N || t < 0 || t > T) continue;
        if (moved[b]) continue;
        double mu, sd;
        mean_std(Ns, S, &mu, &sd);
        double score;
        uint8_t f;
        eval_one(I, p, Ns, O, M, d, mu, sd, b, t, Np, &score, &f, NULL, NULL, NULL);
        int ok = (f & OR_PREC_OK) && !(f & OR_NOOP);
        if (hard_capacity) ok = ok && (f & OR_MINE_OK) && (f & OR_PROC_OK);
        if (!ok || !(score > 0.0)) continue;
        int32_t pb = p[b];
        for (int32_t s = 0; s < S; ++s)
            Ns[s] += val(I, s, b) * (wdisc(I, d, s, t) - wdisc(I, d, s, pb));
        for (int32_t s = 0; s < S; ++s) {
            if (!ore(I, s, b)) continue;
            if (pb < T) O[(int64_t)s * T + pb] -= I->ton[b];
            if (t < T) O[(int64_t)s * T + t] += I->ton[b];
        }
        if (pb < T) M[pb] -= I->ton[b];
        if (t < T) M[t] += I->ton[b];
        p[b] = (int8_t)t;
        moved[b] = 1;
        if (accepted) accepted[i] = 1;
        ++applied;
    }
    if (J_out) {
        or_objective(I, p, &obj, NULL, NULL, NULL);
        *J_out = obj.J;
    }
    free(d); free(Ns); free(Np); free(O); free(M); free(moved);
    return applied;
}

/* ---- relaxed, differentiable objective ------------------------------------
 * x[b,t] in [0,1] is the cumulative fraction of block b mined by the end of
 * period t; y[b,t] = x[b,t] - x[b,t-1] (x[b,-1] = 0) is the fraction mined in
 * period t.  Per-scenario NPV, period tonnages and the penalised objective:
 *   NPV_s  = sum_b v[s,b] sum_t d(t) y[b,t]
 *   Ot[s,t] = sum_b ton_b ore[s,b] y[b,t],   Mt[t] = sum_b ton_b y[b,t]
 *   J = mu - lambda sigma - (mu_proc/S) sum_{s,t} max(0, Ot - Pcap)^2
 *       - mu_mine sum_t max(0, Mt - Mcap)^2
 *       - mu_prec sum_b sum_{a in Pred(b)} sum_t max(0, x[b,t] - x[a,t])^2
 * The gradient is the exact derivative of this expression (the std term uses
 * w_s = 1/S - lambda (NPV_s - mu)/(S sigma), and 1/S where sigma vanishes). */
double or_relaxed_d(const or_inst *I, const double *x, const or_relax_t *rp,
                    double *grad) {
    int64_t N = n_blocks(I);
    int32_t S = I->S, T = I->T;
    double *d = malloc(sizeof(double) * (T + 1));
    double *y = malloc(sizeof(double) * N * T);
    double *Db = malloc(sizeof(double) * N);
    double *npv = malloc(sizeof(double) * S);
    double *Ot = calloc((size_t)S * T, sizeof(double));
    double *Mt = calloc((size_t)T, sizeof(double));
    or_discount(T, I->rate, d);
    for (int64_t b = 0; b < N; ++b) {
        double acc = 0.0;
        for (int32_t t = 0; t < T; ++t) {
            double prev = t > 0 ? x[b * T + t - 1] : 0.0;
            y[b * T + t] = x[b * T + t] - prev;
            acc += d[t] * y[b * T + t];
        }
        Db[b] = acc;
    }
    for (int32_t s = 0; s < S; ++s) {
        double acc = 0.0;
        for (int64_t b = 0; b < N; ++b) acc += val(I, s, (int32_t)b) * Db[b];
        npv[s] = acc;
    }
    for (int64_t b = 0; b < N; ++b)
        for (int32_t t = 0; t < T; ++t) {
            double tw = I->ton[b] * y[b * T + t];
            Mt[t] += tw;
            for (int32_t s = 0; s < S; ++s)
                if (ore(I, s, (int32_t)b)) Ot[(int64_t)s * T + t] += tw;
        }
    double mu, sd;
    mean_std(npv, S, &mu, &sd);
    double pp = 0.0, pm = 0.0, pr = 0.0;
    for (int64_t i = 0; i < (int64_t)S * T; ++i) {
        double e = hinge(Ot[i], I->pcap);
        pp += e * e;
    }
    pp = rp->mu_proc * pp / S;
    for (int32_t t = 0; t < T; ++t) {
        double e = hinge(Mt[t], I->mcap);
        pm += e * e;
    }
    pm = rp->mu_mine * pm;
    for (int64_t b = 0; b < N; ++b) {
        int32_t pa[OR_MAX_DEG];
        int32_t np = or_predecessors(I, (int32_t)b, pa);
        for (int32_t k = 0; k < np; ++k)
            for (int32_t t = 0; t < T; ++t) {
                double e = x[b * T + t] - x[(int64_t)pa[k] * T + t];
                if (e > 0.0) pr += e * e;
            }
    }
    pr = rp->mu_prec * pr;
    double J = mu - I->lambda * sd - pp - pm - pr;

    if (grad) {
        double *w = malloc(sizeof(double) * S);
        double *gy = malloc(sizeof(double) * T);
        int degenerate = !(sd > 1e-12 * (fabs(mu) > 1.0 ? fabs(mu) : 1.0));
        for (int32_t s = 0; s < S; ++s)
            w[s] = degenerate ? 1.0 / S
                              : 1.0 / S - I->lambda * (npv[s] - mu) / (S * sd);
        for (int64_t b = 0; b < N; ++b) {
            double u = 0.0;
            for (int32_t s = 0; s < S; ++s) u += w[s] * val(I, s, (int32_t)b);
            for (int32_t t = 0; t < T; ++t) {
                double cp = 0.0;
                for (int32_t s = 0; s < S; ++s)
                    if (ore(I, s, (int32_t)b)) cp += hinge(Ot[(int64_t)s * T + t], I->pcap);
                double cap = (2.0 * rp->mu_proc / S) * cp +
                             2.0 * rp->mu_mine * hinge(Mt[t], I->mcap);
                gy[t] = d[t] * u - I->ton[b] * cap;
            }
            for (int32_t t = 0; t < T; ++t)
                grad[b * T + t] = gy[t] - (t + 1 < T ? gy[t + 1] : 0.0);
        }
        for (int64_t b = 0; b < N; ++b) {
            int32_t nb[OR_MAX_DEG];
            int32_t np = or_predecessors(I, (int32_t)b, nb);
            for (int32_t t = 0; t < T; ++t) {
                double acc = 0.0;
                for (int32_t k = 0; k < np; ++k)
                    acc += hinge(x[b * T + t] - x[(int64_t)nb[k] * T + t], 0.0);
                grad[b * T + t] -= 2.0 * rp->mu_prec * acc;
            }
            np = or_successors(I, (int32_t)b, nb);
            for (int32_t t = 0; t < T; ++t) {
                double acc = 0.0;
                for (int32_t k = 0; k < np; ++k)
                    acc += hinge(x[(int64_t)nb[k] * T + t] - x[b * T + t], 0.0);
                grad[b * T + t] += 2.0 * rp->mu_prec * acc;
            }
        }
        free(w); free(gy);
    }
    free(d); free(y); free(Db); free(npv); free(Ot); free(Mt);
    return J;
}

double or_relaxed(const or_inst *I, const float *x, const or_relax_t *rp,
                  double *grad) {
    int64_t n = n_blocks(I) * I->T;
    double *xd = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) xd[i] = x[i];
    double J = or_relaxed_d(I, xd, rp, grad);
    free(xd);
    return J;
}

/* ---- gradient ranking ------------------------------------------------------
 * Moving b from p_b to t changes x(p)[b,u] by +1 on [t, p_b) or by -1 on
 * [p_b, t), so its first-order gain is Gc[b,p_b] - Gc[b,t] with
 * Gc[b,t] = sum_{u<t} dJ/dx[b,u]. */
int32_t or_rank_moves(const or_inst *I, const int8_t *p, const double *grad,
                      int32_t k, int32_t *block, int8_t *period, double *gain) {
    int64_t N = n_blocks(I);
    int32_t T = I->T, D = T + 1;
    sidx_t *a = malloc(sizeof(sidx_t) * N * D);
    double *Gc = malloc(sizeof(double) * D);
    int64_t m = 0;
    int32_t nb[OR_MAX_DEG];
    for (int64_t b = 0; b < N; ++b) {
        Gc[0] = 0.0;
        for (int32_t t = 0; t < T; ++t) Gc[t + 1] = Gc[t] + grad[b * T + t];
        /* moves that keep the schedule precedence-feasible (Eq. 15):
         * p[a] <= t' for every predecessor a, t' <= p[c] for every successor */
        int32_t lo = 0, hi = T;
        int32_t np_ = or_predecessors(I, (int32_t)b, nb);
        for (int32_t j = 0; j < np_; ++j) if (p[nb[j]] > lo) lo = p[nb[j]];
        int32_t ns_ = or_successors(I, (int32_t)b, nb);
        for (int32_t j = 0; j < ns_; ++j) if (p[nb[j]] < hi) hi = p[nb[j]];
        for (int32_t t = 0; t < D; ++t) {
            if (t == p[b] || t < lo || t > hi) continue;
            a[m].s = Gc[p[b]] - Gc[t];
            a[m].i = b * D + t;
            ++m;
        }
    }
    qsort(a, (size_t)m, sizeof(sidx_t), cmp_sidx);
    int32_t c = (int32_t)(m < k ? m : k);
    for (int32_t j = 0; j < c; ++j) {
        block[j] = (int32_t)(a[j].i / D);
        period[j] = (int8_t)(a[j].i % D);
        if (gain) gain[j] = a[j].s;
    }
    free(a); free(Gc);
    return c;
}

/* ---- search loops ----------------------------------------------------------
 * Exhaustive: evaluate all N(T+1) moves, take the top k feasible non-no-op
 * moves, repair with them; stop when a repair applies nothing.
 * Gradient-ranked: rank all moves by the relaxed gradient at x(p), evaluate
 * only the top k exactly, take the top k of those, repair; when a round
 * applies nothing, one exhaustive round certifies (and continues if it
 * applied something). */
static int32_t exhaustive_round(const or_inst *I, int8_t *p, int32_t k,
                                int64_t *n_eval, int32_t nt) {
    int64_t N = n_blocks(I);
    int32_t D = I->T + 1;
    int64_t nm = N * D;
    double *sc = malloc(sizeof(double) * nm);
    uint8_t *fl = malloc((size_t)nm);
    int64_t *idx = malloc(sizeof(int64_t) * k);
    int32_t *cb = malloc(sizeof(int32_t) * k);
    int8_t *ct = malloc((size_t)k);
    or_eval_moves(I, p, 1, 1, 0, NULL, NULL, sc, fl, NULL, NULL, NULL, nt);
    *n_eval += nm;
    int32_t c = or_topk(sc, fl, nm, k, OR_PREC_OK, OR_NOOP | OR_BAD, idx, NULL);
    for (int32_t j = 0; j < c; ++j) {
        cb[j] = (int32_t)(idx[j] / D);
        ct[j] = (int8_t)(idx[j] % D);
    }
    int32_t applied = or_repair(I, p, c, cb, ct, 0, NULL, NULL);
    free(sc); free(fl); free(idx); free(cb); free(ct);
    return applied;
}

static int32_t gradient_round(const or_inst *I, int8_t *p, int32_t k,
                              const or_relax_t *rp, int64_t *n_eval, int32_t nt) {
    int64_t N = n_blocks(I);
    int32_t T = I->T;
    double *x = malloc(sizeof(double) * N * T);
    double *g = malloc(sizeof(double) * N * T);
    int32_t *rb = malloc(sizeof(int32_t) * k);
    int8_t *rt = malloc((size_t)k);
    double *sc = malloc(sizeof(double) * k);
    uint8_t *fl = malloc((size_t)k);
    int64_t *idx = malloc(sizeof(int64_t) * k);
    int32_t *cb = malloc(sizeof(int32_t) * k);
    int8_t *ct = malloc((size_t)k);
    for (int64_t b = 0; b < N; ++b)
        for (int32_t t = 0; t < T; ++t) x[b * T + t] = t >= p[b] ? 1.0 : 0.0;
    or_relaxed_d(I, x, rp, g);
    int32_t m = or_rank_moves(I, p, g, k, rb, rt, NULL);
    or_eval_moves(I, p, 0, 1, m, rb, rt, sc, fl, NULL, NULL, NULL, nt);
    *n_eval += m;
    int32_t c = or_topk(sc, fl, m, k, OR_PREC_OK, OR_NOOP | OR_BAD, idx, NULL);
    for (int32_t j = 0; j < c; ++j) {
        cb[j] = rb[idx[j]];
        ct[j] = rt[idx[j]];
    }
    int32_t applied = or_repair(I, p, c, cb, ct, 0, NULL, NULL);
    free(x); free(g); free(rb); free(rt); free(sc); free(fl); free(idx);
    free(cb); free(ct);
    return applied;
}

double or_search(const or_inst *I, int8_t *p, int32_t mode, int32_t k,
                 const or_relax_t *rp, int32_t max_iter, int64_t *stats,
                 int32_t n_threads) {
    int64_t iters = 0, n_eval = 0, applied_total = 0;
    while (iters < max_iter) {
        int32_t a;
        if (mode == 0) {
            a = exhaustive_round(I, p, k, &n_eval, n_threads);
            ++iters;
            applied_total += a;
            if (a == 0) break;
        } else {
            a = gradient_round(I, p, k, rp, &n_eval, n_threads);
            ++iters;
            applied_total += a;
            if (a == 0) {
                a = exhaustive_round(I, p, k, &n_eval, n_threads);
                ++iters;
                applied_total += a;
                if (a == 0) break;
            }
        }
    }
    if (stats) {
        stats[0] = iters;
        stats[1] = n_eval;
        stats[2] = applied_total;
    }
    or_objective_t obj;
    or_objective(I, p, &obj, NULL, NULL, NULL);
    return obj.J;
}

/* ---- exhaustive optimum over feasible schedules (tiny grids only) -------- */
typedef struct {
    const or_inst *I;
    int8_t *p, *best;
    double J_best;
    int64_t count;
    int have;
} opt_ctx;

static void opt_rec(opt_ctx *c, int32_t b) {
    const or_inst *I = c->I;
    int64_t N = n_blocks(I);
    if (b == N) {
        or_objective_t o;
        or_objective(I, c->p, &o, NULL, NULL, NULL);
        ++c->count;
        if (!c->have || o.J > c->J_best) {
            c->have = 1;
            c->J_best = o.J;
            memcpy(c->best, c->p, (size_t)N);
        }
        return;
    }
    int32_t pr[OR_MAX_DEG];
    int32_t np = or_predecessors(I, b, pr);
    int32_t lo = 0;
    for (int32_t k = 0; k < np; ++k)   /* predecessors have smaller indices (checked) */
        if (c->p[pr[k]] > lo) lo = c->p[pr[k]];
    for (int32_t t = lo; t <= I->T; ++t) {
        c->p[b] = (int8_t)t;
        opt_rec(c, b + 1);
    }
}

double or_optimum(const or_inst *I, int8_t *p_best, int64_t *n_feasible) {
    int64_t N = n_blocks(I);
    for (int64_t b = 0; b < N; ++b) {
        int32_t pr[OR_MAX_DEG];
        int32_t np = or_predecessors(I, (int32_t)b, pr);
        for (int32_t k = 0; k < np; ++k)
            if (pr[k] >= b) return NAN;
    }
    opt_ctx c;
    c.I = I;
    c.p = calloc((size_t)N, 1);
    c.best = p_best;
    c.J_best = -INFINITY;
    c.count = 0;
    c.have = 0;
    opt_rec(&c, 0);
    free(c.p);
    if (n_feasible) *n_feasible = c.count;
    return c.J_best;
}

/* ---- greedy initializer (Alg. 3 with every uncertainty factor equal to 1) --
 * Blocks are ranked by value density, here the block's expected value
 * vd[b] = mean_s v[s,b] (grade times mass priced by the value model), in
 * descending order with ties to the smaller index.  Starting from "nothing
 * mined", each block in that order takes the earliest period t < T in which
 * it is feasible against the schedule built so far: every predecessor mined
 * in t or earlier (an unplaced predecessor counts as never mined), every
 * placed successor in t or later, the mining tonnage of t plus the block
 * within Mcap, and in every scenario in which the block is ore the processed
 * tonnage of t plus the block within Pcap -- the PREC_OK, MINE_OK and PROC_OK
 * conditions of a move (b, t).  A block with no such period stays unplaced.
 * The printed loop is one pass; a block whose predecessors rank below it can
 * only be placed in a later pass, so passes repeat over the unplaced blocks,
 * in the same order, until one places nothing (or max_pass passes ran). */
typedef struct { double vd; int32_t b; } vdb_t;

static int cmp_vdb(const void *pa, const void *pb) {
    const vdb_t *a = pa, *b = pb;
    if (a->vd > b->vd) return -1;
    if (a->vd < b->vd) return 1;
    return (a->b > b->b) - (a->b < b->b);
}

int32_t or_greedy_init(const or_inst *I, int8_t *p, int32_t max_pass, int64_t *n_placed) {
    int64_t N = n_blocks(I);
    int32_t S = I->S, T = I->T;
    vdb_t *ord = malloc(sizeof(vdb_t) * (N > 0 ? N : 1));
    double *O = calloc((size_t)S * T, sizeof(double));
    double *M = calloc((size_t)T, sizeof(double));
    for (int64_t b = 0; b < N; ++b) {
        double acc = 0.0;
        for (int32_t s = 0; s < S; ++s) acc += val(I, s, (int32_t)b);
        ord[b].vd = acc / S;
        ord[b].b = (int32_t)b;
        p[b] = (int8_t)T;
    }
    qsort(ord, (size_t)N, sizeof(vdb_t), cmp_vdb);
    int32_t passes = 0;
    int64_t placed = 0;
    while (passes < max_pass) {
        ++passes;
        int64_t now = 0;
        for (int64_t i = 0; i < N; ++i) {
            int32_t b = ord[i].b;
            if (p[b] != T) continue;
            double ton = I->ton[b];
            int32_t nb[OR_MAX_DEG];
            for (int32_t t = 0; t < T; ++t) {
                int ok = 1;
                int32_t n = or_predecessors(I, b, nb);
                for (int32_t k = 0; k < n; ++k)
                    if (p[nb[k]] > t) ok = 0;
                n = or_successors(I, b, nb);
                for (int32_t k = 0; k < n; ++k)
                    if (t > p[nb[k]]) ok = 0;
                if (!(M[t] + ton <= I->mcap)) ok = 0;
                for (int32_t s = 0; s < S && ok; ++s)
                    if (ore(I, s, b) && !(O[(int64_t)s * T + t] + ton <= I->pcap)) ok = 0;
                if (!ok) continue;
                p[b] = (int8_t)t;
                M[t] += ton;
                for (int32_t s = 0; s < S; ++s)
                    if (ore(I, s, b)) O[(int64_t)s * T + t] += ton;
                ++now;
                break;
            }
        }
        placed += now;
        if (now == 0) break;
    }
    if (n_placed) *n_placed = placed;
    free(ord); free(O); free(M);
    return passes;
}

/* ---- cascading repair (Alg. 4 with its fallback) ----------------------------
 * The greedy repair walk, where a candidate (b, t') that precedence forbids is
 * not skipped but taken together with the blocks that forbid it: moving b
 * earlier (t' < p_b) takes along every ancestor a reached through
 * predecessors with p_a > t', moving it later takes along every descendant c
 * reached through successors with p_c < t'; the whole set goes to t'.  The
 * set is found breadth-first (predecessor or successor lists in their order)
 * and holds b first.  The composite move is scored exactly: every N'_s, mu',
 * sigma' from scratch, and the hinge terms of every period the set leaves or
 * enters re-derived.  It is applied iff the set has at most max_set blocks,
 * none of them was moved earlier in this call, the resulting schedule
 * satisfies Eq. 15 at every moved block, (with hard_capacity) the mining
 * tonnage of t' stays within Mcap and the processed tonnage of t' within
 * Pcap in every scenario, and the score is positive.  A candidate that needs
 * no companions is exactly the plain repair's move. */
int32_t or_repair_cascade(const or_inst *I, int8_t *p, int32_t n_cand,
                          const int32_t *cand_block, const int8_t *cand_period,
                          int32_t hard_capacity, int32_t max_set, double *J_out,
                          uint8_t *accepted, int32_t *set_size) {
    int64_t N = n_blocks(I);
    int32_t S = I->S, T = I->T;
    double *d = malloc(sizeof(double) * (T + 1));
    double *Ns = malloc(sizeof(double) * S);
    double *Np = malloc(sizeof(double) * S);
    double *O = malloc(sizeof(double) * S * T);
    double *Op = malloc(sizeof(double) * S * T);
    double *M = malloc(sizeof(double) * T);
    double *Mp = malloc(sizeof(double) * T);
    uint8_t *moved = calloc((size_t)N, 1);
    uint8_t *inset = calloc((size_t)N, 1);
    int32_t *set = malloc(sizeof(int32_t) * (N > 0 ? N : 1));
    or_discount(T, I->rate, d);
    or_objective_t obj;
    or_objective(I, p, &obj, Ns, O, M);
    int32_t applied = 0;
    for (int32_t i = 0; i < n_cand; ++i) {
        int32_t b = cand_block[i], t = cand_period[i];
        if (accepted) accepted[i] = 0;
        if (set_size) set_size[i] = 0;
        if (b < 0 || b >= N || t < 0 || t > T) continue;
        if (moved[b] || t == p[b]) continue;
        /* the set: b, then breadth-first the blocks that must move with it */
        int32_t n = 0, too_big = 0;
        set[n++] = b;
        inset[b] = 1;
        int earlier = t < p[b];
        for (int32_t q = 0; q < n && !too_big; ++q) {
            int32_t nb[OR_MAX_DEG];
            int32_t k = earlier ? or_predecessors(I, set[q], nb) : or_successors(I, set[q], nb);
            for (int32_t j = 0; j < k; ++j) {
                int32_t a = nb[j];
                if (inset[a]) continue;
                if (earlier ? p[a] > t : p[a] < t) {
                    if (n == max_set) { too_big = 1; break; }
                    set[n++] = a;
                    inset[a] = 1;
                }
            }
        }
        if (set_size) set_size[i] = too_big ? -1 : n;
        int ok = !too_big;
        for (int32_t q = 0; q < n && ok; ++q)
            if (moved[set[q]]) ok = 0;
        /* Eq. 15 at every moved block of the composite schedule */
        for (int32_t q = 0; q < n && ok; ++q) {
            int32_t x = set[q], nb[OR_MAX_DEG];
            int32_t k = or_predecessors(I, x, nb);
            for (int32_t j = 0; j < k; ++j)
                if ((inset[nb[j]] ? t : p[nb[j]]) > t) ok = 0;
            k = or_successors(I, x, nb);
            for (int32_t j = 0; j < k; ++j)
                if (t > (inset[nb[j]] ? t : p[nb[j]])) ok = 0;
        }
        double score = 0.0;
        if (ok) {
            /* N'_s from scratch: N_s plus every moved block's change */
            for (int32_t s = 0; s < S; ++s) {
                double acc = Ns[s];
                for (int32_t q = 0; q < n; ++q)
                    acc += val(I, s, set[q]) * (wdisc(I, d, s, t) - wdisc(I, d, s, p[set[q]]));
                Np[s] = acc;
            }
            double mu, sd, mu2, sd2;
            mean_std(Ns, S, &mu, &sd);
            mean_std(Np, S, &mu2, &sd2);
            double dR = risk_value(I, Np, mu2, sd2) - risk_value(I, Ns, mu, sd);
            /* tonnages after the move, then the hinge terms of every period */
            memcpy(Op, O, sizeof(double) * S * T);
            memcpy(Mp, M, sizeof(double) * T);
            for (int32_t q = 0; q < n; ++q) {
                int32_t x = set[q], u = p[x];
                double ton = I->ton[x];
                if (u < T) Mp[u] -= ton;
                if (t < T) Mp[t] += ton;
                for (int32_t s = 0; s < S; ++s) {
                    if (!ore(I, s, x)) continue;
                    if (u < T) Op[(int64_t)s * T + u] -= ton;
                    if (t < T) Op[(int64_t)s * T + t] += ton;
                }
            }
            double acc = 0.0, am = 0.0;
            for (int32_t u = 0; u < T; ++u) {
                int touched = (u == t);
                for (int32_t q = 0; q < n && !touched; ++q)
                    if (p[set[q]] == u) touched = 1;
                if (!touched) continue;
                for (int32_t s = 0; s < S; ++s)
                    acc += hinge(Op[(int64_t)s * T + u], I->pcap) -
                           hinge(O[(int64_t)s * T + u], I->pcap);
                am += hinge(Mp[u], I->mcap) - hinge(M[u], I->mcap);
            }
            double dPp = I->pen_proc * acc / S, dPm = I->pen_mine * am;
            score = dR - dPp - dPm;
            if (hard_capacity && t < T) {
                if (!(Mp[t] <= I->mcap)) ok = 0;
                for (int32_t s = 0; s < S && ok; ++s)
                    if (!(Op[(int64_t)s * T + t] <= I->pcap)) ok = 0;
            }
        }
        if (ok && score > 0.0) {
            memcpy(Ns, Np, sizeof(double) * S);
            memcpy(O, Op, sizeof(double) * S * T);
            memcpy(M, Mp, sizeof(double) * T);
            for (int32_t q = 0; q < n; ++q) {
                p[set[q]] = (int8_t)t;
                moved[set[q]] = 1;
            }
            if (accepted) accepted[i] = 1;
            ++applied;
        }
        for (int32_t q = 0; q < n; ++q) inset[set[q]] = 0;
    }
    if (J_out) {
        or_objective(I, p, &obj, NULL, NULL, NULL);
        *J_out = obj.J;
    }
    free(d); free(Ns); free(Np); free(O); free(Op); free(M); free(Mp);
    free(moved); free(inset); free(set);
    return applied;
}

/* ---- LNS + simulated annealing driver (Alg. 2 without its GA and RL parts) --
 * Neighbourhoods: the x-y tiles of nb x nb block columns (every bench), in
 * row-major tile order.  One step on neighbourhood i at iteration it:
 *   destroy: the region = the tile's blocks and every descendant of them
 *     (through successor lists) is set to "never" (the result stays
 *     precedence-feasible: a block outside the region has no predecessor in
 *     it);
 *   repair: up to max_rounds rounds of {evaluate every move (b, t), b in the
 *     region by increasing index, t = 0..T-1 in order; take the top k by
 *     score (PREC_OK required, NOOP and BAD forbidden); greedy repair with
 *     them}, stopping after a round that applies nothing;
 *   fitness with the eps-relaxed constraints: the capacity violation of a
 *     schedule is its penalty P = Pp + Pm, and f(S) = R(S) - max(0, P(S) - eps)
 *     with eps = eps_max (1 - it / n_iter), decreasing linearly (at eps = 0,
 *     f = J);
 *   simulated-annealing transition: the candidate replaces the current
 *     schedule iff f(cand) > f(cur) - u temp, u the step's uniform draw in
 *     [0,1) (given), temp the temperature of the iteration (temp0 times
 *     cool^it); otherwise the current schedule is kept.
 * The best schedule by J (eps = 0) over the run, starting with the input, is
 * returned in p.  traj (may be NULL) receives per step: J, R, P of the
 * candidate, and 1/0 for accepted.  stats: steps, accepted, moves evaluated,
 * moves applied. */
static void region_of_tile(const or_inst *I, int32_t tx, int32_t ty, int32_t nb,
                           uint8_t *reg) {
    int64_t N = n_blocks(I);
    for (int64_t b = 0; b < N; ++b) {
        int32_t x = (int32_t)(b % I->nx), y = (int32_t)((b / I->nx) % I->ny);
        reg[b] = (x / nb == tx && y / nb == ty) ? 1 : 0;
    }
    int changed = 1;
    while (changed) {   /* descendants: a block with a predecessor in the region */
        changed = 0;
        for (int64_t c = 0; c < N; ++c) {
            if (reg[c]) continue;
            int32_t pr[OR_MAX_DEG];
            int32_t np = or_predecessors(I, (int32_t)c, pr);
            for (int32_t k = 0; k < np; ++k)
                if (reg[pr[k]]) {
                    reg[c] = 1;
                    changed = 1;
                    break;
                }
        }
    }
}

double or_lns_sa(const or_inst *I, int8_t *p, int32_t n_iter, int32_t nb, int32_t k,
                 int32_t max_rounds, double eps_max, double temp0, double cool,
                 const double *u, double *traj, int64_t *stats, int32_t n_threads) {
    int64_t N = n_blocks(I);
    int32_t T = I->T;
    int32_t kx = (I->nx + nb - 1) / nb, ky = (I->ny + nb - 1) / nb, K = kx * ky;
    int8_t *cur = malloc((size_t)N), *cand = malloc((size_t)N), *best = malloc((size_t)N);
    uint8_t *reg = malloc((size_t)N);
    int32_t *lb = malloc(sizeof(int32_t) * N * T > 0 ? sizeof(int32_t) * N * T : 4);
    int8_t *lt = malloc((size_t)N * T > 0 ? (size_t)N * T : 1);
    double *sc = malloc(sizeof(double) * (N * T > 0 ? N * T : 1));
    uint8_t *fl = malloc((size_t)(N * T > 0 ? N * T : 1));
    int64_t *idx = malloc(sizeof(int64_t) * k);
    int32_t *cb = malloc(sizeof(int32_t) * k);
    int8_t *ct = malloc((size_t)k);
    memcpy(cur, p, (size_t)N);
    memcpy(best, p, (size_t)N);
    or_objective_t o;
    or_objective(I, cur, &o, NULL, NULL, NULL);
    double J_best = o.J;
    double R_cur = o.R, P_cur = o.Pp + o.Pm;
    int64_t steps = 0, acc_n = 0, n_eval = 0, n_app = 0;
    for (int32_t it = 0; it < n_iter; ++it) {
        double eps = eps_max * (1.0 - (double)it / n_iter);
        double temp = temp0;
        for (int32_t j = 0; j < it; ++j) temp *= cool;
        for (int32_t i = 0; i < K; ++i) {
            region_of_tile(I, i % kx, i / kx, nb, reg);
            memcpy(cand, cur, (size_t)N);
            int64_t m = 0;
            for (int64_t b = 0; b < N; ++b) {
                if (!reg[b]) continue;
                cand[b] = (int8_t)T;
                for (int32_t t = 0; t < T; ++t) {
                    lb[m] = (int32_t)b;
                    lt[m] = (int8_t)t;
                    ++m;
                }
            }
            for (int32_t r = 0; r < max_rounds; ++r) {
                or_eval_moves(I, cand, 0, 1, m, lb, lt, sc, fl, NULL, NULL, NULL, n_threads);
                n_eval += m;
                int32_t c = or_topk(sc, fl, m, k, OR_PREC_OK, OR_NOOP | OR_BAD, idx, NULL);
                for (int32_t q = 0; q < c; ++q) {
                    cb[q] = lb[idx[q]];
                    ct[q] = lt[idx[q]];
                }
                int32_t a = or_repair(I, cand, c, cb, ct, 0, NULL, NULL);
                n_app += a;
                if (a == 0) break;
            }
            or_objective(I, cand, &o, NULL, NULL, NULL);
            double P_cand = o.Pp + o.Pm;
            double f_cand = o.R - (P_cand - eps > 0.0 ? P_cand - eps : 0.0);
            double f_cur = R_cur - (P_cur - eps > 0.0 ? P_cur - eps : 0.0);
            double uu = u[(int64_t)it * K + i];
            int accept = f_cand > f_cur - uu * temp;
            if (traj) {
                traj[steps * 4 + 0] = o.J;
                traj[steps * 4 + 1] = o.R;
                traj[steps * 4 + 2] = P_cand;
                traj[steps * 4 + 3] = accept ? 1.0 : 0.0;
            }
            ++steps;
            if (accept) {
                memcpy(cur, cand, (size_t)N);
                R_cur = o.R;
                P_cur = P_cand;
                ++acc_n;
                if (o.J > J_best) {
                    J_best = o.J;
                    memcpy(best, cand, (size_t)N);
                }
            }
        }
    }
    memcpy(p, best, (size_t)N);
    if (stats) {
        stats[0] = steps;
        stats[1] = acc_n;
        stats[2] = n_eval;
        stats[3] = n_app;
    }
    free(cur); free(cand); free(best); free(reg); free(lb); free(lt); free(sc); free(fl);
    free(idx); free(cb); free(ct);
    return J_best;
}
