/* sanitize_check.c -- runs every oracle entry point on small seeded
 * instances (grid stencil, explicit lists, objective variants), for a build
 * of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer.  TEST
 * INFRASTRUCTURE ONLY.  Exit status 0 and "ok" on success; the sanitizers
 * abort on the first invalid access. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void) {   /* splitmix64 */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) / 9007199254740992.0;
}

static void run(or_inst *I, const char *label) {
    int32_t N = I->nx * I->ny * I->nz, S = I->S, T = I->T, D = T + 1;
    int8_t *p = malloc(N), *q = malloc(N);
    /* a feasible schedule: periods non-decreasing along every list */
    for (int32_t b = 0; b < N; ++b) {
        int32_t pr[OR_MAX_DEG], lo = 0;
        int32_t n = or_predecessors(I, b, pr);
        for (int32_t k = 0; k < n; ++k) lo = p[pr[k]] > lo ? p[pr[k]] : lo;
        int32_t u = (int32_t)(urand() * (T + 1));
        p[b] = (int8_t)(u > lo ? u : lo);
    }
    or_objective_t o;
    double *Ns = malloc(sizeof(double) * S), *O = malloc(sizeof(double) * S * T),
           *M = malloc(sizeof(double) * T);
    or_objective(I, p, &o, Ns, O, M);
    int64_t nm = (int64_t)N * D;
    double *sc = malloc(sizeof(double) * nm), *c1 = malloc(sizeof(double) * nm),
           *c2 = malloc(sizeof(double) * nm), *c3 = malloc(sizeof(double) * nm);
    uint8_t *fl = malloc(nm);
    or_eval_moves(I, p, 1, 1, 0, NULL, NULL, sc, fl, c1, c2, c3, 2);
    int32_t nl = 50, *lb = malloc(sizeof(int32_t) * nl);
    int8_t *lt = malloc(nl);
    for (int32_t i = 0; i < nl; ++i) {
        lb[i] = (int32_t)(urand() * (N + 2)) - 1;   /* some out of range */
        lt[i] = (int8_t)((int32_t)(urand() * (T + 3)) - 1);
    }
    or_eval_moves(I, p, 0, 1, nl, lb, lt, sc, fl, NULL, NULL, NULL, 1);
    (void)or_eval_bruteforce(I, p, 0, T);
    or_eval_moves(I, p, 1, 1, 0, NULL, NULL, sc, fl, NULL, NULL, NULL, 2);
    int32_t k = 40;
    int64_t *idx = malloc(sizeof(int64_t) * nm);
    double *ts = malloc(sizeof(double) * nm);
    int32_t c = or_topk(sc, fl, nm, k, OR_PREC_OK, OR_NOOP | OR_BAD, idx, ts);
    int32_t *cb = malloc(sizeof(int32_t) * nm);
    int8_t *ct = malloc(nm);
    for (int32_t i = 0; i < c; ++i) {
        cb[i] = (int32_t)(idx[i] / D);
        ct[i] = (int8_t)(idx[i] % D);
    }
    uint8_t *acc = malloc(nm);
    int32_t *size = malloc(sizeof(int32_t) * nm);
    double J;
    memcpy(q, p, N);
    or_repair(I, q, c, cb, ct, 1, &J, acc);
    c = or_topk(sc, fl, nm, k, 0, OR_NOOP | OR_BAD, idx, NULL);
    for (int32_t i = 0; i < c; ++i) {
        cb[i] = (int32_t)(idx[i] / D);
        ct[i] = (int8_t)(idx[i] % D);
    }
    memcpy(q, p, N);
    or_repair_cascade(I, q, c, cb, ct, 0, 4, &J, acc, size);
    or_relax_t rp = {0.003, 0.003, 1.5e6};
    float *x = malloc(sizeof(float) * N * T);
    double *xd = malloc(sizeof(double) * N * T), *g = malloc(sizeof(double) * N * T);
    for (int32_t b = 0; b < N; ++b) {
        double run = 0.0;
        for (int32_t t = 0; t < T; ++t) {
            run += urand() / T;
            x[b * T + t] = (float)run;
            xd[b * T + t] = run;
        }
    }
    (void)or_relaxed(I, x, &rp, g);
    (void)or_relaxed_d(I, xd, &rp, g);
    int8_t *rt = malloc(nm);
    (void)or_rank_moves(I, p, g, k, cb, rt, ts);
    int64_t st[4];
    memcpy(q, p, N);
    (void)or_search(I, q, 0, 16, &rp, 50, st, 1);
    memcpy(q, p, N);
    (void)or_search(I, q, 1, 16, &rp, 50, st, 1);
    int64_t placed;
    (void)or_greedy_init(I, q, 100, &placed);
    int32_t nb = 2, kx = (I->nx + nb - 1) / nb, ky = (I->ny + nb - 1) / nb;
    double *u = malloc(sizeof(double) * 2 * kx * ky), *traj = malloc(sizeof(double) * 8 * kx * ky);
    for (int32_t i = 0; i < 2 * kx * ky; ++i) u[i] = urand();
    memcpy(q, p, N);
    (void)or_lns_sa(I, q, 2, nb, 16, 3, 1e6, 1e5, 0.9, u, traj, st, 1);
    (void)or_cvar(Ns, S, 0.1);
    (void)or_cvar(Ns, S, 1.0);
    printf("%s: J %.6g\n", label, o.J);
    free(p); free(q); free(Ns); free(O); free(M); free(sc); free(c1); free(c2); free(c3);
    free(fl); free(lb); free(lt); free(idx); free(ts); free(cb); free(ct); free(acc);
    free(size); free(x); free(xd); free(g); free(rt); free(u); free(traj);
}

int main(void) {
    const int32_t nx = 5, ny = 4, nz = 3, S = 7, T = 4, N = nx * ny * nz;
    float *v = malloc(sizeof(float) * S * N);
    uint8_t *ore = malloc(S * N);
    double *ton = malloc(sizeof(double) * N);
    for (int32_t i = 0; i < S * N; ++i) {
        ore[i] = urand() < 0.8;
        v[i] = (float)(ore[i] ? 1e5 * urand() : -46800.0);
    }
    for (int32_t b = 0; b < N; ++b) ton[b] = 15600.0;
    or_inst I;
    memset(&I, 0, sizeof(I));
    I.nx = nx; I.ny = ny; I.nz = nz; I.S = S; I.T = T;
    I.rate = 0.08; I.lambda = 0.5; I.pen_proc = 100.0; I.pen_mine = 100.0;
    I.pcap = 0.8 * N * 15600.0 / T; I.mcap = 1.1 * N * 15600.0 / T;
    I.v = v; I.ore = ore; I.ton = ton; I.alpha = 0.1;
    run(&I, "grid");
    /* explicit lists: the 1-9 cone */
    int32_t *pp = malloc(sizeof(int32_t) * (N + 1)), *pi = malloc(sizeof(int32_t) * 9 * N);
    int32_t *sp = malloc(sizeof(int32_t) * (N + 1)), *si = malloc(sizeof(int32_t) * 9 * N);
    int32_t e = 0;
    for (int32_t b = 0; b < N; ++b) {
        pp[b] = e;
        int32_t x = b % nx, y = (b / nx) % ny, z = b / (nx * ny);
        if (z > 0)
            for (int32_t dy = -1; dy <= 1; ++dy)
                for (int32_t dx = -1; dx <= 1; ++dx)
                    if (x + dx >= 0 && x + dx < nx && y + dy >= 0 && y + dy < ny)
                        pi[e++] = (x + dx) + nx * ((y + dy) + ny * (z - 1));
    }
    pp[N] = e;
    or_successor_csr(N, pp, pi, sp, si);
    I.pred_ptr = pp; I.pred_idx = pi; I.succ_ptr = sp; I.succ_idx = si;
    run(&I, "cone");
    /* objective variants */
    double *mult = malloc(sizeof(double) * S * T);
    for (int32_t i = 0; i < S * T; ++i) mult[i] = 0.6 + 0.8 * urand();
    I.mult = mult;
    I.risk = 1;
    run(&I, "variants");
    /* exhaustive optimum of a 3x2x1 bench, T = 2 */
    or_inst J2 = I;
    J2.nx = 3; J2.ny = 2; J2.nz = 1; J2.T = 2;
    J2.pred_ptr = J2.pred_idx = J2.succ_ptr = J2.succ_idx = NULL;
    J2.mult = NULL;
    J2.risk = 0;
    int8_t best[6];
    int64_t nf;
    (void)or_optimum(&J2, best, &nf);
    free(v); free(ore); free(ton); free(pp); free(pi); free(sp); free(si); free(mult);
    printf("ok\n");
    return 0;
}
