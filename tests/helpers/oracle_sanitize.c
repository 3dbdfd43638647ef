/* Drives every entry point of the CPU oracle over a spread of shapes (even
 * and odd L from 2, one to 64 temperatures, a field, both flip-draw streams,
 * PT on and off, the per-class counters and the running-energy check), for a
 * build under AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status
 * 0 when every sweep kept its running energy equal to the recomputed one;
 * a sanitizer report aborts the run.  Used only by the test suite. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ea_oracle.h"

static int run_case(int L, int n_T, int R, int rng, double h, int sweeps, int swap_every, uint64_t seed)
{
    const int N = L * L * L;
    int8_t *J = malloc((size_t)R * N * 3);
    int8_t *spins = malloc((size_t)R * 2 * n_T * N);
    int32_t *perm = malloc(sizeof(int32_t) * (size_t)R * 2 * n_T);
    int32_t *rid = malloc(sizeof(int32_t) * (size_t)R);
    double *betas = malloc(sizeof(double) * (size_t)n_T);
    int64_t *Urun = malloc(sizeof(int64_t) * (size_t)R * 2 * n_T);
    int64_t *ft = calloc((size_t)n_T * 7, sizeof(int64_t)), *fa = calloc((size_t)n_T * 7, sizeof(int64_t));
    int64_t *st = calloc((size_t)n_T, sizeof(int64_t)), *sa = calloc((size_t)n_T, sizeof(int64_t));
    int32_t *E = malloc(sizeof(int32_t) * (size_t)R * 2 * n_T), *q = malloc(sizeof(int32_t) * (size_t)R * n_T);
    int32_t *M = malloc(sizeof(int32_t) * (size_t)R * 2 * n_T);
    int64_t *cnt = calloc((size_t)R * n_T, sizeof(int64_t)), *q2 = calloc((size_t)R * n_T, sizeof(int64_t));
    uint64_t *q4 = calloc((size_t)R * n_T * 2, sizeof(uint64_t));
    int64_t *cc = calloc((size_t)R * n_T * L, sizeof(int64_t));
    if (!J || !spins || !perm || !rid || !betas || !Urun || !ft || !fa || !st || !sa || !E || !q || !M || !cnt ||
        !q2 || !q4 || !cc) {
        fprintf(stderr, "allocation failed\n");
        return 1;
    }
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
    for (size_t b = 0; b < (size_t)R * N * 3; ++b) {
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;
        J[b] = (x & 1) ? 1 : -1;
    }
    for (int r = 0; r < R; ++r) rid[r] = 3 * r + 1;
    for (int k = 0; k < n_T; ++k) betas[k] = n_T == 1 ? 1.0 : 2.5 - 2.0 * k / (n_T - 1);
    orc_sim s = {0};
    s.L = L; s.n_T = n_T; s.R = R; s.rng = rng; s.seed = seed; s.t = 0;
    s.rid = rid; s.J = J; s.betas = betas; s.spins = spins; s.temp_of_slot = perm;
    s.Urun = Urun; s.flip_tries = ft; s.flip_acc = fa; s.swap_tries = st; s.swap_acc = sa; s.h = h;
    orc_init(&s);
    orc_reset_running_energy(&s);
    int rc = orc_sweep(&s, sweeps, swap_every);
    if (rc == 0) rc = orc_sweep(&s, sweeps / 2 + 1, swap_every ? swap_every + 1 : 0);
    orc_observables(&s, E, q);
    orc_magnetization(&s, M);
    orc_measure(&s, cnt, q2, q4, cc);
    for (int k = 0; k < n_T; ++k) (void)orc_flip_threshold_h(betas[k], k % 7, k & 1, h);
    free(J); free(spins); free(perm); free(rid); free(betas); free(Urun); free(ft); free(fa); free(st); free(sa);
    free(E); free(q); free(M); free(cnt); free(q2); free(q4); free(cc);
    if (rc != 0) fprintf(stderr, "case L=%d n_T=%d R=%d rng=%d h=%g: orc_sweep returned %d\n", L, n_T, R, rng, h, rc);
    return rc != 0;
}

int main(void)
{
    int bad = 0, cases = 0;
    static const int Ls[] = {2, 3, 4, 5, 6, 7, 8};
    static const int nTs[] = {1, 2, 5, 16, 33, 64};
    for (unsigned a = 0; a < sizeof Ls / sizeof Ls[0]; ++a)
        for (unsigned b = 0; b < sizeof nTs / sizeof nTs[0]; ++b) {
            const int L = Ls[a], n_T = nTs[b];
            const int rng = (a + b) % 2 && n_T >= 1 ? 1 : 0;
            const double h = rng ? 0.0 : ((a + b) % 3 == 0 ? 0.75 : 0.0);
            bad += run_case(L, n_T, 1 + (int)(a % 2), rng, h, 7, (int)(b % 3), 1000 + 17 * a + b);
            ++cases;
        }
    /* a larger lattice, both streams, PT every sweep */
    bad += run_case(16, 32, 1, 0, 0.0, 3, 1, 77);
    bad += run_case(16, 32, 1, 1, 0.0, 3, 1, 78);
    bad += run_case(9, 48, 2, 0, -1.25, 4, 2, 79);
    cases += 3;
    printf("oracle sanitize: %d cases, %d failed\n", cases, bad);
    return bad != 0;
}
