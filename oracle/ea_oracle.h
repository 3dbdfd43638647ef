/*
 * CPU oracle for the +-J Edwards-Anderson parallel-tempering Metropolis
 * simulation (arXiv:1311.5582).  TEST INFRASTRUCTURE ONLY: loaded by the test
 * suite, the smoke check and the benchmark's CPU-baseline leg, never by the
 * library.  See ea_oracle.c for the definition it implements.
 */
#ifndef EA_ORACLE_H
#define EA_ORACLE_H

#include <stdint.h>

#define ORC_MAX_TEMPS 64

/* flip-draw streams */
#define ORC_RNG_WORDS  0  /* one 32-bit word per (slot, site, sweep)                    */
#define ORC_RNG_PLANES 1  /* the slot's 32-bit uniform read from bit planes of 16 slots */

/* All arrays are owned by the caller.  Spins are stored one per byte (+1/-1),
 * indexed by slot; temp_of_slot maps each slot to its temperature index. */
typedef struct {
    int L;                   /* lattice side, >= 2                              */
    int n_T;                 /* temperatures (= slots) per copy, 1..64          */
    int R;                   /* realizations held in this state                 */
    int rng;                 /* ORC_RNG_WORDS (0) or ORC_RNG_PLANES (1)          */
    uint64_t seed;           /* Philox key                                      */
    int64_t t;               /* sweeps done (global sweep index of the next)    */
    const int32_t *rid;      /* [R] realization id used as Philox counter word 2 */
    const int8_t *J;         /* [R][N][3] couplings +-1, bond (i, i + e_mu)      */
    const double *betas;     /* [n_T] inverse temperatures, index 0 = ladder start */
    int8_t *spins;           /* [R][2][n_T][N]                                   */
    int32_t *temp_of_slot;   /* [R][2][n_T]                                      */
    int64_t *Urun;           /* [R][2][n_T] running unsatisfied-bond count or NULL */
    int64_t *flip_tries;     /* [n_T][7] attempts by (temperature, u) or NULL    */
    int64_t *flip_acc;       /* [n_T][7] accepted flips (with flip_tries)        */
    int64_t *swap_tries;     /* [n_T-1] swap attempts per pair or NULL           */
    int64_t *swap_acc;       /* [n_T-1] accepted swaps (with swap_tries)         */
    double h;                /* external field, a multiple of 1/4 (|h| <= 8)     */
} orc_sim;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t orc_flip_threshold(double beta, int u);
/* the flip draw of (realization id r, copy c, slot, sweep t, site i) under stream `rng` */
uint32_t orc_flip_draw(uint64_t seed, int rng, uint32_t i, uint32_t t, uint32_t r, int c, int slot);
uint32_t orc_swap_threshold(double dbeta_abs, int64_t n);
int orc_n_phases(int L);
int orc_colour(int L, int x, int y, int z);
int orc_local_unsat(int L, const int8_t *J, const int8_t *s, int i);
int64_t orc_unsat_bonds(int L, const int8_t *J, const int8_t *s);
void orc_init(orc_sim *sim);
void orc_reset_running_energy(orc_sim *sim);
/* returns 0; -1 if the running energy disagrees with the recomputed one after
 * a sweep; -2 on invalid sizes */
int orc_sweep(orc_sim *sim, int64_t n_sweeps, int swap_every);
/* energy [R][2][n_T] by temperature index; overlap [R][n_T] (either may be NULL) */
void orc_observables(const orc_sim *sim, int32_t *energy, int32_t *overlap);
/* magnetization sum_i s_i [R][2][n_T] by temperature index */
void orc_magnetization(const orc_sim *sim, int32_t *magnetization);
/* flip cost 12 - 4u + 2h(2S - 1) for a spin with bit S (s = 2S - 1) and u
 * unsatisfied bonds; the flip is certain when it is <= 0, otherwise it is
 * taken iff draw < floor(2^32 exp(-beta cost)) */
uint32_t orc_flip_threshold_h(double beta, int u, int S, double h);

/* one measurement of the overlap moments and plane-sum autocorrelations,
 * added to count/sum_q2 [R][n_T], sum_q4 [R][n_T][2] (lo, hi), sum_c [R][n_T][L] */
void orc_measure(const orc_sim *sim, int64_t *count, int64_t *sum_q2, uint64_t *sum_q4, int64_t *sum_c);

#endif
