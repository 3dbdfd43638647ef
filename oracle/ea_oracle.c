/*
 * CPU oracle for the parallel-tempering Metropolis simulation of the
 * three-dimensional +-J Edwards-Anderson model (Fang et al., "Parallel
 * Tempering Simulation of the three-dimensional Edwards-Anderson Model with
 * Compact Asynchronous Multispin Coding on GPU", arXiv:1311.5582).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code with the HIP path: it has its own Philox, its own threshold formulas
 * and its own lattice indexing, and it stores one spin per byte (int8, +-1).
 *
 * What it computes (paper sections in brackets):
 *   - H = -sum_<ij> J_ij s_i s_j - h sum_i s_i over the 3N nearest-neighbour
 *     bonds of a periodic L^3 simple cubic lattice [Sec. 2.2, Eq. 1]; the
 *     field h is a multiple of 1/4 so that every energy difference the swap
 *     step needs is an exact multiple of 1/2.
 *   - Single-spin-flip Metropolis with acceptance min(1, exp(-beta dE))
 *     [Sec. 2.3], visited as a checkerboard of sublattices updated one after
 *     the other [Sec. 3.1]; odd L uses three colour classes (see below).
 *   - dE is a function of the number u of unsatisfied bonds around the site
 *     and of its spin: dE = 12 - 4u + 2h s (the XOR form of the local energy,
 *     Sec. 4.3, Eq. e; the spin enters through the 2E+S column, Sec. 4.3.1).
 *   - The flip probability is taken from a table indexed by temperature and
 *     local energy [Sec. 4.3.1], converted to 32-bit unsigned integers and
 *     compared with the raw integer output of the random number generator
 *     [Sec. 4.3.2]: flip iff draw < floor(2^32 exp(-beta dE)), clamped to
 *     2^32-1, and always when dE <= 0.
 *   - Random numbers: Philox4x32 with 10 rounds (Salmon et al., SC'11, the
 *     counter-based generator family evaluated in Sec. 4.3.2).  Counter words
 *     and key are laid out below; every draw is a pure function of
 *     (seed, realization, copy, slot, sweep, site), so the visiting order
 *     inside a colour class does not matter.
 *   - Parallel tempering [Sec. 2.4, Sec. 4.1]: after every swap_every-th
 *     sweep, one ascending pass over adjacent temperature pairs; the pair
 *     (k, k+1) exchanges temperatures with probability
 *     min(1, exp((beta_k - beta_{k+1}) (E_a - E_b))), and an accepted swap
 *     exchanges the two temperatures' table rows, not the spins
 *     [Sec. 4.3.1].
 *   - Two independent copies per realization, each with its own ladder, so
 *     that the overlap q between copies can be measured.
 *
 * Readings where the paper is silent or garbled (each is documented in the
 * design notes of the repository):
 *   - Coupling sign: textbook H = -sum J s s with J = +1 ferromagnetic.
 *     Bit form: spin bit = (s == +1), coupling bit = (J == -1); a bond is
 *     unsatisfied iff spin_i XOR spin_j XOR J_bit = 1.
 *   - Metropolis compare: flip iff draw < threshold (Eq. r read as R < P).
 *   - Odd L (not bipartite): colour(x,y,z) = (g(x)+g(y)+g(z)) mod 3 with
 *     g(x) = x & 1 for x < L-1 and g(L-1) = 2, a proper colouring.
 *   - Swap pass order: k = 0 .. n_T-2 ascending, sequential.
 *
 * Philox counter layout (c0, c1, c2, c3), key = (lo32(seed), hi32(seed)):
 *   flip  draw (r, c, slot, t, site i): ctr (i, t, r, 0<<28 | c<<24 | slot>>2), word slot&3
 *   swap  draw (r, c, pair k, t)      : ctr (k, t, r, 1<<28 | c<<24), word 0
 *   init  spin (r, c, slot, site i)   : ctr (i, 0, r, 2<<28 | c<<24 | slot>>2), word slot&3, bit 0
 *
 * Second flip-draw stream (ORC_RNG_PLANES), same acceptance law: the slot's
 * 32-bit uniform is spread over 32 bit planes.  Slots form halves of 16
 * (h = slot >> 4); plane p of half h (p = 0 holds the most significant bit)
 * is the 16-bit field p & 1 (low field first) of word (p & 7) >> 1 of
 *   ctr (i, t, r, 4<<28 | c<<24 | h<<8 | p>>3),
 * and bit slot & 15 of plane p is bit 31 - p of the slot's uniform.  The
 * comparison draw < threshold is then decided at the first plane where the
 * two differ, which lets a bit-parallel implementation stop early.
 *
 * Build: gcc -O2 -fPIC -shared (see oracle/build.py).  No threads, no SIMD
 * intrinsics, no blocking or fusion.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#include "ea_oracle.h"

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 4 "Philox").     */
/* Round: (c0,c1,c2,c3) -> (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1,  */
/* lo(M0*c0)); the key is bumped by the Weyl constants between rounds.     */
/* ---------------------------------------------------------------------- */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u
#define ORC_PHILOX_ROUNDS 10

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < ORC_PHILOX_ROUNDS; ++round) {
        if (round > 0) {
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One 32-bit word of the stream: block(ctr)[word]. */
static uint32_t orc_draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int word)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[word];
}

#define ORC_DOMAIN_FLIP 0u
#define ORC_DOMAIN_SWAP 1u
#define ORC_DOMAIN_INIT 2u
#define ORC_DOMAIN_PLANE 4u

static uint32_t orc_c3(uint32_t domain, int copy, int slot_group)
{
    return (domain << 28) | ((uint32_t)copy << 24) | (uint32_t)slot_group;
}

/* The flip draw of one (realization, copy, slot, sweep, site). */
uint32_t orc_flip_draw(uint64_t seed, int rng, uint32_t i, uint32_t t, uint32_t r, int c, int slot)
{
    if (rng != ORC_RNG_PLANES) return orc_draw(seed, i, t, r, orc_c3(ORC_DOMAIN_FLIP, c, slot >> 2), slot & 3);
    uint32_t uniform = 0u;
    for (int p = 0; p < 32; ++p) {
        uint32_t w = orc_draw(seed, i, t, r, orc_c3(ORC_DOMAIN_PLANE, c, ((slot >> 4) << 8) | (p >> 3)),
                              (p & 7) >> 1);
        uint32_t plane = (w >> (16 * (p & 1))) & 0xFFFFu;
        uniform |= ((plane >> (slot & 15)) & 1u) << (31 - p);
    }
    return uniform;
}

/* ---------------------------------------------------------------------- */
/* Integer probability tables (Sec. 4.3.1 table, Sec. 4.3.2 integers).     */
/* ---------------------------------------------------------------------- */
static uint32_t orc_prob_to_u32(double p)
{
    double x = floor(ldexp(p, 32));
    if (x >= 4294967295.0) return 0xFFFFFFFFu;
    if (x <= 0.0) return 0u;
    return (uint32_t)x;
}

/* Metropolis threshold for a site with u unsatisfied bonds (u in 0..2):
 * dE = 12 - 4u > 0 and P = exp(-beta dE).  For u >= 3, dE <= 0 and the flip
 * is always taken; the table is never consulted. */
uint32_t orc_flip_threshold(double beta, int u)
{
    if (u >= 3) return 0xFFFFFFFFu;
    double dE = (double)(12 - 4 * u);
    return orc_prob_to_u32(exp(-(beta * dE)));
}

uint32_t orc_flip_threshold_h(double beta, int u, int S, double h)
{
    double dE = (double)(12 - 4 * u) + 2.0 * h * (double)(2 * S - 1);
    if (dE <= 0.0) return 0xFFFFFFFFu;
    return orc_prob_to_u32(exp(-(beta * dE)));
}

/* Swap threshold for |beta_k - beta_{k+1}| = dbeta_abs and |U_a - U_b| = n:
 * the energy difference is 2n, so P = exp(-2 |dbeta| n) when the move is
 * unfavourable. */
uint32_t orc_swap_threshold(double dbeta_abs, int64_t n)
{
    return orc_prob_to_u32(exp(-(2.0 * dbeta_abs * (double)n)));
}

/* ---------------------------------------------------------------------- */
/* Lattice.  Site i = x + L*(y + L*z); bond (i, mu) joins i and i + e_mu.  */
/* ---------------------------------------------------------------------- */
static int orc_wrap(int a, int L)
{
    if (a < 0) return a + L;
    if (a >= L) return a - L;
    return a;
}

static int orc_site(int L, int x, int y, int z)
{
    return x + L * (y + L * z);
}

/* neighbour of i along axis mu (0=x, 1=y, 2=z) in direction dir (+1 or -1) */
static int orc_neighbour(int L, int i, int mu, int dir)
{
    int x = i % L, y = (i / L) % L, z = i / (L * L);
    if (mu == 0) x = orc_wrap(x + dir, L);
    if (mu == 1) y = orc_wrap(y + dir, L);
    if (mu == 2) z = orc_wrap(z + dir, L);
    return orc_site(L, x, y, z);
}

int orc_n_phases(int L)
{
    return (L % 2 == 0) ? 2 : 3;
}

static int orc_g(int a, int L)
{
    return (a == L - 1) ? 2 : (a & 1);
}

int orc_colour(int L, int x, int y, int z)
{
    if (L % 2 == 0) return (x + y + z) & 1;
    return (orc_g(x, L) + orc_g(y, L) + orc_g(z, L)) % 3;
}

/* Number of unsatisfied bonds among the six incidences of site i.  The bond
 * (i, j) with coupling J contributes iff J s_i s_j = -1. */
int orc_local_unsat(int L, const int8_t *J, const int8_t *s, int i)
{
    int u = 0;
    for (int mu = 0; mu < 3; ++mu) {
        int jp = orc_neighbour(L, i, mu, +1);
        int jm = orc_neighbour(L, i, mu, -1);
        if (J[3 * i + mu] * s[i] * s[jp] < 0) ++u;   /* bond (i, mu)      */
        if (J[3 * jm + mu] * s[i] * s[jm] < 0) ++u;  /* bond (i - e_mu, mu) */
    }
    return u;
}

/* Total number of unsatisfied bonds U; the energy is E = 2U - 3N. */
int64_t orc_unsat_bonds(int L, const int8_t *J, const int8_t *s)
{
    int N = L * L * L;
    int64_t U = 0;
    for (int i = 0; i < N; ++i)
        for (int mu = 0; mu < 3; ++mu) {
            int jp = orc_neighbour(L, i, mu, +1);
            if (J[3 * i + mu] * s[i] * s[jp] < 0) ++U;
        }
    return U;
}

/* ---------------------------------------------------------------------- */
/* Simulation state helpers.                                               */
/* ---------------------------------------------------------------------- */
static int8_t *orc_spins(const orc_sim *sim, int r, int c, int slot)
{
    int N = sim->L * sim->L * sim->L;
    return sim->spins + (((size_t)r * 2 + c) * sim->n_T + slot) * (size_t)N;
}

static int32_t *orc_perm(const orc_sim *sim, int r, int c)
{
    return sim->temp_of_slot + ((size_t)r * 2 + c) * sim->n_T;
}

static const int8_t *orc_couplings(const orc_sim *sim, int r)
{
    int N = sim->L * sim->L * sim->L;
    return sim->J + (size_t)r * N * 3;
}

void orc_init(orc_sim *sim)
{
    int L = sim->L, N = L * L * L;
    for (int r = 0; r < sim->R; ++r)
        for (int c = 0; c < 2; ++c) {
            for (int slot = 0; slot < sim->n_T; ++slot) {
                int8_t *s = orc_spins(sim, r, c, slot);
                for (int i = 0; i < N; ++i) {
                    uint32_t w = orc_draw(sim->seed, (uint32_t)i, 0u, (uint32_t)sim->rid[r],
                                          orc_c3(ORC_DOMAIN_INIT, c, slot >> 2), slot & 3);
                    s[i] = (w & 1u) ? (int8_t)1 : (int8_t)-1;
                }
            }
            for (int slot = 0; slot < sim->n_T; ++slot) orc_perm(sim, r, c)[slot] = slot;
        }
    sim->t = 0;
    orc_reset_running_energy(sim);
}

void orc_reset_running_energy(orc_sim *sim)
{
    if (!sim->Urun) return;
    for (int r = 0; r < sim->R; ++r)
        for (int c = 0; c < 2; ++c)
            for (int slot = 0; slot < sim->n_T; ++slot)
                sim->Urun[((size_t)r * 2 + c) * sim->n_T + slot] =
                    orc_unsat_bonds(sim->L, orc_couplings(sim, r), orc_spins(sim, r, c, slot));
}

/* One Metropolis stage over the sites of one colour class, for every slot of
 * every (realization, copy) ladder. */
static void orc_stage(orc_sim *sim, int colour, uint32_t t)
{
    int L = sim->L;
    for (int r = 0; r < sim->R; ++r) {
        const int8_t *J = orc_couplings(sim, r);
        for (int c = 0; c < 2; ++c) {
            const int32_t *temp_of_slot = orc_perm(sim, r, c);
            for (int slot = 0; slot < sim->n_T; ++slot) {
                int k = temp_of_slot[slot];
                double beta = sim->betas[k];
                int8_t *s = orc_spins(sim, r, c, slot);
                for (int z = 0; z < L; ++z)
                    for (int y = 0; y < L; ++y)
                        for (int x = 0; x < L; ++x) {
                            if (orc_colour(L, x, y, z) != colour) continue;
                            int i = orc_site(L, x, y, z);
                            int u = orc_local_unsat(L, J, s, i);
                            int S = s[i] > 0;
                            double dE = (double)(12 - 4 * u) + 2.0 * sim->h * (double)(2 * S - 1);
                            int flip;
                            if (dE <= 0.0) {
                                flip = 1;
                            } else {
                                uint32_t draw = orc_flip_draw(sim->seed, sim->rng, (uint32_t)i, t,
                                                              (uint32_t)sim->rid[r], c, slot);
                                flip = draw < orc_flip_threshold_h(beta, u, S, sim->h);
                            }
                            if (sim->flip_tries) {
                                sim->flip_tries[k * 7 + u] += 1;
                                if (flip) sim->flip_acc[k * 7 + u] += 1;
                            }
                            if (flip) {
                                s[i] = (int8_t)(-s[i]);
                                /* u unsatisfied incidences become satisfied and
                                 * the other 6 - u become unsatisfied */
                                if (sim->Urun)
                                    sim->Urun[((size_t)r * 2 + c) * sim->n_T + slot] += 6 - 2 * u;
                            }
                        }
            }
        }
    }
}

/* Replica-exchange pass after sweep t for ladder (r, c).  U is recomputed
 * from scratch for every slot. */
static void orc_swap_pass(orc_sim *sim, int r, int c, uint32_t t)
{
    int n_T = sim->n_T;
    const int8_t *J = orc_couplings(sim, r);
    int32_t *temp_of_slot = orc_perm(sim, r, c);
    int32_t slot_of_temp[ORC_MAX_TEMPS];
    int64_t U[ORC_MAX_TEMPS], up[ORC_MAX_TEMPS];
    int N = sim->L * sim->L * sim->L;
    int64_t m = (int64_t)(4.0 * sim->h);   /* exact: h is a multiple of 1/4 */
    for (int slot = 0; slot < n_T; ++slot) {
        slot_of_temp[temp_of_slot[slot]] = slot;
        const int8_t *s = orc_spins(sim, r, c, slot);
        U[slot] = orc_unsat_bonds(sim->L, J, s);
        up[slot] = 0;
        for (int i = 0; i < N; ++i) up[slot] += s[i] > 0;
    }
    for (int k = 0; k + 1 < n_T; ++k) {
        int a = slot_of_temp[k], b = slot_of_temp[k + 1];
        /* E = 2U - 3N - h M with M = 2 up - N, so 2 (E_a - E_b) = D exactly */
        int64_t D = 4 * (U[a] - U[b]) - m * (up[a] - up[b]);
        double dbeta = sim->betas[k] - sim->betas[k + 1];
        /* accept with min(1, exp(dbeta (E_a - E_b))): certain when
         * dbeta * D >= 0, decided from the signs so that no rounding enters */
        int favourable = (dbeta == 0.0) || (D == 0) || ((dbeta > 0.0) == (D > 0));
        int accept;
        if (favourable) {
            accept = 1;
        } else {
            uint32_t draw = orc_draw(sim->seed, (uint32_t)k, t, (uint32_t)sim->rid[r],
                                     orc_c3(ORC_DOMAIN_SWAP, c, 0), 0);
            double dEabs = 0.5 * (double)(D < 0 ? -D : D);   /* |E_a - E_b| */
            accept = draw < orc_prob_to_u32(exp(-(fabs(dbeta) * dEabs)));
        }
        if (sim->swap_tries) {
            sim->swap_tries[k] += 1;
            if (accept) sim->swap_acc[k] += 1;
        }
        if (accept) {
            slot_of_temp[k] = b;
            slot_of_temp[k + 1] = a;
            temp_of_slot[a] = k + 1;
            temp_of_slot[b] = k;
        }
    }
}

static int orc_check_running_energy(const orc_sim *sim)
{
    if (!sim->Urun) return 0;
    for (int r = 0; r < sim->R; ++r)
        for (int c = 0; c < 2; ++c)
            for (int slot = 0; slot < sim->n_T; ++slot) {
                int64_t U = orc_unsat_bonds(sim->L, orc_couplings(sim, r), orc_spins(sim, r, c, slot));
                if (U != sim->Urun[((size_t)r * 2 + c) * sim->n_T + slot]) return -1;
            }
    return 0;
}

int orc_sweep(orc_sim *sim, int64_t n_sweeps, int swap_every)
{
    if (sim->n_T < 1 || sim->n_T > ORC_MAX_TEMPS || sim->L < 2) return -2;
    int phases = orc_n_phases(sim->L);
    for (int64_t n = 0; n < n_sweeps; ++n) {
        uint32_t t = (uint32_t)sim->t;
        for (int colour = 0; colour < phases; ++colour) orc_stage(sim, colour, t);
        if (sim->Urun && orc_check_running_energy(sim) != 0) return -1;
        if (swap_every > 0 && ((int64_t)t + 1) % swap_every == 0)
            for (int r = 0; r < sim->R; ++r)
                for (int c = 0; c < 2; ++c) orc_swap_pass(sim, r, c, t);
        sim->t += 1;
    }
    return 0;
}

void orc_observables(const orc_sim *sim, int32_t *energy, int32_t *overlap)
{
    int L = sim->L, N = L * L * L, n_T = sim->n_T;
    for (int r = 0; r < sim->R; ++r) {
        int32_t slot_of_temp[2][ORC_MAX_TEMPS];
        for (int c = 0; c < 2; ++c) {
            const int32_t *temp_of_slot = orc_perm(sim, r, c);
            for (int slot = 0; slot < n_T; ++slot) slot_of_temp[c][temp_of_slot[slot]] = slot;
            for (int k = 0; k < n_T; ++k) {
                int64_t U = orc_unsat_bonds(L, orc_couplings(sim, r), orc_spins(sim, r, c, slot_of_temp[c][k]));
                if (energy) energy[((size_t)r * 2 + c) * n_T + k] = (int32_t)(2 * U - 3 * (int64_t)N);
            }
        }
        if (overlap)
            for (int k = 0; k < n_T; ++k) {
                const int8_t *s0 = orc_spins(sim, r, 0, slot_of_temp[0][k]);
                const int8_t *s1 = orc_spins(sim, r, 1, slot_of_temp[1][k]);
                int32_t q = 0;
                for (int i = 0; i < N; ++i) q += s0[i] * s1[i];
                overlap[(size_t)r * n_T + k] = q;
            }
    }
}

/* ---------------------------------------------------------------------- */
/* Measurements of the spin-glass order [Sec. 5: Binder ratio of the      */
/* overlap, correlation length].  For realization r and temperature index */
/* k, with q_i = s_i(copy 0 at T_k) s_i(copy 1 at T_k):                   */
/*   q        = sum_i q_i                                                  */
/*   Q_a[p]   = sum of q_i over the sites whose coordinate a (x, y, z) is p */
/*   C[d]     = sum_a sum_p Q_a[p] Q_a[(p + d) mod L],  d = 0 .. L-1        */
/* so that |sum_i q_i e^{i k x_a}|^2 summed over the three axes equals     */
/* sum_d C[d] cos(k d) for k = 2 pi m / L.  One call adds one measurement: */
/* count += 1, sum_q2 += q^2, sum_q4 += q^4 (exact, 128 bits as lo, hi),   */
/* sum_c[d] += C[d].                                                        */
/* ---------------------------------------------------------------------- */
void orc_measure(const orc_sim *sim, int64_t *count, int64_t *sum_q2, uint64_t *sum_q4, int64_t *sum_c)
{
    int L = sim->L, n_T = sim->n_T;
    int64_t Q[3][32];
    for (int r = 0; r < sim->R; ++r) {
        int32_t slot_of_temp[2][ORC_MAX_TEMPS];
        for (int c = 0; c < 2; ++c) {
            const int32_t *temp_of_slot = orc_perm(sim, r, c);
            for (int slot = 0; slot < n_T; ++slot) slot_of_temp[c][temp_of_slot[slot]] = slot;
        }
        for (int k = 0; k < n_T; ++k) {
            const int8_t *s0 = orc_spins(sim, r, 0, slot_of_temp[0][k]);
            const int8_t *s1 = orc_spins(sim, r, 1, slot_of_temp[1][k]);
            int64_t q = 0;
            for (int a = 0; a < 3; ++a)
                for (int p = 0; p < L; ++p) Q[a][p] = 0;
            for (int z = 0; z < L; ++z)
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x) {
                        int i = orc_site(L, x, y, z);
                        int qi = s0[i] * s1[i];
                        q += qi;
                        Q[0][x] += qi;
                        Q[1][y] += qi;
                        Q[2][z] += qi;
                    }
            size_t rk = (size_t)r * n_T + k;
            count[rk] += 1;
            sum_q2[rk] += q * q;
            /* q^4 < 2^61 for N <= 32^3; 128-bit sum as two words */
            uint64_t q4 = (uint64_t)(q * q) * (uint64_t)(q * q);
            uint64_t lo = sum_q4[2 * rk] + q4;
            sum_q4[2 * rk + 1] += (lo < q4) ? 1u : 0u;
            sum_q4[2 * rk] = lo;
            for (int d = 0; d < L; ++d) {
                int64_t cd = 0;
                for (int a = 0; a < 3; ++a)
                    for (int p = 0; p < L; ++p) cd += Q[a][p] * Q[a][(p + d) % L];
                sum_c[rk * (size_t)L + d] += cd;
            }
        }
    }
}

void orc_magnetization(const orc_sim *sim, int32_t *magnetization)
{
    int N = sim->L * sim->L * sim->L, n_T = sim->n_T;
    for (int r = 0; r < sim->R; ++r)
        for (int c = 0; c < 2; ++c) {
            const int32_t *temp_of_slot = orc_perm(sim, r, c);
            for (int slot = 0; slot < n_T; ++slot) {
                const int8_t *s = orc_spins(sim, r, c, slot);
                int32_t M = 0;
                for (int i = 0; i < N; ++i) M += s[i];
                magnetization[((size_t)r * 2 + c) * n_T + temp_of_slot[slot]] = M;
            }
        }
}
