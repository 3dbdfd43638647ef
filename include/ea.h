/*
 * ea.h - C ABI of the MI355X (gfx950) parallel-tempering Metropolis library
 * for the three-dimensional +-J Edwards-Anderson model over bit-packed
 * temperature replicas (Fang et al., arXiv:1311.5582).
 *
 * Model (Sec. 2.2, Eq. 1, h = 0): H = -sum over the 3N nearest-neighbour
 * bonds of a periodic L x L x L simple cubic lattice of J_b s_i s_j, with
 * s, J in {+1, -1}.  Site i = x + L*(y + L*z); couplings[r][i][mu] is the bond
 * between i and its +mu neighbour (mu = 0:x, 1:y, 2:z).  J = +1 is
 * ferromagnetic, so the all-ferro ground state has E = -3N.
 *
 * Dynamics: checkerboard single-spin-flip Metropolis (Sec. 2.3, 3.1) with
 * integer thresholds looked up by temperature and the 4-bit column 2E+S
 * (Sec. 4.3.1, 4.3.2), Philox4x32-10 random numbers (the counter-based family
 * of Sec. 4.3.2), and parallel-tempering swaps of adjacent temperatures
 * (Sec. 2.4, 4.1) that exchange table rows, not spins.  Each realization
 * carries two independent copies ("replicas" in the spin-glass sense) so that
 * the overlap q can be measured.  Results are a pure function of the inputs
 * and the seed: they do not depend on launch shape, batching, or how the
 * sweeps are split across calls.
 *
 * The random stream, with key (lo32(seed), hi32(seed)) and counter words
 * (c0, c1, c2, c3):
 *   flip draw for (realization r, copy c, slot s, sweep t, site i):
 *       block(i, t, r, c<<24 | s>>2)[s & 3]; the flip is taken iff u >= 3 or
 *       draw < floor(2^32 exp(-beta_k (12 - 4u))) (clamped to 2^32-1), where
 *       u is the number of unsatisfied bonds at i and k = temp_of_slot[s].
 *   swap draw for pair (k, k+1) after sweep t: block(k, t, r, 1<<28 | c<<24)[0].
 *   initial spin: s = +1 iff block(i, 0, r, 2<<28 | c<<24 | s>>2)[s & 3] & 1.
 * A swap pass follows sweep t iff swap_every > 0 and (t+1) % swap_every == 0;
 * it visits k = 0 .. n_T-2 in order, accepting when (beta_k - beta_{k+1}) *
 * (E_a - E_b) >= 0 and otherwise iff draw < floor(2^32 exp(-2|beta_k -
 * beta_{k+1}| |U_a - U_b|)), with U the number of unsatisfied bonds.  Odd L
 * (not bipartite) is updated in three colour classes (g(x)+g(y)+g(z)) mod 3,
 * g(x) = x & 1 for x < L-1, g(L-1) = 2; even L in the two parity classes,
 * parity 0 first.
 *
 * Conventions for every function below:
 *   - Every function returns EA_OK (0) or a negative status; ea_last_error()
 *     then returns a thread-local message.  No C++ exception crosses the ABI.
 *   - Input arrays are caller-owned host memory, read during the call only.
 *     Output arrays are caller-allocated host memory of the documented shape.
 *   - A handle is not thread-safe; distinct handles may be used concurrently
 *     from different threads.
 *   - Device memory is owned by the handle and released by ea_destroy.
 */
#ifndef EA_H
#define EA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define EA_OK        0
#define EA_EINVAL   -1   /* an argument is out of range; nothing was changed      */
#define EA_ENOMEM   -2   /* a device or host allocation failed                    */
#define EA_EDEVICE  -3   /* a HIP call failed (message names it)                  */
#define EA_ESTATE   -4   /* the handle cannot do this now (e.g. sweep counter full) */
#define EA_EBUSY    -5   /* the job is held by another live plan (ea_plan_create)  */

/* spin layouts (Sec. 4.3.3) */
#define EA_LAYOUT_CAMSC 0  /* 1 bit per temperature slot, 32 slots per 32-bit word; the
                              bond energies are widened to 4-bit segments only to sum */
#define EA_LAYOUT_AMSC4 1  /* 4-bit segment per slot (spin in bit 0), 8 slots per word */
#define EA_LAYOUT_AMSC3 2  /* 3-bit segment per slot (spin in bit 0), 10 slots per word; the
                              local energy is summed in the segments and joined with S slot by
                              slot                                                            */
#define EA_LAYOUT_AMSC1 3  /* 1 bit per slot, 32 slots per word (stored like CAMSC); the local
                              energy of each slot is summed on its own                        */

/* flip-draw streams (Sec. 4.3.2: raw 32-bit integers against 32-bit thresholds) */
#define EA_RNG_WORDS  0    /* one Philox output word per (slot, site, sweep), as in the
                              stream description above                                  */
#define EA_RNG_PLANES 1    /* the same 32-bit uniform per (slot, site, sweep), stored
                              bit-sliced: slots form halves of 16 (h = slot >> 4); bit
                              31 - p of slot s's uniform is bit s & 15 of the 16-bit
                              field p & 1 of word (p & 7) >> 1 of
                              block(i, t, r, 4<<28 | c<<24 | h<<8 | p>>3).  The compare
                              is decided at the first differing bit, so the kernel
                              draws only the planes it needs                             */

#define EA_MAX_TEMPS 64    /* temperatures (slots) per copy                           */
#define EA_MAX_L     32    /* lattice side                                            */

typedef struct ea_sim ea_sim;   /* opaque handle: one job of R realizations x 2 copies */

typedef struct ea_options {
    int layout;          /* EA_LAYOUT_CAMSC (default), _AMSC4, _AMSC3 or _AMSC1         */
    int block_threads;   /* threads per workgroup: 0 = library choice, else a multiple
                            of 64 in [64, 1024]                                        */
    int words_resident;  /* spin words per site held in LDS at once: 0 = as many as fit;
                            fewer makes the kernel stage word groups through HBM       */
    int split;           /* 0 = auto: a job with fewer ladders than CUs (CAMSC, <= 32
                            temperatures, even L) spreads each ladder over 2 or 4
                            workgroups when each keeps >= 2048 site-groups of work per
                            sweep; 1 = never; 2 = whenever possible; 3 = whenever
                            possible, by slot groups only.  Two workgroups of a ladder
                            split it by lattice halves along z, each with every slot
                            (word draws, L >= 4, no field, natural site order; the
                            halves trade their boundary planes after every colour
                            class), otherwise by slot groups, each with the whole
                            lattice (they meet only at swap points).  Batches and
                            plans apply the same rule to all their jobs together       */
    int rng;             /* flip-draw stream: EA_RNG_WORDS (default) or EA_RNG_PLANES
                            (CAMSC only); both give each flip the acceptance law
                            P(draw < threshold) = threshold / 2^32                      */
    double field;        /* external field h of Eq. 1 (H gains -h sum_i s_i): a multiple of
                            1/4 in [-8, 8], so that every energy difference the swap step
                            needs is exact; default 0.  The flip cost becomes
                            12 - 4u + 2h s and the swap step compares E = 2U - 3N - h M.
                            Needs EA_RNG_WORDS                                              */
    void *stream;        /* hipStream_t to run on; NULL = the default stream            */
    /* optional device allocator (e.g. backed by a framework's caching allocator);
       both NULL = hipMalloc / hipFree.  dev_alloc returns NULL on failure.            */
    void *(*dev_alloc)(size_t bytes, void *ctx);
    void (*dev_free)(void *ptr, void *ctx);
    void *alloc_ctx;
    int site_order;      /* order of the spin words and coupling bytes in the workgroup's
                            scratchpad, after the allocation schemes of Sec. 4.2.1:
                            EA_ORDER_NATURAL (default; the "unified" lattice) or
                            EA_ORDER_BY_CLASS (the "separated" one: each checkerboard
                            class contiguous, CAMSC and even L only; such a job runs
                            only in launches of its own: ea_sweep, a one-job batch
                            or plan, EA_EINVAL in a mix).  Results never depend on it  */
} ea_options;

#define EA_ORDER_NATURAL  0
#define EA_ORDER_BY_CLASS 1

/* Fill *opt with the defaults (CAMSC, library-chosen launch, default stream,
 * hipMalloc). */
void ea_default_options(ea_options *opt);

/* Create a job (Sec. 2.2 problem statement; Sec. 3.2, 3.3 work mapping).
 *   L            lattice side, 2 <= L <= EA_MAX_L.
 *   couplings    int8 [n_realizations][L^3][3], each +1 or -1 (copied).
 *   betas        double [n_T] inverse temperatures, finite and > 0; index 0 is
 *                "temperature index 0" of the ladder (copied).
 *   n_T          1 <= n_T <= EA_MAX_TEMPS.
 *   n_realizations  >= 1; realization r uses r as its Philox counter word.
 *   seed         64-bit Philox key.
 *   opt          NULL for defaults.
 * Initial state: spins from the initial-spin stream, temp_of_slot[s] = s,
 * sweeps_done = 0.  Errors: EA_EINVAL (argument), EA_ENOMEM, EA_EDEVICE. */
int ea_create(int L, const int8_t *couplings, const double *betas, int n_T,
              int n_realizations, uint64_t seed, const ea_options *opt, ea_sim **out);

/* Run n_sweeps >= 0 sweeps (Sec. 3.1: one sweep = the colour classes in
 * order), with a parallel-tempering pass after every sweep t for which
 * swap_every > 0 and (t+1) % swap_every == 0 (Sec. 4.1); swap_every = 0 turns
 * PT off.  Asynchronous on the handle's stream when one was given, otherwise
 * synchronous.  EA_ESTATE if the total sweep count would reach 2^32.
 * A split job (ea_sim_info: split_parts > 1) runs 2 or 4 workgroups per
 * ladder that wait for each other with a bounded wait, at swap points and,
 * split by lattice halves (ea_sim_split), for boundary words in every colour
 * class (the launch needs only that many of its workgroups resident at once
 * to make progress); should a wait ever time out (for instance when other work holds
 * the device for about a second), this call (or the next ea_observables /
 * ea_state on an asynchronous stream) returns EA_EDEVICE and the state is
 * invalid until ea_set_state. */
int ea_sweep(ea_sim *sim, int64_t n_sweeps, int swap_every);

/* One launch over the ladders of several jobs of uneven size (Sec. 3.3 maps
 * realizations to workgroups; here the ladders of all jobs share one queue).  n_sweeps[j] and
 * swap_every[j] apply to sims[j] exactly as in ea_sweep; each job's results
 * equal those of running it alone.  All sims must live on the current device
 * and share one layout; the launch uses sims[0]'s stream, after the work
 * already queued on every job's own stream, and returns when it is done. */
int ea_sweep_batch(ea_sim *const *sims, int n_sims, const int64_t *n_sweeps,
                   const int *swap_every);

/* For callers that cannot allocate device memory: code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * ordering and results as ea_sweep_batch, but the launch's work-queue counter,
 * job descriptors and ladder list live in a static workspace of the library
 * (about 1.1 MB, one copy per device, held until the process ends) instead of
 * buffers allocated per call; no device memory is allocated or freed.
 * Limits: at most EA_NOALLOC_MAX_JOBS jobs, and at most EA_NOALLOC_MAX_LADDERS
 * ladders (2 x realizations) over the jobs with n_sweeps > 0; beyond them
 * EA_EINVAL and nothing runs.  A single job takes ea_sweep's lone launch,
 * which uses only the job's own buffers.  Every call on one device shares
 * that device's workspace and keeps the last call's contents: calls that
 * overlap in time on one device (several host threads) race and must be
 * serialised by the caller; calls made one after another are safe, since
 * each returns only when its launch is done. */
#define EA_NOALLOC_MAX_JOBS    256
#define EA_NOALLOC_MAX_LADDERS 262144
int ea_sweep_batch_noalloc(ea_sim *const *sims, int n_sims, const int64_t *n_sweeps,
                           const int *swap_every);

/* ---- Launch plans: one step over several jobs, captured once and replayed ----
 * A plan freezes a job list and a step (sweeps_per_step sweeps of every job,
 * with swap_every[j] for job j, as ea_sweep would run them) into one
 * persistent launch whose ladders are ordered largest first, and captures the
 * step in a hipGraph; ea_plan_run replays it.  The jobs' sweep counters live
 * in device memory, so every replay continues each job's random stream: the
 * results equal those of ea_sweep on each job alone.  The workgroup size is
 * opt->block_threads, or picked by timing candidates on scratch copies of the
 * jobs (results never depend on it).  When the jobs together have fewer
 * ladders than the device has compute units and every job can be split (the
 * conditions of ea_options.split, which each job's own setting can turn
 * off), the step spreads each ladder over 2 or 4 workgroups; with autotune
 * the split and unsplit shapes are timed against each other.  A job belongs to at most one live plan
 * (EA_EBUSY otherwise).  Each run is ordered after the work queued on the
 * jobs' own streams, and later work queued there is ordered after the run.
 * Destroying a job while a plan holds it makes ea_plan_run return EA_ESTATE. */
typedef struct ea_plan ea_plan;
typedef struct ea_plan_options {
    int block_threads;   /* 0 = autotune (or, with autotune = 0, the largest planned size) */
    int autotune;        /* 1 = time 256/512/768/1024 threads, each unsplit and split where
                            possible, on scratch copies; cache the best per device
                            architecture and job shapes (also in the file named by
                            the environment variable EA_TUNE_CACHE, if set)          */
    int use_graph;       /* 1 = replay a captured hipGraph (default); 0 = plain launches */
    int reserved_;
    void *stream;        /* hipStream_t; NULL = a stream owned by the plan, runs synchronous */
} ea_plan_options;

void ea_default_plan_options(ea_plan_options *opt);
int ea_plan_create(ea_sim *const *sims, int n_sims, int sweeps_per_step, const int *swap_every,
                   const ea_plan_options *opt, ea_plan **out);
/* Run n_steps >= 0 steps.  EA_ESTATE if a sweep counter would reach 2^32. */
int ea_plan_run(ea_plan *plan, int64_t n_steps);
/* Launch shape of a plan's step: workgroup size, workgroups launched, ladders
 * (units), dynamic LDS bytes, whether a graph is replayed, and workgroups
 * per ladder (1, or 2/4 for split ladders).  Any pointer may be NULL. */
int ea_plan_info(const ea_plan *plan, int *block_threads, int *grid, int *n_units, size_t *lds_bytes,
                 int *uses_graph, int *split_parts);
void ea_plan_destroy(ea_plan *plan);

/* ---- Serving: continuous batching of jobs on one GPU ----
 * Jobs are submitted with host inputs and wait.  Each ea_server_step
 * (1) admits waiting jobs while their device footprint (ea_job_footprint)
 * fits the budget: first fit in arrival order (EA_ADMIT_FIFO), or, until the
 * running jobs hold fill_ladders ladders, shortest remaining work first
 * (sweeps x L^3 x n_T x R; EA_ADMIT_SHORTEST: a long job can wait behind a
 * stream of shorter ones) or highest response ratio first ((waited +
 * estimated service) / estimated service, with the service time from the
 * measured rate of the server's own steps; EA_ADMIT_RESPONSE_RATIO: the
 * longer a job has waited relative to its size, the sooner it runs); the
 * jobs are created while the previous step still
 * runs on the GPU; (2) waits for that step and retires finished jobs:
 * energies and overlaps are measured, device state is freed; (3) launches the
 * next step over every running job and returns without waiting for it.  In a
 * step the running job with the most work per ladder and sweep (L^3 x n_T)
 * runs quantum sweeps and every other job round(quantum x that work / its
 * own) sweeps, so that all ladders of the step take about equally long (at
 * most the sweeps it has left).  With more ladders than compute units the
 * launch takes ceil(ladders / CUs) rounds of such units, the last one partly
 * idle; with pack_rounds the jobs of lowest response ratio (never all) then
 * run shorter units, at least a quarter of the others', sized to fill the
 * idle slots of floor(ladders / CUs) rounds.  A graph-captured plan is
 * replayed while the job set and sweep counts are unchanged.  A job's results are the
 * same alone and in any mix. */
#define EA_ADMIT_FIFO           0
#define EA_ADMIT_SHORTEST       1
#define EA_ADMIT_RESPONSE_RATIO 2
#define EA_JOB_QUEUED    0
#define EA_JOB_RUNNING   1
#define EA_JOB_DONE      2
#define EA_JOB_CANCELLED 3
#define EA_JOB_FAILED    4

typedef struct ea_server ea_server;
typedef struct ea_server_options {
    size_t hbm_budget_bytes;  /* device bytes for job state; 0 = 80% of free memory at creation */
    int quantum_sweeps;       /* sweeps per step of the job with the most work per sweep (400)    */
    int layout;               /* EA_LAYOUT_* of every job                                         */
    int max_active;           /* admitted jobs at once, <= 4095 (0 = 4095)                        */
    int autotune;             /* 1 = tune each job mix's workgroup size (cached by shape); default 0 */
    int keep_state;           /* keep each finished job's spins and permutation on the host       */
    int rng;                  /* EA_RNG_* flip-draw stream of every job (planes: CAMSC only); the
                                 jobs run without a field                                        */
    int policy;               /* EA_ADMIT_RESPONSE_RATIO (default), _SHORTEST or _FIFO            */
    int fill_ladders;         /* SHORTEST, RESPONSE_RATIO: stop admitting once the running jobs hold this
                                 many ladders (2 x realizations); 0 = 4 x the compute units      */
    int pack_rounds;          /* 1 (default): when a step's ladders overfill their last round of
                                 compute units, the least urgent jobs run shorter units in that
                                 round's idle slots; 0: every unit of a step about equally long  */
    void *stream;             /* hipStream_t of the steps; NULL = a stream owned by the server    */
} ea_server_options;

void ea_default_server_options(ea_server_options *opt);
int ea_server_create(const ea_server_options *opt, ea_server **out);
/* Queue a job (inputs as ea_create; copied).  EA_ENOMEM if it alone exceeds the budget. */
int ea_server_submit(ea_server *sv, int L, const int8_t *couplings, const double *betas, int n_T,
                     int n_realizations, uint64_t seed, int64_t n_sweeps, int swap_every, int64_t *job_id);
/* Admit, finish the step in flight, retire, launch the next step.  Counts
 * after the call: running jobs include those of the step just launched. */
int ea_server_step(ea_server *sv, int *n_running, int *n_queued, int *n_finished);
int ea_server_status(ea_server *sv, int64_t job_id, int *status, int64_t *sweeps_done);
/* Results of a DONE job: energy int32 [R][2][n_T], overlap int32 [R][n_T] (as ea_observables). */
int ea_server_result(ea_server *sv, int64_t job_id, int32_t *energy, int32_t *overlap);
/* Final spins [R][2][n_T][L^3] and temp_of_slot [R][2][n_T] of a DONE job (needs keep_state). */
int ea_server_final_state(ea_server *sv, int64_t job_id, int8_t *spins, int32_t *temp_of_slot);
int ea_server_cancel(ea_server *sv, int64_t job_id);    /* queued or running; frees its memory */
int ea_server_release(ea_server *sv, int64_t job_id);   /* forget a finished job's results     */
int ea_server_stats(const ea_server *sv, size_t *hbm_used, size_t *hbm_budget, int64_t *steps,
                    int64_t *plans_built, int64_t *launches_replayed);
void ea_server_destroy(ea_server *sv);

/* Device bytes ea_create allocates for such a job without a field (a field
 * lengthens the swap tables; ea_sim_footprint reports a live job exactly).
 * Includes the boundary exchange of a split by lattice halves for CAMSC jobs
 * of one word per site, even L >= 4 and two workgroups per ladder within the
 * current device's compute units (256 when no device can be queried).
 * Host-only computation. */
int ea_job_footprint(int L, const double *betas, int n_T, int n_realizations, int layout, size_t *bytes);
/* Device bytes a live job holds. */
int ea_sim_footprint(const ea_sim *sim, size_t *bytes);

/* Measurement (Sec. 4.1, separate kernel): energy int32 [R][2][n_T] indexed by
 * temperature index, E = 2U - 3N (the bond part: with a field the total is
 * E - h M, see ea_magnetization); overlap int32 [R][n_T]:
 * q_k = sum_i s_i(copy 0 at temperature k) s_i(copy 1 at temperature k).
 * Either pointer may be NULL.  Synchronous. */
int ea_observables(ea_sim *sim, int32_t *energy, int32_t *overlap);
/* Magnetization M = sum_i s_i [R][2][n_T] by temperature index (with a field
 * the total energy is energy - h M).  Synchronous. */
int ea_magnetization(ea_sim *sim, int32_t *magnetization);

/* Spin dump (Sec. 4.1: the configurations are copied out of the simulation
 * kernel's state for measurements and analysis on the host).  Read the full
 * state: spins int8 [R][2][n_T][L^3] (+1/-1, indexed by slot), temp_of_slot
 * int32 [R][2][n_T] (Sec. 4.3.1: a slot keeps its spins and changes
 * temperature on an accepted swap), sweeps_done.  Any pointer may be NULL.
 * Synchronous.  Uses a temporary device buffer of R*2*n_T*L^3 bytes
 * (EA_ENOMEM if it cannot be had).  With ea_set_state this is
 * checkpoint/resume: the stream is counter-based, so a resumed run continues
 * bit-identically. */
int ea_state(ea_sim *sim, int8_t *spins, int32_t *temp_of_slot, int64_t *sweeps_done);

/* Restore a spin dump (the inverse of ea_state, Sec. 4.1).  Overwrite the
 * state (same shapes; temp_of_slot must be a permutation of 0..n_T-1 in
 * every ladder, sweeps_done in [0, 2^32)).  EA_EINVAL leaves the state
 * unchanged.  The measurement accumulators and swap counts are kept. */
int ea_set_state(ea_sim *sim, const int8_t *spins, const int32_t *temp_of_slot,
                 int64_t sweeps_done);

/* Accepted swaps per (realization, copy, pair k) since creation, uint64
 * [R][2][n_T-1] (n_T = 1: nothing written); the device counts in 64 bits.
 * Synchronous.  (Sec. 2.4: the acceptance rate of each adjacent pair is what
 * a temperature ladder is tuned by.) */
int ea_swap_acceptance(ea_sim *sim, uint64_t *accepted);

/* ---- Measurements of the spin-glass order (Sec. 5: Binder ratio of the overlap,
 * correlation length) ----
 * For realization r and temperature index k, with q_i = s_i(copy 0 at T_k) *
 * s_i(copy 1 at T_k), q = sum_i q_i, and Q_a[p] the sum of q_i over the sites
 * whose coordinate a (x, y, z) equals p:
 *   C[d] = sum_a sum_p Q_a[p] Q_a[(p + d) mod L],   d = 0 .. L-1,
 * so that the axis-summed |sum_i q_i exp(i k x_a)|^2 equals sum_d C[d] cos(k d).
 * ea_measure adds one measurement of the current state to device-resident
 * accumulators: count += 1, sum_q2 += q^2, sum_q4 += q^4 (exact, a 128-bit sum
 * kept as two 64-bit words, low word first), sum_c[d] += C[d].  Asynchronous
 * on the handle's stream when one was given, otherwise synchronous. */
int ea_measure(ea_sim *sim);
/* Copy the accumulators: count and sum_q2 int64 [R][n_T], sum_q4 uint64 [R][n_T][2],
 * sum_c int64 [R][n_T][L]; any pointer may be NULL.  Synchronous. */
int ea_measure_read(ea_sim *sim, int64_t *count, int64_t *sum_q2, uint64_t *sum_q4, int64_t *sum_c);
/* Zero the accumulators (ea_create starts them at zero; ea_set_state keeps them). */
int ea_measure_reset(ea_sim *sim);
/* Per temperature index, from the accumulators with [.] the average over
 * realizations of each realization's time average <.>:
 *   binder[k]    = (3 - [<q^4>] / [<q^2>]^2) / 2,
 *   xi_over_L[k] = sqrt(chi(0) / chi(k_min) - 1) / (2 sin(k_min / 2)) / L,
 * chi(0) = [<q^2>] / N, chi(k_min) = [<sum_d C[d] cos(k_min d)>] / (3 N),
 * k_min = 2 pi / L (NaN where chi(0) < chi(k_min)).  Host arithmetic in double
 * on the exact sums.  EA_ESTATE if a realization has no measurement. */
int ea_binder_xi(ea_sim *sim, double *binder, double *xi_over_L);

/* Shape queries. */
int ea_get_dims(const ea_sim *sim, int *L, int *n_T, int *n_realizations, int *layout);
/* Launch plan of a lone ea_sweep: workgroup size, spin words resident in LDS,
 * workgroups per ladder (1, or 2/4 when split), dynamic LDS bytes. */
int ea_sim_info(const ea_sim *sim, int *block_threads, int *words_resident, int *split_parts, size_t *lds_bytes);
/* How a lone ea_sweep splits the job's ladders: workgroups per ladder (1: not
 * split) and whether they split it by lattice halves (1) or by slot groups (0). */
int ea_sim_split(const ea_sim *sim, int *split_parts, int *by_halves);

/* Release the handle and its device memory (NULL is a no-op). */
void ea_destroy(ea_sim *sim);

/* Thread-local message for the last non-OK status on this thread. */
const char *ea_last_error(void);

/* Host-side table helpers (no device use), the same formulas the library
 * uses (Sec. 4.3.1, 4.3.2):
 *   flip_thr[k][u] = min(floor(2^32 exp(-betas[k] (12 - 4u))), 2^32-1), u = 0..2,
 *   written as uint32 [n_T][3];
 *   swap threshold = min(floor(2^32 exp(-2 dbeta_abs n)), 2^32-1). */
int ea_flip_thresholds(const double *betas, int n_T, uint32_t *flip_thr);
uint32_t ea_swap_threshold(double dbeta_abs, int64_t n);

/* Library build identification (static string). */
const char *ea_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EA_H */
