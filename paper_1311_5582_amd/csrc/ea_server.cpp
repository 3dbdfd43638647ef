// Serving loop: continuous batching of simulation jobs on one GPU.
//
// Jobs are submitted with host inputs and wait.  Each step (1) admits waiting
// jobs while their exact HBM footprint fits the budget - first fit in arrival
// order, or shortest remaining work first until the running jobs hold enough
// ladders to fill the device - creating them on an admission stream while the
// previous step still runs on the GPU, (2) waits for that step and retires
// finished jobs (energies and overlaps measured, device state released, which
// admits the next jobs), and (3) launches the next step over every running
// job, each for about as much work per ladder as `quantum` sweeps of the job
// with the most work per sweep (capped by the sweeps it has left; with more
// ladders than compute units the least urgent jobs get shorter units that fill
// the last round's idle slots, ea_sched.h), replaying a graph-captured plan
// while the job set and sweep counts are unchanged.
// Results are a pure function of each job's inputs (counter-based stream,
// device-resident sweep counters), so a job's result is the same alone and in
// any mix.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "ea.h"
#include "ea_host.h"
#include "ea_sched.h"

using namespace ea;

namespace {

struct Job {
    int64_t id = 0;
    int status = EA_JOB_QUEUED;
    int L = 0, n_T = 0, R = 0, swap_every = 0;
    uint64_t seed = 0;
    int64_t n_sweeps = 0, done = 0;
    double arrival = 0.0;                      // host clock at submission, seconds
    size_t footprint = 0;
    std::vector<int8_t> J;
    std::vector<double> betas;
    ea_sim *sim = nullptr;
    std::vector<int32_t> energy, overlap;      // results once DONE
    std::vector<int8_t> spins;                 // final state (keep_state)
    std::vector<int32_t> perm;
    std::string error;
};

}  // namespace

constexpr int kMaxStepSweeps = 1 << 20;   // sweeps of one job in one step, at most

struct ea_server {
    ea_server_options opt{};
    int device = 0;
    int fill_ladders = 0;             // shortest-first admission stops once the running jobs hold this many
    int cus = 0;                      // compute units of the device
    hipStream_t stream = nullptr;     // steps
    hipStream_t admit = nullptr;      // job creation, measurement and readout
    size_t used = 0;
    int64_t next_id = 1;
    std::map<int64_t, std::unique_ptr<Job>> jobs;
    std::deque<int64_t> queue;        // waiting, arrival order
    std::vector<int64_t> active;      // admitted, running
    int64_t active_ladders = 0;
    // plan cache: valid while the active set and the per-job sweep counts are unchanged
    ea_plan *plan = nullptr;
    std::vector<int64_t> plan_ids;
    std::vector<int> plan_sweeps;
    // the step launched by the last ea_server_step, not yet waited for
    bool in_flight = false;
    std::vector<int64_t> flight_ids;
    std::vector<int> flight_sweeps;
    double flight_flips = 0.0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // around each step, for the measured service rate
    double s_per_flip = 1e-12;                 // running estimate of the GPU time per flip attempt
    int64_t steps = 0, launches_replayed = 0, plans_built = 0;
};

static void drop_plan(ea_server *sv)
{
    if (sv->plan) ea_plan_destroy(sv->plan);
    sv->plan = nullptr;
    sv->plan_ids.clear();
    sv->plan_sweeps.clear();
}

// Wait for the step in flight and credit its sweeps.
static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static int finish_step(ea_server *sv)
{
    if (!sv->in_flight) return EA_OK;
    sv->in_flight = false;
    EA_HIP(hipStreamSynchronize(sv->stream));
    float ms = 0.0f;
    if (sv->flight_flips > 0.0 && hipEventElapsedTime(&ms, sv->ev0, sv->ev1) == hipSuccess && ms > 0.0f)
        sv->s_per_flip = 0.8 * sv->s_per_flip + 0.2 * (1e-3 * ms / sv->flight_flips);
    for (size_t k = 0; k < sv->flight_ids.size(); ++k) {
        auto it = sv->jobs.find(sv->flight_ids[k]);
        if (it != sv->jobs.end()) it->second->done += sv->flight_sweeps[k];
    }
    ++sv->steps;
    return EA_OK;
}

static int64_t remaining_work(const Job *j)
{
    return (j->n_sweeps - j->done) * (int64_t)j->L * j->L * j->L * j->n_T * j->R;
}

// Response ratio of a job: (time since it arrived + its estimated remaining
// service time) / that estimate, the service time from the measured rate.
static double response_ratio(const ea_server *sv, const Job *j, double now)
{
    const double est = std::max(1e-6, (double)remaining_work(j) * 2.0 * sv->s_per_flip);
    return (now - j->arrival + est) / est;
}

static void release_job_device(ea_server *sv, Job *j)
{
    if (j->sim) {
        ea_destroy(j->sim);
        j->sim = nullptr;
        sv->used -= j->footprint;
        sv->active_ladders -= 2 * (int64_t)j->R;
    }
}

extern "C" {

void ea_default_server_options(ea_server_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->quantum_sweeps = 400;
    opt->layout = EA_LAYOUT_CAMSC;
    opt->autotune = 0;   // the job mix changes at every arrival; tuning each mix would cost more than it saves
    opt->policy = EA_ADMIT_RESPONSE_RATIO;
    opt->fill_ladders = 0;
    opt->pack_rounds = 1;
}

int ea_server_create(const ea_server_options *opt_in, ea_server **out)
{
    if (!out) return fail(EA_EINVAL, "ea_server_create: out is NULL");
    *out = nullptr;
    ea_server_options opt;
    ea_default_server_options(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.quantum_sweeps < 1) return fail(EA_EINVAL, "quantum_sweeps < 1");
    if (opt.layout < EA_LAYOUT_CAMSC || opt.layout > EA_LAYOUT_AMSC1) return fail(EA_EINVAL, "unknown layout");
    if (opt.rng != EA_RNG_WORDS && opt.rng != EA_RNG_PLANES) return fail(EA_EINVAL, "unknown rng");
    if (opt.rng == EA_RNG_PLANES && opt.layout != EA_LAYOUT_CAMSC)
        return fail(EA_EINVAL, "plane draws need the CAMSC layout");
    if (opt.max_active < 0 || opt.max_active > 4095) return fail(EA_EINVAL, "max_active outside [0, 4095]");
    if (opt.policy < EA_ADMIT_FIFO || opt.policy > EA_ADMIT_RESPONSE_RATIO) return fail(EA_EINVAL, "unknown policy");
    if (opt.fill_ladders < 0) return fail(EA_EINVAL, "fill_ladders < 0");
    ea_server *sv = new (std::nothrow) ea_server;
    if (!sv) return fail(EA_ENOMEM, "host allocation failed");
    sv->opt = opt;
    if (sv->opt.max_active == 0) sv->opt.max_active = 4095;
    hipError_t e = hipGetDevice(&sv->device);
    if (e == hipSuccess && sv->opt.hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        e = hipMemGetInfo(&free_b, &total_b);
        sv->opt.hbm_budget_bytes = free_b / 10 * 8;
    }
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, sv->device);
    sv->fill_ladders = opt.fill_ladders > 0 ? opt.fill_ladders : 4 * cus;
    sv->cus = cus;
    if (e == hipSuccess && opt.stream == nullptr) e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->admit, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&sv->ev0);
    if (e == hipSuccess) e = hipEventCreate(&sv->ev1);
    if (e != hipSuccess) {
        if (sv->ev0) (void)hipEventDestroy(sv->ev0);
        if (sv->ev1) (void)hipEventDestroy(sv->ev1);
        if (sv->admit) (void)hipStreamDestroy(sv->admit);
        if (opt.stream == nullptr && sv->stream) (void)hipStreamDestroy(sv->stream);
        delete sv;
        return fail(EA_EDEVICE, "server set-up failed: %s", hipGetErrorString(e));
    }
    if (opt.stream) sv->stream = (hipStream_t)opt.stream;
    *out = sv;
    return EA_OK;
}

int ea_server_submit(ea_server *sv, int L, const int8_t *couplings, const double *betas, int n_T, int R, uint64_t seed,
                     int64_t n_sweeps, int swap_every, int64_t *job_id)
{
    if (!sv || !job_id) return fail(EA_EINVAL, "ea_server_submit: NULL argument");
    if (n_sweeps < 0 || n_sweeps >= ((int64_t)1 << 32)) return fail(EA_EINVAL, "n_sweeps out of range");
    if (swap_every < 0) return fail(EA_EINVAL, "swap_every < 0");
    size_t fp = 0;
    if (int rc = ea_job_footprint(L, betas, n_T, R, sv->opt.layout, &fp)) return rc;
    if (fp > sv->opt.hbm_budget_bytes)
        return fail(EA_ENOMEM, "job needs %zu device bytes, more than the whole budget %zu", fp,
                    sv->opt.hbm_budget_bytes);
    if (!couplings) return fail(EA_EINVAL, "couplings is NULL");
    const size_t nJ = (size_t)R * L * L * L * 3;
    for (size_t b = 0; b < nJ; ++b)
        if (couplings[b] != 1 && couplings[b] != -1) return fail(EA_EINVAL, "couplings[%zu] is not +-1", b);
    std::unique_ptr<Job> j(new (std::nothrow) Job);
    if (!j) return fail(EA_ENOMEM, "host allocation failed");
    j->id = sv->next_id++;
    j->L = L; j->n_T = n_T; j->R = R; j->seed = seed; j->n_sweeps = n_sweeps; j->swap_every = swap_every;
    j->footprint = fp;
    j->arrival = now_s();
    j->J.assign(couplings, couplings + nJ);
    j->betas.assign(betas, betas + n_T);
    *job_id = j->id;
    sv->queue.push_back(j->id);
    sv->jobs[j->id] = std::move(j);
    return EA_OK;
}

int ea_server_step(ea_server *sv, int *n_running, int *n_queued, int *n_finished)
{
    if (!sv) return fail(EA_EINVAL, "ea_server_step: NULL server");
    EA_HIP(hipSetDevice(sv->device));
    int finished = 0;
    // 1. admission, on the host and the admission stream while the step in flight runs
    std::vector<int64_t> order(sv->queue.begin(), sv->queue.end());
    if (sv->opt.policy == EA_ADMIT_SHORTEST) {
        std::stable_sort(order.begin(), order.end(), [sv](int64_t a, int64_t b) {
            return remaining_work(sv->jobs[a].get()) < remaining_work(sv->jobs[b].get());
        });
    } else if (sv->opt.policy == EA_ADMIT_RESPONSE_RATIO) {
        const double now = now_s();
        std::vector<std::pair<double, int64_t>> keyed;
        for (int64_t id : order) keyed.push_back({-response_ratio(sv, sv->jobs[id].get(), now), id});
        std::stable_sort(keyed.begin(), keyed.end(),
                         [](const std::pair<double, int64_t> &a, const std::pair<double, int64_t> &b) {
                             return a.first < b.first;
                         });
        for (size_t k = 0; k < keyed.size(); ++k) order[k] = keyed[k].second;
    }
    for (int64_t id : order) {
        Job *j = sv->jobs[id].get();
        if ((int)sv->active.size() >= sv->opt.max_active) break;
        if (sv->opt.policy != EA_ADMIT_FIFO && !sv->active.empty() && sv->active_ladders >= sv->fill_ladders)
            break;
        if (sv->used + j->footprint > sv->opt.hbm_budget_bytes) continue;
        ea_options o;
        ea_default_options(&o);
        o.layout = sv->opt.layout;
        o.rng = sv->opt.rng;
        o.stream = sv->admit;
        sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), id));
        const int rc = ea_create(j->L, j->J.data(), j->betas.data(), j->n_T, j->R, j->seed, &o, &j->sim);
        if (rc != EA_OK) {
            j->status = EA_JOB_FAILED;
            j->error = ea_last_error();
            ++finished;
            continue;
        }
        sv->used += j->footprint;
        sv->active_ladders += 2 * (int64_t)j->R;
        j->status = EA_JOB_RUNNING;
        j->J.clear();
        j->J.shrink_to_fit();
        sv->active.push_back(id);
    }
    // 2. wait for the step in flight, retire finished jobs
    if (int rc = finish_step(sv)) return rc;
    std::vector<int64_t> still;
    for (int64_t id : sv->active) {
        Job *j = sv->jobs[id].get();
        if (j->done < j->n_sweeps) {
            still.push_back(id);
            continue;
        }
        j->energy.assign((size_t)j->R * 2 * j->n_T, 0);
        j->overlap.assign((size_t)j->R * j->n_T, 0);
        int rc = ea_observables(j->sim, j->energy.data(), j->overlap.data());
        if (rc == EA_OK && sv->opt.keep_state) {
            j->spins.assign((size_t)j->R * 2 * j->n_T * j->L * j->L * j->L, 0);
            j->perm.assign((size_t)j->R * 2 * j->n_T, 0);
            rc = ea_state(j->sim, j->spins.data(), j->perm.data(), nullptr);
        }
        if (rc != EA_OK) {
            j->status = EA_JOB_FAILED;
            j->error = ea_last_error();
        } else {
            j->status = EA_JOB_DONE;
        }
        drop_plan(sv);   // the cached plan references this job's buffers
        release_job_device(sv, j);
        ++finished;
    }
    sv->active.swap(still);
    // 3. launch the next step over every running job (not waited for here)
    if (!sv->active.empty()) {
        // Sweeps per step in inverse proportion to a ladder's work per sweep
        // (sites x temperatures): the job with the most work per sweep runs
        // `quantum` sweeps, and every ladder of the step takes about as long,
        // so a job with cheap sweeps is not held to the pace of an expensive
        // one and the launch's units are of one size; with packing, the least
        // urgent jobs fill the last round's idle slots with shorter units.
        const double now = now_s();
        std::vector<StepJob> sj;
        std::vector<ea_sim *> sims;
        std::vector<int> se;
        for (int64_t id : sv->active) {
            const Job *j = sv->jobs[id].get();
            sj.push_back({2 * (int64_t)j->R, (double)j->L * j->L * j->L * j->n_T, j->n_sweeps - j->done,
                          response_ratio(sv, j, now)});
            sims.push_back(j->sim);
            se.push_back(j->swap_every);
        }
        const std::vector<int> q =
            step_sweeps(sj, sv->opt.quantum_sweeps, sv->cus, sv->opt.pack_rounds != 0, kMaxStepSweeps);
        if (sv->plan == nullptr || sv->plan_ids != sv->active || sv->plan_sweeps != q) {
            drop_plan(sv);
            ea_plan_options po;
            ea_default_plan_options(&po);
            po.autotune = sv->opt.autotune;
            po.stream = sv->stream;
            if (int rc = plan_create(sims.data(), (int)sims.size(), q.data(), se.data(), &po, &sv->plan)) return rc;
            sv->plan_ids = sv->active;
            sv->plan_sweeps = q;
            ++sv->plans_built;
        } else {
            ++sv->launches_replayed;
        }
        EA_HIP(hipEventRecord(sv->ev0, sv->stream));
        if (int rc = ea_plan_run(sv->plan, 1)) return rc;
        EA_HIP(hipEventRecord(sv->ev1, sv->stream));
        sv->in_flight = true;
        sv->flight_ids = sv->active;
        sv->flight_sweeps = q;
        sv->flight_flips = 0.0;
        for (size_t k = 0; k < sv->active.size(); ++k) {
            const Job *j = sv->jobs[sv->active[k]].get();
            sv->flight_flips += (double)q[k] * j->L * j->L * j->L * j->n_T * 2.0 * j->R;
        }
    }
    if (n_running) *n_running = (int)sv->active.size();
    if (n_queued) *n_queued = (int)sv->queue.size();
    if (n_finished) *n_finished = finished;
    return EA_OK;
}

int ea_server_status(ea_server *sv, int64_t id, int *status, int64_t *sweeps_done)
{
    if (!sv) return fail(EA_EINVAL, "ea_server_status: NULL server");
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return fail(EA_EINVAL, "unknown job %lld", (long long)id);
    if (status) *status = it->second->status;
    if (sweeps_done) *sweeps_done = it->second->done;
    return EA_OK;
}

int ea_server_result(ea_server *sv, int64_t id, int32_t *energy, int32_t *overlap)
{
    if (!sv) return fail(EA_EINVAL, "ea_server_result: NULL server");
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return fail(EA_EINVAL, "unknown job %lld", (long long)id);
    const Job *j = it->second.get();
    if (j->status != EA_JOB_DONE) return fail(EA_ESTATE, "job %lld is not done", (long long)id);
    if (energy) std::memcpy(energy, j->energy.data(), j->energy.size() * sizeof(int32_t));
    if (overlap) std::memcpy(overlap, j->overlap.data(), j->overlap.size() * sizeof(int32_t));
    return EA_OK;
}

int ea_server_final_state(ea_server *sv, int64_t id, int8_t *spins, int32_t *temp_of_slot)
{
    if (!sv) return fail(EA_EINVAL, "ea_server_final_state: NULL server");
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return fail(EA_EINVAL, "unknown job %lld", (long long)id);
    const Job *j = it->second.get();
    if (j->status != EA_JOB_DONE || j->spins.empty()) return fail(EA_ESTATE, "no final state kept for job %lld", (long long)id);
    if (spins) std::memcpy(spins, j->spins.data(), j->spins.size());
    if (temp_of_slot) std::memcpy(temp_of_slot, j->perm.data(), j->perm.size() * sizeof(int32_t));
    return EA_OK;
}

int ea_server_cancel(ea_server *sv, int64_t id)
{
    if (!sv) return fail(EA_EINVAL, "ea_server_cancel: NULL server");
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return fail(EA_EINVAL, "unknown job %lld", (long long)id);
    Job *j = it->second.get();
    if (j->status == EA_JOB_QUEUED) {
        sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), id));
    } else if (j->status == EA_JOB_RUNNING) {
        if (int rc = finish_step(sv)) return rc;
        drop_plan(sv);
        release_job_device(sv, j);
        sv->active.erase(std::find(sv->active.begin(), sv->active.end(), id));
    } else {
        return fail(EA_ESTATE, "job %lld already finished", (long long)id);
    }
    j->status = EA_JOB_CANCELLED;
    return EA_OK;
}

int ea_server_release(ea_server *sv, int64_t id)
{
    if (!sv) return fail(EA_EINVAL, "ea_server_release: NULL server");
    auto it = sv->jobs.find(id);
    if (it == sv->jobs.end()) return fail(EA_EINVAL, "unknown job %lld", (long long)id);
    const int st = it->second->status;
    if (st == EA_JOB_QUEUED || st == EA_JOB_RUNNING) return fail(EA_ESTATE, "job %lld has not finished", (long long)id);
    sv->jobs.erase(it);
    return EA_OK;
}

int ea_server_stats(const ea_server *sv, size_t *hbm_used, size_t *hbm_budget, int64_t *steps, int64_t *plans_built,
                    int64_t *launches_replayed)
{
    if (!sv) return fail(EA_EINVAL, "ea_server_stats: NULL server");
    if (hbm_used) *hbm_used = sv->used;
    if (hbm_budget) *hbm_budget = sv->opt.hbm_budget_bytes;
    if (steps) *steps = sv->steps;
    if (plans_built) *plans_built = sv->plans_built;
    if (launches_replayed) *launches_replayed = sv->launches_replayed;
    return EA_OK;
}

void ea_server_destroy(ea_server *sv)
{
    if (!sv) return;
    (void)hipSetDevice(sv->device);
    (void)finish_step(sv);
    drop_plan(sv);
    (void)hipStreamSynchronize(sv->stream);
    for (auto &kv : sv->jobs) release_job_device(sv, kv.second.get());
    if (sv->opt.stream == nullptr) (void)hipStreamDestroy(sv->stream);
    (void)hipStreamDestroy(sv->admit);
    (void)hipEventDestroy(sv->ev0);
    (void)hipEventDestroy(sv->ev1);
    delete sv;
}

}  // extern "C"
