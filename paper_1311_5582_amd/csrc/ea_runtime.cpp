// Runtime around the sweep kernel: launch sets over several jobs of uneven
// size (one persistent launch, largest ladders first), launch plans whose
// step is captured once in a hipGraph and replayed, and an autotuner that
// picks the workgroup size by timing candidates on scratch copies of the jobs.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ea.h"
#include "ea_host.h"
#include "ea_internal.h"

namespace ea {

// Device arrays of one launch: descriptors, unit list, work-queue counter.
struct LaunchSet {
    int layout = 0;   // kernel variant (kernel_variant of the jobs' layout and draw stream)
    int parts = 1;    // workgroups per ladder (split ladders when > 1)
    int sep = 0;      // spin words in LDS by colour class (a launch over one job only)
    int n_jobs = 0;
    int n_units = 0;
    int bt = 0;
    int grid = 0;
    size_t lds = 0;
    JobDesc *d_descs = nullptr;
    uint32_t *d_units = nullptr;
    uint32_t *d_queue = nullptr;
    std::vector<JobDesc> descs;
};

static void launchset_free(LaunchSet &ls)
{
    if (ls.d_descs) (void)hipFree(ls.d_descs);
    if (ls.d_units) (void)hipFree(ls.d_units);
    if (ls.d_queue) (void)hipFree(ls.d_queue);
    ls.d_descs = nullptr;
    ls.d_units = nullptr;
    ls.d_queue = nullptr;
}

static int min_block_threads(int N)
{
    return ((N + 84) / 85 + 63) / 64 * 64;
}

// Host part of a launch over descs (descs[j] describes job j with n_sweeps and
// swap_every already set): the unit list, ladders of the most work first, the
// workgroup size (bt = 0: the largest planned size among the jobs), LDS bytes
// and grid.
static int launchset_plan(LaunchSet &ls, const std::vector<JobDesc> &descs, const std::vector<size_t> &lds_per_job,
                          int layout, int bt, int split_opt, std::vector<uint32_t> *units)
{
    ls.layout = layout;
    ls.n_jobs = (int)descs.size();
    ls.descs = descs;
    ls.sep = 0;
    for (const JobDesc &d : descs)
        if (d.site_order != 0) {
            if (descs.size() > 1)
                return fail(EA_EINVAL, "a job with its spin words in LDS by colour class runs only alone");
            ls.sep = d.site_order;
        }
    std::vector<std::pair<double, uint32_t>> order;
    int want_bt = 0, need_bt = 64;
    size_t lds = 0;
    for (int j = 0; j < ls.n_jobs; ++j) {
        const JobDesc &d = descs[j];
        if (d.n_sweeps == 0) continue;
        want_bt = std::max(want_bt, d.block_threads);
        need_bt = std::max(need_bt, min_block_threads(d.N));
        lds = std::max(lds, lds_per_job[j]);
        const double work = (double)d.N * d.n_T * (double)d.n_sweeps;
        for (int l = 0; l < d.ladders; ++l) order.push_back({-work, ((uint32_t)j << 20) | (uint32_t)l});
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, uint32_t> &a, const std::pair<double, uint32_t> &b) {
                         return a.first < b.first;
                     });
    ls.bt = bt > 0 ? bt : want_bt;
    if (ls.bt < need_bt) return fail(EA_EINVAL, "block_threads=%d is below %d needed by a job", ls.bt, need_bt);
    ls.lds = lds;
    ls.n_units = (int)order.size();
    units->resize(order.size());
    for (size_t k = 0; k < order.size(); ++k) (*units)[k] = order[k].second;
    if (ls.n_units == 0) return EA_OK;
    // split ladders when the launch alone would leave compute units idle
    std::vector<JobDesc> live;
    for (const JobDesc &d : descs)
        if (d.n_sweeps > 0) live.push_back(d);
    ls.parts = choose_split_parts(live.data(), (int)live.size(), ls.bt, ls.lds, layout, split_opt);
    if (ls.parts > 1) ls.layout = split_variant(live.data(), (int)live.size(), layout, ls.parts, split_opt);
    if (ls.parts > 1)
        ls.grid = split_grid(ls.n_units, ls.parts);
    else if (int rc = device_grid(layout, ls.bt, ls.lds, ls.n_units, &ls.grid))
        return rc;
    EA_HIP(sweep_set_lds(ls.layout, ls.parts, ls.lds));   // before any capture: not a stream operation
    return EA_OK;
}

// The split choice of a launch over several jobs: never if any job asks for
// never, whenever possible if every job asks for that (by slot groups if every
// job asks for slot groups), otherwise automatic.
static int batch_split_opt(ea_sim *const *sims, int n)
{
    bool all_force = true, all_slots = true;
    for (int j = 0; j < n; ++j) {
        if (sims[j]->split_opt == 1) return 1;
        if (sims[j]->split_opt != 2 && sims[j]->split_opt != 3) all_force = false;
        if (sims[j]->split_opt != 3) all_slots = false;
    }
    return all_slots ? 3 : (all_force ? 2 : 0);
}

// Plan a launch and give it device arrays of its own.
static int launchset_build(LaunchSet &ls, const std::vector<JobDesc> &descs, const std::vector<size_t> &lds_per_job,
                           int layout, int bt, int split_opt, hipStream_t st)
{
    std::vector<uint32_t> units;
    if (int rc = launchset_plan(ls, descs, lds_per_job, layout, bt, split_opt, &units)) return rc;
    if (ls.n_units == 0) return EA_OK;
    EA_HIP(hipMalloc(&ls.d_descs, descs.size() * sizeof(JobDesc)));
    EA_HIP(hipMalloc(&ls.d_units, units.size() * sizeof(uint32_t)));
    EA_HIP(hipMalloc(&ls.d_queue, kQueueWords * sizeof(uint32_t)));
    EA_HIP(hipMemcpyAsync(ls.d_descs, descs.data(), descs.size() * sizeof(JobDesc), hipMemcpyHostToDevice, st));
    EA_HIP(hipMemcpyAsync(ls.d_units, units.data(), units.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    EA_HIP(hipMemsetAsync(ls.d_queue, 0, kQueueWords * sizeof(uint32_t), st));   // armed once; each launch re-arms them
    EA_HIP(hipStreamSynchronize(st));
    return EA_OK;
}

static int launchset_launch(const LaunchSet &ls, hipStream_t st)
{
    if (ls.n_units == 0) return EA_OK;
    EA_HIP(launch_sweep(ls.d_descs, ls.n_jobs, ls.d_units, ls.n_units, ls.d_queue, ls.layout, ls.parts, ls.sep, ls.bt,
                        ls.lds, ls.grid, st));
    return EA_OK;
}

static int validate_jobs(ea_sim *const *sims, int n_sims, const int64_t *n_sweeps, const int *swap_every)
{
    if (!sims || n_sims < 1 || !n_sweeps || !swap_every) return fail(EA_EINVAL, "bad job list");
    if (n_sims > 4095) return fail(EA_EINVAL, "at most 4095 jobs per launch");
    for (int j = 0; j < n_sims; ++j) {
        const ea_sim *s = sims[j];
        if (!s) return fail(EA_EINVAL, "sims[%d] is NULL", j);
        if (s->layout != sims[0]->layout) return fail(EA_EINVAL, "sims[%d] has a different layout", j);
        if (s->h.rng != sims[0]->h.rng) return fail(EA_EINVAL, "sims[%d] has a different flip-draw stream", j);
        if (s->device != sims[0]->device) return fail(EA_EINVAL, "sims[%d] lives on another device", j);
        if (n_sweeps[j] < 0 || n_sweeps[j] > 0x7FFFFFFF) return fail(EA_EINVAL, "n_sweeps[%d] out of range", j);
        if (swap_every[j] < 0) return fail(EA_EINVAL, "swap_every[%d] < 0", j);
        for (int i = 0; i < j; ++i)
            if (sims[i] == s) return fail(EA_EINVAL, "sims[%d] appears twice", j);
    }
    return EA_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: workgroup size for a set of jobs, timed on scratch copies.
// ---------------------------------------------------------------------------
// A tuned launch shape: workgroup size and split choice (1 = one workgroup per ladder).
struct Tuned {
    int bt = 0;
    int split_opt = 1;
};
static std::mutex g_tune_mu;
static std::map<std::string, Tuned> g_tune_cache;
static bool g_tune_loaded = false;

static std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');   // drop feature suffixes such as ":sramecc+:xnack-"
    return colon == std::string::npos ? a : a.substr(0, colon);
}

static std::string tune_key(const std::vector<JobDesc> &descs, int layout, int split_opt)
{
    // shape classes: (L, words, swap on/off) multiset; realization counts do not change the best size
    std::vector<std::string> parts;
    for (const JobDesc &d : descs) {
        char b[64];
        std::snprintf(b, sizeof b, "%d.%d.%d", d.L, d.NW, d.swap_every > 0 ? 1 : 0);
        parts.push_back(b);
    }
    std::sort(parts.begin(), parts.end());
    parts.erase(std::unique(parts.begin(), parts.end()), parts.end());
    std::string k = device_arch() + ":" + std::to_string(layout) + ":s" + std::to_string(split_opt);
    for (const std::string &p : parts) k += ":" + p;
    return k;
}

static void tune_cache_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("EA_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char key[512];
    int bt = 0, split = 0;
    while (std::fscanf(f, "%511s %d %d", key, &bt, &split) == 3) g_tune_cache[key] = {bt, split};
    std::fclose(f);
}

static void tune_cache_store(const std::string &key, Tuned v)
{
    g_tune_cache[key] = v;
    const char *path = std::getenv("EA_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d\n", key.c_str(), v.bt, v.split_opt);
    std::fclose(f);
}

// Time each candidate shape (workgroup size; one workgroup per ladder or
// split ladders where the jobs allow it) on scratch copies of the jobs'
// mutable state (spins, permutation, counters, swap counts, exchange area and
// error flag); the jobs themselves are untouched.  split_opt is the jobs'
// split choice; the tuned shape keeps it or turns splitting off.
static int autotune_shape(const std::vector<JobDesc> &descs, const std::vector<size_t> &lds_per_job, int layout,
                          int split_opt, hipStream_t st, Tuned *best_shape)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_cache_load();
    const std::string key = tune_key(descs, layout, split_opt);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
        *best_shape = it->second;
        return EA_OK;
    }
    int need = 64;
    for (const JobDesc &d : descs) need = std::max(need, min_block_threads(d.N));
    std::vector<JobDesc> scratch = descs;
    std::vector<void *> bufs;
    auto cleanup = [&]() {
        for (void *p : bufs) (void)hipFree(p);
    };
    int64_t work = 0;
    for (JobDesc &d : scratch) {
        const size_t spin_bytes = (size_t)d.ladders * d.NW * d.N * 4;
        const size_t xchg_bytes = (size_t)d.ladders * 2 * kMaxTemps * 8;
        void *sp = nullptr, *pm = nullptr, *ac = nullptr, *ct = nullptr, *xc = nullptr, *er = nullptr;
        hipError_t e = hipMalloc(&sp, spin_bytes);
        if (e == hipSuccess) bufs.push_back(sp), e = hipMalloc(&pm, (size_t)d.ladders * kMaxTemps * 4);
        if (e == hipSuccess) bufs.push_back(pm), e = hipMalloc(&ac, (size_t)d.ladders * kMaxTemps * 8);
        if (e == hipSuccess) bufs.push_back(ac), e = hipMalloc(&ct, 8);
        if (e == hipSuccess) bufs.push_back(ct), e = hipMalloc(&xc, xchg_bytes);
        if (e == hipSuccess) bufs.push_back(xc), e = hipMalloc(&er, 4);
        if (e == hipSuccess) bufs.push_back(er);
        void *hl = nullptr;
        const size_t halo_sz = d.halo ? halo_bytes(d.L, d.n_T, d.ladders / 2, EA_LAYOUT_CAMSC) : 0;
        if (e == hipSuccess && halo_sz) {
            e = hipMalloc(&hl, halo_sz);
            if (e == hipSuccess) bufs.push_back(hl), e = hipMemsetAsync(hl, 0, halo_sz, st);
        }
        // own exchange words: the scratch run's sweep tags must never reach the job's
        if (e == hipSuccess) e = hipMemsetAsync(xc, 0, xchg_bytes, st);
        if (e == hipSuccess) e = hipMemsetAsync(er, 0, 4, st);
        if (e == hipSuccess) e = hipMemcpyAsync(sp, d.spins, spin_bytes, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(pm, d.temp_of_slot, (size_t)d.ladders * kMaxTemps * 4, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemsetAsync(ac, 0, (size_t)d.ladders * kMaxTemps * 8, st);
        if (e == hipSuccess) e = hipMemcpyAsync(ct, d.sweep_ctr, 4, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) {
            cleanup();
            return fail(EA_ENOMEM, "autotune scratch: %s", hipGetErrorString(e));
        }
        d.spins = (uint32_t *)sp;
        d.temp_of_slot = (int32_t *)pm;
        d.swap_acc = (uint64_t *)ac;
        d.sweep_ctr = (uint32_t *)ct;
        d.xchg = (uint64_t *)xc;
        d.error = (uint32_t *)er;
        d.halo = (uint64_t *)hl;
        work += (int64_t)d.ladders * d.N * d.n_T;
    }
    // a few sweeps, enough for ~50 ms-equivalent of the largest config at 1 ps/flip
    const int sweeps = (int)std::max<int64_t>(2, std::min<int64_t>(20, 50000000000LL / std::max<int64_t>(work, 1)));
    for (JobDesc &d : scratch) {
        d.n_sweeps = sweeps;
        d.swap_every = d.swap_every > 0 ? 1 : 0;   // tune with the most PT work
    }
    const int candidates[] = {256, 512, 768, 1024};
    float best_ms = 1e30f;
    Tuned best;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(EA_EDEVICE, "autotune: hipEventCreate failed");
    }
    int rc = EA_OK;
    for (int k = 0; k < 8 && rc == EA_OK; ++k) {
        const int bt = candidates[k / 2];
        const int sopt = (k & 1) ? split_opt : 1;   // unsplit, then split where the jobs allow it
        if (bt < need || ((k & 1) && split_opt == 1)) continue;
        LaunchSet ls;
        rc = launchset_build(ls, scratch, lds_per_job, layout, bt, sopt, st);
        if (rc) break;
        if ((k & 1) && ls.parts == 1) {   // the same launch as the unsplit candidate
            launchset_free(ls);
            continue;
        }
        float ms = 0;
        hipError_t e = hipSuccess;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // first run warms up
            e = hipEventRecord(e0, st);
            if (e == hipSuccess && launchset_launch(ls, st) != EA_OK) e = hipErrorUnknown;
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        }
        launchset_free(ls);
        if (e != hipSuccess) {
            rc = fail(EA_EDEVICE, "autotune run failed: %s", hipGetErrorString(e));
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best.bt = bt;
            best.split_opt = sopt;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // a split scratch run that timed out has no valid timing; report it like a launch failure
    for (const JobDesc &d : scratch) {
        uint32_t err = 0;
        if (rc == EA_OK && hipMemcpy(&err, d.error, 4, hipMemcpyDeviceToHost) == hipSuccess && err)
            rc = fail(EA_EDEVICE, "autotune: a split-ladder exchange timed out");
    }
    cleanup();
    if (rc) return rc;
    if (best.bt == 0) return fail(EA_EINVAL, "no workgroup size fits these jobs");
    tune_cache_store(key, best);
    *best_shape = best;
    return EA_OK;
}

}  // namespace ea

using namespace ea;

// ---------------------------------------------------------------------------
// Launch plans
// ---------------------------------------------------------------------------
struct ea_plan {
    LaunchSet ls;
    std::vector<ea_sim *> sims;
    std::vector<int> sweeps;   // sweeps of each job per step
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool user_stream = false;
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool lost_job = false;   // a job was destroyed while the plan held it
};

namespace ea {
void plan_forget_job(ea_plan *p, ea_sim *s)
{
    (void)hipStreamSynchronize(p->stream);   // no replay may still read the job
    for (size_t j = p->sims.size(); j-- > 0;)
        if (p->sims[j] == s) {
            p->sims.erase(p->sims.begin() + j);
            p->sweeps.erase(p->sweeps.begin() + j);
        }
    p->lost_job = true;
}
}  // namespace ea

extern "C" {

int ea_sweep_batch(ea_sim *const *sims, int n_sims, const int64_t *n_sweeps, const int *swap_every)
{
    if (int rc = validate_jobs(sims, n_sims, n_sweeps, swap_every)) return rc;
    for (int j = 0; j < n_sims; ++j)
        if (sims[j]->t + n_sweeps[j] >= ((int64_t)1 << 32))
            return fail(EA_ESTATE, "sweep counter of sims[%d] would reach 2^32", j);
    ea_sim *s0 = sims[0];
    EA_HIP(hipSetDevice(s0->device));
    hipStream_t st = s0->stream;
    if (n_sims == 1) {
        ea_sim *s = s0;
        if (n_sweeps[0] == 0) return EA_OK;
        s->h.n_sweeps = (int32_t)n_sweeps[0];
        s->h.swap_every = swap_every[0];
        EA_HIP(hipMemcpyAsync(&s->d_job->n_sweeps, &s->h.n_sweeps, 2 * sizeof(int32_t), hipMemcpyHostToDevice, st));
        int kv = kernel_variant(s->layout, s->h.rng);
        const int parts = s->split_parts;
        int grid = 0;
        if (parts > 1) {
            grid = split_grid(s->h.ladders, parts);
            kv = split_variant(&s->h, 1, kv, parts, s->split_opt);
        } else if (int rc = device_grid(kv, s->block_threads, s->lds, s->h.ladders, &grid)) {
            return rc;
        }
        EA_HIP(launch_sweep(s->d_job, 1, s->d_units, s->h.ladders, s->d_counters + 1, kv, parts, s->h.site_order,
                            s->block_threads,
                            s->lds, grid, st));
        if (parts > 1) s->ever_split = true;
        s->t += n_sweeps[0];
        if (!s->user_stream) {
            EA_HIP(hipStreamSynchronize(st));
            return check_split_error(s);
        }
        return EA_OK;
    }
    std::vector<JobDesc> descs(n_sims);
    std::vector<size_t> lds(n_sims);
    for (int j = 0; j < n_sims; ++j) {
        descs[j] = sims[j]->h;
        descs[j].n_sweeps = (int32_t)n_sweeps[j];
        descs[j].swap_every = swap_every[j];
        lds[j] = sims[j]->lds;
    }
    LaunchSet ls;
    int rc = launchset_build(ls, descs, lds, kernel_variant(s0->layout, s0->h.rng), 0, batch_split_opt(sims, n_sims), st);
    // the launch runs on sims[0]'s stream: first let it wait for the other jobs' streams
    if (rc == EA_OK) rc = order_streams(sims, n_sims, st, false);
    if (rc == EA_OK) rc = launchset_launch(ls, st);
    if (rc == EA_OK) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(EA_EDEVICE, "batched sweep failed: %s", hipGetErrorString(e));
    }
    const int parts = ls.parts;
    launchset_free(ls);
    if (rc) return rc;
    for (int j = 0; j < n_sims; ++j) {
        sims[j]->t += n_sweeps[j];
        if (parts > 1 && n_sweeps[j] > 0) sims[j]->ever_split = true;
    }
    if (parts > 1)
        for (int j = 0; j < n_sims; ++j)
            if (int rc2 = check_split_error(sims[j])) return rc2;
    return EA_OK;
}

int ea_sweep_batch_noalloc(ea_sim *const *sims, int n_sims, const int64_t *n_sweeps, const int *swap_every)
{
    if (int rc = validate_jobs(sims, n_sims, n_sweeps, swap_every)) return rc;
    if (n_sims > kNoallocMaxJobs)
        return fail(EA_EINVAL, "ea_sweep_batch_noalloc: %d jobs exceed the workspace limit of %d", n_sims,
                    kNoallocMaxJobs);
    int64_t units = 0;
    for (int j = 0; j < n_sims; ++j) {
        if (sims[j]->t + n_sweeps[j] >= ((int64_t)1 << 32))
            return fail(EA_ESTATE, "sweep counter of sims[%d] would reach 2^32", j);
        if (n_sweeps[j] > 0) units += 2 * (int64_t)sims[j]->R;
    }
    if (units > kNoallocMaxUnits)
        return fail(EA_EINVAL, "ea_sweep_batch_noalloc: %lld ladders exceed the workspace limit of %d",
                    (long long)units, kNoallocMaxUnits);
    // one job: the lone launch uses only the job's own device buffers
    if (n_sims == 1) return ea_sweep_batch(sims, n_sims, n_sweeps, swap_every);
    ea_sim *s0 = sims[0];
    EA_HIP(hipSetDevice(s0->device));
    hipStream_t st = s0->stream;
    std::vector<JobDesc> descs(n_sims);
    std::vector<size_t> lds(n_sims);
    for (int j = 0; j < n_sims; ++j) {
        descs[j] = sims[j]->h;
        descs[j].n_sweeps = (int32_t)n_sweeps[j];
        descs[j].swap_every = swap_every[j];
        lds[j] = sims[j]->lds;
    }
    LaunchSet ls;   // its device arrays are the workspace: never launchset_free it
    std::vector<uint32_t> order;
    if (int rc = launchset_plan(ls, descs, lds, kernel_variant(s0->layout, s0->h.rng), 0,
                                batch_split_opt(sims, n_sims), &order))
        return rc;
    if (ls.n_units > 0) {
        void *ws = nullptr;
        EA_HIP(noalloc_workspace(&ws));
        uint8_t *base = (uint8_t *)ws;
        ls.d_queue = (uint32_t *)(base + kNoallocQueueOff);
        ls.d_descs = (JobDesc *)(base + kNoallocDescOff);
        ls.d_units = (uint32_t *)(base + kNoallocUnitOff);
        // the workspace is rewritten only after the work already queued on every job's stream
        if (int rc = order_streams(sims, n_sims, st, false)) return rc;
        EA_HIP(hipMemcpyAsync(ls.d_descs, descs.data(), descs.size() * sizeof(JobDesc), hipMemcpyHostToDevice, st));
        EA_HIP(hipMemcpyAsync(ls.d_units, order.data(), order.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        // the queue counters must start at zero whatever an earlier call left there
        EA_HIP(hipMemsetAsync(ls.d_queue, 0, kQueueWords * sizeof(uint32_t), st));
        if (int rc = launchset_launch(ls, st)) return rc;
        const hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(EA_EDEVICE, "batched sweep failed: %s", hipGetErrorString(e));
    }
    for (int j = 0; j < n_sims; ++j) {
        sims[j]->t += n_sweeps[j];
        if (ls.parts > 1 && n_sweeps[j] > 0) sims[j]->ever_split = true;
    }
    if (ls.parts > 1)
        for (int j = 0; j < n_sims; ++j)
            if (int rc = check_split_error(sims[j])) return rc;
    return EA_OK;
}

void ea_default_plan_options(ea_plan_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->autotune = 1;
    opt->use_graph = 1;
}

}  // extern "C"

namespace ea {

int plan_create(ea_sim *const *sims, int n_sims, const int *sweeps, const int *swap_every,
                const ea_plan_options *opt_in, ea_plan **out)
{
    if (!out) return fail(EA_EINVAL, "ea_plan_create: out is NULL");
    *out = nullptr;
    if (n_sims < 1 || !sweeps) return fail(EA_EINVAL, "bad job list");
    ea_plan_options opt;
    ea_default_plan_options(&opt);
    if (opt_in) opt = *opt_in;
    std::vector<int64_t> ns(n_sims);
    for (int j = 0; j < n_sims; ++j) {
        if (sweeps[j] < 0) return fail(EA_EINVAL, "sweeps[%d]=%d < 0", j, sweeps[j]);
        ns[j] = sweeps[j];
    }
    if (int rc = validate_jobs(sims, n_sims, ns.data(), swap_every)) return rc;
    if (opt.block_threads != 0 && (opt.block_threads < 64 || opt.block_threads > kMaxBlock || opt.block_threads % 64))
        return fail(EA_EINVAL, "block_threads=%d must be a multiple of 64 in [64, %d]", opt.block_threads, kMaxBlock);
    for (int j = 0; j < n_sims; ++j)
        if (sims[j]->plan) return fail(EA_EBUSY, "sims[%d] is held by another live plan", j);
    EA_HIP(hipSetDevice(sims[0]->device));
    ea_plan *p = new (std::nothrow) ea_plan;
    if (!p) return fail(EA_ENOMEM, "host allocation failed");
    p->sims.assign(sims, sims + n_sims);
    p->sweeps.assign(sweeps, sweeps + n_sims);
    p->device = sims[0]->device;
    p->use_graph = opt.use_graph != 0;
    p->user_stream = opt.stream != nullptr;
    auto bail = [p](int rc) {
        launchset_free(p->ls);
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        if (p->own_stream) (void)hipStreamDestroy(p->stream);
        delete p;
        return rc;
    };
    if (p->user_stream) {
        p->stream = (hipStream_t)opt.stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(fail(EA_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e)));
        p->own_stream = true;
    }
    std::vector<JobDesc> descs(n_sims);
    std::vector<size_t> lds(n_sims);
    for (int j = 0; j < n_sims; ++j) {
        descs[j] = sims[j]->h;
        descs[j].n_sweeps = sweeps[j];
        descs[j].swap_every = swap_every[j];
        lds[j] = sims[j]->lds;
    }
    // all prior work on the jobs' own streams must land before the plan reads them
    for (ea_sim *s : p->sims) {
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return bail(fail(EA_EDEVICE, "job stream failed: %s", hipGetErrorString(e)));
    }
    int bt = opt.block_threads;
    int split_opt = batch_split_opt(sims, n_sims);
    const int kv = kernel_variant(sims[0]->layout, sims[0]->h.rng);
    if (bt == 0 && opt.autotune) {
        Tuned shape;
        if (int rc = autotune_shape(descs, lds, kv, split_opt, p->stream, &shape)) return bail(rc);
        bt = shape.bt;
        split_opt = shape.split_opt;
    }
    if (int rc = launchset_build(p->ls, descs, lds, kv, bt, split_opt, p->stream)) return bail(rc);
    if (p->use_graph && p->ls.n_units > 0) {
        hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const int rc = launchset_launch(p->ls, p->stream);
            hipError_t e2 = hipStreamEndCapture(p->stream, &p->graph);
            if (rc) return bail(rc);
            e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return bail(fail(EA_EDEVICE, "graph capture failed: %s", hipGetErrorString(e)));
    }
    for (ea_sim *s : p->sims) {
        s->plan = p;
        if (p->ls.parts > 1) s->ever_split = true;
    }
    *out = p;
    return EA_OK;
}

}  // namespace ea

extern "C" {

int ea_plan_create(ea_sim *const *sims, int n_sims, int sweeps_per_step, const int *swap_every,
                   const ea_plan_options *opt, ea_plan **out)
{
    if (sweeps_per_step < 1) return fail(EA_EINVAL, "sweeps_per_step=%d < 1", sweeps_per_step);
    if (n_sims < 1 || n_sims > 4095) return fail(EA_EINVAL, "bad job list");
    std::vector<int> sw(n_sims, sweeps_per_step);
    return plan_create(sims, n_sims, sw.data(), swap_every, opt, out);
}

int ea_plan_run(ea_plan *p, int64_t n_steps)
{
    if (!p) return fail(EA_EINVAL, "ea_plan_run: NULL plan");
    if (n_steps < 0) return fail(EA_EINVAL, "n_steps < 0");
    if (p->lost_job) return fail(EA_ESTATE, "a job of this plan was destroyed; destroy the plan");
    for (size_t j = 0; j < p->sims.size(); ++j)
        if (p->sims[j]->t + n_steps * p->sweeps[j] >= ((int64_t)1 << 32))
            return fail(EA_ESTATE, "a job's sweep counter would reach 2^32");
    EA_HIP(hipSetDevice(p->device));
    if (n_steps == 0) return EA_OK;
    // order the replays after the work already queued on the jobs' own streams,
    // and later work on those streams after the replays
    if (int rc = order_streams(p->sims.data(), (int)p->sims.size(), p->stream, false)) return rc;
    for (int64_t k = 0; k < n_steps; ++k) {
        if (p->exec)
            EA_HIP(hipGraphLaunch(p->exec, p->stream));
        else if (int rc = launchset_launch(p->ls, p->stream))
            return rc;
    }
    if (int rc = order_streams(p->sims.data(), (int)p->sims.size(), p->stream, true)) return rc;
    for (size_t j = 0; j < p->sims.size(); ++j) p->sims[j]->t += n_steps * p->sweeps[j];
    if (!p->user_stream) EA_HIP(hipStreamSynchronize(p->stream));
    return EA_OK;
}

int ea_plan_info(const ea_plan *p, int *block_threads, int *grid, int *n_units, size_t *lds_bytes, int *uses_graph,
                 int *split_parts)
{
    if (!p) return fail(EA_EINVAL, "ea_plan_info: NULL plan");
    if (split_parts) *split_parts = p->ls.parts;
    if (block_threads) *block_threads = p->ls.bt;
    if (grid) *grid = p->ls.grid;
    if (n_units) *n_units = p->ls.n_units;
    if (lds_bytes) *lds_bytes = p->ls.lds;
    if (uses_graph) *uses_graph = p->exec != nullptr;
    return EA_OK;
}

void ea_plan_destroy(ea_plan *p)
{
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipStreamSynchronize(p->stream);
    for (ea_sim *s : p->sims)
        if (s->plan == p) s->plan = nullptr;
    launchset_free(p->ls);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->own_stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

}  // extern "C"
