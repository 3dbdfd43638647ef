// Host-side internals shared by the ABI (ea_api.cpp) and the runtime
// (ea_runtime.cpp: launch plans with hipGraph, autotuner, serving loop).
// Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ea.h"
#include "ea_internal.h"

namespace ea {

constexpr size_t kLdsBudget = 160 * 1024 - 1024;   // dynamic LDS per workgroup; the rest is static
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr int kThreadsPerCu = 2048;

extern thread_local std::string g_error;
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define EA_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return ::ea::fail(EA_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

uint32_t prob_to_u32(double p);
uint32_t flip_thr(double beta, int u);
uint32_t swap_thr(double dbeta_abs, int64_t n);
uint32_t flip_thr_h(double beta, int u, int S, double h);
uint32_t swap_thr_g(double dbeta_abs, int64_t n, int g);
int field_scale(int m);   // g = gcd(4, m), 4 for m = 0

struct DeviceAlloc {
    void *(*alloc)(size_t, void *) = nullptr;
    void (*release)(void *, void *) = nullptr;
    void *ctx = nullptr;
};

int wgs_per_cu(size_t lds, int bt);
int build_swap_tables(const double *betas, int n_T, int N, int m, std::vector<uint32_t> *sthr, std::vector<int32_t> *soff,
                      std::vector<int32_t> *slen, std::vector<int32_t> *ssgn, int64_t *total);
size_t job_footprint_bytes(int L, int n_T, int R, int layout, int64_t swap_entries);
size_t halo_bytes(int L, int n_T, int R, int layout);   // exchange area of ladders split by halves (0: none)
int device_grid(int kv, int bt, size_t lds, int n_units, int *grid);   // kv: kernel_variant()
// Workgroups per ladder (1, 2 or 4) for one launch over the jobs descs[0..n)
// with workgroups of bt threads and lds bytes: 2 or 4 when every job can be
// split and the launch alone would leave compute units idle.  split_opt as in
// ea_options (1 = never, 2 = whenever possible, 0 = when each part keeps
// enough work).
int choose_split_parts(const JobDesc *descs, int n, int bt, size_t lds, int kv, int split_opt);
// Kernel variant of a launch split into `parts`: kSlabVariant (ladders split
// by lattice halves) when every job allows it and split_opt is not 3, else kv.
int split_variant(const JobDesc *descs, int n, int kv, int parts, int split_opt);

}  // namespace ea

// One job: R realizations x 2 copies x n_T slots, resident in HBM.
struct ea_sim {
    int L = 0, N = 0, n_T = 0, R = 0, layout = 0, NW = 0;
    int block_threads = 0, words_resident = 0;
    int device = 0;
    uint64_t seed = 0;
    int64_t t = 0;                    // host shadow of the sweep counter
    hipStream_t stream = nullptr;
    bool user_stream = false;
    ea::DeviceAlloc da;
    std::vector<void *> owned;        // device buffers to release
    ea::JobDesc h{};                  // host copy of the descriptor
    ea::JobDesc *d_job = nullptr;
    uint32_t *d_units = nullptr;      // ladders of this job for a lone launch
    uint32_t *d_counters = nullptr;   // [0] sweep counter, [1..8] queue words of a lone launch
    int64_t swap_total = 0;           // entries in the swap tables
    size_t lds = 0;                   // dynamic LDS bytes of this job's sweep workgroups
    size_t footprint = 0;             // device bytes owned by this job
    size_t halo_size = 0;             // bytes of h.halo (0: none)
    int split_parts = 1;              // workgroups per ladder in a lone launch (1, 2 or 4)
    int split_opt = 0;                // ea_options.split: 0 auto, 1 never, 2 whenever possible, 3 by slot groups
    bool ever_split = false;          // a split launch has run this job: its exchange may have timed out
    int64_t *d_meas = nullptr;        // measurement sums: count, q^2 [R][n_T], q^4 [R][n_T][2], C [R][n_T][L]
    int32_t *d_obs = nullptr;         // observables outputs: energy, overlap, magnetization
    hipEvent_t ev = nullptr;          // orders launches on other streams (batches, plans) with this job's stream
    ea_plan *plan = nullptr;          // the live plan that holds this job, if any
};

namespace ea {
int check_split_error(ea_sim *s);
// Make `st` wait for the work queued so far on each job's own stream, or each
// job's stream wait for the work queued so far on `st` (after = true).
int order_streams(ea_sim *const *sims, int n_sims, hipStream_t st, bool after);
// A job held by a live plan is being destroyed: the plan drops it and refuses to run.
void plan_forget_job(ea_plan *p, ea_sim *s);
// ea_plan_create with its own sweep count per job and step (sweeps[j] >= 0).
int plan_create(ea_sim *const *sims, int n_sims, const int *sweeps, const int *swap_every,
                const ea_plan_options *opt, ea_plan **out);
}
