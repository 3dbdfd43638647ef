// Host side of the C ABI declared in include/ea.h: argument validation,
// integer probability tables (Sec. 4.3.1, 4.3.2), lattice colour classes,
// device buffers and launch planning.  All simulation arithmetic runs in the
// kernels of ea_kernels.hip.
#include <algorithm>
#include <cmath>
#include <limits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ea.h"
#include "ea_host.h"
#include "ea_internal.h"

using namespace ea;

namespace ea {

thread_local std::string g_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

// ---------------------------------------------------------------------------
// Integer probability tables
// ---------------------------------------------------------------------------
uint32_t prob_to_u32(double p)
{
    const double x = std::floor(std::ldexp(p, 32));
    if (!(x < 4294967295.0)) return 0xFFFFFFFFu;
    if (x <= 0.0) return 0u;
    return (uint32_t)x;
}

// Metropolis: dE = 12 - 4u for a site with u unsatisfied bonds.
uint32_t flip_thr(double beta, int u)
{
    return prob_to_u32(std::exp(-(beta * (double)(12 - 4 * u))));
}

// Replica exchange: |dE| = 2n for |U_a - U_b| = n.
uint32_t swap_thr(double dbeta_abs, int64_t n)
{
    return prob_to_u32(std::exp(-(2.0 * dbeta_abs * (double)n)));
}

// Flip cost 12 - 4u + 2h(2S - 1); the table entry of a cost <= 0 is never read
// (those flips are certain).
uint32_t flip_thr_h(double beta, int u, int S, double h)
{
    const double dE = (double)(12 - 4 * u) + 2.0 * h * (double)(2 * S - 1);
    if (dE <= 0.0) return 0xFFFFFFFFu;
    return prob_to_u32(std::exp(-(beta * dE)));
}

// Swap threshold for an energy difference |E_a - E_b| = g n / 2, where n
// indexes the table and g = gcd(4, 4h) (g = 4 without a field: |dE| = 2n).
uint32_t swap_thr_g(double dbeta_abs, int64_t n, int g)
{
    return prob_to_u32(std::exp(-(dbeta_abs * (0.5 * (double)((int64_t)g * n)))));
}

int field_scale(int m)
{
    const int a = m < 0 ? -m : m;
    if (a == 0 || a % 4 == 0) return 4;
    return a % 2 == 0 ? 2 : 1;
}

}  // namespace ea

namespace ea {

int dev_alloc(ea_sim *s, size_t bytes, void **out)
{
    bytes = std::max<size_t>(bytes, 16);
    void *p = nullptr;
    if (s->da.alloc) {
        p = s->da.alloc(bytes, s->da.ctx);
        if (!p) return fail(EA_ENOMEM, "device allocator returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) return fail(EA_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    s->owned.push_back(p);
    s->footprint += bytes;
    *out = p;
    return EA_OK;
}

// A temporary device buffer from the job's allocator (not counted in its footprint).
int temp_alloc(ea_sim *s, size_t bytes, void **out)
{
    bytes = std::max<size_t>(bytes, 16);
    void *p = nullptr;
    if (s->da.alloc) {
        p = s->da.alloc(bytes, s->da.ctx);
        if (!p) return fail(EA_ENOMEM, "device allocator returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) return fail(EA_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    *out = p;
    return EA_OK;
}

void temp_free(ea_sim *s, void *p)
{
    if (!p) return;
    if (s->da.release)
        s->da.release(p, s->da.ctx);
    else
        (void)hipFree(p);
}

void release_all(ea_sim *s)
{
    for (void *p : s->owned) {
        if (s->da.release)
            s->da.release(p, s->da.ctx);
        else
            (void)hipFree(p);
    }
    s->owned.clear();
}

template <class T>
int upload(ea_sim *s, const std::vector<T> &v, T **out)
{
    void *p = nullptr;
    int rc = dev_alloc(s, v.size() * sizeof(T), &p);
    if (rc) return rc;
    if (!v.empty()) EA_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = (T *)p;
    return EA_OK;
}

int sync_if_needed(ea_sim *s)
{
    if (!s->user_stream) EA_HIP(hipStreamSynchronize(s->stream));
    return EA_OK;
}

// Colour classes (Sec. 3.1 checkerboard; odd L uses three classes).
void colour_classes(int L, std::vector<uint32_t> &sites, int32_t off[4], int *n_classes)
{
    const int nc = (L % 2 == 0) ? 2 : 3;
    auto g = [L](int a) { return a == L - 1 ? 2 : (a & 1); };
    sites.clear();
    for (int c = 0; c < nc; ++c) {
        off[c] = (int32_t)sites.size();
        for (int z = 0; z < L; ++z)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    const int col = (L % 2 == 0) ? ((x + y + z) & 1) : ((g(x) + g(y) + g(z)) % 3);
                    if (col == c) sites.push_back((uint32_t)x | ((uint32_t)y << 8) | ((uint32_t)z << 16));
                }
    }
    for (int c = nc; c < 4; ++c) off[c] = (int32_t)sites.size();
    *n_classes = nc;
}


// Workgroups of `bt` threads and `lds` bytes that fit on one CU.
int wgs_per_cu(size_t lds, int bt)
{
    const int by_lds = (int)(kLdsPerCu / (lds + 1024));
    return std::max(0, std::min(by_lds, kThreadsPerCu / bt));
}

// Optional LDS copies (swap tables, odd-L site list) are taken only when they
// fit and do not lower the number of workgroups a CU can hold.
void plan_optional_lds(int N, int wr, int bt, bool odd, int64_t swap_entries, uint32_t item_bytes, int *swap_lds,
                       int *sites_lds)
{
    *swap_lds = 0;
    *sites_lds = 0;
    auto total = [&](int sw, int si) { return (size_t)lds_layout(N, wr, sw, si, item_bytes).total; };
    const int base = wgs_per_cu(total(0, 0), bt);
    if (odd && total(0, N) <= kLdsBudget && wgs_per_cu(total(0, N), bt) >= base) *sites_lds = N;
    if (swap_entries > 0 && swap_entries < (1 << 20) && total((int)swap_entries, *sites_lds) <= kLdsBudget &&
        wgs_per_cu(total((int)swap_entries, *sites_lds), bt) >= base)
        *swap_lds = (int)swap_entries;
}

int plan_launch(int N, int NW, const ea_options &opt, int *block_threads, int *words_resident)
{
    // words resident in LDS
    const uint32_t items = opt.rng == EA_RNG_PLANES ? kPlaneItemBytes : 0u;
    const LdsLayout lay = lds_layout(N, 1, 1, 1, items);
    if (lay.mask % 8 != 0 || lay.ptab % 16 != 0 || lay.spin % 16 != 0 || lay.thr % 16 != 0 || lay.stab % 4 != 0 ||
        lay.sites % 4 != 0 || lay.items % 16 != 0)
        return fail(EA_EINVAL, "internal LDS layout misaligned for %d sites", N);
    const size_t fixed = lds_layout(N, 0, 0, 0, items).total;
    if (fixed + (size_t)N * 4 > kLdsBudget)
        return fail(EA_EINVAL, "lattice of %d sites does not fit one spin word in LDS", N);
    int wr_max = (int)((kLdsBudget - fixed) / ((size_t)N * 4));
    int wr = std::min(NW, wr_max);
    if (opt.words_resident < 0) return fail(EA_EINVAL, "words_resident=%d < 0", opt.words_resident);
    if (opt.split < 0 || opt.split > 3) return fail(EA_EINVAL, "split=%d is not 0, 1, 2 or 3", opt.split);
    if (opt.words_resident > 0) {
        if (opt.words_resident > wr_max)
            return fail(EA_EINVAL, "words_resident=%d exceeds the %d words that fit in LDS", opt.words_resident, wr_max);
        wr = std::min(NW, opt.words_resident);
    }
    // threads: one site of a colour class per thread where possible
    int min_bt = ((N + 84) / 85 + 63) / 64 * 64;   // keeps per-lane bond counts below 256
    int bt = opt.block_threads;
    if (bt == 0) {
        bt = std::min(kMaxBlock, std::max(256, (N / 2 + 63) / 64 * 64));
        bt = std::max(bt, min_bt);
    }
    if (bt < 64 || bt > kMaxBlock || bt % 64 != 0)
        return fail(EA_EINVAL, "block_threads=%d must be a multiple of 64 in [64, %d]", bt, kMaxBlock);
    if (bt < min_bt) return fail(EA_EINVAL, "block_threads=%d is below %d for %d sites", bt, min_bt, N);
    *block_threads = bt;
    *words_resident = wr;
    return EA_OK;
}

int device_grid(int kv, int bt, size_t lds, int n_units, int *grid)
{
    int dev = 0;
    EA_HIP(hipGetDevice(&dev));
    int cus = 0;
    EA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = sweep_max_blocks_per_cu(kv, 1, bt, lds);
    if (per_cu < 1) return fail(EA_EDEVICE, "sweep kernel cannot be resident with %d threads and %zu B LDS", bt, lds);
    *grid = std::max(1, std::min(n_units, cus * per_cu));
    return EA_OK;
}

// Swap tables per pair k: entries n = 0.. while the threshold is non-zero
// (|U_a - U_b| <= 3N caps the length).  sthr may be NULL to size only.
int build_swap_tables(const double *betas, int n_T, int N, int m, std::vector<uint32_t> *sthr,
                      std::vector<int32_t> *soff, std::vector<int32_t> *slen, std::vector<int32_t> *ssgn,
                      int64_t *total)
{
    const int g = field_scale(m);
    if (soff) soff->assign(kMaxTemps, 0);
    if (slen) slen->assign(kMaxTemps, 0);
    if (ssgn) ssgn->assign(kMaxTemps, 0);
    if (sthr) sthr->clear();
    int64_t count = 0;
    for (int k = 0; k + 1 < n_T; ++k) {
        const double db = betas[k] - betas[k + 1];
        const int sg = (db > 0.0) - (db < 0.0);
        if (ssgn) (*ssgn)[k] = sg;
        if (soff) (*soff)[k] = (int32_t)count;
        if (sg == 0) continue;
        const double dabs = std::fabs(db);
        // |2 (E_a - E_b)| = |4 dU - m d(up)| <= 12 N + |m| N
        const int64_t cap = (12 * (int64_t)N + (int64_t)(m < 0 ? -m : m) * N) / g;
        int64_t n = 0;
        uint32_t prev = 0xFFFFFFFFu;
        for (; n <= cap; ++n) {
            const uint32_t v = swap_thr_g(dabs, n, g);
            if (v == 0) break;
            // the split by lattice halves turns each pair's test into a cut
            // on n, which needs thresholds that never increase with n
            if (v > prev) return fail(EA_EINVAL, "non-monotone swap table for pair %d", k);
            prev = v;
            if (sthr) sthr->push_back(v);
        }
        // the thresholds decrease with n; check that the zero tail stays zero
        for (int64_t q = n; q <= std::min(cap, n + 64); ++q)
            if (swap_thr_g(dabs, q, g) != 0) return fail(EA_EINVAL, "non-monotone swap table for pair %d", k);
        if (slen) (*slen)[k] = (int32_t)n;
        count += n;
    }
    if (total) *total = count;
    return EA_OK;
}

// Compute units of the current device (256 when no device can be queried).
static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return 256;
    return cus;
}

// Bytes of the boundary-plane exchange of ladders split by lattice halves:
// [ladders][2 parts][2 classes][2 sides][L^2 / 2] tagged words, for jobs of a
// shape that can run so (CAMSC, one word per site, even L >= 4) with few
// enough ladders to be split at all (two workgroups per ladder fit in the
// device's compute units); 0 otherwise.
size_t halo_bytes(int L, int n_T, int R, int layout)
{
    const int64_t ladders = 2 * (int64_t)R;
    if (layout != EA_LAYOUT_CAMSC || n_T > 32 || (L & 1) || L < 4 || 2 * ladders > device_cus()) return 0;
    return (size_t)ladders * 8 * ((size_t)L * L / 2) * sizeof(uint64_t);
}

// Device bytes ea_create allocates for a job (one term per allocation).
size_t job_footprint_bytes(int L, int n_T, int R, int layout, int64_t swap_entries)
{
    auto a = [](size_t b) { return std::max<size_t>(b, 16); };
    const size_t N = (size_t)L * L * L, ladders = 2 * (size_t)R;
    const size_t NW = (size_t)(n_T + slots_per_word(layout) - 1) / slots_per_word(layout);
    const size_t halo = halo_bytes(L, n_T, R, layout);
    return a(ladders * NW * N * 4) + a((size_t)R * N) + a(ladders * kMaxTemps * 4) + a((size_t)n_T * kThrCols * 4) +
           a((size_t)swap_entries * 4) + 3 * a(kMaxTemps * 4) + a(N * 4) + a(kCounterWords * 4) + a(ladders * kMaxTemps * 8) +
           a(ladders * 4) + a(sizeof(JobDesc)) + a(ladders * 2 * kMaxTemps * 8) + a(4) + (halo ? a(halo) : 0) +
           a((size_t)R * n_T * (4 + L) * 8) + a((size_t)R * n_T * 5 * 4);
}

int choose_split_parts(const JobDesc *descs, int n, int bt, size_t lds, int kv, int split_opt)
{
    if (split_opt == 1 || n < 1 || (kv != 0 && kv != 2)) return 1;   // CAMSC word or plane draws only
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
    int64_t ladders = 0;
    for (int j = 0; j < n; ++j) {
        const JobDesc &d = descs[j];
        if (d.NW != 1 || (d.L & 1)) return 1;
        const int per_lane = 6 * ((d.N / 2 + bt - 1) / bt);
        if (per_lane > 255) return 1;   // class energy sums must fit 8 bit planes
        ladders += d.ladders;
    }
    for (int parts : {4, 2}) {
        // never more workgroups than CUs (measured: 4 parts x 512 threads, two per CU, is
        // slower than 2 parts x 1024); a small lattice is latency-bound: the exchange
        // costs more than the split saves unless each part keeps enough work (measured
        // with PT every sweep: 4 parts pay off from 1024 site-groups per part, 2 parts
        // from 2048)
        if (ladders * parts > cus) continue;
        // two parts may split by lattice halves, which needs no even count of slot groups
        const bool halves = parts == 2 && split_variant(descs, n, kv, parts, split_opt) != kv;
        bool ok = true;
        for (int j = 0; j < n && ok; ++j) {
            const int ngr = (descs[j].n_T + 3) >> 2;
            if (ngr % parts != 0 && !halves) ok = false;
            if (split_opt == 0 && (int64_t)descs[j].N * ngr / parts < 4096 / parts) ok = false;
        }
        if (!ok) continue;
        // every workgroup resident at once: each queue's parts meet without waiting for a slot
        const int per_cu = sweep_max_blocks_per_cu(kv, parts, bt, lds);
        if (per_cu < 1 || (int64_t)per_cu * cus < split_grid((int)ladders, parts)) continue;
        return parts;
    }
    return 1;
}

// Kernel variant of a split launch: ladders split by lattice halves
// (kSlabVariant for word draws, kSlabPlanesVariant for plane draws) when every
// job allows it (CAMSC, one word per site, even L >= 4, no field, natural
// order, an exchange area) and the split is two ways, unless split_opt asks
// for slot groups (3); otherwise kv.
int split_variant(const JobDesc *descs, int n, int kv, int parts, int split_opt)
{
    if (parts != 2 || (kv != 0 && kv != 2) || split_opt == 3 || n < 1) return kv;
    for (int j = 0; j < n; ++j) {
        const JobDesc &d = descs[j];
        if (!d.halo || d.NW != 1 || (d.L & 1) || d.L < 4 || d.field_m != 0 || d.site_order != 0) return kv;
    }
    return kv == 0 ? kSlabVariant : kSlabPlanesVariant;
}

// Workgroups per ladder for a lone launch of the job.
static int choose_split(const ea_sim *s, int split_opt)
{
    return choose_split_parts(&s->h, 1, s->block_threads, s->lds, kernel_variant(s->layout, s->h.rng), split_opt);
}

int order_streams(ea_sim *const *sims, int n_sims, hipStream_t st, bool after)
{
    for (int j = 0; j < n_sims; ++j) {
        ea_sim *s = sims[j];
        if (s->stream == st) continue;
        if (after) {
            EA_HIP(hipEventRecord(s->ev, st));
            EA_HIP(hipStreamWaitEvent(s->stream, s->ev, 0));
        } else {
            EA_HIP(hipEventRecord(s->ev, s->stream));
            EA_HIP(hipStreamWaitEvent(st, s->ev, 0));
        }
    }
    return EA_OK;
}

int check_split_error(ea_sim *s)
{
    if (!s->ever_split) return EA_OK;
    uint32_t err = 0;
    EA_HIP(hipMemcpyAsync(&err, s->h.error, sizeof err, hipMemcpyDeviceToHost, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    if (err) return fail(EA_EDEVICE, "a split-ladder exchange timed out; the job's state is not valid");
    return EA_OK;
}

}  // namespace ea

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

void ea_default_options(ea_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->layout = EA_LAYOUT_CAMSC;
}

const char *ea_last_error(void) { return g_error.c_str(); }

const char *ea_version(void) { return "ea-mi355x 0.1 (gfx950, Philox4x32-10, CAMSC/AMSC4)"; }

uint32_t ea_swap_threshold(double dbeta_abs, int64_t n) { return swap_thr(dbeta_abs, n); }

int ea_flip_thresholds(const double *betas, int n_T, uint32_t *out)
{
    if (!betas || !out || n_T < 1 || n_T > EA_MAX_TEMPS) return fail(EA_EINVAL, "ea_flip_thresholds: bad arguments");
    for (int k = 0; k < n_T; ++k)
        for (int u = 0; u < 3; ++u) out[k * 3 + u] = flip_thr(betas[k], u);
    return EA_OK;
}

int ea_create(int L, const int8_t *couplings, const double *betas, int n_T, int n_realizations, uint64_t seed,
              const ea_options *opt_in, ea_sim **out)
{
    if (!out) return fail(EA_EINVAL, "ea_create: out is NULL");
    *out = nullptr;
    ea_options opt;
    ea_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (L < 2 || L > EA_MAX_L) return fail(EA_EINVAL, "L=%d outside [2, %d]", L, EA_MAX_L);
    if (n_T < 1 || n_T > EA_MAX_TEMPS) return fail(EA_EINVAL, "n_T=%d outside [1, %d]", n_T, EA_MAX_TEMPS);
    if (n_realizations < 1 || n_realizations > (1 << 19))
        return fail(EA_EINVAL, "n_realizations=%d outside [1, 2^19]", n_realizations);
    if (!couplings || !betas) return fail(EA_EINVAL, "couplings and betas must not be NULL");
    if (opt.layout < EA_LAYOUT_CAMSC || opt.layout > EA_LAYOUT_AMSC1)
        return fail(EA_EINVAL, "unknown layout %d", opt.layout);
    if (opt.rng != EA_RNG_WORDS && opt.rng != EA_RNG_PLANES) return fail(EA_EINVAL, "unknown rng %d", opt.rng);
    if (opt.rng == EA_RNG_PLANES && opt.layout != EA_LAYOUT_CAMSC)
        return fail(EA_EINVAL, "plane draws need the CAMSC layout");
    if (!(std::fabs(opt.field) <= 8.0) || 4.0 * opt.field != std::floor(4.0 * opt.field))
        return fail(EA_EINVAL, "field %g is not a multiple of 1/4 in [-8, 8]", opt.field);
    if (opt.rng == EA_RNG_PLANES && opt.field != 0.0) return fail(EA_EINVAL, "plane draws need field 0");
    if ((opt.dev_alloc == nullptr) != (opt.dev_free == nullptr))
        return fail(EA_EINVAL, "dev_alloc and dev_free must be given together");
    if (opt.site_order != EA_ORDER_NATURAL && opt.site_order != EA_ORDER_BY_CLASS)
        return fail(EA_EINVAL, "unknown site_order %d", opt.site_order);
    if (opt.site_order == EA_ORDER_BY_CLASS && (opt.layout != EA_LAYOUT_CAMSC || (L & 1)))
        return fail(EA_EINVAL, "site_order by class needs the CAMSC layout and even L");
    for (int k = 0; k < n_T; ++k)
        if (!std::isfinite(betas[k]) || !(betas[k] > 0.0))
            return fail(EA_EINVAL, "betas[%d]=%g must be finite and > 0", k, betas[k]);
    const int N = L * L * L;
    const size_t nJ = (size_t)n_realizations * N * 3;
    for (size_t b = 0; b < nJ; ++b)
        if (couplings[b] != 1 && couplings[b] != -1)
            return fail(EA_EINVAL, "couplings[%zu]=%d is not +1 or -1", b, (int)couplings[b]);

    const int spw = slots_per_word(opt.layout);
    const int NW = (n_T + spw - 1) / spw;
    int bt = 0, wr = 0;
    if (int rc = plan_launch(N, NW, opt, &bt, &wr)) return rc;

    ea_sim *s = new (std::nothrow) ea_sim;
    if (!s) return fail(EA_ENOMEM, "host allocation failed");
    s->L = L; s->N = N; s->n_T = n_T; s->R = n_realizations; s->layout = opt.layout; s->NW = NW;
    s->block_threads = bt; s->words_resident = wr; s->seed = seed;
    s->stream = (hipStream_t)opt.stream;
    s->user_stream = opt.stream != nullptr;
    s->da.alloc = opt.dev_alloc; s->da.release = opt.dev_free; s->da.ctx = opt.alloc_ctx;

    auto bail = [s](int rc) {
        release_all(s);
        if (s->ev) (void)hipEventDestroy(s->ev);
        delete s;
        return rc;
    };
    hipError_t he = hipGetDevice(&s->device);
    if (he != hipSuccess) return bail(fail(EA_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(he)));
    he = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
    if (he != hipSuccess) return bail(fail(EA_EDEVICE, "hipEventCreate failed: %s", hipGetErrorString(he)));

    const int ladders = 2 * n_realizations;
    // tables
    const double hf = opt.field;
    const int m = (int)(4.0 * hf);   // exact: validated as a multiple of 1/4
    // columns 2E + S; a certain flip (cost <= 0) keeps 0: the kernels never read it
    std::vector<uint32_t> fthr((size_t)n_T * kThrCols, 0u);
    int a_first[2] = {7, 7};   // smallest E whose flip is certain, per spin bit S (7: none)
    for (int S = 0; S < 2; ++S)
        for (int E = 6; E >= 0; --E)
            if ((double)(12 - 4 * E) + 2.0 * hf * (double)(2 * S - 1) <= 0.0) a_first[S] = E;
    for (int k = 0; k < n_T; ++k)
        for (int col = 0; col < 14; ++col) {
            const int E = col >> 1, S = col & 1;
            fthr[(size_t)k * kThrCols + col] = E < a_first[S] ? flip_thr_h(betas[k], E, S, hf) : 0u;
        }
    std::vector<int32_t> soff, slen, ssgn;
    std::vector<uint32_t> sthr;
    if (int rc = build_swap_tables(betas, n_T, N, m, &sthr, &soff, &slen, &ssgn, nullptr)) return bail(rc);
    // couplings as 6 incidence bits per site
    std::vector<uint8_t> j6((size_t)n_realizations * N);
    for (int r = 0; r < n_realizations; ++r) {
        const int8_t *J = couplings + (size_t)r * N * 3;
        for (int z = 0; z < L; ++z)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    const int i = x + L * (y + L * z);
                    const int im[3] = {((x + L - 1) % L) + L * (y + L * z), x + L * (((y + L - 1) % L) + L * z),
                                       x + L * (y + L * ((z + L - 1) % L))};
                    uint8_t b = 0;
                    for (int mu = 0; mu < 3; ++mu) {
                        if (J[3 * i + mu] < 0) b |= (uint8_t)(1u << (2 * mu));
                        if (J[3 * im[mu] + mu] < 0) b |= (uint8_t)(1u << (2 * mu + 1));
                    }
                    j6[(size_t)r * N + i] = b;
                }
    }
    std::vector<uint32_t> sites;
    int32_t class_off[4];
    int n_classes = 0;
    colour_classes(L, sites, class_off, &n_classes);

    JobDesc &h = s->h;
    int rc = EA_OK;
    void *p = nullptr;
    if ((rc = dev_alloc(s, (size_t)ladders * NW * N * 4, &p))) return bail(rc);
    h.spins = (uint32_t *)p;
    uint8_t *dj6 = nullptr;
    if ((rc = upload(s, j6, &dj6))) return bail(rc);
    h.j6 = dj6;
    std::vector<int32_t> perm((size_t)ladders * kMaxTemps, 0);
    for (int l = 0; l < ladders; ++l)
        for (int k = 0; k < n_T; ++k) perm[(size_t)l * kMaxTemps + k] = k;
    if ((rc = upload(s, perm, &h.temp_of_slot))) return bail(rc);
    uint32_t *dft = nullptr, *dst = nullptr, *dsites = nullptr;
    int32_t *doff = nullptr, *dlen = nullptr, *dsgn = nullptr;
    if ((rc = upload(s, fthr, &dft)) || (rc = upload(s, sthr, &dst)) || (rc = upload(s, soff, &doff)) ||
        (rc = upload(s, slen, &dlen)) || (rc = upload(s, ssgn, &dsgn)) || (rc = upload(s, sites, &dsites)))
        return bail(rc);
    h.flip_thr = dft; h.swap_thr = dst; h.swap_off = doff; h.swap_len = dlen; h.swap_sgn = dsgn; h.sites = dsites;
    std::vector<uint32_t> counters(kCounterWords, 0u);   // sweep counter, then the launch's queue words
    if ((rc = upload(s, counters, &s->d_counters))) return bail(rc);
    h.sweep_ctr = s->d_counters;
    std::vector<uint64_t> acc((size_t)ladders * kMaxTemps, 0u);
    if ((rc = upload(s, acc, &h.swap_acc))) return bail(rc);
    std::vector<uint64_t> xchg((size_t)ladders * 2 * kMaxTemps, 0);
    std::vector<uint32_t> err(1, 0u);
    if ((rc = upload(s, xchg, &h.xchg)) || (rc = upload(s, err, &h.error)))
        return bail(rc);
    if (const size_t hb = halo_bytes(L, n_T, n_realizations, opt.layout)) {
        std::vector<uint64_t> halo(hb / sizeof(uint64_t), 0);   // tag 0: no sweep has written yet
        if ((rc = upload(s, halo, &h.halo))) return bail(rc);
        s->halo_size = hb;
    }
    std::vector<int64_t> meas((size_t)n_realizations * n_T * (4 + L), 0);
    if ((rc = upload(s, meas, &s->d_meas))) return bail(rc);
    // outputs of the observables kernel: energy and magnetization [R][2][n_T], overlap [R][n_T]
    std::vector<int32_t> obs((size_t)n_realizations * n_T * 5, 0);
    if ((rc = upload(s, obs, &s->d_obs))) return bail(rc);
    std::vector<uint32_t> units(ladders);
    for (int l = 0; l < ladders; ++l) units[l] = (uint32_t)l;   // job 0 of a lone launch
    if ((rc = upload(s, units, &s->d_units))) return bail(rc);
    for (int c = 0; c < 4; ++c) h.class_off[c] = class_off[c];
    h.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
    h.key1 = (uint32_t)(seed >> 32);
    h.L = L; h.N = N; h.n_T = n_T; h.NW = NW; h.n_classes = n_classes; h.words_resident = wr;
    h.n_sweeps = 0; h.swap_every = 0; h.ladders = ladders; h.block_threads = bt;
    h.seg_bits = 4;
    h.rng = opt.rng;
    h.field_m = m;
    h.field_g = field_scale(m);
    h.always_add0 = (uint32_t)(8 - a_first[0]) * 0x11111111u;
    h.always_add1 = (uint32_t)(8 - a_first[1]) * 0x11111111u;
    h.always_col0 = 2 * a_first[0];
    h.always_col1 = 2 * a_first[1] + 1;
    h.site_order = opt.site_order;
    h.invL = 1.0f / (float)L;
    h.invH = 1.0f / (float)(L / 2 > 0 ? L / 2 : 1);
    s->swap_total = (int64_t)sthr.size();
    const uint32_t item_bytes = opt.rng == EA_RNG_PLANES ? kPlaneItemBytes : 0u;
    plan_optional_lds(N, wr, bt, L % 2 != 0, s->swap_total, item_bytes, &h.swap_lds, &h.sites_lds);
    s->lds = lds_layout(N, wr, h.swap_lds, h.sites_lds, item_bytes).total;
    s->split_opt = opt.split;
    s->split_parts = choose_split(s, opt.split);
    std::vector<JobDesc> hv(1, h);
    if ((rc = upload(s, hv, &s->d_job))) return bail(rc);
    he = launch_init_spins(s->d_job, h, s->layout, s->stream);
    if (he != hipSuccess) return bail(fail(EA_EDEVICE, "init kernel launch failed: %s", hipGetErrorString(he)));
    he = hipStreamSynchronize(s->stream);
    if (he != hipSuccess) return bail(fail(EA_EDEVICE, "init kernel failed: %s", hipGetErrorString(he)));
    *out = s;
    return EA_OK;
}

int ea_job_footprint(int L, const double *betas, int n_T, int n_realizations, int layout, size_t *bytes)
{
    if (!betas || !bytes || L < 2 || L > EA_MAX_L || n_T < 1 || n_T > EA_MAX_TEMPS || n_realizations < 1 ||
        (layout < EA_LAYOUT_CAMSC || layout > EA_LAYOUT_AMSC1))
        return fail(EA_EINVAL, "ea_job_footprint: bad arguments");
    int64_t total = 0;
    if (int rc = build_swap_tables(betas, n_T, L * L * L, 0, nullptr, nullptr, nullptr, nullptr, &total)) return rc;
    *bytes = job_footprint_bytes(L, n_T, n_realizations, layout, total);
    return EA_OK;
}

int ea_sim_info(const ea_sim *s, int *block_threads, int *words_resident, int *split_parts, size_t *lds_bytes)
{
    if (!s) return fail(EA_EINVAL, "ea_sim_info: NULL handle");
    if (block_threads) *block_threads = s->block_threads;
    if (words_resident) *words_resident = s->words_resident;
    if (split_parts) *split_parts = s->split_parts;
    if (lds_bytes) *lds_bytes = s->lds;
    return EA_OK;
}

int ea_sim_split(const ea_sim *s, int *split_parts, int *by_halves)
{
    if (!s) return fail(EA_EINVAL, "ea_sim_split: NULL handle");
    if (split_parts) *split_parts = s->split_parts;
    if (by_halves)
        *by_halves = s->split_parts > 1 && split_variant(&s->h, 1, kernel_variant(s->layout, s->h.rng), s->split_parts,
                                                         s->split_opt) != kernel_variant(s->layout, s->h.rng);
    return EA_OK;
}

// ---- measurements (Sec. 5) ----
static void meas_parts(ea_sim *s, int64_t **count, int64_t **q2, uint64_t **q4, int64_t **c)
{
    const size_t rt = (size_t)s->R * s->n_T;
    *count = s->d_meas;
    *q2 = s->d_meas + rt;
    *q4 = (uint64_t *)(s->d_meas + 2 * rt);
    *c = s->d_meas + 4 * rt;
}

int ea_measure(ea_sim *s)
{
    if (!s) return fail(EA_EINVAL, "ea_measure: NULL handle");
    EA_HIP(hipSetDevice(s->device));
    int64_t *count, *q2, *c;
    uint64_t *q4;
    meas_parts(s, &count, &q2, &q4, &c);
    EA_HIP(launch_measure(s->d_job, s->h, s->layout, count, q2, q4, c, s->stream));
    if (!s->user_stream) {
        EA_HIP(hipStreamSynchronize(s->stream));
        return check_split_error(s);
    }
    return EA_OK;
}

int ea_measure_read(ea_sim *s, int64_t *count, int64_t *sum_q2, uint64_t *sum_q4, int64_t *sum_c)
{
    if (!s) return fail(EA_EINVAL, "ea_measure_read: NULL handle");
    EA_HIP(hipSetDevice(s->device));
    const size_t rt = (size_t)s->R * s->n_T;
    std::vector<int64_t> h(rt * (4 + s->L));
    EA_HIP(hipMemcpyAsync(h.data(), s->d_meas, h.size() * 8, hipMemcpyDeviceToHost, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    if (int rc = check_split_error(s)) return rc;
    if (count) std::memcpy(count, h.data(), rt * 8);
    if (sum_q2) std::memcpy(sum_q2, h.data() + rt, rt * 8);
    if (sum_q4) std::memcpy(sum_q4, h.data() + 2 * rt, 2 * rt * 8);
    if (sum_c) std::memcpy(sum_c, h.data() + 4 * rt, rt * s->L * 8);
    return EA_OK;
}

int ea_measure_reset(ea_sim *s)
{
    if (!s) return fail(EA_EINVAL, "ea_measure_reset: NULL handle");
    EA_HIP(hipSetDevice(s->device));
    EA_HIP(hipMemsetAsync(s->d_meas, 0, (size_t)s->R * s->n_T * (4 + s->L) * 8, s->stream));
    if (!s->user_stream) EA_HIP(hipStreamSynchronize(s->stream));
    return EA_OK;
}

int ea_binder_xi(ea_sim *s, double *binder, double *xi_over_L)
{
    if (!s) return fail(EA_EINVAL, "ea_binder_xi: NULL handle");
    const int R = s->R, n_T = s->n_T, L = s->L;
    const size_t rt = (size_t)R * n_T;
    std::vector<int64_t> count(rt), q2(rt), c(rt * L);
    std::vector<uint64_t> q4(2 * rt);
    if (int rc = ea_measure_read(s, count.data(), q2.data(), q4.data(), c.data())) return rc;
    const double N = (double)s->N, kmin = 2.0 * M_PI / L;
    for (int k = 0; k < n_T; ++k) {
        double m2 = 0, m4 = 0, ck = 0;
        for (int r = 0; r < R; ++r) {
            const size_t rk = (size_t)r * n_T + k;
            if (count[rk] <= 0) return fail(EA_ESTATE, "no measurement taken for realization %d", r);
            const double n = (double)count[rk];
            m2 += (double)q2[rk] / n;
            m4 += ((double)q4[2 * rk] + std::ldexp((double)q4[2 * rk + 1], 64)) / n;
            double sk = 0;
            for (int d = 0; d < L; ++d) sk += (double)c[rk * L + d] * std::cos(kmin * d);
            ck += sk / n;
        }
        m2 /= R;
        m4 /= R;
        ck /= R;
        if (binder) binder[k] = 0.5 * (3.0 - m4 / (m2 * m2));
        if (xi_over_L) {
            const double ratio = (m2 / N) / (ck / (3.0 * N));
            xi_over_L[k] = ratio >= 1.0 ? std::sqrt(ratio - 1.0) / (2.0 * std::sin(kmin / 2.0)) / L
                                        : std::numeric_limits<double>::quiet_NaN();
        }
    }
    return EA_OK;
}

int ea_sim_footprint(const ea_sim *s, size_t *bytes)
{
    if (!s || !bytes) return fail(EA_EINVAL, "ea_sim_footprint: NULL argument");
    *bytes = s->footprint;
    return EA_OK;
}

void ea_destroy(ea_sim *s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    if (s->plan) plan_forget_job(s->plan, s);
    release_all(s);
    if (s->ev) (void)hipEventDestroy(s->ev);
    delete s;
}

int ea_get_dims(const ea_sim *s, int *L, int *n_T, int *R, int *layout)
{
    if (!s) return fail(EA_EINVAL, "ea_get_dims: NULL handle");
    if (L) *L = s->L;
    if (n_T) *n_T = s->n_T;
    if (R) *R = s->R;
    if (layout) *layout = s->layout;
    return EA_OK;
}

int ea_sweep(ea_sim *s, int64_t n_sweeps, int swap_every)
{
    return ea_sweep_batch(&s, 1, &n_sweeps, &swap_every);
}

int ea_observables(ea_sim *s, int32_t *energy, int32_t *overlap)
{
    if (!s) return fail(EA_EINVAL, "ea_observables: NULL handle");
    EA_HIP(hipSetDevice(s->device));
    const size_t ne = (size_t)s->R * 2 * s->n_T, nq = (size_t)s->R * s->n_T;
    int32_t *d = s->d_obs;
    hipError_t e = launch_observables(s->d_job, s->h, s->layout, d, d + ne, nullptr, s->stream);
    if (e == hipSuccess && energy) e = hipMemcpyAsync(energy, d, ne * sizeof(int32_t), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && overlap) e = hipMemcpyAsync(overlap, d + ne, nq * sizeof(int32_t), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(EA_EDEVICE, "observables failed: %s", hipGetErrorString(e));
    return check_split_error(s);
}

int ea_magnetization(ea_sim *s, int32_t *magnetization)
{
    if (!s || !magnetization) return fail(EA_EINVAL, "ea_magnetization: NULL argument");
    EA_HIP(hipSetDevice(s->device));
    const size_t ne = (size_t)s->R * 2 * s->n_T, nq = (size_t)s->R * s->n_T;
    int32_t *d = s->d_obs + ne + nq;
    hipError_t e = launch_observables(s->d_job, s->h, s->layout, nullptr, nullptr, d, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(magnetization, d, ne * sizeof(int32_t), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(EA_EDEVICE, "magnetization failed: %s", hipGetErrorString(e));
    return check_split_error(s);
}

int ea_state(ea_sim *s, int8_t *spins, int32_t *temp_of_slot, int64_t *sweeps_done)
{
    if (!s) return fail(EA_EINVAL, "ea_state: NULL handle");
    EA_HIP(hipSetDevice(s->device));
    const int ladders = 2 * s->R;
    hipError_t e = hipSuccess;
    if (spins) {
        const size_t n = (size_t)ladders * s->n_T * s->N;
        void *d = nullptr;
        if (int rc = temp_alloc(s, n, &d)) return rc;
        e = launch_unpack(s->d_job, s->h, s->layout, (int8_t *)d, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(spins, d, n, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        temp_free(s, d);
        if (e != hipSuccess) return fail(EA_EDEVICE, "state readout failed: %s", hipGetErrorString(e));
    }
    if (temp_of_slot) {
        std::vector<int32_t> perm((size_t)ladders * kMaxTemps);
        EA_HIP(hipMemcpyAsync(perm.data(), s->h.temp_of_slot, perm.size() * 4, hipMemcpyDeviceToHost, s->stream));
        EA_HIP(hipStreamSynchronize(s->stream));
        for (int l = 0; l < ladders; ++l)
            for (int k = 0; k < s->n_T; ++k) temp_of_slot[(size_t)l * s->n_T + k] = perm[(size_t)l * kMaxTemps + k];
    }
    if (int rc = check_split_error(s)) return rc;
    if (sweeps_done) {
        uint32_t t = 0;
        EA_HIP(hipMemcpyAsync(&t, s->d_counters, sizeof t, hipMemcpyDeviceToHost, s->stream));
        EA_HIP(hipStreamSynchronize(s->stream));
        *sweeps_done = (int64_t)t;
    }
    return EA_OK;
}

int ea_set_state(ea_sim *s, const int8_t *spins, const int32_t *temp_of_slot, int64_t sweeps_done)
{
    if (!s || !spins || !temp_of_slot) return fail(EA_EINVAL, "ea_set_state: NULL argument");
    if (sweeps_done < 0 || sweeps_done >= ((int64_t)1 << 32)) return fail(EA_EINVAL, "sweeps_done out of range");
    const int ladders = 2 * s->R;
    const size_t n = (size_t)ladders * s->n_T * s->N;
    for (size_t b = 0; b < n; ++b)
        if (spins[b] != 1 && spins[b] != -1) return fail(EA_EINVAL, "spins[%zu]=%d is not +1 or -1", b, (int)spins[b]);
    std::vector<int32_t> perm((size_t)ladders * kMaxTemps, 0);
    for (int l = 0; l < ladders; ++l) {
        std::vector<int> seen(s->n_T, 0);
        for (int k = 0; k < s->n_T; ++k) {
            const int32_t v = temp_of_slot[(size_t)l * s->n_T + k];
            if (v < 0 || v >= s->n_T || seen[v]) return fail(EA_EINVAL, "temp_of_slot of ladder %d is not a permutation", l);
            seen[v] = 1;
            perm[(size_t)l * kMaxTemps + k] = v;
        }
    }
    EA_HIP(hipSetDevice(s->device));
    void *d = nullptr;
    if (int rc = temp_alloc(s, n, &d)) return rc;
    const uint32_t t = (uint32_t)sweeps_done;
    hipError_t e = hipMemcpyAsync(d, spins, n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = launch_pack(s->d_job, s->h, s->layout, (const int8_t *)d, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h.temp_of_slot, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d_counters, &t, sizeof t, hipMemcpyHostToDevice, s->stream);
    // exchange words carry sweep tags: a rewound counter must not meet stale ones
    if (e == hipSuccess) e = hipMemsetAsync(s->h.xchg, 0, (size_t)ladders * 2 * kMaxTemps * sizeof(uint64_t), s->stream);
    if (e == hipSuccess && s->h.halo)
        e = hipMemsetAsync(s->h.halo, 0, s->halo_size, s->stream);
    // a valid state clears an earlier exchange timeout
    if (e == hipSuccess) e = hipMemsetAsync(s->h.error, 0, sizeof(uint32_t), s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    temp_free(s, d);
    if (e != hipSuccess) return fail(EA_EDEVICE, "state upload failed: %s", hipGetErrorString(e));
    s->t = sweeps_done;
    return EA_OK;
}

int ea_swap_acceptance(ea_sim *s, uint64_t *accepted)
{
    if (!s || !accepted) return fail(EA_EINVAL, "ea_swap_acceptance: NULL argument");
    EA_HIP(hipSetDevice(s->device));
    const int ladders = 2 * s->R;
    std::vector<uint64_t> acc((size_t)ladders * kMaxTemps);
    EA_HIP(hipMemcpyAsync(acc.data(), s->h.swap_acc, acc.size() * 8, hipMemcpyDeviceToHost, s->stream));
    EA_HIP(hipStreamSynchronize(s->stream));
    for (int l = 0; l < ladders; ++l)
        for (int k = 0; k + 1 < s->n_T; ++k)
            accepted[(size_t)l * (s->n_T - 1) + k] = acc[(size_t)l * kMaxTemps + k];
    return EA_OK;
}

}  // extern "C"
