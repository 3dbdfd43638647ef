// Internal declarations shared by the host side (ea_api.cpp) and the HIP
// kernels (ea_kernels.hip) of the library.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ea {

// Philox4x32 constants (Salmon et al., SC'11): multipliers and Weyl key bumps.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;
constexpr int kPhiloxRounds = 10;

// Stream domains, counter word 3 bits 28..31.
constexpr uint32_t kDomainFlip = 0u;
constexpr uint32_t kDomainSwap = 1u;
constexpr uint32_t kDomainInit = 2u;
constexpr uint32_t kDomainPlane = 4u;   // bit-plane flip draws (EA_RNG_PLANES)

constexpr int kMaxTemps = 64;
constexpr int kThrCols = 16;          // threshold row: column 2E+S, E in 0..6, S in 0..1
constexpr int kMaxBlock = 1024;
constexpr int kMaxWaves = kMaxBlock / 64;
constexpr int kQueueWords = 8;        // work-queue counters of a launch (one per XCD for split ladders)
constexpr int kCounterWords = 16;     // a job's device counters: [0] sweeps done, [1..8] its lone launch's queues

// Layout parameters: slots per 32-bit word and the bit stride between slots.
template <int LAYOUT> struct Layout;
// kKeep marks the spin bit of every slot.
template <> struct Layout<0> {   // CAMSC
    static constexpr int kSlotsPerWord = 32; static constexpr int kStride = 1; static constexpr uint32_t kKeep = 0xFFFFFFFFu;
};
template <> struct Layout<1> {   // AMSC4
    static constexpr int kSlotsPerWord = 8;  static constexpr int kStride = 4; static constexpr uint32_t kKeep = 0x11111111u;
};
template <> struct Layout<2> {   // AMSC3
    static constexpr int kSlotsPerWord = 10; static constexpr int kStride = 3; static constexpr uint32_t kKeep = 0x09249249u;
};
template <> struct Layout<3> {   // AMSC1 (stored like CAMSC)
    static constexpr int kSlotsPerWord = 32; static constexpr int kStride = 1; static constexpr uint32_t kKeep = 0xFFFFFFFFu;
};

inline int slots_per_word(int layout) { return layout == 1 ? 8 : (layout == 2 ? 10 : 32); }

// One job (an ea_sim) as the kernels see it.  Lives in device memory.
struct JobDesc {
    uint32_t *spins;          // [ladders][NW][N] packed words, ladder = 2r + copy
    const uint8_t *j6;        // [R][N] bit d set iff incidence d has J = -1;
                              // d = 0:+x 1:-x 2:+y 3:-y 4:+z 5:-z
    int32_t *temp_of_slot;    // [ladders][kMaxTemps]
    const uint32_t *flip_thr; // [n_T][kThrCols] by column 2E+S (columns >= 6 are 0)
    const uint32_t *swap_thr; // concatenated per-pair tables, entry n = |U_a - U_b|
    const int32_t *swap_off;  // [kMaxTemps] start of pair k's table in swap_thr
    const int32_t *swap_len;  // [kMaxTemps] entries of pair k (beyond: threshold 0)
    const int32_t *swap_sgn;  // [kMaxTemps] sign of beta_k - beta_{k+1}
    const uint32_t *sites;    // [N] packed x | y<<8 | z<<16, grouped by colour class
    uint32_t *sweep_ctr;      // sweeps done (next sweep index); advanced after each launch
    uint64_t *swap_acc;       // [ladders][kMaxTemps] accepted swaps per pair
    int32_t class_off[4];     // colour class c = sites[class_off[c] .. class_off[c+1])
    uint32_t key0, key1;      // Philox key
    int32_t L, N, n_T, NW;    // NW = words per site
    int32_t n_classes;
    int32_t words_resident;   // words held in LDS at once (== NW: load once per launch)
    int32_t n_sweeps;         // sweeps in this launch
    int32_t swap_every;       // 0 = no PT
    int32_t ladders;          // 2R
    int32_t block_threads;    // workgroup size this job was planned for
    int32_t swap_lds;         // swap-table entries copied to LDS (0: read from HBM)
    int32_t sites_lds;        // odd L: site list entries copied to LDS (0: read from HBM)
    float invL, invH;         // 1/L and 1/(L/2), exact quotients for indices < 2^15
    uint32_t seg_bits;        // 4: width of a 2E+S segment (a runtime value on purpose: a
                              // constant width lets the compiler split v_bfe_u32 into shift+mask)
    uint64_t *xchg;           // [ladders][2][kMaxTemps] (sweep index + 1) << 32 | slot energy, split workgroups
    uint32_t *error;          // set to non-zero if a split exchange timed out
    int32_t rng;              // EA_RNG_WORDS or EA_RNG_PLANES (CAMSC only)
    int32_t field_m;          // 4h (the field h is a multiple of 1/4); 0 without a field
    int32_t field_g;          // gcd(4, field_m): slot value W = (4U - m up) / g indexes the swap tables
    uint32_t always_add0;     // (8 - a_S) in every 4-bit segment: E + this >= 8 iff E >= a_S,
    uint32_t always_add1;     //   a_S = smallest E whose flip is certain for spin bit S
    int32_t always_col0;      // the same as a column 2E+S: certain iff 2E+S >= always_col[S]
    int32_t always_col1;
    int32_t site_order;       // LDS order of spin words and coupling bytes: 0 natural, 1 by colour class (even L)
    uint64_t *halo;           // [ladders][2 parts][2 classes][2 sides][L*L/2] (sweep index + 1) << 32 | spin word:
                              // boundary planes of a ladder split by lattice halves (NULL if never split so)
};

// Dynamic LDS carve-up of the sweep kernel, one definition for host and
// device.  The fixed-size tables come first so that every region is naturally
// aligned whatever N is (the 64-bit accept masks need 8-byte alignment).
struct LdsLayout {
    uint32_t thr;     // [kMaxTemps][kThrCols] u32 threshold rows by slot
    uint32_t fthr;    // [kMaxTemps][kThrCols] u32 threshold rows by temperature
    uint32_t U;       // [kMaxTemps] i32 unsatisfied bonds per slot
    uint32_t perm;    // [kMaxTemps] i32 temp_of_slot
    uint32_t sot;     // [kMaxTemps] i32 slot_of_temp
    uint32_t draw;    // [kMaxTemps] u32 swap draws
    uint32_t soff;    // [kMaxTemps] i32 swap table offsets
    uint32_t slen;    // [kMaxTemps] i32 swap table lengths
    uint32_t ssgn;    // [kMaxTemps] i32 sign of beta_k - beta_{k+1}
    uint32_t acc;     // [kMaxTemps] u32 accepted swaps of this unit
    uint32_t mask;    // [kMaxTemps] u64 speculative accept bits
    uint32_t ptab;    // [2 words][3 E][32 planes] u32 bit-sliced thresholds by slot (EA_RNG_PLANES)
    uint32_t up;      // [kMaxTemps] i32 spins up per slot (with a field)
    uint32_t items;   // [kMaxWaves][3][kItemCap] u32 halves still undecided after 8 planes (plane draws)
    uint32_t spin;    // [words][N] u32 spin words
    uint32_t stab;    // [swap_entries] u32 swap tables (optional)
    uint32_t sites;   // [site_entries] u32 packed coordinates (optional)
    uint32_t j6;      // [N] u8 coupling bits
    uint32_t total;
};

// Plane draws: every wave keeps up to kItemCap 16-slot halves that 8 planes
// left undecided, as three u32 fields each, and finishes them 64 at a time
// once more than kItemFlush wait (kItemFlush + 64 <= kItemCap).
constexpr int kItemCap = 96;
constexpr int kItemFlush = 32;
constexpr uint32_t kPlaneItemBytes = (uint32_t)kMaxWaves * 3u * (uint32_t)kItemCap * 4u;

__host__ __device__ inline LdsLayout lds_layout(int N, int words, int swap_entries, int site_entries,
                                                uint32_t item_bytes = 0)
{
    LdsLayout l;
    l.thr = 0;
    l.fthr = l.thr + kMaxTemps * kThrCols * 4;
    l.U = l.fthr + kMaxTemps * kThrCols * 4;
    l.perm = l.U + kMaxTemps * 4;
    l.sot = l.perm + kMaxTemps * 4;
    l.draw = l.sot + kMaxTemps * 4;
    l.soff = l.draw + kMaxTemps * 4;
    l.slen = l.soff + kMaxTemps * 4;
    l.ssgn = l.slen + kMaxTemps * 4;
    l.acc = l.ssgn + kMaxTemps * 4;
    l.mask = l.acc + kMaxTemps * 4;
    l.ptab = l.mask + kMaxTemps * 8;
    l.up = l.ptab + 2 * 3 * 32 * 4;
    l.items = l.up + kMaxTemps * 4;
    l.spin = l.items + item_bytes;
    l.stab = l.spin + (uint32_t)words * (uint32_t)N * 4u;
    l.sites = l.stab + (uint32_t)swap_entries * 4u;
    l.j6 = l.sites + (uint32_t)site_entries * 4u;
    l.total = l.j6 + ((uint32_t)N + 15u) / 16u * 16u;
    return l;
}

// Host-side launchers (ea_kernels.hip).  Each returns the first HIP error.
hipError_t launch_init_spins(const JobDesc *d_job, const JobDesc &h_job, int layout, hipStream_t s);
// Sweep kernel variant: 0 CAMSC, 1 AMSC4, 2 CAMSC with plane draws, 3 AMSC3, 4 AMSC1;
// kSlabVariant / kSlabPlanesVariant: CAMSC word / plane draws with ladders split by
// lattice halves (launches only).
inline int kernel_variant(int layout, int rng)
{
    return layout == 0 ? (rng ? 2 : 0) : (layout == 1 ? 1 : (layout == 2 ? 3 : 4));
}
constexpr int kSlabVariant = 5;
constexpr int kSlabPlanesVariant = 6;
// One sweep launch over n_units ladders (units[k] = job << 20 | ladder), then
// the sweep counters advance and the queue words are re-armed.  parts = 1:
// persistent workgroups pull ladders from queue[0]; parts = 2 or 4 (CAMSC
// jobs with one word per site and even L): `parts` workgroups per ladder,
// tickets from queue[blockIdx % 8], grid = split_grid(n_units, parts).
// sep = 1: spin words in LDS by colour class (one CAMSC job only).
hipError_t launch_sweep(const JobDesc *d_jobs, int n_jobs, const uint32_t *d_units, int n_units,
                        uint32_t *d_queue, int kv, int parts, int sep, int block_threads, size_t lds, int grid,
                        hipStream_t s);
// Workgroups of a split launch: every queue gets as many as its ladders have parts.
inline int split_grid(int n_units, int parts) { return (n_units + 7) / 8 * 8 * parts; }
hipError_t launch_observables(const JobDesc *d_job, const JobDesc &h_job, int layout, int32_t *d_energy,
                              int32_t *d_overlap, int32_t *d_magnet, hipStream_t s);
hipError_t launch_unpack(const JobDesc *d_job, const JobDesc &h_job, int layout, int8_t *d_spins, hipStream_t s);
hipError_t launch_measure(const JobDesc *d_job, const JobDesc &h_job, int layout, int64_t *count, int64_t *sum_q2,
                          uint64_t *sum_q4, int64_t *sum_c, hipStream_t s);
hipError_t launch_pack(const JobDesc *d_job, const JobDesc &h_job, int layout, const int8_t *d_spins, hipStream_t s);
hipError_t sweep_set_lds(int kv, int parts, size_t lds);
int sweep_max_blocks_per_cu(int kv, int parts, int block_threads, size_t lds);

// Static workspace of the allocation-free batch launch (ea_sweep_batch_noalloc):
// work-queue counter, job descriptors and unit list of one launch, at fixed
// offsets.  One copy per device, held until the process ends.
constexpr int kNoallocMaxJobs = 256;
constexpr int kNoallocMaxUnits = 1 << 18;
constexpr size_t kNoallocQueueOff = 0;
constexpr size_t kNoallocDescOff = 256;
constexpr size_t kNoallocUnitOff = (kNoallocDescOff + kNoallocMaxJobs * sizeof(JobDesc) + 255) / 256 * 256;
constexpr size_t kNoallocBytes = kNoallocUnitOff + (size_t)kNoallocMaxUnits * 4;
// Device address of the workspace on the current device (looked up once per device).
hipError_t noalloc_workspace(void **ptr);

}  // namespace ea
