// HIP kernels for gfx950: parallel-tempering Metropolis sweeps of the 3D
// +-J Edwards-Anderson model over multispin-coded temperature replicas
// (Fang et al., arXiv:1311.5582).
//
// Work mapping (Sec. 3): one workgroup owns one ladder (a realization's copy
// with all its temperature slots) at a time, pulled from a device work queue;
// the lattice sites of one colour class are spread over the workgroup's
// threads (Sec. 3.1); the temperature slots are the bits of a word (Sec. 3.2,
// 4.3.3).  The ladder's spin words stay in LDS across all sweeps of a launch
// (Sec. 4.2.2 "integer cube" in the scratchpad); when they do not fit, word
// groups are staged through HBM once per swap interval, which is legal because
// different slots never interact between swap points.
//
// Per site and word (Sec. 4.3, Eq. e and the look-up table of Sec. 4.3.1):
//   e_d   = S xor S_nbr(d) xor Jmask_d            for the six incidences d
//   E     = sum_d e_d, widened to 4-bit segments (CAMSC) or native (AMSC4)
//   col   = 2E + S per slot, the table column; the row is the slot's current
//           temperature, rebuilt when PT exchanges temperatures
//   flip  = (E >= 3) or draw < thr[slot][col], draw = Philox4x32-10 output
//           compared as a raw 32-bit integer (Sec. 4.3.2)
// After every swap_every-th sweep the unsatisfied-bond count U of every slot
// is reduced (bit-plane counters + wave ballots) and the ascending swap pass
// is evaluated: all acceptance bits that the sequential pass could need are
// computed in parallel, then one lane walks the pairs in order.
#include "ea_internal.h"

namespace ea {

namespace {

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);   // truth table of a ^ b ^ c
}

// Philox4x32-10 block.  In the sweep, counter words 1..3 are uniform across
// the wavefront (sweep, realization, slot group) and only word 0 (the site)
// varies, so the first rounds are left as plain xors for the compiler to
// evaluate on the scalar unit and share between slot groups; from the fourth
// round on every operand is per-lane and the two xors fuse into one bitop3.
__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < kPhiloxRounds; ++round) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)c2;
        uint32_t n0, n2;
        if (round < 3) {
            n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        } else {
            n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
            n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        }
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return {c0, c1, c2, c3};
}

// 4-bit field of a segment word, as a plain v_bfe_u32 (kept out of the
// compiler's shift/mask canonicalisation so that the scaled LDS address is
// one v_lshl_add_u32 away).
__device__ __forceinline__ uint32_t field4(uint32_t x, int shift)
{
    uint32_t r;
    asm("v_bfe_u32 %0, %1, %2, 4" : "=v"(r) : "v"(x), "i"(shift));
    return r;
}

// Site index and the six neighbour indices (periodic) from packed coordinates.
struct Nbrs {
    int i, xp, xm, yp, ym, zp, zm;
};

__device__ __forceinline__ Nbrs neighbours(uint32_t xyz, int L)
{
    const int x = xyz & 0xFF, y = (xyz >> 8) & 0xFF, z = xyz >> 16;
    const int LL = L * L;
    Nbrs n;
    n.i = x + L * y + LL * z;
    n.xp = (x == L - 1) ? n.i - (L - 1) : n.i + 1;
    n.xm = (x == 0) ? n.i + (L - 1) : n.i - 1;
    n.yp = (y == L - 1) ? n.i - (L - 1) * L : n.i + L;
    n.ym = (y == 0) ? n.i + (L - 1) * L : n.i - L;
    n.zp = (z == L - 1) ? n.i - (L - 1) * LL : n.i + LL;
    n.zm = (z == 0) ? n.i + (L - 1) * LL : n.i - LL;
    return n;
}

// LDS regions of the sweep kernel (offsets from lds_layout()).
struct Smem {
    uint32_t *spin;   // [words_resident][N]
    uint8_t *j6;      // [N]
    uint32_t *thr;    // [kMaxTemps][kThrCols] rows by slot
    int32_t *U;       // [kMaxTemps]
    int32_t *perm;    // temp_of_slot
    int32_t *sot;     // slot_of_temp
    uint32_t *draw;   // swap draws per pair
    uint64_t *mask;   // speculative accept bits per pair
};

__device__ __forceinline__ Smem carve(uint8_t *base, int N, int words)
{
    const LdsLayout l = lds_layout(N, words);
    Smem s;
    s.thr = (uint32_t *)(base + l.thr);
    s.U = (int32_t *)(base + l.U);
    s.perm = (int32_t *)(base + l.perm);
    s.sot = (int32_t *)(base + l.sot);
    s.draw = (uint32_t *)(base + l.draw);
    s.mask = (uint64_t *)(base + l.mask);
    s.spin = (uint32_t *)(base + l.spin);
    s.j6 = base + l.j6;
    return s;
}

// ---------------------------------------------------------------------------
// Metropolis decisions for one word.  NG = number of 4-slot groups (Philox
// blocks) the word holds; a compile-time NG keeps all blocks in one basic
// block so their independent chains interleave.
// ---------------------------------------------------------------------------
struct Ctr {
    uint32_t t, r, c3, k0, k1;   // sweep, realization, domain|copy|group base, key
};

// CAMSC: X[k] holds 2E+S of slot 4j+k in segment j.  Returns the flip bits of
// the 4*NG slots, bit s = slot s of the word.
template <int NG>
__device__ __forceinline__ uint32_t camsc_decide(const uint32_t X[4], const uint32_t *rows, uint32_t site,
                                                 const Ctr &c)
{
    uint32_t F = 0;
#pragma unroll
    for (int g = NG - 1; g >= 0; --g) {
        const U4 rr = philox10(site, c.t, c.r, c.c3 | (uint32_t)g, c.k0, c.k1);
        const uint32_t *row = rows + 4 * g * kThrCols;
        F = (F << 1) | (rr.w < row[3 * kThrCols + field4(X[3], 4 * g)] ? 1u : 0u);
        F = (F << 1) | (rr.z < row[2 * kThrCols + field4(X[2], 4 * g)] ? 1u : 0u);
        F = (F << 1) | (rr.y < row[1 * kThrCols + field4(X[1], 4 * g)] ? 1u : 0u);
        F = (F << 1) | (rr.x < row[0 * kThrCols + field4(X[0], 4 * g)] ? 1u : 0u);
    }
    return F;
}

// AMSC4: X holds 2E+S of slot j in segment j.  Flip bit of slot j at bit 4j.
template <int NG>
__device__ __forceinline__ uint32_t amsc4_decide(uint32_t X, const uint32_t *rows, uint32_t site, const Ctr &c)
{
    uint32_t F = 0;
#pragma unroll
    for (int g = NG - 1; g >= 0; --g) {
        const U4 rr = philox10(site, c.t, c.r, c.c3 | (uint32_t)g, c.k0, c.k1);
        const uint32_t *row = rows + 4 * g * kThrCols;
        F = (F << 4) | (rr.w < row[3 * kThrCols + field4(X, 16 * g + 12)] ? 1u : 0u);
        F = (F << 4) | (rr.z < row[2 * kThrCols + field4(X, 16 * g + 8)] ? 1u : 0u);
        F = (F << 4) | (rr.y < row[1 * kThrCols + field4(X, 16 * g + 4)] ? 1u : 0u);
        F = (F << 4) | (rr.x < row[0 * kThrCols + field4(X, 16 * g)] ? 1u : 0u);
    }
    return F;
}

// ---------------------------------------------------------------------------
// Metropolis update of one site for the `gw` resident words (word index g0..).
// ---------------------------------------------------------------------------
template <int LAYOUT>
__device__ __forceinline__ void update_site(const Smem &sm, const Nbrs &nb, int N, int gw, int g0, int n_T,
                                            uint32_t t, uint32_t r, uint32_t c3base, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M = 0x11111111u;
    const uint32_t j6 = sm.j6[nb.i];
    // all-ones mask for an antiferromagnetic incidence ("multiply the coupling
    // with a bit-mask to match the pattern of S", Sec. 4.3.3)
    uint32_t m[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) m[d] = 0u - ((j6 >> d) & 1u);
    if (LAYOUT == 1) {
#pragma unroll
        for (int d = 0; d < 6; ++d) m[d] &= M;
    }
    for (int w = 0; w < gw; ++w) {
        uint32_t *sw = sm.spin + (size_t)w * N;
        const uint32_t S = sw[nb.i];
        const uint32_t e0 = S ^ sw[nb.xp] ^ m[0];
        const uint32_t e1 = S ^ sw[nb.xm] ^ m[1];
        const uint32_t e2 = S ^ sw[nb.yp] ^ m[2];
        const uint32_t e3 = S ^ sw[nb.ym] ^ m[3];
        const uint32_t e4 = S ^ sw[nb.zp] ^ m[4];
        const uint32_t e5 = S ^ sw[nb.zm] ^ m[5];
        const int wg = __builtin_amdgcn_readfirstlane(g0 + w);
        if (LAYOUT == 0) {
            // CAMSC: widen each 1-bit bond word into four 4-bit-segment words
            // (segment j of word k holds slot 4j + k), sum, append S.
            uint32_t X[4];
            uint32_t always = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t E = ((e0 >> k) & M) + ((e1 >> k) & M) + ((e2 >> k) & M) + ((e3 >> k) & M) +
                                   ((e4 >> k) & M) + ((e5 >> k) & M);
                X[k] = (E << 1) | ((S >> k) & M);
                always |= (((X[k] + 0x22222222u) >> 3) & M) << k;   // 2E+S >= 6  <=>  E >= 3
            }
            const int slot0 = wg * 32;
            const int left = n_T - slot0;
            const int ngr = left >= 32 ? 8 : (left + 3) >> 2;
            const uint32_t valid = left >= 32 ? 0xFFFFFFFFu : ((1u << left) - 1u);
            const uint32_t *rows = sm.thr + slot0 * kThrCols;
            const Ctr c{t, r, c3base | (uint32_t)(wg * 8), k0, k1};
            uint32_t F;
            switch (ngr) {
                case 8: F = camsc_decide<8>(X, rows, nb.i, c); break;
                case 7: F = camsc_decide<7>(X, rows, nb.i, c); break;
                case 6: F = camsc_decide<6>(X, rows, nb.i, c); break;
                case 5: F = camsc_decide<5>(X, rows, nb.i, c); break;
                case 4: F = camsc_decide<4>(X, rows, nb.i, c); break;
                case 3: F = camsc_decide<3>(X, rows, nb.i, c); break;
                case 2: F = camsc_decide<2>(X, rows, nb.i, c); break;
                default: F = camsc_decide<1>(X, rows, nb.i, c); break;
            }
            sw[nb.i] = S ^ ((F | always) & valid);
        } else {
            // AMSC4: 4-bit segments throughout; 2E+S is formed for all slots at once.
            const uint32_t E = e0 + e1 + e2 + e3 + e4 + e5;
            const uint32_t X = (E << 1) | S;
            const uint32_t always = ((X + 0x22222222u) >> 3) & M;
            const int slot0 = wg * 8;
            const int left = n_T - slot0;
            const uint32_t valid = left >= 8 ? M : (M & ((1u << (4 * left)) - 1u));
            const uint32_t *rows = sm.thr + slot0 * kThrCols;
            const Ctr c{t, r, c3base | (uint32_t)(wg * 2), k0, k1};
            const uint32_t F = left > 4 ? amsc4_decide<2>(X, rows, nb.i, c) : amsc4_decide<1>(X, rows, nb.i, c);
            sw[nb.i] = S ^ ((F | always) & valid);
        }
    }
}

// ---------------------------------------------------------------------------
// Unsatisfied-bond counts per slot for one word (forward bonds of every site),
// added into U[slot0 + b].  Each lane keeps vertical bit-plane counters; the
// planes are reduced across the wave with ballot + popcount.
// ---------------------------------------------------------------------------
template <int LAYOUT>
__device__ void count_unsat_word(const uint32_t *words, const uint8_t *j6, const uint32_t *sites, int N, int L,
                                 int slot0, int n_T, int np, int *U)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr int STR = Layout<LAYOUT>::kStride;
    const uint32_t keep = LAYOUT == 0 ? 0xFFFFFFFFu : 0x11111111u;
    uint32_t P[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int idx = threadIdx.x; idx < N; idx += blockDim.x) {
        const Nbrs nb = neighbours(sites[idx], L);
        const uint32_t S = words[nb.i];
        const uint32_t jb = j6[nb.i];
        const uint32_t ex = S ^ words[nb.xp] ^ ((0u - (jb & 1u)) & keep);
        const uint32_t ey = S ^ words[nb.yp] ^ ((0u - ((jb >> 2) & 1u)) & keep);
        const uint32_t ez = S ^ words[nb.zp] ^ ((0u - ((jb >> 4) & 1u)) & keep);
        // full adder: ex + ey + ez = 2c + s
        const uint32_t s = ex ^ ey ^ ez;
        const uint32_t c = (ex & ey) | (ez & (ex ^ ey));
        uint32_t carry = P[0] & s;
        P[0] ^= s;
        const uint32_t t1 = P[1] ^ c;
        uint32_t c2 = (P[1] & c) | (carry & t1);
        P[1] = t1 ^ carry;
#pragma unroll
        for (int p = 2; p < 8; ++p) {
            if (p < np) {
                const uint32_t tt = P[p] & c2;
                P[p] ^= c2;
                c2 = tt;
            }
        }
    }
    const int lane = threadIdx.x & 63;
    const int nslots = min(SPW, n_T - slot0);
    for (int b = 0; b < nslots; ++b) {
        int cnt = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            if (p < np) cnt += __popcll(__ballot((P[p] >> (b * STR)) & 1u)) << p;
        }
        if (lane == 0 && cnt) atomicAdd(&U[slot0 + b], cnt);
    }
}

// Bit planes needed so that no lane's per-slot count overflows.
__device__ __forceinline__ int planes_for(int N, int nthr)
{
    const int per_lane = 3 * ((N + nthr - 1) / nthr);
    int np = 2;
    while ((1 << np) <= per_lane) ++np;
    return np;
}

// ---------------------------------------------------------------------------
// Sweep kernel: persistent workgroups pulling ladders from a queue.
// ---------------------------------------------------------------------------
template <int LAYOUT>
__global__ void __launch_bounds__(kMaxBlock) sweep_kernel(const JobDesc *__restrict__ jobs,
                                                          const uint32_t *__restrict__ units, int n_units,
                                                          uint32_t *queue)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    extern __shared__ __align__(16) uint8_t smem_raw[];
    __shared__ uint32_t s_next;
    __shared__ int32_t s_fin[kMaxTemps];
    __shared__ uint32_t s_acc[kMaxTemps];

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;

    for (;;) {
        if (tid == 0) s_next = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t u = __builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
        if (u >= (uint32_t)n_units) break;
        const uint32_t unit = units[u];
        const JobDesc &jd = jobs[unit >> 20];
        const int ladder = unit & 0xFFFFF;
        const int N = jd.N, L = jd.L, NW = jd.NW, WR = jd.words_resident, n_T = jd.n_T;
        const int n_classes = jd.n_classes;
        const uint32_t r = (uint32_t)(ladder >> 1);
        const uint32_t copy = (uint32_t)(ladder & 1);
        const uint32_t c3flip = (kDomainFlip << 28) | (copy << 24);
        const uint32_t k0 = jd.key0, k1 = jd.key1;
        const Smem sm = carve(smem_raw, N, WR);
        uint32_t *g_spin = jd.spins + (size_t)ladder * NW * N;

        // couplings, permutation and threshold rows of this ladder
        const uint8_t *g_j6 = jd.j6 + (size_t)r * N;
        for (int idx = tid; idx < N; idx += nthr) sm.j6[idx] = g_j6[idx];
        if (tid < kMaxTemps) {
            sm.perm[tid] = tid < n_T ? jd.temp_of_slot[ladder * kMaxTemps + tid] : 0;
            s_acc[tid] = 0;
        }
        __syncthreads();
        if (tid < n_T) sm.sot[sm.perm[tid]] = tid;
        for (int idx = tid; idx < kMaxTemps * kThrCols; idx += nthr) {
            const int slot = idx / kThrCols;
            sm.thr[idx] = slot < n_T ? jd.flip_thr[sm.perm[slot] * kThrCols + (idx % kThrCols)] : 0u;
        }
        const int n_groups = (NW + WR - 1) / WR;
        if (n_groups == 1)
            for (int idx = tid; idx < NW * N; idx += nthr) sm.spin[idx] = g_spin[idx];
        __syncthreads();

        uint32_t t = __builtin_amdgcn_readfirstlane(*jd.sweep_ctr);
        int remaining = jd.n_sweeps;
        const int se = jd.swap_every;
        const int np = planes_for(N, nthr);
        while (remaining > 0) {
            int chunk = remaining;
            bool swap_now = false;
            if (se > 0) {
                const int to_swap = se - (int)(t % (uint32_t)se);
                if (to_swap <= remaining) {
                    chunk = to_swap;
                    swap_now = true;
                }
            }
            if (swap_now) {
                if (tid < kMaxTemps) sm.U[tid] = 0;
                __syncthreads();
            }
            for (int g0 = 0; g0 < NW; g0 += WR) {
                const int gw = min(WR, NW - g0);
                if (n_groups > 1) {
                    for (int idx = tid; idx < gw * N; idx += nthr) sm.spin[idx] = g_spin[(size_t)g0 * N + idx];
                    __syncthreads();
                }
                for (int s = 0; s < chunk; ++s) {
                    const uint32_t ts = t + (uint32_t)s;
                    for (int c = 0; c < n_classes; ++c) {
                        const int end = jd.class_off[c + 1];
                        for (int it = jd.class_off[c] + tid; it < end; it += nthr) {
                            const Nbrs nb = neighbours(jd.sites[it], L);
                            update_site<LAYOUT>(sm, nb, N, gw, g0, n_T, ts, r, c3flip, k0, k1);
                        }
                        __syncthreads();
                    }
                }
                if (swap_now) {
                    for (int w = 0; w < gw; ++w)
                        count_unsat_word<LAYOUT>(sm.spin + (size_t)w * N, sm.j6, jd.sites, N, L, (g0 + w) * SPW,
                                                 n_T, np, sm.U);
                }
                if (n_groups > 1) {
                    __syncthreads();
                    for (int idx = tid; idx < gw * N; idx += nthr) g_spin[(size_t)g0 * N + idx] = sm.spin[idx];
                }
            }
            if (swap_now && n_T > 1) {
                // ---- replica-exchange pass after sweep t + chunk - 1 ----
                const uint32_t tswap = t + (uint32_t)chunk - 1u;
                const int pairs = n_T - 1;
                if (tid < pairs)
                    sm.draw[tid] = philox10((uint32_t)tid, tswap, r, (kDomainSwap << 28) | (copy << 24), k0, k1).x;
                if (tid < kMaxTemps) sm.mask[tid] = 0;
                __syncthreads();
                // acceptance of "configuration now at position j reaches pair k"
                for (int p = tid; p < pairs * 64; p += nthr) {
                    const int k = p >> 6, j = p & 63;
                    if (j > k) continue;
                    const int d = sm.U[sm.sot[j]] - sm.U[sm.sot[k + 1]];
                    const int sg = jd.swap_sgn[k];
                    bool acc = (sg == 0) || (d == 0) || ((sg > 0) == (d > 0));
                    if (!acc) {
                        const int n = d < 0 ? -d : d;
                        const uint32_t thr = n < jd.swap_len[k] ? jd.swap_thr[jd.swap_off[k] + n] : 0u;
                        acc = sm.draw[k] < thr;
                    }
                    if (acc) atomicOr((unsigned long long *)&sm.mask[k], 1ull << j);
                }
                __syncthreads();
                if (tid == 0) {
                    int cj = 0;   // position (in the old order) of the configuration carried upwards
                    for (int k = 0; k < pairs; ++k) {
                        if ((sm.mask[k] >> cj) & 1ull) {
                            s_fin[k] = sm.sot[k + 1];
                            s_acc[k] += 1;
                        } else {
                            s_fin[k] = sm.sot[cj];
                            cj = k + 1;
                        }
                    }
                    s_fin[pairs] = sm.sot[cj];
                }
                __syncthreads();
                if (tid < n_T) {
                    sm.sot[tid] = s_fin[tid];
                    sm.perm[s_fin[tid]] = tid;
                }
                __syncthreads();
                for (int idx = tid; idx < kMaxTemps * kThrCols; idx += nthr) {
                    const int slot = idx / kThrCols;
                    sm.thr[idx] = slot < n_T ? jd.flip_thr[sm.perm[slot] * kThrCols + (idx % kThrCols)] : 0u;
                }
                __syncthreads();
            }
            t += (uint32_t)chunk;
            remaining -= chunk;
        }
        if (n_groups == 1)
            for (int idx = tid; idx < NW * N; idx += nthr) g_spin[idx] = sm.spin[idx];
        if (tid < n_T) {
            jd.temp_of_slot[ladder * kMaxTemps + tid] = sm.perm[tid];
            if (tid < n_T - 1) jd.swap_acc[ladder * kMaxTemps + tid] += s_acc[tid];
        }
        __syncthreads();
    }
}

// Advance each job's sweep counter and re-arm the queue for the next launch.
__global__ void advance_kernel(const JobDesc *__restrict__ jobs, int n_jobs, uint32_t *queue)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_jobs) *jobs[j].sweep_ctr += (uint32_t)jobs[j].n_sweeps;
    if (j == 0) *queue = 0;
}

// ---------------------------------------------------------------------------
// Initial spins from the initial-spin stream.
// ---------------------------------------------------------------------------
template <int LAYOUT>
__global__ void init_spins_kernel(const JobDesc *__restrict__ jd_ptr)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr int STR = Layout<LAYOUT>::kStride;
    const JobDesc &jd = *jd_ptr;
    const size_t total = (size_t)jd.ladders * jd.NW * jd.N;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % jd.N);
        const int w = (int)((idx / jd.N) % jd.NW);
        const int ladder = (int)(idx / ((size_t)jd.N * jd.NW));
        const uint32_t c3 = (kDomainInit << 28) | ((uint32_t)(ladder & 1) << 24);
        uint32_t word = 0;
        for (int g = 0; g < SPW / 4; ++g) {
            const int slot = w * SPW + 4 * g;
            if (slot >= jd.n_T) break;
            const U4 rr = philox10((uint32_t)i, 0u, (uint32_t)(ladder >> 1), c3 | (uint32_t)(slot >> 2), jd.key0, jd.key1);
            const uint32_t v[4] = {rr.x, rr.y, rr.z, rr.w};
            for (int k = 0; k < 4 && slot + k < jd.n_T; ++k) word |= (v[k] & 1u) << ((4 * g + k) * STR);
        }
        jd.spins[idx] = word;
    }
}

// ---------------------------------------------------------------------------
// Measurement kernel (Sec. 4.1): one workgroup per realization.
// ---------------------------------------------------------------------------
template <int LAYOUT>
__global__ void __launch_bounds__(512) observables_kernel(const JobDesc *__restrict__ jd_ptr, int32_t *energy,
                                                          int32_t *overlap)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr int STR = Layout<LAYOUT>::kStride;
    __shared__ int s_U[2][kMaxTemps];
    __shared__ int s_diff[kMaxTemps];
    __shared__ int s_sot[2][kMaxTemps];
    const JobDesc &jd = *jd_ptr;
    const int r = blockIdx.x;
    const int N = jd.N, n_T = jd.n_T, NW = jd.NW;
    const int tid = threadIdx.x;
    if (tid < kMaxTemps) {
        s_U[0][tid] = s_U[1][tid] = 0;
        s_diff[tid] = 0;
    }
    __syncthreads();
    if (tid < 2 * n_T) {
        const int c = tid / n_T, s = tid % n_T;
        s_sot[c][jd.temp_of_slot[(2 * r + c) * kMaxTemps + s]] = s;
    }
    __syncthreads();
    const int np = planes_for(N, blockDim.x);
    const uint8_t *j6 = jd.j6 + (size_t)r * N;
    for (int c = 0; c < 2; ++c)
        for (int w = 0; w < NW; ++w)
            count_unsat_word<LAYOUT>(jd.spins + ((size_t)(2 * r + c) * NW + w) * N, j6, jd.sites, N, jd.L, w * SPW,
                                     n_T, np, s_U[c]);
    // overlap between the copies at equal temperature index
    const uint32_t *s0 = jd.spins + (size_t)(2 * r) * NW * N;
    const uint32_t *s1 = jd.spins + (size_t)(2 * r + 1) * NW * N;
    for (int k = 0; k < n_T; ++k) {
        const int a = s_sot[0][k], b = s_sot[1][k];
        const uint32_t *wa = s0 + (size_t)(a / SPW) * N;
        const uint32_t *wb = s1 + (size_t)(b / SPW) * N;
        const int sa = (a % SPW) * STR, sb = (b % SPW) * STR;
        int diff = 0;
        for (int i = tid; i < N; i += blockDim.x) diff += ((wa[i] >> sa) ^ (wb[i] >> sb)) & 1u;
        for (int off = 32; off > 0; off >>= 1) diff += __shfl_down(diff, off, 64);
        if ((tid & 63) == 0) atomicAdd(&s_diff[k], diff);
    }
    __syncthreads();
    if (tid < 2 * n_T) {
        const int c = tid / n_T, k = tid % n_T;
        if (energy) energy[((size_t)r * 2 + c) * n_T + k] = 2 * s_U[c][s_sot[c][k]] - 3 * N;
    }
    if (tid < n_T && overlap) overlap[(size_t)r * n_T + tid] = N - 2 * s_diff[tid];
}

// ---------------------------------------------------------------------------
// Pack / unpack between words and one int8 spin per (ladder, slot, site).
// ---------------------------------------------------------------------------
template <int LAYOUT>
__global__ void unpack_kernel(const JobDesc *__restrict__ jd_ptr, int8_t *out)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr int STR = Layout<LAYOUT>::kStride;
    const JobDesc &jd = *jd_ptr;
    const size_t total = (size_t)jd.ladders * jd.n_T * jd.N;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % jd.N);
        const int slot = (int)((idx / jd.N) % jd.n_T);
        const size_t ladder = idx / ((size_t)jd.N * jd.n_T);
        const uint32_t word = jd.spins[(ladder * jd.NW + slot / SPW) * jd.N + i];
        out[idx] = ((word >> ((slot % SPW) * STR)) & 1u) ? (int8_t)1 : (int8_t)-1;
    }
}

template <int LAYOUT>
__global__ void pack_kernel(const JobDesc *__restrict__ jd_ptr, const int8_t *in)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr int STR = Layout<LAYOUT>::kStride;
    const JobDesc &jd = *jd_ptr;
    const size_t total = (size_t)jd.ladders * jd.NW * jd.N;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % jd.N);
        const int w = (int)((idx / jd.N) % jd.NW);
        const size_t ladder = idx / ((size_t)jd.N * jd.NW);
        uint32_t word = 0;
        for (int j = 0; j < SPW; ++j) {
            const int slot = w * SPW + j;
            if (slot >= jd.n_T) break;
            if (in[(ladder * jd.n_T + slot) * jd.N + i] > 0) word |= 1u << (j * STR);
        }
        jd.spins[idx] = word;
    }
}

int grid_for(size_t total, int block)
{
    const size_t g = (total + block - 1) / block;
    return (int)(g < 65536 ? (g ? g : 1) : 65536);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_init_spins(const JobDesc *d_job, const JobDesc &h, int layout, hipStream_t s)
{
    const size_t total = (size_t)h.ladders * h.NW * h.N;
    if (layout == 0)
        hipLaunchKernelGGL(init_spins_kernel<0>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job);
    else
        hipLaunchKernelGGL(init_spins_kernel<1>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job);
    return hipGetLastError();
}

hipError_t launch_sweep(const JobDesc *d_jobs, int n_jobs, const uint32_t *d_units, int n_units, uint32_t *d_queue,
                        int layout, int block_threads, size_t lds, int grid, hipStream_t s)
{
    if (layout == 0) {
        hipError_t e = hipFuncSetAttribute((const void *)sweep_kernel<0>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(sweep_kernel<0>, dim3(grid), dim3(block_threads), lds, s, d_jobs, d_units, n_units,
                           d_queue);
    } else {
        hipError_t e = hipFuncSetAttribute((const void *)sweep_kernel<1>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(sweep_kernel<1>, dim3(grid), dim3(block_threads), lds, s, d_jobs, d_units, n_units,
                           d_queue);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(advance_kernel, dim3((n_jobs + 255) / 256), dim3(256), 0, s, d_jobs, n_jobs, d_queue);
    return hipGetLastError();
}

hipError_t launch_observables(const JobDesc *d_job, const JobDesc &h, int layout, int32_t *d_energy,
                              int32_t *d_overlap, hipStream_t s)
{
    const int R = h.ladders / 2;
    if (layout == 0)
        hipLaunchKernelGGL(observables_kernel<0>, dim3(R), dim3(512), 0, s, d_job, d_energy, d_overlap);
    else
        hipLaunchKernelGGL(observables_kernel<1>, dim3(R), dim3(512), 0, s, d_job, d_energy, d_overlap);
    return hipGetLastError();
}

hipError_t launch_unpack(const JobDesc *d_job, const JobDesc &h, int layout, int8_t *d_spins, hipStream_t s)
{
    const size_t total = (size_t)h.ladders * h.n_T * h.N;
    if (layout == 0)
        hipLaunchKernelGGL(unpack_kernel<0>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins);
    else
        hipLaunchKernelGGL(unpack_kernel<1>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins);
    return hipGetLastError();
}

hipError_t launch_pack(const JobDesc *d_job, const JobDesc &h, int layout, const int8_t *d_spins, hipStream_t s)
{
    const size_t total = (size_t)h.ladders * h.NW * h.N;
    if (layout == 0)
        hipLaunchKernelGGL(pack_kernel<0>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins);
    else
        hipLaunchKernelGGL(pack_kernel<1>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins);
    return hipGetLastError();
}

int sweep_max_blocks_per_cu(int layout, int block_threads, size_t lds)
{
    int n = 0;
    hipError_t e;
    if (layout == 0)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_kernel<0>, block_threads, lds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_kernel<1>, block_threads, lds);
    return e == hipSuccess ? n : 0;
}

}  // namespace ea
