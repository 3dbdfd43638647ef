// HIP kernels for gfx950: parallel-tempering Metropolis sweeps of the 3D
// +-J Edwards-Anderson model over multispin-coded temperature replicas
// (Fang et al., arXiv:1311.5582).
//
// Work mapping (Sec. 3): one workgroup owns one ladder (a realization's copy
// with all its temperature slots) at a time, pulled from a device work queue;
// the lattice sites of one colour class are spread over the workgroup's
// threads (Sec. 3.1); the temperature slots are the bits of a word (Sec. 3.2,
// 4.3.3).  The ladder's spin words stay in LDS across all sweeps of a launch
// (the block-resident integer array of Sec. 4.2.2); when they do not fit, word
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
#include <atomic>

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

// Segment field of a 2E+S word: v_bfe_u32 with the width in a register.
__device__ __forceinline__ uint32_t field4(uint32_t x, int shift, uint32_t width)
{
    return __builtin_amdgcn_ubfe(x, (uint32_t)shift, width);
}

// A site's LDS word index, its six neighbours' LDS word indices (periodic),
// and its natural index g = x + L(y + Lz), which keys the random stream.  In
// the natural order the LDS index is g.
struct Nbrs {
    int i, xp, xm, yp, ym, zp, zm;
    int g;
};

__device__ __forceinline__ Nbrs neighbours(int x, int y, int z, int L)
{
    const int LL = L * L;
    Nbrs n;
    n.i = x + L * y + LL * z;
    n.g = n.i;
    n.xp = (x == L - 1) ? n.i - (L - 1) : n.i + 1;
    n.xm = (x == 0) ? n.i + (L - 1) : n.i - 1;
    n.yp = (y == L - 1) ? n.i - (L - 1) * L : n.i + L;
    n.ym = (y == 0) ? n.i + (L - 1) * L : n.i - L;
    n.zp = (z == L - 1) ? n.i - (L - 1) * LL : n.i + LL;
    n.zm = (z == 0) ? n.i + (L - 1) * LL : n.i - LL;
    return n;
}

__device__ __forceinline__ Nbrs neighbours_packed(uint32_t xyz, int L)
{
    return neighbours(xyz & 0xFF, (xyz >> 8) & 0xFF, xyz >> 16, L);
}

// floor(j / d) for 0 <= j < 2^15 and d <= 32 given inv = 1.0f / d: the
// float product of j + 1/2 and inv lands strictly inside (q, q + 1).
__device__ __forceinline__ int qdiv(int j, float inv)
{
    return (int)(((float)j + 0.5f) * inv);
}

// Item j of checkerboard class c (even L): rows (y, z) hold L/2 class sites
// at x = 2 xh + ((c + y + z) & 1).
__device__ __forceinline__ Nbrs checker_site(int j, int c, int L, float invH, float invL)
{
    const int w = qdiv(j, invH);
    const int xh = j - w * (L >> 1);
    const int z = qdiv(w, invL);
    const int y = w - z * L;
    return neighbours(2 * xh + ((c + y + z) & 1), y, z, L);
}

__device__ __forceinline__ Nbrs natural_site(int i, int L, float invL)
{
    const int w = qdiv(i, invL);
    const int z = qdiv(w, invL);
    return neighbours(i - w * L, w - z * L, z, L);
}

// Natural index of item j of checkerboard class c (even L).
__device__ __forceinline__ int checker_index(int j, int c, int L, float invH, float invL)
{
    const int w = qdiv(j, invH);
    const int xh = j - w * (L >> 1);
    const int z = qdiv(w, invL);
    const int y = w - z * L;
    return 2 * xh + ((c + y + z) & 1) + L * w;
}

// LDS order of the spin words and coupling bytes of an even lattice:
// natural (sep = 0: word g at g), or by colour class (sep = 1: class c in words
// c N/2 .. c N/2 + N/2 - 1, the class-c site g at c N/2 + g / 2, which is its
// position j in checker_site's enumeration).  By class, the sites that
// consecutive threads update are consecutive words, and so are their
// neighbours along x.
struct Order {
    int sep, nh;   // nh = N / 2
    int base;      // natural order: the LDS word of site g is g - base (0 but in a split by lattice halves)
};

// Item j of class c with LDS indices in order SEP.
template <int SEP>
__device__ __forceinline__ Nbrs class_site(const Order &o, int j, int c, int L, float invH, float invL)
{
    Nbrs n = checker_site(j, c, L, invH, invL);
    if (SEP) {
        const int other = (1 - c) * o.nh;
        n.i = c * o.nh + j;
        n.xp = other + (n.xp >> 1);
        n.xm = other + (n.xm >> 1);
        n.yp = other + (n.yp >> 1);
        n.ym = other + (n.ym >> 1);
        n.zp = other + (n.zp >> 1);
        n.zm = other + (n.zm >> 1);
    }
    return n;
}


// Natural index of LDS word k.
__device__ __forceinline__ int natural_of(const Order &o, int k, int L, float invH, float invL)
{
    if (!o.sep) return k;
    const int c = k >= o.nh ? 1 : 0;
    return checker_index(k - c * o.nh, c, L, invH, invL);
}

// Site of LDS word k with LDS indices (any order; for whole-lattice passes).
__device__ __forceinline__ Nbrs lds_site(const Order &o, int k, int L, float invH, float invL)
{
    if (!o.sep) return natural_site(k, L, invL);
    const int c = k >= o.nh ? 1 : 0;
    return class_site<1>(o, k - c * o.nh, c, L, invH, invL);
}

// LDS regions of the sweep kernel (offsets from lds_layout()).
struct Smem {
    uint32_t *thr;    // [kMaxTemps][kThrCols] rows by slot
    uint32_t *fthr;   // [kMaxTemps][kThrCols] rows by temperature
    int32_t *U;       // unsatisfied bonds per slot
    int32_t *perm;    // temp_of_slot
    int32_t *sot;     // slot_of_temp
    uint32_t *draw;   // per pair: its swap draw (split by lattice halves: its cut, swap_cut)
    int32_t *soff, *slen, *ssgn;   // swap tables: offset, length, sign of dbeta
    uint32_t *acc;    // accepted swaps per pair in this unit
    uint64_t *mask;   // speculative accept bits per pair
    uint32_t *ptab;   // [2][3][32] bit-sliced thresholds by slot (plane draws)
    int32_t *up;      // spins up per slot (with a field)
    uint32_t *items;  // plane draws: per wave, the halves waiting for more planes
    uint32_t *spin;   // [words_resident][N]
    uint32_t *stab;   // swap tables (when cached)
    uint32_t *sites;  // odd-L site list (when cached)
    uint8_t *j6;      // [N]
    Order ord;        // LDS order of spin words and coupling bytes
};

__device__ __forceinline__ Smem carve(uint8_t *base, int N, int words, int swap_entries, int site_entries,
                                      uint32_t item_bytes, int sep)
{
    const LdsLayout l = lds_layout(N, words, swap_entries, site_entries, item_bytes);
    Smem s;
    s.thr = (uint32_t *)(base + l.thr);
    s.fthr = (uint32_t *)(base + l.fthr);
    s.U = (int32_t *)(base + l.U);
    s.perm = (int32_t *)(base + l.perm);
    s.sot = (int32_t *)(base + l.sot);
    s.draw = (uint32_t *)(base + l.draw);
    s.ptab = (uint32_t *)(base + l.ptab);
    s.up = (int32_t *)(base + l.up);
    s.items = (uint32_t *)(base + l.items);
    s.soff = (int32_t *)(base + l.soff);
    s.slen = (int32_t *)(base + l.slen);
    s.ssgn = (int32_t *)(base + l.ssgn);
    s.acc = (uint32_t *)(base + l.acc);
    s.mask = (uint64_t *)(base + l.mask);
    s.spin = (uint32_t *)(base + l.spin);
    s.stab = (uint32_t *)(base + l.stab);
    s.sites = (uint32_t *)(base + l.sites);
    s.j6 = base + l.j6;
    s.ord.sep = sep;
    s.ord.nh = N >> 1;
    s.ord.base = 0;
    return s;
}

// ---------------------------------------------------------------------------
// Metropolis decisions for one word.  NG = number of 4-slot groups (Philox
// blocks) the word holds; a compile-time NG keeps all blocks in one basic
// block so their independent chains interleave.
// ---------------------------------------------------------------------------
struct Ctr {
    uint32_t t, r, c3, k0, k1;   // sweep, realization, domain|copy|group base, key
    uint32_t w;                  // segment width (4)
};

// CAMSC: X[k] holds 2E+S of slot 4j+k in segment j.  Returns the flip bits of
// the 4*NG slots, bit s = slot s of the word.  With PRE the NG blocks were
// drawn beforehand (pre[g] = the block of group g).
template <int NG, bool PRE = false>
__device__ __forceinline__ uint32_t camsc_decide(const uint32_t X[4], const uint32_t *rows, uint32_t site,
                                                 const Ctr &c, const U4 *pre = nullptr)
{
    uint32_t F = 0;
#pragma unroll
    for (int g = NG - 1; g >= 0; --g) {
        const U4 rr = PRE ? pre[g] : philox10(site, c.t, c.r, c.c3 + (uint32_t)g, c.k0, c.k1);
        const uint32_t *row = rows + 4 * g * kThrCols;
        F = (F << 1) | (rr.w < row[3 * kThrCols + field4(X[3], 4 * g, c.w)] ? 1u : 0u);
        F = (F << 1) | (rr.z < row[2 * kThrCols + field4(X[2], 4 * g, c.w)] ? 1u : 0u);
        F = (F << 1) | (rr.y < row[1 * kThrCols + field4(X[1], 4 * g, c.w)] ? 1u : 0u);
        F = (F << 1) | (rr.x < row[0 * kThrCols + field4(X[0], 4 * g, c.w)] ? 1u : 0u);
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
        const U4 rr = philox10(site, c.t, c.r, c.c3 + (uint32_t)g, c.k0, c.k1);
        const uint32_t *row = rows + 4 * g * kThrCols;
        F = (F << 4) | (rr.w < row[3 * kThrCols + field4(X, 16 * g + 12, c.w)] ? 1u : 0u);
        F = (F << 4) | (rr.z < row[2 * kThrCols + field4(X, 16 * g + 8, c.w)] ? 1u : 0u);
        F = (F << 4) | (rr.y < row[1 * kThrCols + field4(X, 16 * g + 4, c.w)] ? 1u : 0u);
        F = (F << 4) | (rr.x < row[0 * kThrCols + field4(X, 16 * g, c.w)] ? 1u : 0u);
    }
    return F;
}

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);   // truth table of majority(a, b, c)
}

// CAMSC with bit-plane draws.  The uniform of slot s is bit-sliced over 32
// planes (plane p holds bit 31 - p); plane p of the 16-slot half h is the
// 16-bit field p & 1 of word (p & 7) >> 1 of block (site, t, r,
// domain | copy | h << 8 | p >> 3).  `draw < threshold` is decided at the
// first plane where the two differ, so the slots still undecided are compared
// plane by plane against their thresholds, which ptab holds bit-sliced by slot
// (pt[e * 32 + p] = bit 31 - p of the threshold at E = e, e = 0..2; m1 / m2
// select the slots with E = 1 / 2).

// Bit-sliced thresholds by slot for the plane draws, from the rows by slot:
// ptab[w][e][p] bit b = bit 31 - p of the threshold of slot 32 w + b at E = e
// (column 2e; with h = 0 both columns of an E are equal).  Rows of slots past
// the ladder are zero.  One ballot per (e, p), shared out over the waves.
__device__ __forceinline__ void build_ptab(const Smem &sm, int NW, int wave, int nwaves, int lane)
{
    const uint32_t v0 = sm.thr[lane * kThrCols + 0];
    const uint32_t v1 = sm.thr[lane * kThrCols + 2];
    const uint32_t v2 = sm.thr[lane * kThrCols + 4];
    for (int item = wave; item < 96; item += nwaves) {
        const int e = item >> 5, p = item & 31;
        const uint32_t v = e == 0 ? v0 : (e == 1 ? v1 : v2);
        const uint64_t b = __ballot((v >> (31 - p)) & 1u);
        if (lane == 0) {
            sm.ptab[item] = (uint32_t)b;
            if (NW > 1) sm.ptab[96 + item] = (uint32_t)(b >> 32);
        }
    }
}

// Plane draws, first round: planes 0..7 of NH halves from one block each
// (block index 0 of the stream above), for the slots in `und`.  Returns the
// slots found below their threshold; `und` keeps the slots these planes left
// undecided (their draw and threshold agree in the top 8 bits; probability
// 2^-8 each), which finish later from the half's next blocks.
// (planes8_compare takes the two blocks drawn already: a = half h0's, b =
// the next half's when NH = 2.)
template <int NH>
__device__ __forceinline__ uint32_t planes8_compare(uint32_t &und, uint32_t m1, uint32_t m2, const uint32_t *pt,
                                                    const U4 &a, const U4 &b, int lo)
{
    uint32_t lt = 0;
    const uint32_t sel_even = lo ? 0x01000C0Cu : 0x0C0C0100u;
    const uint32_t sel_odd = lo ? 0x03020C0Cu : 0x0C0C0302u;
    const uint32_t wa[4] = {a.x, a.y, a.z, a.w};
    const uint32_t wb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        uint32_t R;
        if (NH == 2)
            R = __builtin_amdgcn_perm(wb[q >> 1], wa[q >> 1], (q & 1) ? 0x07060302u : 0x05040100u);
        else
            R = __builtin_amdgcn_perm(wa[q >> 1], wa[q >> 1], (q & 1) ? sel_odd : sel_even);
        const uint32_t t01 = (m1 & pt[32 + q]) | (~m1 & pt[q]);
        const uint32_t T = (m2 & pt[64 + q]) | (~m2 & t01);
        const uint32_t x = und & (R ^ T);
        lt |= x & T;
        und ^= x;
    }
    return lt;
}

template <int NH>
__device__ __forceinline__ uint32_t camsc_planes8(uint32_t &und, uint32_t m1, uint32_t m2, const uint32_t *pt,
                                                  uint32_t site, uint32_t t, uint32_t r, uint32_t c3, uint32_t k0,
                                                  uint32_t k1, int lo)
{
    const U4 a = philox10(site, t, r, c3, k0, k1);
    U4 b = a;
    if (NH == 2) b = philox10(site, t, r, c3 + (1u << 8), k0, k1);
    return planes8_compare<NH>(und, m1, m2, pt, a, b, lo);
}

// A wave's list of halves that the first 8 planes left undecided, in LDS:
// field 0 = site | local word << 15 | half << 17 | next block << 18, field 1 =
// undecided slots | E==1 slots << 16, field 2 = E==2 slots (16-bit masks of the
// half).  Working through them a whole wave at a time keeps the lanes busy:
// the wave-wide alternative, drawing the next planes for every lane while any
// lane still needs them, spends most of its Philox blocks on decided slots.
struct PlaneQueue {
    uint32_t *f;   // this wave's fields: f[k], f[kItemCap + k], f[2 kItemCap + k]
    int count;     // halves waiting (uniform across the wave)
};

__device__ __forceinline__ PlaneQueue plane_queue(const Smem &sm, int wave)
{
    PlaneQueue q;
    q.f = sm.items + wave * 3 * kItemCap;
    q.count = 0;
    return q;
}

// Append this lane's half if it has undecided slots; every lane of the wave calls it.
__device__ __forceinline__ void plane_push(PlaneQueue &q, uint32_t und16, uint32_t m1_16, uint32_t m2_16, uint32_t key)
{
    const uint64_t b = __ballot(und16 != 0u);
    if (b == 0ull) return;
    const int below = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
    if (und16 != 0u) {
        const int pos = q.count + below;
        q.f[pos] = key;
        q.f[kItemCap + pos] = und16 | (m1_16 << 16);
        q.f[2 * kItemCap + pos] = m2_16;
    }
    q.count = __builtin_amdgcn_readfirstlane(q.count + (int)__builtin_popcountll(b));
}

// Take up to 64 waiting halves, one per lane, and compare them against their
// next 8 planes (block `next block` of the half); xor the flips found into the
// spin words (other bits than the first round's, so the order is free) and put
// back the halves still undecided.  A half whose 32 planes all agree has a draw
// equal to its threshold: not below it, so no flip.  Every lane calls it.
__device__ __forceinline__ void plane_drain(const Smem &sm, PlaneQueue &q, int lane, int N, int g0, int cls,
                                            uint32_t t, uint32_t r, uint32_t c3base, uint32_t k0, uint32_t k1)
{
    const int n = min(q.count, 64);
    const int base = q.count - n;
    q.count = base;
    uint32_t key = 0, und = 0, m1 = 0, m2 = 0;
    if (lane < n) {
        key = q.f[base + lane];
        const uint32_t y = q.f[kItemCap + base + lane];
        und = y & 0xFFFFu;
        m1 = y >> 16;
        m2 = q.f[2 * kItemCap + base + lane];
    }
    const uint32_t blk = key >> 18;
    if (lane < n) {
        const uint32_t site = key & 0x7FFFu, wl = (key >> 15) & 3u, hb = (key >> 17) & 1u;
        const uint32_t wg = (uint32_t)g0 + wl;
        const U4 a = philox10(site, t, r, c3base | ((2u * wg + hb) << 8) | blk, k0, k1);
        const uint32_t w4[4] = {a.x, a.y, a.z, a.w};
        const uint32_t *pt = sm.ptab + wg * 96u + 8u * blk;
        const uint32_t sh = 16u * hb;
        const uint32_t m0 = ~(m1 | m2);
        uint32_t lt = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t R = (w4[p >> 1] >> (16 * (p & 1))) & 0xFFFFu;
            const uint32_t T = ((m0 & (pt[p] >> sh)) | (m1 & (pt[32 + p] >> sh)) | (m2 & (pt[64 + p] >> sh))) & 0xFFFFu;
            const uint32_t x = und & (R ^ T);
            lt |= x & T;
            und ^= x;
        }
        const uint32_t at = sm.ord.sep ? (uint32_t)(cls * sm.ord.nh) + (site >> 1) : site - sm.ord.base;   // LDS word
        if (lt) atomicXor(sm.spin + wl * (uint32_t)N + at, lt << sh);
    }
    plane_push(q, blk < 3u ? und : 0u, m1, m2, (key & 0x3FFFFu) | ((blk + 1u) << 18));
}

// One site (all resident words) with plane draws, outside the summing class:
// the first 8 planes of each half decide here, the rest go to the wave's list.
// Every lane of the wave calls it; `live` lanes hold a site.
template <bool SPLIT>
__device__ __forceinline__ void update_site_planes(const Smem &sm, PlaneQueue &q, bool live, const Nbrs &nb, int N,
                                                   int gw, int g0, int cls, int n_T, uint32_t t, uint32_t r,
                                                   uint32_t c3base, uint32_t k0, uint32_t k1, int gb, int ngr_own,
                                                   int lane)
{
    const uint32_t j6 = live ? sm.j6[nb.i] : 0u;
    for (int w = 0; w < gw; ++w) {
        const int wg = g0 + w;
        const int left = n_T - wg * 32;
        uint32_t valid = left >= 32 ? 0xFFFFFFFFu : ((1u << left) - 1u);
        int h0 = 2 * wg, nh = left > 16 ? 2 : 1, lo = 0;
        if (SPLIT) {
            const int a = 4 * gb, b = 4 * (gb + ngr_own) - 1;
            valid &= (ngr_own >= 8 ? 0xFFFFFFFFu : ((1u << (4 * ngr_own)) - 1u)) << (4 * gb);
            h0 = 2 * wg + (a >> 4);
            nh = (b >> 4) - (a >> 4) + 1;
            lo = nh == 1 ? (a & 16) : 0;
        }
        uint32_t und = 0, m1 = 0, m2 = 0;
        if (live) {
            uint32_t *sw = sm.spin + (size_t)w * N;
            const uint32_t S = sw[nb.i];
            const uint32_t e0 = xor3(S, sw[nb.xp], (0u - (j6 & 1u)));
            const uint32_t e1 = xor3(S, sw[nb.xm], (0u - ((j6 >> 1) & 1u)));
            const uint32_t e2 = xor3(S, sw[nb.yp], (0u - ((j6 >> 2) & 1u)));
            const uint32_t e3 = xor3(S, sw[nb.ym], (0u - ((j6 >> 3) & 1u)));
            const uint32_t e4 = xor3(S, sw[nb.zp], (0u - ((j6 >> 4) & 1u)));
            const uint32_t e5 = xor3(S, sw[nb.zm], (0u - ((j6 >> 5) & 1u)));
            const uint32_t s1 = xor3(e0, e1, e2), c1 = maj3(e0, e1, e2);
            const uint32_t s2 = xor3(e3, e4, e5), c2 = maj3(e3, e4, e5);
            const uint32_t E0 = s1 ^ s2, kk = s1 & s2;
            const uint32_t E1 = xor3(c1, c2, kk), E2 = maj3(c1, c2, kk);
            const uint32_t always = E2 | (E1 & E0);   // E >= 3
            m1 = E0 & ~E1;
            m2 = E1 & ~E0;
            und = valid & ~always;
            const uint32_t *pt = sm.ptab + wg * 96;
            const uint32_t c3 = c3base | ((uint32_t)h0 << 8);
            const uint32_t lt = nh == 2 ? camsc_planes8<2>(und, m1, m2, pt, nb.g, t, r, c3, k0, k1, 0)
                                        : camsc_planes8<1>(und, m1, m2, pt, nb.g, t, r, c3, k0, k1, lo);
            sw[nb.i] = S ^ ((lt | always) & valid);
        }
        const uint32_t key = (uint32_t)nb.g | ((uint32_t)w << 15) | (1u << 18);
        if (nh == 2) {
            plane_push(q, und & 0xFFFFu, m1 & 0xFFFFu, m2 & 0xFFFFu, key);
            while (q.count > kItemFlush) plane_drain(sm, q, lane, N, g0, cls, t, r, c3base, k0, k1);
            plane_push(q, und >> 16, m1 >> 16, m2 >> 16, key | (1u << 17));
        } else {
            plane_push(q, (und >> lo) & 0xFFFFu, (m1 >> lo) & 0xFFFFu, (m2 >> lo) & 0xFFFFu,
                       key | ((uint32_t)(lo >> 4) << 17));
        }
        while (q.count > kItemFlush) plane_drain(sm, q, lane, N, g0, cls, t, r, c3base, k0, k1);
    }
}

// Exchange the bits of a selected by m << sh with the bits of b selected by m.
__device__ __forceinline__ void swap_bits(uint32_t &a, uint32_t &b, int sh, uint32_t m)
{
    const uint32_t t = ((a >> sh) ^ b) & m;
    b ^= t;
    a ^= t << sh;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_src(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// P += shifted copy of P (NQ planes in, carry grows the top plane).
template <int NQ, int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_add_planes(uint32_t (&P)[14])
{
    uint32_t Q[NQ];
#pragma unroll
    for (int p = 0; p < NQ; ++p) Q[p] = dpp_src<CTRL, ROW_MASK>(P[p]);
    uint32_t c = P[0] & Q[0];
    P[0] ^= Q[0];
#pragma unroll
    for (int p = 1; p < NQ; ++p) {
        const uint32_t sum = xor3(P[p], Q[p], c);
        c = maj3(P[p], Q[p], c);
        P[p] = sum;
    }
    P[NQ] = c;   // planes above NQ are zero before this step
}

// P += s0 + 2 s1 + 4 s2 per bit position (a per-slot count of 0..7), np planes
// (NPC > 0: exactly NPC planes, known at compile time).
template <int NPC = 0>
__device__ __forceinline__ void planes_add3(uint32_t (&P)[8], uint32_t s0, uint32_t s1, uint32_t s2, int np)
{
    if (NPC > 0) np = NPC;
    uint32_t carry = P[0] & s0;
    P[0] ^= s0;
    const uint32_t n1 = xor3(P[1], s1, carry);
    carry = maj3(P[1], s1, carry);
    P[1] = n1;
    const uint32_t n2 = xor3(P[2], s2, carry);
    carry = maj3(P[2], s2, carry);
    P[2] = n2;
#pragma unroll
    for (int p = 3; p < 8; ++p) {
        if (p < np) {
            const uint32_t tt = P[p] & carry;
            P[p] ^= carry;
            carry = tt;
        }
    }
}

// Wave-sum NP plane counters (DPP) and add slot b's total into U[slot0 + b]
// for the slots of one word (bit position b * STR).
template <int NP, int STR>
__device__ __forceinline__ void reduce_planes_add(uint32_t (&P)[14], int nslots, int *U, int first = 0)
{
    dpp_add_planes<NP + 0, 0x111, 0xF>(P);   // row_shr:1
    dpp_add_planes<NP + 1, 0x112, 0xF>(P);   // row_shr:2
    dpp_add_planes<NP + 2, 0x114, 0xF>(P);   // row_shr:4
    dpp_add_planes<NP + 3, 0x118, 0xF>(P);   // row_shr:8
    dpp_add_planes<NP + 4, 0x142, 0xA>(P);   // row_bcast:15 into rows 1, 3
    dpp_add_planes<NP + 5, 0x143, 0xC>(P);   // row_bcast:31 into rows 2, 3
    const int lane = threadIdx.x & 63;
    const int shift = (lane < nslots ? first + lane : 0) * STR;
    int cnt = 0;
#pragma unroll
    for (int p = 0; p < NP + 6; ++p) {
        const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)P[p], 63);
        cnt += (int)((w >> shift) & 1u) << p;
    }
    if (lane < nslots && cnt) atomicAdd(&U[first + lane], cnt);
}

// slots first .. first + nslots - 1 of the word (bit positions (first + b) * STR)
template <int STR>
__device__ __forceinline__ void reduce_planes8_add(const uint32_t (&P8)[8], int np, int nslots, int *U, int first = 0)
{
    uint32_t P[14];
#pragma unroll
    for (int p = 0; p < 14; ++p) P[p] = p < 8 ? P8[p] : 0u;
    switch (np) {
        case 2: reduce_planes_add<2, STR>(P, nslots, U, first); break;
        case 3: reduce_planes_add<3, STR>(P, nslots, U, first); break;
        case 4: reduce_planes_add<4, STR>(P, nslots, U, first); break;
        case 5: reduce_planes_add<5, STR>(P, nslots, U, first); break;
        case 6: reduce_planes_add<6, STR>(P, nslots, U, first); break;
        case 7: reduce_planes_add<7, STR>(P, nslots, U, first); break;
        default: reduce_planes_add<8, STR>(P, nslots, U, first); break;
    }
}

// Wave-sum of four plane counters whose per-lane counts stay below 16, for the
// nslots <= 16 slots first .. first + nslots - 1 (first a multiple of 4),
// added into U[first + b].  The planes become one byte per slot (a bit
// transpose inside each nibble), DPP sums inside each row of 16 lanes keep a
// byte below 256, and the four row sums are added in 16-bit fields.
__device__ __forceinline__ void reduce_planes4_bytes_add(const uint32_t (&P8)[8], int nslots, int *U, int first)
{
    uint32_t X[4] = {P8[0], P8[1], P8[2], P8[3]};
    // nibble m of X[q] <- the count of slot 4m + q
    swap_bits(X[0], X[2], 2, 0x33333333u);
    swap_bits(X[1], X[3], 2, 0x33333333u);
    swap_bits(X[0], X[1], 1, 0x55555555u);
    swap_bits(X[2], X[3], 1, 0x55555555u);
    // byte m of Z[q] <- the count of slot first + 4m + q
    uint32_t Z[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t y = (X[q] >> first) & 0xFFFFu;
        const uint32_t t = (y | (y << 8)) & 0x00FF00FFu;
        Z[q] = (t | (t << 4)) & 0x0F0F0F0Fu;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) Z[q] += dpp_src<0x111, 0xF>(Z[q]);   // row_shr:1
#pragma unroll
    for (int q = 0; q < 4; ++q) Z[q] += dpp_src<0x112, 0xF>(Z[q]);   // row_shr:2
#pragma unroll
    for (int q = 0; q < 4; ++q) Z[q] += dpp_src<0x114, 0xF>(Z[q]);   // row_shr:4
#pragma unroll
    for (int q = 0; q < 4; ++q) Z[q] += dpp_src<0x118, 0xF>(Z[q]);   // row_shr:8
    // W[2q + h] fields f = 0, 1 <- byte 2f + h of Z[q]: slot first + 4(2f + h) + q
    uint32_t W[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        W[2 * q] = Z[q] & 0x00FF00FFu;
        W[2 * q + 1] = (Z[q] >> 8) & 0x00FF00FFu;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) W[k] += dpp_src<0x142, 0xA>(W[k]);   // row_bcast:15 into rows 1, 3
#pragma unroll
    for (int k = 0; k < 8; ++k) W[k] += dpp_src<0x143, 0xC>(W[k]);   // row_bcast:31 into rows 2, 3
    // lane b: slot first + b = first + 4m + q with m = 2f + h (selects on
    // values, not on array elements, so that nothing goes to scratch memory)
    const int b = threadIdx.x & 15;
    const int q = b & 3, h = (b >> 2) & 1, f = b >> 3;
    const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)W[0], 63);
    const uint32_t w1 = (uint32_t)__builtin_amdgcn_readlane((int)W[1], 63);
    const uint32_t w2 = (uint32_t)__builtin_amdgcn_readlane((int)W[2], 63);
    const uint32_t w3 = (uint32_t)__builtin_amdgcn_readlane((int)W[3], 63);
    const uint32_t w4 = (uint32_t)__builtin_amdgcn_readlane((int)W[4], 63);
    const uint32_t w5 = (uint32_t)__builtin_amdgcn_readlane((int)W[5], 63);
    const uint32_t w6 = (uint32_t)__builtin_amdgcn_readlane((int)W[6], 63);
    const uint32_t w7 = (uint32_t)__builtin_amdgcn_readlane((int)W[7], 63);
    const uint32_t a0 = h ? w1 : w0, a1 = h ? w3 : w2;
    const uint32_t a2 = h ? w5 : w4, a3 = h ? w7 : w6;
    const uint32_t c0 = (q & 1) ? a1 : a0, c1 = (q & 1) ? a3 : a2;
    const uint32_t v = (q & 2) ? c1 : c0;
    const int cnt = (int)((v >> (16 * f)) & 0xFFFFu);
    const int lane = threadIdx.x & 63;
    if (lane < nslots && cnt) atomicAdd(&U[first + lane], cnt);
}

// Certain flips (cost <= 0).  Without a field they are the slots with E >= 3;
// with a field h the bound depends on the spin: E >= a_S for spin bit S.
struct Field {
    bool on;
    uint32_t add0, add1;   // (8 - a_S) per 4-bit segment
    int col0, col1;        // certain iff column 2E+S >= col_S
};

__device__ __forceinline__ Field field_of(const JobDesc &jd)
{
    return Field{jd.field_m != 0, jd.always_add0, jd.always_add1, jd.always_col0, jd.always_col1};
}

// Segments (4 bits, bit 0 = S in Sb) of E >= a_S: E + (8 - a_S) reaches bit 3
// without leaving the segment (E <= 6).
__device__ __forceinline__ uint32_t certain_segments(uint32_t E, uint32_t Sb, const Field &fd)
{
    constexpr uint32_t M = 0x11111111u;
    const uint32_t ge0 = ((E + fd.add0) >> 3) & M;
    const uint32_t ge1 = ((E + fd.add1) >> 3) & M;
    return (ge1 & Sb) | (ge0 & ~Sb);
}

// ---------------------------------------------------------------------------
// Metropolis update of one site for the `gw` resident words (word index g0..).
// ---------------------------------------------------------------------------
// With ACC (CAMSC, even L, last colour class of a swap sweep) the six bond
// bits of the site after the update are added into the per-lane plane counters
// of its word: on a bipartite lattice every bond has exactly one endpoint in
// that class, so these sums are the slots' unsatisfied-bond counts U.
//
// With SPLIT (CAMSC, one word per site) this workgroup owns only the slot
// groups [gb, gb + ngr_own) of the word; the other groups' bits in its LDS
// copy are never read for its own decisions (slots do not interact).
// NPC > 0 fixes the number of plane counters at compile time.
//
// With PRE (CAMSC words, SPLIT) the Philox blocks of the own groups were drawn
// beforehand: pre[g] is the block of own group g (at most four).
template <int LAYOUT, bool ACC = false, bool SPLIT = false, int RNG = 0, bool PRE = false, int NPC = 0>
__device__ __forceinline__ void update_site(const Smem &sm, const Nbrs &nb, int N, int gw, int g0, int n_T,
                                            uint32_t t, uint32_t r, uint32_t c3base, uint32_t k0, uint32_t k1,
                                            uint32_t segw, const Field &fd, uint32_t (*P)[8] = nullptr, int np = 0,
                                            int gb = 0, int ngr_own = 0, const U4 *pre = nullptr)
{
    static_assert(!PRE || (SPLIT && LAYOUT == 0 && RNG == 0), "pre-drawn blocks: split CAMSC words only");
    constexpr uint32_t M = 0x11111111u;
    const uint32_t j6 = sm.j6[nb.i];
    // all-ones mask for an antiferromagnetic incidence: the coupling, widened
    // to every slot bit, is applied to S by XOR (Sec. 4.3.3)
    uint32_t m[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) m[d] = 0u - ((j6 >> d) & 1u);
    if (LAYOUT == 1 || LAYOUT == 2) {
#pragma unroll
        for (int d = 0; d < 6; ++d) m[d] &= Layout<LAYOUT>::kKeep;
    }
    for (int w = 0; w < gw; ++w) {
        uint32_t *sw = sm.spin + (size_t)w * N;
        const uint32_t S = sw[nb.i];
        const uint32_t e0 = xor3(S, sw[nb.xp], m[0]);
        const uint32_t e1 = xor3(S, sw[nb.xm], m[1]);
        const uint32_t e2 = xor3(S, sw[nb.yp], m[2]);
        const uint32_t e3 = xor3(S, sw[nb.ym], m[3]);
        const uint32_t e4 = xor3(S, sw[nb.zp], m[4]);
        const uint32_t e5 = xor3(S, sw[nb.zm], m[5]);
        const int wg = __builtin_amdgcn_readfirstlane(g0 + w);
        if (LAYOUT == 0) {
            static_assert(RNG == 0, "plane draws update sites through class_pass_planes");
            // CAMSC: sum the six 1-bit bond words as three bit planes (full
            // adders, one bitop3 each), then widen into four 4-bit-segment words
            // (segment j of word k holds slot 4j + k) that carry 2E+S:
            // S | E0 << 1 | E1 << 2 | E2 << 3 of that slot.
            const uint32_t s1 = xor3(e0, e1, e2), c1 = maj3(e0, e1, e2);
            const uint32_t s2 = xor3(e3, e4, e5), c2 = maj3(e3, e4, e5);
            const uint32_t E0 = s1 ^ s2, kk = s1 & s2;
            const uint32_t E1 = xor3(c1, c2, kk), E2 = maj3(c1, c2, kk);
            // word p bit k of every nibble -> word k bit p: a 4 x 4 bit transpose
            // inside each nibble by two rounds of masked swaps
            uint32_t X[4] = {S, E0, E1, E2};
            swap_bits(X[0], X[2], 2, 0x33333333u);
            swap_bits(X[1], X[3], 2, 0x33333333u);
            swap_bits(X[0], X[1], 1, 0x55555555u);
            swap_bits(X[2], X[3], 1, 0x55555555u);
            uint32_t always = 0;
            if (!fd.on) {
                always = E2 | (E1 & E0);   // E >= 3, bit s = slot s
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) always |= certain_segments((X[k] >> 1) & 0x77777777u, X[k] & M, fd) << k;
            }
            const int slot0 = wg * 32;
            const int left = n_T - slot0;
            int ngr = left >= 32 ? 8 : (left + 3) >> 2;
            uint32_t valid = left >= 32 ? 0xFFFFFFFFu : ((1u << left) - 1u);
            const uint32_t *rows = sm.thr + slot0 * kThrCols;
            Ctr c{t, r, c3base + (uint32_t)(wg * 8), k0, k1, segw};
            if (SPLIT) {
                // own groups only: shift them down to group 0, decide, shift the flips back
#pragma unroll
                for (int k = 0; k < 4; ++k) X[k] >>= 4 * gb;
                rows += 4 * gb * kThrCols;
                c.c3 += (uint32_t)gb;
                ngr = ngr_own;
                valid &= (ngr_own >= 8 ? 0xFFFFFFFFu : ((1u << (4 * ngr_own)) - 1u)) << (4 * gb);
            }
            uint32_t F;
            if (SPLIT) {   // a split ladder owns at most four groups
                switch (ngr) {
                    case 4: F = camsc_decide<4, PRE>(X, rows, nb.g, c, pre); break;
                    case 3: F = camsc_decide<3, PRE>(X, rows, nb.g, c, pre); break;
                    case 2: F = camsc_decide<2, PRE>(X, rows, nb.g, c, pre); break;
                    default: F = camsc_decide<1, PRE>(X, rows, nb.g, c, pre); break;
                }
            } else {
                switch (ngr) {
                    case 8: F = camsc_decide<8>(X, rows, nb.g, c); break;
                    case 7: F = camsc_decide<7>(X, rows, nb.g, c); break;
                    case 6: F = camsc_decide<6>(X, rows, nb.g, c); break;
                    case 5: F = camsc_decide<5>(X, rows, nb.g, c); break;
                    case 4: F = camsc_decide<4>(X, rows, nb.g, c); break;
                    case 3: F = camsc_decide<3>(X, rows, nb.g, c); break;
                    case 2: F = camsc_decide<2>(X, rows, nb.g, c); break;
                    default: F = camsc_decide<1>(X, rows, nb.g, c); break;
                }
            }
            if (SPLIT) F <<= 4 * gb;
            const uint32_t flip = (F | always) & valid;
            sw[nb.i] = S ^ flip;
            if (ACC) {
                // unsatisfied bonds after the update: E if kept, 6 - E if flipped
                // (bit planes of 6 - E as in the plane-draw branch above)
                const uint32_t C1 = (flip & ~(E1 ^ E0)) | (~flip & E1);
                const uint32_t C2 = (flip & ~(E2 ^ (E1 & E0))) | (~flip & E2);
                planes_add3<NPC>(*P, E0, C1, C2, np);
            }
        } else if (LAYOUT == 1) {
            // AMSC4: 4-bit segments throughout; 2E+S is formed for all slots at once.
            const uint32_t E = e0 + e1 + e2 + e3 + e4 + e5;
            const uint32_t X = (E << 1) | S;
            const uint32_t always = fd.on ? certain_segments(E, S, fd) : ((X + 0x22222222u) >> 3) & M;
            const int slot0 = wg * 8;
            const int left = n_T - slot0;
            const uint32_t valid = left >= 8 ? M : (M & ((1u << (4 * left)) - 1u));
            const uint32_t *rows = sm.thr + slot0 * kThrCols;
            const Ctr c{t, r, c3base + (uint32_t)(wg * 2), k0, k1, segw};
            const uint32_t F = left > 4 ? amsc4_decide<2>(X, rows, nb.g, c) : amsc4_decide<1>(X, rows, nb.g, c);
            sw[nb.i] = S ^ ((F | always) & valid);
        } else {
            // AMSC3 / AMSC1 (Sec. 4.3.3): 2E+S is joined slot by slot.  AMSC3
            // sums the six bond words in its 3-bit segments first (E <= 6 never
            // carries out of a segment); AMSC1 sums each slot's six bond bits
            // on their own.  One Philox block serves four consecutive slots.
            constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
            constexpr int STR = Layout<LAYOUT>::kStride;
            const uint32_t E3 = LAYOUT == 2 ? e0 + e1 + e2 + e3 + e4 + e5 : 0u;
            const int slot0 = wg * SPW;
            const int n = min(SPW, n_T - slot0);
            const uint32_t *rows = sm.thr + slot0 * kThrCols;
            uint32_t flip = 0;
            U4 blk{0u, 0u, 0u, 0u};
            int cur = -1;
            for (int j = 0; j < n; ++j) {
                const int slot = slot0 + j;
                if ((slot >> 2) != cur) {   // uniform across the wave
                    cur = slot >> 2;
                    blk = philox10(nb.g, t, r, c3base + (uint32_t)cur, k0, k1);
                }
                uint32_t E;
                if (LAYOUT == 2)
                    E = (E3 >> (3 * j)) & 7u;
                else
                    E = ((e0 >> j) & 1u) + ((e1 >> j) & 1u) + ((e2 >> j) & 1u) + ((e3 >> j) & 1u) +
                        ((e4 >> j) & 1u) + ((e5 >> j) & 1u);
                const uint32_t sbit = (S >> (j * STR)) & 1u;
                const uint32_t col = (E << 1) | sbit;
                const int q = slot & 3;
                const uint32_t dr = q == 0 ? blk.x : (q == 1 ? blk.y : (q == 2 ? blk.z : blk.w));
                const bool f = (int)col >= (sbit ? fd.col1 : fd.col0) || dr < rows[j * kThrCols + col];
                flip |= (f ? 1u : 0u) << (j * STR);
            }
            sw[nb.i] = S ^ flip;
        }
    }
}

// ---------------------------------------------------------------------------
// Unsatisfied-bond counts per slot for one word (forward bonds of every site),
// added into U[slot0 + b].
//
// Each lane sums its sites' bond bits in NP vertical bit planes (plane p holds
// bit p of every slot's count).  The wave then adds the lanes' plane counters
// with DPP: row_shr 1, 2, 4, 8 leave each row's total in its lane 15, and
// row_bcast 15 / 31 fold the rows into lane 63; every step is a vertical
// ripple add, two bitop3 per plane.  Finally the planes are broadcast from
// lane 63 and lane b assembles slot b's count, so the whole reduction is
// vector work plus one LDS atomic per wave.
// ---------------------------------------------------------------------------
template <int LAYOUT, int NP>
__device__ void count_unsat_word_np(const Order &o, const uint32_t *words, const uint8_t *j6, int N, int L, float invH,
                                    float invL, int slot0, int n_T, int *U)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr int STR = Layout<LAYOUT>::kStride;
    const uint32_t keep = Layout<LAYOUT>::kKeep;
    uint32_t P[14];
#pragma unroll
    for (int p = 0; p < 14; ++p) P[p] = 0;
    for (int idx = threadIdx.x; idx < N; idx += blockDim.x) {
        const Nbrs nb = lds_site(o, idx, L, invH, invL);
        const uint32_t S = words[nb.i];
        const uint32_t jb = j6[nb.i];
        const uint32_t ex = S ^ words[nb.xp] ^ ((0u - (jb & 1u)) & keep);
        const uint32_t ey = S ^ words[nb.yp] ^ ((0u - ((jb >> 2) & 1u)) & keep);
        const uint32_t ez = S ^ words[nb.zp] ^ ((0u - ((jb >> 4) & 1u)) & keep);
        // ex + ey + ez = 2c + s, added into the planes
        const uint32_t s = xor3(ex, ey, ez);
        const uint32_t c = maj3(ex, ey, ez);
        const uint32_t carry0 = P[0] & s;
        P[0] ^= s;
        uint32_t carry = maj3(P[1], c, carry0);
        P[1] = xor3(P[1], c, carry0);
#pragma unroll
        for (int p = 2; p < NP; ++p) {
            const uint32_t tt = P[p] & carry;
            P[p] ^= carry;
            carry = tt;
        }
    }
    reduce_planes_add<NP, STR>(P, min(SPW, n_T - slot0), U + slot0);
}

// One ballot of the swap pass's acceptance words for up to 32 temperatures:
// lane k of half hf (lane = 32 hf + k) evaluates pair k for the start position
// j = 2i + hf, so the ballot holds col[2i] in its low and col[2i + 1] in its
// high 32 bits; bit k of col[j] is set when pair k (k >= j) would swap the
// configuration carried up from position j.  uj: energy at position j;
// u_next: energy at position k + 1; the pair's draw, sign of dbeta, table
// length and offset in drk, sg, len, off.  Without GUARD the table is in LDS
// and is read unconditionally (an index past its end still falls inside the
// workgroup's LDS, and the value is then unused).
template <bool GUARD>
__device__ __forceinline__ uint64_t swap_ballot(const uint32_t *tab, int uj, int u_next, uint32_t drk, int sg,
                                                int len, int off, int k, int j, bool live)
{
    const int d = uj - u_next;
    const int n = d < 0 ? -d : d;
    const int lenm1 = len > 0 ? len - 1 : 0;
    uint32_t thr;
    if (GUARD)
        thr = len > 0 ? tab[off + min(n, lenm1)] : 0u;
    else
        thr = tab[off + min(n, lenm1)];
    const bool favourable = (sg == 0) || (d == 0) || ((sg > 0) == (d > 0));
    return __ballot(live && k >= j && (favourable || (n < len && drk < thr)));
}

// The Philox blocks of the NG own groups (counter groups c3 .. c3 + NG - 1) of
// sweep t at site j of colour class 0 (j < half).
template <int NG>
__device__ __forceinline__ void predraw_site(U4 (&st)[4], int j, int L, float invH, float invL, uint32_t t,
                                             uint32_t r, uint32_t c3, uint32_t k0, uint32_t k1)
{
    // the site is the same at every swap point: keep the compiler from hoisting
    // its partial rounds out of the sweep loop (they would stay live through
    // every sweep)
    asm volatile("" : "+v"(j));
    const uint32_t site = checker_site(j, 0, L, invH, invL).i;
#pragma unroll
    for (int g = 0; g < NG; ++g) st[g] = philox10(site, t, r, c3 + (uint32_t)g, k0, k1);
}

// Bit planes needed so that no lane's per-slot count overflows.
__device__ __forceinline__ int planes_for(int N, int nthr)
{
    const int per_lane = 3 * ((N + nthr - 1) / nthr);
    int np = 2;
    while ((1 << np) <= per_lane) ++np;
    return np;
}

// Planes for per-lane sums of six bond bits over the sites of one colour class.
__device__ __forceinline__ int planes_for_class(int n_sites, int nthr)
{
    const int per_lane = 6 * ((n_sites + nthr - 1) / nthr);
    int np = 3;
    while ((1 << np) <= per_lane) ++np;
    return np;
}

// Two sites of one colour class at once (CAMSC, one word per site, word draws,
// no field): the same steps as update_site, with both sites' loads first and
// both stores last so that their Philox chains share one straight-line block.
// Legal because two sites of one class are never neighbours: neither reads the
// other's spin.  NG = the slot groups decided (the own groups when SPLIT);
// with PRE the blocks were drawn beforehand (prea, preb as in update_site).
template <bool ACC, bool SPLIT, int NG, int NPC, bool PRE = false>
__device__ __forceinline__ void update_pair_camsc(const Smem &sm, const Nbrs &na, const Nbrs &nb, int n_T,
                                                  uint32_t t, uint32_t r, uint32_t c3base, uint32_t k0, uint32_t k1,
                                                  uint32_t segw, uint32_t (*P)[8], int np, int gb, int ngr_own,
                                                  const U4 *prea = nullptr, const U4 *preb = nullptr)
{
    const Nbrs nn[2] = {na, nb};
    uint32_t *sw = sm.spin;
    uint32_t S[2], V[2][6], J[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        J[q] = sm.j6[nn[q].i];
        S[q] = sw[nn[q].i];
        V[q][0] = sw[nn[q].xp];
        V[q][1] = sw[nn[q].xm];
        V[q][2] = sw[nn[q].yp];
        V[q][3] = sw[nn[q].ym];
        V[q][4] = sw[nn[q].zp];
        V[q][5] = sw[nn[q].zm];
    }
    uint32_t valid = n_T >= 32 ? 0xFFFFFFFFu : ((1u << n_T) - 1u);
    const uint32_t *rows = sm.thr;
    Ctr c{t, r, c3base, k0, k1, segw};
    if (SPLIT) {
        rows += 4 * gb * kThrCols;
        c.c3 += (uint32_t)gb;
        valid &= (ngr_own >= 8 ? 0xFFFFFFFFu : ((1u << (4 * ngr_own)) - 1u)) << (4 * gb);
    }
    uint32_t out[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        uint32_t e[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) e[d] = xor3(S[q], V[q][d], 0u - ((J[q] >> d) & 1u));
        const uint32_t s1 = xor3(e[0], e[1], e[2]), c1 = maj3(e[0], e[1], e[2]);
        const uint32_t s2 = xor3(e[3], e[4], e[5]), c2 = maj3(e[3], e[4], e[5]);
        const uint32_t E0 = s1 ^ s2, kk = s1 & s2;
        const uint32_t E1 = xor3(c1, c2, kk), E2 = maj3(c1, c2, kk);
        uint32_t X[4] = {S[q], E0, E1, E2};
        swap_bits(X[0], X[2], 2, 0x33333333u);
        swap_bits(X[1], X[3], 2, 0x33333333u);
        swap_bits(X[0], X[1], 1, 0x55555555u);
        swap_bits(X[2], X[3], 1, 0x55555555u);
        const uint32_t always = E2 | (E1 & E0);   // E >= 3
        if (SPLIT) {
#pragma unroll
            for (int k = 0; k < 4; ++k) X[k] >>= 4 * gb;
        }
        uint32_t F = camsc_decide<NG, PRE>(X, rows, (uint32_t)nn[q].g, c, q == 0 ? prea : preb);
        if (SPLIT) F <<= 4 * gb;
        const uint32_t flip = (F | always) & valid;
        out[q] = S[q] ^ flip;
        if (ACC) {
            const uint32_t C1 = (flip & ~(E1 ^ E0)) | (~flip & E1);
            const uint32_t C2 = (flip & ~(E2 ^ (E1 & E0))) | (~flip & E2);
            planes_add3<NPC>(*P, E0, C1, C2, np);
        }
    }
    sw[nn[0].i] = out[0];
    sw[nn[1].i] = out[1];
}

// One colour class of an even lattice: a split ladder with word draws and no
// field takes the sites of a thread two at a time, everything else one at a
// time (pairing measured slower where a workgroup holds the whole ladder).
template <int LAYOUT, bool ACC, bool SPLIT, int RNG, int NPC, int NG, int SEP>
__device__ __forceinline__ void class_pass_ng(const Smem &sm, int c, int tid, int nthr, int half, int L, float invH,
                                              float invL, int N, int gw, int g0, int n_T, uint32_t t, uint32_t r,
                                              uint32_t c3base, uint32_t k0, uint32_t k1, uint32_t segw,
                                              const Field &fd, uint32_t (*P)[8], int np, int gb, int ngr_own)
{
    int j = tid;
    for (; j + nthr < half; j += 2 * nthr)
        update_pair_camsc<ACC, SPLIT, NG, NPC>(sm, class_site<SEP>(sm.ord, j, c, L, invH, invL),
                                               class_site<SEP>(sm.ord, j + nthr, c, L, invH, invL), n_T, t, r, c3base,
                                               k0, k1,
                                               segw, P, np, gb, ngr_own);
    if (j < half)
        update_site<LAYOUT, ACC, SPLIT, RNG, false, NPC>(sm, class_site<SEP>(sm.ord, j, c, L, invH, invL), N, gw, g0, n_T, t, r,
                                                        c3base, k0, k1, segw, fd, P, np, gb, ngr_own);
}

// One colour class with plane draws: sites in wave-uniform rounds so that
// every lane takes part in the list's ballots, then the wave finishes its
// list before the class barrier.  `slist` = the odd-L site list (NULL:
// checkerboard class c of an even lattice, `count` sites); otherwise entries
// first..first+count-1 of it.  ACC (the summing class of an even lattice, one
// word per site): once the wave's list is empty its sites are final, and each
// lane adds the unsatisfied incidences of its sites, recounted from the
// updated spins, into its bit-plane counters.
template <bool SPLIT, bool ACC = false, int NPC = 0, int SEP = 0>
__device__ void class_pass_planes(const Smem &sm, int c, int tid, int nthr, int count, const uint32_t *slist,
                                  int first, int L, float invH, float invL, int N, int gw, int g0, int n_T, uint32_t t,
                                  uint32_t r, uint32_t c3base, uint32_t k0, uint32_t k1, int gb, int ngr_own,
                                  uint32_t (*P)[8] = nullptr, int np = 0)
{
    const int lane = tid & 63;
    PlaneQueue q = plane_queue(sm, tid >> 6);
    for (int jb = tid - lane; jb < count; jb += nthr) {   // the same trip count for the whole wave
        const int j = jb + lane;
        const bool live = j < count;
        const int jj = live ? j : 0;
        const Nbrs nb = slist ? neighbours_packed(slist[first + jj], L) : class_site<SEP>(sm.ord, jj, c, L, invH, invL);
        update_site_planes<SPLIT>(sm, q, live, nb, N, gw, g0, c, n_T, t, r, c3base, k0, k1, gb, ngr_own, lane);
    }
    while (q.count > 0) plane_drain(sm, q, lane, N, g0, c, t, r, c3base, k0, k1);
    if (ACC) {
        // a wave's list holds only its own sites: once it is empty they are final
        for (int j = tid; j < count; j += nthr) {
            const Nbrs nb = class_site<SEP>(sm.ord, j, c, L, invH, invL);
            const uint32_t j6 = sm.j6[nb.i];
            const uint32_t *sw = sm.spin;
            const uint32_t S = sw[nb.i];
            const uint32_t e0 = xor3(S, sw[nb.xp], (0u - (j6 & 1u)));
            const uint32_t e1 = xor3(S, sw[nb.xm], (0u - ((j6 >> 1) & 1u)));
            const uint32_t e2 = xor3(S, sw[nb.yp], (0u - ((j6 >> 2) & 1u)));
            const uint32_t e3 = xor3(S, sw[nb.ym], (0u - ((j6 >> 3) & 1u)));
            const uint32_t e4 = xor3(S, sw[nb.zp], (0u - ((j6 >> 4) & 1u)));
            const uint32_t e5 = xor3(S, sw[nb.zm], (0u - ((j6 >> 5) & 1u)));
            const uint32_t s1 = xor3(e0, e1, e2), c1 = maj3(e0, e1, e2);
            const uint32_t s2 = xor3(e3, e4, e5), c2 = maj3(e3, e4, e5);
            const uint32_t kk = s1 & s2;
            planes_add3<NPC>(*P, s1 ^ s2, xor3(c1, c2, kk), maj3(c1, c2, kk), np);
        }
    }
}

template <int LAYOUT, bool ACC, bool SPLIT, int RNG, int NPC = 0, int SEP = 0>
__device__ __forceinline__ void class_pass(const Smem &sm, int c, int tid, int nthr, int half, int L, float invH,
                                           float invL, int N, int NW, int gw, int g0, int n_T, uint32_t t, uint32_t r,
                                           uint32_t c3base, uint32_t k0, uint32_t k1, uint32_t segw, const Field &fd,
                                           uint32_t (*P)[8], int np, int gb, int ngr_own)
{
    if constexpr (LAYOUT == 0 && RNG == 1) {
        class_pass_planes<SPLIT, ACC, NPC, SEP>(sm, c, tid, nthr, half, nullptr, 0, L, invH, invL, N, gw, g0, n_T, t,
                                                r, c3base, k0, k1, gb, ngr_own, P, np);
        return;
    } else {
    if (SPLIT && LAYOUT == 0 && NW == 1 && !fd.on) {
        const int ng = ngr_own;
#define EA_PASS(G) class_pass_ng<LAYOUT, ACC, SPLIT, RNG, NPC, G, SEP>(sm, c, tid, nthr, half, L, invH, invL, N, gw, g0, \
                       n_T, t, r, c3base, k0, k1, segw, fd, P, np, gb, ngr_own)
        switch (ng) {
            case 1: EA_PASS(1); return;
            case 2: EA_PASS(2); return;
            case 3: EA_PASS(3); return;
            default: EA_PASS(4); return;   // a split ladder owns at most four groups
        }
#undef EA_PASS
    }
    for (int j = tid; j < half; j += nthr)
        update_site<LAYOUT, ACC, SPLIT, RNG, false, NPC>(sm, class_site<SEP>(sm.ord, j, c, L, invH, invL), N, gw, g0, n_T, t, r,
                                                        c3base, k0, k1, segw, fd, P, np, gb, ngr_own);
    }
}

template <int LAYOUT>
__device__ __forceinline__ void count_unsat_word(const Order &o, const uint32_t *words, const uint8_t *j6, int N, int L,
                                                 float invH, float invL,
                                                 int slot0, int n_T, int np, int *U)
{
    switch (np) {
        case 2: count_unsat_word_np<LAYOUT, 2>(o, words, j6, N, L, invH, invL, slot0, n_T, U); break;
        case 3: count_unsat_word_np<LAYOUT, 3>(o, words, j6, N, L, invH, invL, slot0, n_T, U); break;
        case 4: count_unsat_word_np<LAYOUT, 4>(o, words, j6, N, L, invH, invL, slot0, n_T, U); break;
        case 5: count_unsat_word_np<LAYOUT, 5>(o, words, j6, N, L, invH, invL, slot0, n_T, U); break;
        case 6: count_unsat_word_np<LAYOUT, 6>(o, words, j6, N, L, invH, invL, slot0, n_T, U); break;
        case 7: count_unsat_word_np<LAYOUT, 7>(o, words, j6, N, L, invH, invL, slot0, n_T, U); break;
        default: count_unsat_word_np<LAYOUT, 8>(o, words, j6, N, L, invH, invL, slot0, n_T, U); break;
    }
}


// Spins up per slot for one word, added into U[slot0 + b] (the same plane
// counters and wave reduction as the bond counts, one bit per site).
template <int LAYOUT, int NP>
__device__ void count_up_word_np(const uint32_t *words, int N, int slot0, int n_T, int *U)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr int STR = Layout<LAYOUT>::kStride;
    uint32_t P[14];
#pragma unroll
    for (int p = 0; p < 14; ++p) P[p] = 0;
    for (int idx = threadIdx.x; idx < N; idx += blockDim.x) {
        uint32_t carry = words[idx] & Layout<LAYOUT>::kKeep;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const uint32_t tt = P[p] & carry;
            P[p] ^= carry;
            carry = tt;
        }
    }
    reduce_planes_add<NP, STR>(P, min(SPW, n_T - slot0), U + slot0);
}

template <int LAYOUT>
__device__ __forceinline__ void count_up_word(const uint32_t *words, int N, int slot0, int n_T, int np, int *U)
{
    switch (np) {
        case 2: count_up_word_np<LAYOUT, 2>(words, N, slot0, n_T, U); break;
        case 3: count_up_word_np<LAYOUT, 3>(words, N, slot0, n_T, U); break;
        case 4: count_up_word_np<LAYOUT, 4>(words, N, slot0, n_T, U); break;
        case 5: count_up_word_np<LAYOUT, 5>(words, N, slot0, n_T, U); break;
        case 6: count_up_word_np<LAYOUT, 6>(words, N, slot0, n_T, U); break;
        case 7: count_up_word_np<LAYOUT, 7>(words, N, slot0, n_T, U); break;
        default: count_up_word_np<LAYOUT, 8>(words, N, slot0, n_T, U); break;
    }
}

// ---------------------------------------------------------------------------
// Sweep kernel.
//
// PARTS = 1: persistent workgroups pulling ladders from a queue (units[k] =
// job << 20 | ladder).  With PARTS > 1, UNITS = false runs one job's ladders
// in order (job 0, ladder = list index) and UNITS = true reads the list.
// PARTS > 1 (CAMSC, one word per site, even L): PARTS workgroups share a
// ladder, each holding all of its words in LDS but deciding only its own slot
// groups.  At a swap point they publish their slots' energies through a
// double-buffered exchange in HBM (64-bit words tagged with the sweep index,
// so readers need no fence; the wait is bounded and a timeout is reported
// through an error flag, so a launch always ends), then all run the identical
// swap pass.  Workgroups take tickets from one of eight queues, queue
// blockIdx mod 8, and the PARTS consecutive tickets of a queue are the parts
// of one ladder (blocks are meant to be dealt to the eight XCDs round robin,
// which would put partners on one XCD; nothing relies on it: the exchange
// words are agent-scope atomics, coherent across XCDs).
// Tickets go to workgroups in the order they start: only the most recently
// opened ladder of a queue can lack a part, so the launch needs no
// co-residency guarantee to make progress, only PARTS workgroups per queue.
// ---------------------------------------------------------------------------
constexpr uint32_t kSpinLimit = 1u << 20;   // polls of a partner's flag before giving up

// A pair with draw dr swaps at energy-difference index n (against the
// temperatures' order) when n < len and dr < tab[n].  The table does not
// increase with n (the host checks it), so those n are a prefix of the
// table: the cut returned is the first n whose threshold is at or below dr
// (len if there is none), and the test becomes n < cut.
__device__ __forceinline__ int swap_cut(const uint32_t *tab, int len, uint32_t dr)
{
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tab[mid] > dr)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// The pairs' swap draws of the swap point after sweep tswap, taken by one
// wave ahead of the swap step (the class barriers in between publish them):
// with the tables in LDS each pair's cut (swap_cut), else the draw itself
// (a search over a table in HBM would hold that wave up for longer than the
// swap step saves).
__device__ __forceinline__ void swap_draws_ahead(const Smem &sm, const uint32_t *stab, bool cuts, int n_T,
                                                 uint32_t tswap, uint32_t r, uint32_t c3swap, uint32_t k0, uint32_t k1,
                                                 int wave, int nwaves, int lane)
{
    if (n_T > 1 && wave == (nwaves >> 1) && lane < n_T - 1) {
        const uint32_t dr = philox10((uint32_t)lane, tswap, r, c3swap, k0, k1).x;
        sm.draw[lane] = cuts ? (uint32_t)swap_cut(stab + sm.soff[lane], sm.slen[lane], dr) : dr;
    }
}

// The ascending swap pass of one ladder once every slot's value is in U and
// the pairs' draws are in `draw` (both in LDS; with CUT, `draw` holds each
// pair's cut instead, see swap_cut): acceptance words over all (start, pair)
// combinations, then the walk over the rejections in wave 0, which moves the
// temperature rows to their new slots.  Ends after a barrier; U is consumed
// (zero again).  (CUT is a template argument: a run-time choice inside the
// pass measured 1.8% slower at PT after every sweep.)
template <bool CUT>
__device__ __forceinline__ void swap_pass_words(const Smem &sm, const uint32_t *stab, int n_T, int wave, int nwaves,
                                                int lane)
{
    const int pairs = n_T - 1;
    // Bit k of col[j]: would pair k swap if the configuration that
    // sat at position j before the pass had been carried up to k
    // (j <= k)?  Waves take start positions j in turn, lanes the
    // pairs k, so one ballot is col[j].  No data-dependent branch:
    // a pair's table length is uniform and a non-empty table has
    // entry 0.
    {
        const int k = lane;
        const bool live = k < pairs;
        const int kk = live ? k : 0;
        const int u_next = sm.U[sm.sot[kk + 1]];
        const int sg = sm.ssgn[kk];
        const int len = sm.slen[kk];
        const int off = sm.soff[kk];
        const uint32_t dr = sm.draw[kk];
        const int u_here = sm.U[sm.sot[lane < n_T ? lane : 0]];   // lane j: energy at position j
        for (int j = wave; j < pairs; j += nwaves) {
            const int d = __builtin_amdgcn_readlane(u_here, j) - u_next;
            const int n = d < 0 ? -d : d;
            const bool favourable = (sg == 0) || (d == 0) || ((sg > 0) == (d > 0));
            bool by_draw;
            if constexpr (CUT) {
                by_draw = n < (int)dr;
            } else {
                const uint32_t thr = len > 0 ? stab[off + min(n, len - 1)] : 0u;
                by_draw = n < len && dr < thr;
            }
            const bool acc = live && k >= j && (favourable || by_draw);
            const uint64_t col = __ballot(acc);
            if (lane == 0) sm.mask[j] = col;
        }
    }
    __syncthreads();
    if (wave == 0) {
        // The ascending pass, visiting only its rejections: from
        // restart point j the next rejected pair is the first k >= j
        // whose bit is clear in col[j], and after a rejection at k
        // the carried configuration restarts at k + 1.
        const uint64_t col = sm.mask[lane];
        sm.mask[lane] = 0ull;   // consumed; ready for the next swap point
        const uint64_t open = ~col & ((1ull << pairs) - 1ull) & (~0ull << lane);   // pairs <= 63
        const int nr = open ? (int)__builtin_ctzll(open) : 64;
        // a run of pairs rejected right at their restart point is one step
        const uint64_t imm = __ballot(lane < pairs && !((col >> lane) & 1ull));
        uint64_t rej = 0;
        int cj = 0;
        for (;;) {   // cj grows every turn: at most `pairs` turns
            const int run = __builtin_ctzll(~(imm >> cj));   // imm has no bit at or above pairs
            rej |= ((1ull << run) - 1ull) << cj;
            cj += run;
            const int r = __builtin_amdgcn_readlane(nr, cj);
            if (r >= pairs) break;
            rej |= 1ull << r;
            cj = r + 1;
        }
        // lane k: pair k accepted -> the configuration from position k+1
        // comes down; rejected -> the carried one stays (it started at the
        // last restart point at or below k)
        int src;
        if (lane < pairs && !((rej >> lane) & 1ull)) {
            src = lane + 1;
        } else {
            const uint64_t starts = ((rej << 1) | 1ull) & (lane >= 63 ? ~0ull : ((2ull << lane) - 1ull));
            src = 63 - __clzll((long long)starts);
        }
        if (lane == pairs) src = cj;
        const int newslot = lane < n_T ? sm.sot[src] : 0;
        if (lane < pairs && src == lane + 1) sm.acc[lane] += 1u;
        if (lane < n_T) {
            sm.sot[lane] = newslot;
            sm.perm[newslot] = lane;
            // the slot now at temperature `lane` takes that temperature's row
            const uint4 *from = (const uint4 *)(sm.fthr + lane * kThrCols);
            uint4 *to = (uint4 *)(sm.thr + newslot * kThrCols);
#pragma unroll
            for (int c = 0; c < kThrCols / 4; ++c) to[c] = from[c];
        }
        sm.U[lane] = 0;   // consumed
    }
    __syncthreads();
}


template <int LAYOUT, int PARTS, int RNG, bool UNITS = false, int SEP = 0>
__global__ void __launch_bounds__(kMaxBlock) sweep_kernel(const JobDesc *__restrict__ jobs,
                                                          const uint32_t *__restrict__ units, int n_units,
                                                          uint32_t *queue)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr bool SPLIT = PARTS > 1;
    // Split ladders with word draws run the swap pass in wave 0 alone while
    // the other waves draw the next sweep's first colour class.
    constexpr bool PREDRAW = SPLIT && RNG == 0;
    static_assert(!SPLIT || LAYOUT == 0, "split ladders are CAMSC only");
    static_assert(RNG == 0 || LAYOUT == 0, "plane draws are CAMSC only");
    static_assert(SEP == 0 || (LAYOUT == 0 && !UNITS), "the class order runs lone CAMSC launches only");
    extern __shared__ __align__(16) uint8_t smem_raw[];
    __shared__ uint32_t s_next;

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nwaves = nthr >> 6;

    for (int iter = 0;; ++iter) {
        uint32_t unit;
        int part = 0;
        if (SPLIT) {
            // one ticket per workgroup: the grid gives every queue as many
            // workgroups as its ladders have parts
            if (iter > 0) break;
            const uint32_t xq = blockIdx.x & 7u;
            if (tid == 0) s_next = atomicAdd(queue + xq, 1u);
            __syncthreads();
            const uint32_t tk = __builtin_amdgcn_readfirstlane(s_next);
            __syncthreads();
            part = (int)(tk % (uint32_t)PARTS);
            const uint32_t li = (tk / (uint32_t)PARTS) * 8u + xq;   // this queue's (tk / PARTS)-th ladder
            if (li >= (uint32_t)n_units) break;   // its partners' tickets are past the end too
            // a lone job's ladders in order need no list (and an index the
            // compiler can recompute keeps fewer registers live than a loaded one)
            unit = UNITS ? units[li] : li;
        } else {
            if (tid == 0) s_next = atomicAdd(queue, 1u);
            __syncthreads();
            const uint32_t u = __builtin_amdgcn_readfirstlane(s_next);
            __syncthreads();
            if (u >= (uint32_t)n_units) break;
            unit = units[u];
        }
        const JobDesc &jd = jobs[unit >> 20];
        const int ladder = unit & 0xFFFFF;
        const int N = jd.N, L = jd.L, NW = jd.NW, WR = jd.words_resident, n_T = jd.n_T;
        const bool even = (L & 1) == 0;
        const float invL = jd.invL, invH = jd.invH;
        const uint32_t r = (uint32_t)(ladder >> 1);
        const uint32_t copy = (uint32_t)(ladder & 1);
        const uint32_t c3flip = ((RNG == 1 ? kDomainPlane : kDomainFlip) << 28) | (copy << 24);
        const uint32_t c3swap = (kDomainSwap << 28) | (copy << 24);
        const uint32_t k0 = jd.key0, k1 = jd.key1;
        const uint32_t segw = jd.seg_bits;
        const int n_swap_lds = jd.swap_lds, n_sites_lds = jd.sites_lds;
        const Smem sm = carve(smem_raw, N, WR, n_swap_lds, n_sites_lds, RNG == 1 ? kPlaneItemBytes : 0u, SEP);
        uint32_t *g_spin = jd.spins + (size_t)ladder * NW * N;
        const int n_groups = (NW + WR - 1) / WR;

        // couplings, tables and permutation of this ladder
        const uint8_t *g_j6 = jd.j6 + (size_t)r * N;
        for (int idx = tid; idx < N; idx += nthr) sm.j6[idx] = g_j6[natural_of(sm.ord, idx, L, invH, invL)];
        for (int idx = tid; idx < n_T * kThrCols; idx += nthr) sm.fthr[idx] = jd.flip_thr[idx];
        for (int idx = tid; idx < n_swap_lds; idx += nthr) sm.stab[idx] = jd.swap_thr[idx];
        for (int idx = tid; idx < n_sites_lds; idx += nthr) sm.sites[idx] = jd.sites[idx];
        if (tid < kMaxTemps) {
            sm.perm[tid] = tid < n_T ? jd.temp_of_slot[ladder * kMaxTemps + tid] : 0;
            sm.acc[tid] = 0;
            sm.U[tid] = 0;
            sm.up[tid] = 0;
            sm.mask[tid] = 0ull;
            sm.soff[tid] = jd.swap_off[tid];
            sm.slen[tid] = jd.swap_len[tid];
            sm.ssgn[tid] = jd.swap_sgn[tid];
        }
        if (n_groups == 1)
            for (int idx = tid; idx < N; idx += nthr) {
                const int nat = natural_of(sm.ord, idx, L, invH, invL);
                for (int w = 0; w < NW; ++w) sm.spin[(size_t)w * N + idx] = g_spin[(size_t)w * N + nat];
            }
        __syncthreads();
        if (tid < n_T) sm.sot[sm.perm[tid]] = tid;
        for (int idx = tid; idx < kMaxTemps * kThrCols; idx += nthr) {
            const int slot = idx / kThrCols;
            sm.thr[idx] = slot < n_T ? sm.fthr[sm.perm[slot] * kThrCols + (idx % kThrCols)] : 0u;
        }
        __syncthreads();
        if (RNG == 1) {
            build_ptab(sm, NW, wave, nwaves, lane);
            __syncthreads();
        }
        const uint32_t *stab = n_swap_lds ? sm.stab : jd.swap_thr;
        const bool cuts = n_swap_lds > 0;   // swap tests as cuts (swap_cut) when the tables sit in LDS
        const uint32_t *slist = n_sites_lds ? sm.sites : jd.sites;

        uint32_t t = __builtin_amdgcn_readfirstlane(*jd.sweep_ctr);
        int remaining = jd.n_sweeps;
        const int se = jd.swap_every;
        const int np = planes_for(N, nthr);
        const int half = N >> 1;
        // CAMSC on a bipartite lattice with every word resident: the slot
        // energies come out of the last colour class of the swap sweep
        const int np_b = planes_for_class(half, nthr);
        const Field fd = field_of(jd);
        const bool fused_energy = LAYOUT == 0 && even && NW == 1 && np_b <= 8 && !fd.on;
        // slot groups this workgroup decides (all of them unless split)
        const int ngr_own = SPLIT ? ((n_T + 3) >> 2) / PARTS : 0;
        const int gb = SPLIT ? part * ngr_own : 0;
        const int s_lo = SPLIT ? 4 * gb : 0;
        const int s_hi = SPLIT ? min(n_T, 4 * (gb + ngr_own)) : n_T;
        bool c0_done = false;   // class 0 of sweep t already ran (after the last swap pass)
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
            // this chunk's swap draws (cuts), off the swap step's path (the
            // split by slot groups with word draws draws them in its swap step)
            if (!PREDRAW && swap_now)
                swap_draws_ahead(sm, stab, cuts, n_T, t + (uint32_t)chunk - 1u, r, c3swap, k0, k1, wave, nwaves, lane);
            uint32_t P[1][8];
#pragma unroll
            for (int p = 0; p < 8; ++p) P[0][p] = 0u;
            for (int g0 = 0; g0 < NW; g0 += WR) {
                const int gw = min(WR, NW - g0);
                if (n_groups > 1) {
                    for (int idx = tid; idx < N; idx += nthr) {
                        const int nat = natural_of(sm.ord, idx, L, invH, invL);
                        for (int w = 0; w < gw; ++w) sm.spin[(size_t)w * N + idx] = g_spin[(size_t)(g0 + w) * N + nat];
                    }
                    __syncthreads();
                }
                for (int s = 0; s < chunk; ++s) {
                    const uint32_t ts = t + (uint32_t)s;
                    if (even) {
                        if (!(PREDRAW && s == 0 && c0_done)) {
                            class_pass<LAYOUT, false, SPLIT, RNG, 0, SEP>(sm, 0, tid, nthr, half, L, invH, invL, N, NW, gw, g0,
                                                                  n_T, ts, r, c3flip, k0, k1, segw, fd, nullptr, 0, gb,
                                                                  ngr_own);
                            __syncthreads();
                        }
                        if (fused_energy && swap_now && s == chunk - 1) {
                            if (RNG == 0 && np_b == 4)   // at most two sites per lane
                                class_pass<LAYOUT, true, SPLIT, RNG, 4, SEP>(sm, 1, tid, nthr, half, L, invH, invL, N, NW,
                                                                        gw, g0, n_T, ts, r, c3flip, k0, k1, segw, fd, P,
                                                                        np_b, gb, ngr_own);
                            else
                                class_pass<LAYOUT, true, SPLIT, RNG, 0, SEP>(sm, 1, tid, nthr, half, L, invH, invL, N, NW, gw,
                                                                     g0, n_T, ts, r, c3flip, k0, k1, segw, fd, P, np_b,
                                                                     gb, ngr_own);
                        } else {
                            class_pass<LAYOUT, false, SPLIT, RNG, 0, SEP>(sm, 1, tid, nthr, half, L, invH, invL, N, NW, gw, g0,
                                                                  n_T, ts, r, c3flip, k0, k1, segw, fd, nullptr, 0, gb,
                                                                  ngr_own);
                        }
                        // after the summing class a wave goes straight on to reduce its
                        // own counters (registers and atomics on U only); the barrier
                        // that follows the reduction covers the spins as well
                        if (!(fused_energy && swap_now && s == chunk - 1)) __syncthreads();
                    } else {
                        for (int c = 0; c < jd.n_classes; ++c) {
                            const int beg = jd.class_off[c], end = jd.class_off[c + 1];
                            if constexpr (RNG == 1)
                                class_pass_planes<false>(sm, c, tid, nthr, end - beg, slist, beg, L, invH, invL, N, gw,
                                                         g0, n_T, ts, r, c3flip, k0, k1, 0, 0);
                            else
                                for (int it = beg + tid; it < end; it += nthr)
                                    update_site<LAYOUT, false, false, RNG>(sm, neighbours_packed(slist[it], L), N, gw,
                                                                          g0, n_T, ts, r, c3flip, k0, k1, segw, fd);
                            __syncthreads();
                        }
                    }
                }
                if (swap_now) {
                    if (fused_energy) {
                        if (np_b == 4 && s_hi - s_lo <= 16)
                            reduce_planes4_bytes_add(P[0], s_hi - s_lo, sm.U, s_lo);
                        else
                            reduce_planes8_add<1>(P[0], np_b, s_hi - s_lo, sm.U, s_lo);
                    } else {
                        for (int w = 0; w < gw; ++w) {
                            count_unsat_word<LAYOUT>(sm.ord, sm.spin + (size_t)w * N, sm.j6, N, L, invH, invL,
                                                     (g0 + w) * SPW, n_T, np, sm.U);
                            if (fd.on) count_up_word<LAYOUT>(sm.spin + (size_t)w * N, N, (g0 + w) * SPW, n_T, np, sm.up);
                        }
                    }
                }
                if (n_groups > 1) {
                    __syncthreads();
                    for (int idx = tid; idx < N; idx += nthr) {
                        const int nat = natural_of(sm.ord, idx, L, invH, invL);
                        for (int w = 0; w < gw; ++w) g_spin[(size_t)(g0 + w) * N + nat] = sm.spin[(size_t)w * N + idx];
                    }
                }
            }
            c0_done = false;
            if (swap_now && n_T > 1) {
                // ---- replica-exchange pass after sweep t + chunk - 1 ----
                const uint32_t tswap = t + (uint32_t)chunk - 1u;
                const int pairs = n_T - 1;
                if constexpr (PREDRAW) {
                    // Wave 0 publishes this workgroup's slot values and draws the
                    // next sweep's first colour class (as every wave does) before
                    // it collects the partners' values; then all waves compute the
                    // acceptance words and wave 0 walks the pass.
                    __syncthreads();   // own slots' energies are complete
                    const bool next = remaining > chunk;
                    const uint32_t tag = tswap + 1u;
                    uint64_t *xb = jd.xchg + ((size_t)ladder * 2 + ((tswap / (uint32_t)se) & 1u)) * kMaxTemps;
                    int u = 0;
                    if (wave == 0) {
                        u = sm.U[lane];
                        if (fd.on) u = (4 * u - jd.field_m * sm.up[lane]) / jd.field_g;   // W, as below
                        if (lane >= s_lo && lane < s_hi)
                            __hip_atomic_store(&xb[lane], ((uint64_t)tag << 32) | (uint32_t)u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (wave == nwaves - 1 && lane < pairs)
                        sm.draw[lane] = philox10((uint32_t)lane, tswap, r, c3swap, k0, k1).x;
                    // the next sweep's draws at this thread's first site of class 0
                    // now, at its second one while wave 0 walks the pass
                    U4 st[2][4];
                    const uint32_t tn = tswap + 1u, c3n = c3flip + (uint32_t)gb;
                    if (next && tid < half) {
                        switch (ngr_own) {
                            case 4: predraw_site<4>(st[0], tid, L, invH, invL, tn, r, c3n, k0, k1); break;
                            case 3: predraw_site<3>(st[0], tid, L, invH, invL, tn, r, c3n, k0, k1); break;
                            case 2: predraw_site<2>(st[0], tid, L, invH, invL, tn, r, c3n, k0, k1); break;
                            default: predraw_site<1>(st[0], tid, L, invH, invL, tn, r, c3n, k0, k1); break;
                        }
                    }
                    if (wave == 0) {
                        if (lane < n_T && (lane < s_lo || lane >= s_hi)) {
                            uint32_t spins = 0;
                            uint64_t v;
                            while ((uint32_t)((v = __hip_atomic_load(&xb[lane], __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT)) >> 32) != tag) {
                                if (++spins > kSpinLimit ||
                                    ((spins & 255u) == 0u &&
                                     __hip_atomic_load(jd.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
                                    atomicOr(jd.error, 1u);
                                    v = 0;
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(1);
                            }
                            u = (int32_t)(uint32_t)v;
                        }
                        sm.U[lane] = u;   // every slot's value (n_T <= 32 here: one word per site)
                    }
                    __syncthreads();   // slot values and the pairs' draws are in
                    {
                        // acceptance words: wave w takes the ballots i = w, w + nwaves, ... < 16
                        const int k = lane & 31, hf = lane >> 5;
                        const bool live = k < pairs;
                        const int kk = live ? k : 0;
                        const int u_next = sm.U[sm.sot[kk + 1]];
                        const int sg = sm.ssgn[kk], len = sm.slen[kk], off = sm.soff[kk];
                        const uint32_t drk = sm.draw[kk];
                        for (int i = wave; i < 16; i += nwaves) {
                            const int j = 2 * i + hf;
                            const int uj = sm.U[sm.sot[j < n_T ? j : 0]];
                            const uint64_t b =
                                n_swap_lds ? swap_ballot<false>(sm.stab, uj, u_next, drk, sg, len, off, k, j, live)
                                           : swap_ballot<true>(jd.swap_thr, uj, u_next, drk, sg, len, off, k, j, live);
                            if (lane == 0) sm.mask[i] = b;
                        }
                    }
                    __syncthreads();   // acceptance words are in
                    if (wave == 0) {
                        // lane j: col[j]; the ascending pass over its rejections, as below
                        const uint64_t w2 = sm.mask[lane >> 1];
                        const uint32_t colv = lane < 32 ? ((lane & 1) ? (uint32_t)(w2 >> 32) : (uint32_t)w2) : 0u;
                        const uint32_t open = lane < 32 ? ~colv & ((1u << pairs) - 1u) & (~0u << lane) : 0u;
                        const int nr = open ? (int)__builtin_ctz(open) : 64;
                        // pairs rejected right at their restart point: a run of them is
                        // taken in one step (common among the low temperatures)
                        const uint32_t imm = (uint32_t)__ballot(lane < pairs && !((colv >> lane) & 1u));
                        uint32_t rej = 0;
                        int cj = 0;
                        for (;;) {   // cj grows every turn: at most `pairs` turns
                            const int run = __builtin_ctz(~(imm >> cj));   // imm has no bit at or above pairs
                            rej |= ((1u << run) - 1u) << cj;
                            cj += run;
                            const int rr = __builtin_amdgcn_readlane(nr, cj);
                            if (rr >= pairs) break;
                            rej |= 1u << rr;
                            cj = rr + 1;
                        }
                        int src;
                        if (lane < pairs && !((rej >> lane) & 1u)) {
                            src = lane + 1;
                        } else {
                            const uint32_t starts = ((rej << 1) | 1u) & (lane >= 31 ? ~0u : ((2u << lane) - 1u));
                            src = 31 - __clz((int)starts);
                        }
                        if (lane == pairs) src = cj;
                        const int newslot = lane < n_T ? sm.sot[src] : 0;
                        if (lane < pairs && src == lane + 1) sm.acc[lane] += 1u;
                        if (lane < n_T) {
                            sm.sot[lane] = newslot;
                            sm.perm[newslot] = lane;
                            const uint4 *from = (const uint4 *)(sm.fthr + lane * kThrCols);
                            uint4 *to = (uint4 *)(sm.thr + newslot * kThrCols);
#pragma unroll
                            for (int c = 0; c < kThrCols / 4; ++c) to[c] = from[c];
                        }
                        sm.U[lane] = 0;   // consumed
                        sm.up[lane] = 0;
                    }
                    if (next && tid + nthr < half) {
                        const int j1 = tid + nthr;
                        switch (ngr_own) {
                            case 4: predraw_site<4>(st[1], j1, L, invH, invL, tn, r, c3n, k0, k1); break;
                            case 3: predraw_site<3>(st[1], j1, L, invH, invL, tn, r, c3n, k0, k1); break;
                            case 2: predraw_site<2>(st[1], j1, L, invH, invL, tn, r, c3n, k0, k1); break;
                            default: predraw_site<1>(st[1], j1, L, invH, invL, tn, r, c3n, k0, k1); break;
                        }
                    }
                    __syncthreads();   // temperature rows of the new permutation are in
                    if (next) {
                        // class 0 of the next sweep (so that the blocks need not
                        // stay live across the loop)
                        int j0 = tid;
                        asm volatile("" : "+v"(j0));   // as in predraw_site
                        if (j0 + nthr < half && !fd.on) {   // both sites in one block, as in class_pass
                            const Nbrs na = class_site<SEP>(sm.ord, j0, 0, L, invH, invL);
                            const Nbrs nb = class_site<SEP>(sm.ord, j0 + nthr, 0, L, invH, invL);
#define EA_PAIR(G) update_pair_camsc<false, SPLIT, G, 0, PREDRAW>(sm, na, nb, n_T, tn, r, c3flip, k0, k1, segw, \
                                                                 nullptr, 0, gb, ngr_own, st[0], st[1])
                            switch (ngr_own) {
                                case 1: EA_PAIR(1); break;
                                case 2: EA_PAIR(2); break;
                                case 3: EA_PAIR(3); break;
                                default: EA_PAIR(4); break;
                            }
#undef EA_PAIR
                        } else {
                            if (j0 < half)
                                update_site<LAYOUT, false, SPLIT, RNG, PREDRAW>(sm, class_site<SEP>(sm.ord, j0, 0, L, invH, invL),
                                                                                N, 1, 0, n_T, tn, r, c3flip, k0, k1,
                                                                                segw, fd, nullptr, 0, gb, ngr_own,
                                                                                st[0]);
                            if (j0 + nthr < half)
                                update_site<LAYOUT, false, SPLIT, RNG, PREDRAW>(sm, class_site<SEP>(sm.ord, j0 + nthr, 0, L,
                                                                                               invH, invL),
                                                                                N, 1, 0, n_T, tn, r, c3flip, k0, k1,
                                                                                segw, fd, nullptr, 0, gb, ngr_own,
                                                                                st[1]);
                        }
                        for (int j = tid + 2 * nthr; j < half; j += nthr)
                            update_site<LAYOUT, false, SPLIT, RNG>(sm, class_site<SEP>(sm.ord, j, 0, L, invH, invL), N, 1, 0, n_T,
                                                                  tn, r, c3flip, k0, k1, segw, fd, nullptr, 0, gb,
                                                                  ngr_own);
                        __syncthreads();
                        c0_done = true;
                    }
                } else {
                    if (fd.on) {
                        // with a field the slot value is W = (4U - m up) / g, so that
                        // 2 (E_a - E_b) = g (W_a - W_b) (exact: g divides both terms)
                        __syncthreads();
                        if (tid < kMaxTemps) {
                            sm.U[tid] = (4 * sm.U[tid] - jd.field_m * sm.up[tid]) / jd.field_g;
                            sm.up[tid] = 0;
                        }
                    }
                    if (SPLIT) {
                        // Publish own slots' energies and collect the partners'.
                        // Each word carries its sweep tag, so plain relaxed
                        // atomics suffice: no fence, no cache write-back.
                        __syncthreads();   // own energies are complete
                        const uint32_t tag = tswap + 1u;
                        uint64_t *xb = jd.xchg + ((size_t)ladder * 2 + ((tswap / (uint32_t)se) & 1u)) * kMaxTemps;
                        if (tid >= s_lo && tid < s_hi)
                            __hip_atomic_store(&xb[tid], ((uint64_t)tag << 32) | (uint32_t)sm.U[tid], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        if (tid < n_T && (tid < s_lo || tid >= s_hi)) {
                            uint32_t spins = 0;
                            uint64_t v;
                            // bounded: after any timeout (error set) nobody waits long again
                            while ((uint32_t)((v = __hip_atomic_load(&xb[tid], __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT)) >> 32) != tag) {
                                if (++spins > kSpinLimit ||
                                    ((spins & 255u) == 0u &&
                                     __hip_atomic_load(jd.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
                                    atomicOr(jd.error, 1u);
                                    v = 0;
                                    break;
                                }
                                __builtin_amdgcn_s_sleep(1);
                            }
                            sm.U[tid] = (int32_t)(uint32_t)v;
                        }
                    }
                    __syncthreads();   // slot energies U are in (the pairs' draws since the chunk began)
                    if (cuts)
                        swap_pass_words<true>(sm, stab, n_T, wave, nwaves, lane);
                    else
                        swap_pass_words<false>(sm, stab, n_T, wave, nwaves, lane);
                    if (RNG == 1) {
                        build_ptab(sm, NW, wave, nwaves, lane);
                        __syncthreads();
                    }
                }
            } else if (swap_now) {
                __syncthreads();
                if (tid < kMaxTemps) {
                    sm.U[tid] = 0;
                    sm.up[tid] = 0;
                }
                __syncthreads();
            }
            t += (uint32_t)chunk;
            remaining -= chunk;
        }
        if (SPLIT) {
            // merge own slots' bits: the partners change disjoint bits, so the xors commute
            const uint32_t own = (ngr_own >= 8 ? 0xFFFFFFFFu : ((1u << (4 * ngr_own)) - 1u)) << s_lo;
            for (int idx = tid; idx < N; idx += nthr) {
                const int nat = natural_of(sm.ord, idx, L, invH, invL);
                const uint32_t delta = (sm.spin[idx] ^ g_spin[nat]) & own;
                if (delta) atomicXor(&g_spin[nat], delta);
            }
        } else if (n_groups == 1) {
            for (int idx = tid; idx < N; idx += nthr) {
                const int nat = natural_of(sm.ord, idx, L, invH, invL);
                for (int w = 0; w < NW; ++w) g_spin[(size_t)w * N + nat] = sm.spin[(size_t)w * N + idx];
            }
        }
        if (tid < n_T && part == 0) {
            jd.temp_of_slot[ladder * kMaxTemps + tid] = sm.perm[tid];
            if (tid < n_T - 1) jd.swap_acc[ladder * kMaxTemps + tid] += sm.acc[tid];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Ladders split by lattice halves (CAMSC, word draws, one word per site, even
// L >= 4, no field, natural order).  Two workgroups share a ladder: part p
// owns the planes z0 = p L/2 .. z0 + L/2 - 1 with every slot, so that no bond
// word, site index or random block is formed twice (a split by slot groups
// forms every site's bond words in each part).  A part keeps its planes and
// one halo plane on either side in LDS (LDS plane zl + 1 holds local plane zl
// = -1 .. L/2).  Each site of its first or last plane publishes its new word,
// tagged with the sweep index, as soon as it is updated; before its own
// update it takes the one halo word it needs, the partner's newest word of the
// other class across the boundary (the partner's last plane lies below this
// part's first, its first plane above this part's last).  So the halves meet
// word by word and only where they touch, and no class waits for the whole
// boundary.  At a swap point each part's slot energies are sums over its own
// sites of the summing class; the parts exchange and add them (the next
// sweep's first draws are made meanwhile) and run the identical swap pass.
// Tickets as in sweep_kernel with two parts.
// ---------------------------------------------------------------------------
struct Slab {
    int L, H, LL, hp, hc, z0;   // H = L / 2 planes, hp = L L / 2 sites of a class per plane, hc = H hp
    float invH, invL;
};

// Item j (0 <= j < hc) of class c in a part: local plane zl = j / hp, then
// row y and the x of the class's parity; LDS indices with the halo planes.
__device__ __forceinline__ Nbrs slab_site(const Slab &s, int j, int c)
{
    const int w = qdiv(j, s.invH);   // y + L zl
    const int xh = j - w * (s.L >> 1);
    const int zl = qdiv(w, s.invL);
    const int y = w - zl * s.L;
    const int x = 2 * xh + ((c + y + s.z0 + zl) & 1);
    const int row = x + s.L * y;
    Nbrs n;
    n.i = row + s.LL * (zl + 1);
    n.g = row + s.LL * (s.z0 + zl);
    n.xp = (x == s.L - 1) ? n.i - (s.L - 1) : n.i + 1;
    n.xm = (x == 0) ? n.i + (s.L - 1) : n.i - 1;
    n.yp = (y == s.L - 1) ? n.i - (s.L - 1) * s.L : n.i + s.L;
    n.ym = (y == 0) ? n.i + (s.L - 1) * s.L : n.i - s.L;
    n.zp = n.i + s.LL;
    n.zm = n.i - s.LL;
    return n;
}

// The low word of a tagged 64-bit word once its tag has arrived.  Bounded like
// the energy exchange: after a timeout (error set) nobody waits long again and
// the value is 0.
__device__ __forceinline__ uint32_t wait_tagged(const uint64_t *w, uint32_t tag, uint32_t *error)
{
    uint32_t spins = 0;
    uint64_t v;
    while ((uint32_t)((v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 32) != tag) {
        if (++spins > kSpinLimit ||
            ((spins & 255u) == 0u && __hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
            atomicOr(error, 1u);
            return 0u;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return (uint32_t)v;
}

// The blocks of item j of class 0 at sweep t for all eight slot groups of the
// word (those past the ladder go unused), drawn during a swap step: the swap
// pass changes thresholds, not draws.  A fixed count keeps the blocks in
// registers.
__device__ __forceinline__ void slab_predraw(U4 (&st)[8], uint32_t site, uint32_t t, uint32_t r, uint32_t c3,
                                             uint32_t k0, uint32_t k1)
{
    asm volatile("" : "+v"(site));   // as in predraw_site: keep the rounds where they are written
#pragma unroll
    for (int q = 0; q < 8; ++q) st[q] = philox10(site, t, r, c3 + (uint32_t)q, k0, k1);
}

// The part of a CAMSC site update that needs only the spins (one word per
// site, no field), as in update_site: the site's word S, its segment words X
// (segment j of X[k] = 2E+S of slot 4j + k) and the certain flips (E >= 3).
struct CamscPrep {
    uint32_t S, always;
    uint32_t X[4];
};

__device__ __forceinline__ CamscPrep camsc_prepare(const Smem &sm, const Nbrs &nb)
{
    const uint32_t j6 = sm.j6[nb.i];
    const uint32_t *sw = sm.spin;
    CamscPrep p;
    p.S = sw[nb.i];
    const uint32_t e0 = xor3(p.S, sw[nb.xp], (0u - (j6 & 1u)));
    const uint32_t e1 = xor3(p.S, sw[nb.xm], (0u - ((j6 >> 1) & 1u)));
    const uint32_t e2 = xor3(p.S, sw[nb.yp], (0u - ((j6 >> 2) & 1u)));
    const uint32_t e3 = xor3(p.S, sw[nb.ym], (0u - ((j6 >> 3) & 1u)));
    const uint32_t e4 = xor3(p.S, sw[nb.zp], (0u - ((j6 >> 4) & 1u)));
    const uint32_t e5 = xor3(p.S, sw[nb.zm], (0u - ((j6 >> 5) & 1u)));
    const uint32_t s1 = xor3(e0, e1, e2), c1 = maj3(e0, e1, e2);
    const uint32_t s2 = xor3(e3, e4, e5), c2 = maj3(e3, e4, e5);
    const uint32_t E0 = s1 ^ s2, kk = s1 & s2;
    const uint32_t E1 = xor3(c1, c2, kk), E2 = maj3(c1, c2, kk);
    p.X[0] = p.S;
    p.X[1] = E0;
    p.X[2] = E1;
    p.X[3] = E2;
    swap_bits(p.X[0], p.X[2], 2, 0x33333333u);
    swap_bits(p.X[1], p.X[3], 2, 0x33333333u);
    swap_bits(p.X[0], p.X[1], 1, 0x55555555u);
    swap_bits(p.X[2], p.X[3], 1, 0x55555555u);
    p.always = E2 | (E1 & E0);
    return p;
}

// The rest: decisions against the rows by slot with the blocks drawn
// beforehand; returns the new spin word.
__device__ __forceinline__ uint32_t camsc_finish(const Smem &sm, const CamscPrep &p, int n_T, const Ctr &c,
                                                 const U4 *pre)
{
    const int ngr = n_T >= 32 ? 8 : (n_T + 3) >> 2;
    const uint32_t valid = n_T >= 32 ? 0xFFFFFFFFu : ((1u << n_T) - 1u);
    uint32_t F;
    switch (ngr) {
        case 8: F = camsc_decide<8, true>(p.X, sm.thr, 0u, c, pre); break;
        case 7: F = camsc_decide<7, true>(p.X, sm.thr, 0u, c, pre); break;
        case 6: F = camsc_decide<6, true>(p.X, sm.thr, 0u, c, pre); break;
        case 5: F = camsc_decide<5, true>(p.X, sm.thr, 0u, c, pre); break;
        case 4: F = camsc_decide<4, true>(p.X, sm.thr, 0u, c, pre); break;
        case 3: F = camsc_decide<3, true>(p.X, sm.thr, 0u, c, pre); break;
        case 2: F = camsc_decide<2, true>(p.X, sm.thr, 0u, c, pre); break;
        default: F = camsc_decide<1, true>(p.X, sm.thr, 0u, c, pre); break;
    }
    return p.S ^ ((F | p.always) & valid);
}

// Where item j of a class sits on the part's boundary: first plane (side 0),
// last plane (side 1) or neither; k = its index within that plane.
struct SlabEdge {
    bool first, last;
    int k;
};

__device__ __forceinline__ SlabEdge slab_edge(const Slab &g, int j)
{
    SlabEdge e;
    e.first = j < g.hp;
    e.last = j >= g.hc - g.hp;   // exclusive with first: L/2 >= 2 planes
    e.k = e.first ? j : j - (g.hc - g.hp);
    return e;
}

// One colour class of a part at sweep t, items j0, j0 + nthr, ...  mine =
// this part's words of class c (side 0 = its first plane, side 1 = its last),
// theirs = the partner's words of the other class, whose newest tag is `want`;
// with poll = false (the launch's first class) the halo planes loaded from HBM
// are current.  A site on the first or last plane reads one halo cell, which
// only it reads, and its wave runs at a raised priority: its words are the
// partner's halo.  (Its blocks drawn while the partner's word travels measured
// faster without a swap step but slower with one: the extra live registers
// spill.)  With ACC the sites' bond counts after the update go into the plane
// counters P (the summing class).
template <bool ACC>
__device__ __forceinline__ void slab_class(const Smem &sm, const Slab &g, int c, int j0, int nthr, int NL, int n_T,
                                           uint32_t t, uint32_t r, uint32_t c3flip, uint32_t k0, uint32_t k1,
                                           uint32_t segw, uint64_t *mine, const uint64_t *theirs, uint32_t want,
                                           bool poll, uint32_t *error, uint32_t (*P)[8], int np)
{
    const Field fd{false, 0u, 0u, 0, 0};
    const uint64_t tag = (uint64_t)(t + 1u) << 32;
    for (int j = j0; j < g.hc; j += nthr) {
        const Nbrs nb = slab_site(g, j, c);
        const SlabEdge e = slab_edge(g, j);
        const bool edge = __ballot(e.first || e.last) != 0ull;
        if (edge) __builtin_amdgcn_s_setprio(2);
        if (poll && (e.first || e.last))
            sm.spin[e.first ? nb.zm : nb.zp] = wait_tagged(&theirs[e.first ? g.hp + e.k : e.k], want, error);
        update_site<0, ACC>(sm, nb, NL, 1, 0, n_T, t, r, c3flip, k0, k1, segw, fd, P, np);
        if (e.first || e.last)
            __hip_atomic_store(&mine[e.first ? e.k : g.hp + e.k], tag | sm.spin[nb.i], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (edge) __builtin_amdgcn_s_setprio(0);
    }
}

// One colour class of a part with plane draws (as class_pass_planes): items
// in wave-uniform rounds, each boundary site first taking its halo word; once
// a wave's list of undecided halves is empty its sites are final, and it
// publishes its boundary words and (ACC, the summing class) adds the bond
// counts of its sites into the plane counters P.
template <bool ACC>
__device__ void slab_class_planes(const Smem &sm, const Slab &g, int c, int tid, int nthr, int NL, int n_T,
                                  uint32_t t, uint32_t r, uint32_t c3base, uint32_t k0, uint32_t k1, uint64_t *mine,
                                  const uint64_t *theirs, uint32_t want, bool poll, uint32_t *error,
                                  uint32_t (*P)[8], int np)
{
    const int lane = tid & 63;
    PlaneQueue q = plane_queue(sm, (int)(threadIdx.x >> 6));   // tid may start past the first nthr sites
    for (int jb = tid - lane; jb < g.hc; jb += nthr) {   // the same trip count for the whole wave
        const int j = jb + lane;
        const bool live = j < g.hc;
        const Nbrs nb = slab_site(g, live ? j : 0, c);
        const SlabEdge e = slab_edge(g, j);
        if (live && poll && (e.first || e.last))
            sm.spin[e.first ? nb.zm : nb.zp] = wait_tagged(&theirs[e.first ? g.hp + e.k : e.k], want, error);
        update_site_planes<false>(sm, q, live, nb, NL, 1, 0, c, n_T, t, r, c3base, k0, k1, 0, 0, lane);
    }
    while (q.count > 0) plane_drain(sm, q, lane, NL, 0, c, t, r, c3base, k0, k1);
    const uint64_t tag = (uint64_t)(t + 1u) << 32;
    for (int j = tid; j < g.hc; j += nthr) {
        const SlabEdge e = slab_edge(g, j);
        if (!ACC && !(e.first || e.last)) continue;
        const Nbrs nb = slab_site(g, j, c);
        const uint32_t *sw = sm.spin;
        const uint32_t S = sw[nb.i];
        if (e.first || e.last)
            __hip_atomic_store(&mine[e.first ? e.k : g.hp + e.k], tag | S, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ACC) {
            const uint32_t j6 = sm.j6[nb.i];
            const uint32_t e0 = xor3(S, sw[nb.xp], (0u - (j6 & 1u)));
            const uint32_t e1 = xor3(S, sw[nb.xm], (0u - ((j6 >> 1) & 1u)));
            const uint32_t e2 = xor3(S, sw[nb.yp], (0u - ((j6 >> 2) & 1u)));
            const uint32_t e3 = xor3(S, sw[nb.ym], (0u - ((j6 >> 3) & 1u)));
            const uint32_t e4 = xor3(S, sw[nb.zp], (0u - ((j6 >> 4) & 1u)));
            const uint32_t e5 = xor3(S, sw[nb.zm], (0u - ((j6 >> 5) & 1u)));
            const uint32_t s1 = xor3(e0, e1, e2), c1 = maj3(e0, e1, e2);
            const uint32_t s2 = xor3(e3, e4, e5), c2 = maj3(e3, e4, e5);
            const uint32_t kk = s1 & s2;
            planes_add3<0>(*P, s1 ^ s2, xor3(c1, c2, kk), maj3(c1, c2, kk), np);
        }
    }
}

// Plane draws ahead of a swap step (split by lattice halves, one word per
// site): a site's bond sums, its E >= 3 mask and the first-round blocks of its
// halves (block 0 of each), none of which depends on the temperatures.
struct PlanePrep {
    uint32_t S, always, m1, m2, und;
    U4 a, b;
};

__device__ __forceinline__ PlanePrep plane_prepare(const Smem &sm, const Nbrs &nb, int n_T, uint32_t t, uint32_t r,
                                                   uint32_t c3base, uint32_t k0, uint32_t k1)
{
    PlanePrep p;
    const uint32_t *sw = sm.spin;
    const uint32_t j6 = sm.j6[nb.i];
    p.S = sw[nb.i];
    const uint32_t e0 = xor3(p.S, sw[nb.xp], (0u - (j6 & 1u)));
    const uint32_t e1 = xor3(p.S, sw[nb.xm], (0u - ((j6 >> 1) & 1u)));
    const uint32_t e2 = xor3(p.S, sw[nb.yp], (0u - ((j6 >> 2) & 1u)));
    const uint32_t e3 = xor3(p.S, sw[nb.ym], (0u - ((j6 >> 3) & 1u)));
    const uint32_t e4 = xor3(p.S, sw[nb.zp], (0u - ((j6 >> 4) & 1u)));
    const uint32_t e5 = xor3(p.S, sw[nb.zm], (0u - ((j6 >> 5) & 1u)));
    const uint32_t s1 = xor3(e0, e1, e2), c1 = maj3(e0, e1, e2);
    const uint32_t s2 = xor3(e3, e4, e5), c2 = maj3(e3, e4, e5);
    const uint32_t E0 = s1 ^ s2, kk = s1 & s2;
    const uint32_t E1 = xor3(c1, c2, kk), E2 = maj3(c1, c2, kk);
    p.always = E2 | (E1 & E0);   // E >= 3
    p.m1 = E0 & ~E1;
    p.m2 = E1 & ~E0;
    const uint32_t valid = n_T >= 32 ? 0xFFFFFFFFu : ((1u << n_T) - 1u);
    p.und = valid & ~p.always;
    p.a = philox10((uint32_t)nb.g, t, r, c3base, k0, k1);
    p.b = n_T > 16 ? philox10((uint32_t)nb.g, t, r, c3base + (1u << 8), k0, k1) : p.a;
    return p;
}

// The prepared site's first round against the thresholds after the swap pass
// (update_site_planes with the blocks drawn); undecided halves go to the
// wave's list.  Every lane of the wave calls it; `live` lanes hold a site.
__device__ __forceinline__ void plane_finish(const Smem &sm, PlaneQueue &q, bool live, PlanePrep p, int site, int i0,
                                             int NL, int n_T, uint32_t t, uint32_t r, uint32_t c3base, uint32_t k0,
                                             uint32_t k1, int lane)
{
    const uint32_t valid = n_T >= 32 ? 0xFFFFFFFFu : ((1u << n_T) - 1u);
    uint32_t und = live ? p.und : 0u, m1 = live ? p.m1 : 0u, m2 = live ? p.m2 : 0u;
    if (live) {
        const uint32_t lt = n_T > 16 ? planes8_compare<2>(und, m1, m2, sm.ptab, p.a, p.b, 0)
                                     : planes8_compare<1>(und, m1, m2, sm.ptab, p.a, p.a, 0);
        sm.spin[i0] = p.S ^ ((lt | p.always) & valid);
    }
    const uint32_t key = (uint32_t)site | (1u << 18);
    plane_push(q, und & 0xFFFFu, m1 & 0xFFFFu, m2 & 0xFFFFu, key);
    while (q.count > kItemFlush) plane_drain(sm, q, lane, NL, 0, 0, t, r, c3base, k0, k1);
    if (n_T > 16) {
        plane_push(q, und >> 16, m1 >> 16, m2 >> 16, key | (1u << 17));
        while (q.count > kItemFlush) plane_drain(sm, q, lane, NL, 0, 0, t, r, c3base, k0, k1);
    }
}

template <bool UNITS, int RNG>
__global__ void __launch_bounds__(kMaxBlock) slab_kernel(const JobDesc *__restrict__ jobs,
                                                         const uint32_t *__restrict__ units, int n_units,
                                                         uint32_t *queue)
{
    extern __shared__ __align__(16) uint8_t smem_raw[];
    __shared__ uint32_t s_next;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nwaves = nthr >> 6;

    // one ticket per workgroup: the two consecutive tickets of a queue are the
    // halves of one ladder (see sweep_kernel)
    const uint32_t xq = blockIdx.x & 7u;
    if (tid == 0) s_next = atomicAdd(queue + xq, 1u);
    __syncthreads();
    const uint32_t tk = __builtin_amdgcn_readfirstlane(s_next);
    const int part = (int)(tk & 1u);
    const uint32_t li = (tk >> 1) * 8u + xq;
    if (li >= (uint32_t)n_units) return;   // the partner's ticket is past the end too
    const uint32_t unit = UNITS ? units[li] : li;
    const JobDesc &jd = jobs[unit >> 20];
    const int ladder = unit & 0xFFFFF;
    const int L = jd.L, N = jd.N, n_T = jd.n_T;
    Slab g;
    g.L = L;
    g.H = L >> 1;
    g.LL = L * L;
    g.hp = g.LL >> 1;
    g.hc = g.H * g.hp;
    g.z0 = part * g.H;
    g.invH = jd.invH;
    g.invL = jd.invL;
    const int NL = (g.H + 2) * g.LL;   // own planes and the two halo planes
    const uint32_t r = (uint32_t)(ladder >> 1);
    const uint32_t copy = (uint32_t)(ladder & 1);
    const uint32_t c3flip = ((RNG == 1 ? kDomainPlane : kDomainFlip) << 28) | (copy << 24);
    const uint32_t c3swap = (kDomainSwap << 28) | (copy << 24);
    const uint32_t k0 = jd.key0, k1 = jd.key1;
    const uint32_t segw = jd.seg_bits;
    const int n_swap_lds = jd.swap_lds;
    Smem sm = carve(smem_raw, NL, 1, n_swap_lds, 0, RNG == 1 ? kPlaneItemBytes : 0u, 0);
    sm.ord.base = (g.z0 - 1) * g.LL;   // own site g sits at LDS word g - base
    uint32_t *g_spin = jd.spins + (size_t)ladder * N;
    const uint8_t *g_j6 = jd.j6 + (size_t)r * N;
    uint64_t *hx = jd.halo + (size_t)ladder * 8u * (uint32_t)g.hp;   // [part][class][side][hp]

    for (int idx = tid; idx < NL; idx += nthr) {
        const int pl = qdiv(qdiv(idx, g.invL), g.invL);   // LDS plane: local plane pl - 1
        int zg = g.z0 + pl - 1;
        zg = zg < 0 ? zg + L : (zg >= L ? zg - L : zg);
        const int nat = idx + (zg - pl) * g.LL;
        sm.spin[idx] = g_spin[nat];
        sm.j6[idx] = g_j6[nat];
    }
    for (int idx = tid; idx < n_T * kThrCols; idx += nthr) sm.fthr[idx] = jd.flip_thr[idx];
    for (int idx = tid; idx < n_swap_lds; idx += nthr) sm.stab[idx] = jd.swap_thr[idx];
    if (tid < kMaxTemps) {
        sm.perm[tid] = tid < n_T ? jd.temp_of_slot[ladder * kMaxTemps + tid] : 0;
        sm.acc[tid] = 0;
        sm.U[tid] = 0;
        sm.up[tid] = 0;
        sm.mask[tid] = 0ull;
        sm.soff[tid] = jd.swap_off[tid];
        sm.slen[tid] = jd.swap_len[tid];
        sm.ssgn[tid] = jd.swap_sgn[tid];
    }
    __syncthreads();
    if (tid < n_T) sm.sot[sm.perm[tid]] = tid;
    for (int idx = tid; idx < kMaxTemps * kThrCols; idx += nthr) {
        const int slot = idx / kThrCols;
        sm.thr[idx] = slot < n_T ? sm.fthr[sm.perm[slot] * kThrCols + (idx % kThrCols)] : 0u;
    }
    __syncthreads();
    if (RNG == 1) {
        build_ptab(sm, 1, wave, nwaves, lane);
        __syncthreads();
    }
    const uint32_t *stab = n_swap_lds ? sm.stab : jd.swap_thr;
    const bool cuts = n_swap_lds > 0;   // swap tests as cuts (swap_cut) when the tables sit in LDS

    uint32_t t = __builtin_amdgcn_readfirstlane(*jd.sweep_ctr);
    int remaining = jd.n_sweeps;
    const int se = jd.swap_every;
    const int np_b = planes_for_class(g.hc, nthr);   // at most 8 (the host checks)
    const int other = 1 - part;
    bool poll = false;     // the launch's first class reads the halo planes loaded from HBM
    bool c0_done = false;  // class 0 of sweep t already ran (after the last swap pass)
    U4 st[8];
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
        // this chunk's swap draws (cuts), off the swap step's path
        if (swap_now) swap_draws_ahead(sm, stab, cuts, n_T, t + (uint32_t)chunk - 1u, r, c3swap, k0, k1, wave, nwaves, lane);
        uint32_t P[1][8];
#pragma unroll
        for (int p = 0; p < 8; ++p) P[0][p] = 0u;
        for (int s = 0; s < chunk; ++s) {
            const uint32_t ts = t + (uint32_t)s;
            for (int c = 0; c < 2; ++c) {
                if (c == 0 && s == 0 && c0_done) continue;
                uint64_t *mine = hx + (size_t)((part * 2 + c) * 2) * g.hp;
                const uint64_t *theirs = hx + (size_t)((other * 2 + 1 - c) * 2) * g.hp;
                const uint32_t want = c == 0 ? ts : ts + 1u;   // the partner's last class-(1 - c) update
                if (c == 1 && swap_now && s == chunk - 1) {
                    if constexpr (RNG == 1)
                        slab_class_planes<true>(sm, g, c, tid, nthr, NL, n_T, ts, r, c3flip, k0, k1, mine, theirs,
                                                want, poll, jd.error, P, np_b);
                    else
                        slab_class<true>(sm, g, c, tid, nthr, NL, n_T, ts, r, c3flip, k0, k1, segw, mine, theirs, want,
                                         poll, jd.error, P, np_b);
                    reduce_planes8_add<1>(P[0], np_b, n_T, sm.U, 0);
                } else {
                    if constexpr (RNG == 1)
                        slab_class_planes<false>(sm, g, c, tid, nthr, NL, n_T, ts, r, c3flip, k0, k1, mine, theirs,
                                                 want, poll, jd.error, nullptr, 0);
                    else
                        slab_class<false>(sm, g, c, tid, nthr, NL, n_T, ts, r, c3flip, k0, k1, segw, mine, theirs, want,
                                          poll, jd.error, nullptr, 0);
                }
                poll = true;
                __syncthreads();
            }
        }
        c0_done = false;
        if (swap_now && n_T > 1) {
            // this part's energies are complete (the class barrier); add the partner's
            const uint32_t tswap = t + (uint32_t)chunk - 1u;
            const uint32_t tag = tswap + 1u;
            const uint32_t tn = tswap + 1u;
            const bool next = remaining > chunk;
            uint64_t *xb = jd.xchg + ((size_t)ladder * 2 + ((tswap / (uint32_t)se) & 1u)) * kMaxTemps;
            if (tid < n_T)
                __hip_atomic_store(&xb[part * 32 + tid], ((uint64_t)tag << 32) | (uint32_t)sm.U[tid],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // While the sums travel: this thread's first class-0 site of the next
            // sweep takes its halo word, draws its blocks and forms its segment
            // words (none of which depends on the temperatures); after the swap
            // pass only its decisions remain.
            // (plane draws: the bond sums and the first-round blocks of the site)
            const bool ahead = next && tid < g.hc;
            const SlabEdge e0 = slab_edge(g, tid);
            CamscPrep prep;
            PlanePrep pp;
            int i0 = 0, site0 = 0;
            if (ahead) {
                const Nbrs nb = slab_site(g, tid, 0);
                if (e0.first || e0.last)
                    sm.spin[e0.first ? nb.zm : nb.zp] = wait_tagged(
                        hx + (size_t)(other * 4 + 2) * g.hp + (e0.first ? g.hp + e0.k : e0.k), tn, jd.error);
                if constexpr (RNG == 0) {
                    slab_predraw(st, (uint32_t)nb.g, tn, r, c3flip, k0, k1);
                    prep = camsc_prepare(sm, nb);
                } else {
                    pp = plane_prepare(sm, nb, n_T, tn, r, c3flip, k0, k1);
                }
                i0 = nb.i;
                site0 = nb.g;
            }
            if (tid < n_T) sm.U[tid] += (int32_t)wait_tagged(&xb[other * 32 + tid], tag, jd.error);
            __syncthreads();   // slot energies U are in (the pairs' draws since the chunk began)
            if (cuts)
                swap_pass_words<true>(sm, stab, n_T, wave, nwaves, lane);
            else
                swap_pass_words<false>(sm, stab, n_T, wave, nwaves, lane);
            if (RNG == 1) {
                build_ptab(sm, 1, wave, nwaves, lane);
                __syncthreads();
            }
            if (next) {
                // class 0 of the next sweep: the first sites only decide
                uint64_t *mine = hx + (size_t)(part * 4) * g.hp;
                if constexpr (RNG == 0) {
                    if (ahead) {
                        const Ctr cc{tn, r, c3flip, k0, k1, segw};
                        const uint32_t v = camsc_finish(sm, prep, n_T, cc, st);
                        sm.spin[i0] = v;
                        if (e0.first || e0.last)
                            __hip_atomic_store(&mine[e0.first ? e0.k : g.hp + e0.k], ((uint64_t)(tn + 1u) << 32) | v,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    slab_class<false>(sm, g, 0, tid + nthr, nthr, NL, n_T, tn, r, c3flip, k0, k1, segw, mine,
                                      hx + (size_t)(other * 4 + 2) * g.hp, tn, true, jd.error, nullptr, 0);
                } else {
                    // the list of undecided halves is empty before the boundary
                    // words go out (their late flips land from it)
                    PlaneQueue q = plane_queue(sm, wave);
                    plane_finish(sm, q, ahead, pp, site0, i0, NL, n_T, tn, r, c3flip, k0, k1, lane);
                    while (q.count > 0) plane_drain(sm, q, lane, NL, 0, 0, tn, r, c3flip, k0, k1);
                    if (ahead && (e0.first || e0.last))
                        __hip_atomic_store(&mine[e0.first ? e0.k : g.hp + e0.k],
                                           ((uint64_t)(tn + 1u) << 32) | sm.spin[i0], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    slab_class_planes<false>(sm, g, 0, tid + nthr, nthr, NL, n_T, tn, r, c3flip, k0, k1, mine,
                                             hx + (size_t)(other * 4 + 2) * g.hp, tn, true, jd.error, nullptr, 0);
                }
                __syncthreads();
                c0_done = true;
            }
        } else if (swap_now) {
            if (tid < kMaxTemps) sm.U[tid] = 0;
            __syncthreads();
        }
        t += (uint32_t)chunk;
        remaining -= chunk;
    }
    // own planes back: they are contiguous in both orders
    for (int idx = g.LL + tid; idx < (g.H + 1) * g.LL; idx += nthr) g_spin[idx + (g.z0 - 1) * g.LL] = sm.spin[idx];
    if (tid < n_T && part == 0) {
        jd.temp_of_slot[ladder * kMaxTemps + tid] = sm.perm[tid];
        if (tid < n_T - 1) jd.swap_acc[ladder * kMaxTemps + tid] += sm.acc[tid];
    }
}

// Advance each job's sweep counter and re-arm the queues for the next launch.
__global__ void advance_kernel(const JobDesc *__restrict__ jobs, int n_jobs, uint32_t *queue)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_jobs) *jobs[j].sweep_ctr += (uint32_t)jobs[j].n_sweeps;
    if (j < kQueueWords) queue[j] = 0;
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
        U4 rr{0u, 0u, 0u, 0u};
        int cur = -1;
        for (int j = 0; j < SPW; ++j) {   // slot groups of 4 need not align with words (AMSC3)
            const int slot = w * SPW + j;
            if (slot >= jd.n_T) break;
            if ((slot >> 2) != cur) {
                cur = slot >> 2;
                rr = philox10((uint32_t)i, 0u, (uint32_t)(ladder >> 1), c3 | (uint32_t)cur, jd.key0, jd.key1);
            }
            const int q = slot & 3;
            const uint32_t v = q == 0 ? rr.x : (q == 1 ? rr.y : (q == 2 ? rr.z : rr.w));
            word |= (v & 1u) << (j * STR);
        }
        jd.spins[idx] = word;
    }
}

// ---------------------------------------------------------------------------
// Overlap measurement (Sec. 5: Binder ratio and correlation length of the
// spin-glass order): one workgroup per (realization, temperature index).
// q_i = +1 where the two copies at that temperature agree, -1 elsewhere; its
// plane sums along x, y and z are formed in LDS (a thread per x-line), and the
// measurement adds q^2, q^4 (as a 128-bit sum) and the plane-sum
// autocorrelation C[d] = sum_a sum_p Q_a[p] Q_a[(p + d) mod L] into
// accumulators that only this workgroup touches, so every sum is exact.
// ---------------------------------------------------------------------------
template <int LAYOUT>
__global__ void __launch_bounds__(256) measure_kernel(const JobDesc *__restrict__ jd_ptr, int64_t *count,
                                                      int64_t *sum_q2, uint64_t *sum_q4, int64_t *sum_c)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr int STR = Layout<LAYOUT>::kStride;
    __shared__ int s_Q[3][32];
    __shared__ int s_slot[2];
    const JobDesc &jd = *jd_ptr;
    const int n_T = jd.n_T, N = jd.N, L = jd.L, NW = jd.NW;
    const int r = blockIdx.x / n_T, k = blockIdx.x % n_T;
    const int tid = threadIdx.x;
    if (tid < 96) s_Q[tid / 32][tid % 32] = 0;
    if (tid < 2 * n_T) {
        const int c = tid / n_T, s = tid % n_T;
        if (jd.temp_of_slot[(2 * r + c) * kMaxTemps + s] == k) s_slot[c] = s;
    }
    __syncthreads();
    const int a = s_slot[0], b = s_slot[1];
    const uint32_t *wa = jd.spins + ((size_t)(2 * r) * NW + a / SPW) * N;
    const uint32_t *wb = jd.spins + ((size_t)(2 * r + 1) * NW + b / SPW) * N;
    const int sa = (a % SPW) * STR, sb = (b % SPW) * STR;
    for (int line = tid; line < L * L; line += blockDim.x) {
        const int y = line % L, z = line / L;
        int sum = 0;
        for (int x = 0; x < L; ++x) {
            const int i = x + L * line;
            const int qi = 1 - 2 * (int)(((wa[i] >> sa) ^ (wb[i] >> sb)) & 1u);
            sum += qi;
            atomicAdd(&s_Q[0][x], qi);
        }
        atomicAdd(&s_Q[1][y], sum);
        atomicAdd(&s_Q[2][z], sum);
    }
    __syncthreads();
    const size_t rk = (size_t)r * n_T + k;
    if (tid < L) {
        int64_t cd = 0;
        for (int ax = 0; ax < 3; ++ax)
            for (int p = 0; p < L; ++p) cd += (int64_t)s_Q[ax][p] * s_Q[ax][(p + tid) % L];
        sum_c[rk * L + tid] += cd;
    }
    if (tid == 0) {
        int64_t q = 0;
        for (int p = 0; p < L; ++p) q += s_Q[0][p];
        count[rk] += 1;
        sum_q2[rk] += q * q;
        const uint64_t q4 = (uint64_t)(q * q) * (uint64_t)(q * q);   // < 2^61 for N <= 2^15
        const uint64_t lo = sum_q4[2 * rk] + q4;
        sum_q4[2 * rk + 1] += lo < q4 ? 1u : 0u;
        sum_q4[2 * rk] = lo;
    }
}

// ---------------------------------------------------------------------------
// Measurement kernel (Sec. 4.1): one workgroup per realization.
// ---------------------------------------------------------------------------
template <int LAYOUT>
__global__ void __launch_bounds__(512) observables_kernel(const JobDesc *__restrict__ jd_ptr, int32_t *energy,
                                                          int32_t *overlap, int32_t *magnet)
{
    constexpr int SPW = Layout<LAYOUT>::kSlotsPerWord;
    constexpr int STR = Layout<LAYOUT>::kStride;
    __shared__ int s_U[2][kMaxTemps];
    __shared__ int s_diff[kMaxTemps];
    __shared__ int s_sot[2][kMaxTemps];
    __shared__ int s_up[2][kMaxTemps];
    const JobDesc &jd = *jd_ptr;
    const int r = blockIdx.x;
    const int N = jd.N, n_T = jd.n_T, NW = jd.NW;
    const int tid = threadIdx.x;
    if (tid < kMaxTemps) {
        s_U[0][tid] = s_U[1][tid] = 0;
        s_up[0][tid] = s_up[1][tid] = 0;
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
        {
            count_unsat_word<LAYOUT>(Order{0, N >> 1, 0}, jd.spins + ((size_t)(2 * r + c) * NW + w) * N, j6, N, jd.L,
                                     jd.invH, jd.invL, w * SPW, n_T, np, s_U[c]);   // HBM holds the natural order
            if (magnet) count_up_word<LAYOUT>(jd.spins + ((size_t)(2 * r + c) * NW + w) * N, N, w * SPW, n_T, np, s_up[c]);
        }
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
        if (magnet) magnet[((size_t)r * 2 + c) * n_T + k] = 2 * s_up[c][s_sot[c][k]] - N;
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
// Storage of a layout's words (AMSC1 words are CAMSC words).
static int storage_layout(int layout) { return layout == 3 ? 0 : layout; }

hipError_t launch_init_spins(const JobDesc *d_job, const JobDesc &h, int layout, hipStream_t s)
{
    const size_t total = (size_t)h.ladders * h.NW * h.N;
    // AMSC1 words are stored like CAMSC words
    switch (storage_layout(layout)) {
        case 0: hipLaunchKernelGGL(init_spins_kernel<0>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job); break;
        case 1: hipLaunchKernelGGL(init_spins_kernel<1>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job); break;
        default: hipLaunchKernelGGL(init_spins_kernel<2>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job); break;
    }
    return hipGetLastError();
}

// Sweep kernel variants: kv = 0 CAMSC, 1 AMSC4, 2 CAMSC with plane draws, 3 AMSC3, 4 AMSC1;
// split ladders (parts 2 or 4, CAMSC) read the unit list when `listed`; sep =
// spin words in LDS by colour class (lone CAMSC launches); kSlabVariant =
// ladders split by lattice halves (two parts).
static const void *sweep_fn(int kv, int parts, bool listed = false, int sep = 0)
{
    if (kv == kSlabVariant) return listed ? (const void *)slab_kernel<true, 0> : (const void *)slab_kernel<false, 0>;
    if (kv == kSlabPlanesVariant)
        return listed ? (const void *)slab_kernel<true, 1> : (const void *)slab_kernel<false, 1>;
    if (kv == 1) return (const void *)sweep_kernel<1, 1, 0>;
    if (kv == 3) return (const void *)sweep_kernel<2, 1, 0>;
    if (kv == 4) return (const void *)sweep_kernel<3, 1, 0>;
    if (sep) {
        if (kv == 2)
            return parts == 4 ? (const void *)sweep_kernel<0, 4, 1, false, 1>
                              : (parts == 2 ? (const void *)sweep_kernel<0, 2, 1, false, 1>
                                            : (const void *)sweep_kernel<0, 1, 1, false, 1>);
        return parts == 4 ? (const void *)sweep_kernel<0, 4, 0, false, 1>
                          : (parts == 2 ? (const void *)sweep_kernel<0, 2, 0, false, 1>
                                        : (const void *)sweep_kernel<0, 1, 0, false, 1>);
    }
    if (kv == 2) {
        if (parts == 4) return listed ? (const void *)sweep_kernel<0, 4, 1, true> : (const void *)sweep_kernel<0, 4, 1>;
        if (parts == 2) return listed ? (const void *)sweep_kernel<0, 2, 1, true> : (const void *)sweep_kernel<0, 2, 1>;
        return (const void *)sweep_kernel<0, 1, 1>;
    }
    if (parts == 4) return listed ? (const void *)sweep_kernel<0, 4, 0, true> : (const void *)sweep_kernel<0, 4, 0>;
    if (parts == 2) return listed ? (const void *)sweep_kernel<0, 2, 0, true> : (const void *)sweep_kernel<0, 2, 0>;
    return (const void *)sweep_kernel<0, 1, 0>;
}

hipError_t sweep_set_lds(int kv, int parts, size_t lds)
{
    // the attribute is process-wide per kernel; raise it only when a launch needs more
    static std::atomic<size_t> set_max[kSlabPlanesVariant + 1][3] = {};
    const int pi = parts == 4 ? 2 : (parts == 2 ? 1 : 0);
    std::atomic<size_t> &cur = set_max[kv][pi];
    if (lds <= cur.load()) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(sweep_fn(kv, parts), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess && parts > 1)
        e = hipFuncSetAttribute(sweep_fn(kv, parts, true), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess && (kv == 0 || kv == 2))
        e = hipFuncSetAttribute(sweep_fn(kv, parts, false, 1), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) {
        size_t prev = cur.load();
        while (prev < lds && !cur.compare_exchange_weak(prev, lds)) {
        }
    }
    return e;
}

hipError_t launch_sweep(const JobDesc *d_jobs, int n_jobs, const uint32_t *d_units, int n_units, uint32_t *d_queue,
                        int kv, int parts, int sep, int block_threads, size_t lds, int grid, hipStream_t s)
{
    hipError_t e = sweep_set_lds(kv, parts, lds);
    if (e != hipSuccess) return e;
    void *args[] = {(void *)&d_jobs, (void *)&d_units, (void *)&n_units, (void *)&d_queue};
    // one job's units are its ladders in order (a launch set of one job keeps them so)
    if (sep && (n_jobs > 1 || (kv != 0 && kv != 2))) return hipErrorInvalidValue;   // lone CAMSC launches only
    e = hipLaunchKernel(sweep_fn(kv, parts, n_jobs > 1, sep), dim3(grid), dim3(block_threads), args, lds, s);
    if (e != hipSuccess) return e;
    const int adv = n_jobs > kQueueWords ? n_jobs : kQueueWords;
    hipLaunchKernelGGL(advance_kernel, dim3((adv + 255) / 256), dim3(256), 0, s, d_jobs, n_jobs, d_queue);
    return hipGetLastError();
}

int sweep_max_blocks_per_cu(int kv, int parts, int block_threads, size_t lds)
{
    int n = 0, m = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sweep_fn(kv, parts), block_threads, lds);
    if (e == hipSuccess && parts > 1)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, sweep_fn(kv, parts, true), block_threads, lds);
    else
        m = n;
    return e == hipSuccess ? (n < m ? n : m) : 0;
}

hipError_t launch_observables(const JobDesc *d_job, const JobDesc &h, int layout, int32_t *d_energy,
                              int32_t *d_overlap, int32_t *d_magnet, hipStream_t s)
{
    const int R = h.ladders / 2;
    // AMSC1 words are stored like CAMSC words
    switch (storage_layout(layout)) {
        case 0: hipLaunchKernelGGL(observables_kernel<0>, dim3(R), dim3(512), 0, s, d_job, d_energy, d_overlap, d_magnet); break;
        case 1: hipLaunchKernelGGL(observables_kernel<1>, dim3(R), dim3(512), 0, s, d_job, d_energy, d_overlap, d_magnet); break;
        default: hipLaunchKernelGGL(observables_kernel<2>, dim3(R), dim3(512), 0, s, d_job, d_energy, d_overlap, d_magnet); break;
    }
    return hipGetLastError();
}

hipError_t launch_measure(const JobDesc *d_job, const JobDesc &h, int layout, int64_t *count, int64_t *sum_q2,
                          uint64_t *sum_q4, int64_t *sum_c, hipStream_t s)
{
    const int blocks = h.ladders / 2 * h.n_T;
    // AMSC1 words are stored like CAMSC words
    switch (storage_layout(layout)) {
        case 0: hipLaunchKernelGGL(measure_kernel<0>, dim3(blocks), dim3(256), 0, s, d_job, count, sum_q2, sum_q4, sum_c); break;
        case 1: hipLaunchKernelGGL(measure_kernel<1>, dim3(blocks), dim3(256), 0, s, d_job, count, sum_q2, sum_q4, sum_c); break;
        default: hipLaunchKernelGGL(measure_kernel<2>, dim3(blocks), dim3(256), 0, s, d_job, count, sum_q2, sum_q4, sum_c); break;
    }
    return hipGetLastError();
}

hipError_t launch_unpack(const JobDesc *d_job, const JobDesc &h, int layout, int8_t *d_spins, hipStream_t s)
{
    const size_t total = (size_t)h.ladders * h.n_T * h.N;
    // AMSC1 words are stored like CAMSC words
    switch (storage_layout(layout)) {
        case 0: hipLaunchKernelGGL(unpack_kernel<0>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins); break;
        case 1: hipLaunchKernelGGL(unpack_kernel<1>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins); break;
        default: hipLaunchKernelGGL(unpack_kernel<2>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins); break;
    }
    return hipGetLastError();
}

hipError_t launch_pack(const JobDesc *d_job, const JobDesc &h, int layout, const int8_t *d_spins, hipStream_t s)
{
    const size_t total = (size_t)h.ladders * h.NW * h.N;
    // AMSC1 words are stored like CAMSC words
    switch (storage_layout(layout)) {
        case 0: hipLaunchKernelGGL(pack_kernel<0>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins); break;
        case 1: hipLaunchKernelGGL(pack_kernel<1>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins); break;
        default: hipLaunchKernelGGL(pack_kernel<2>, dim3(grid_for(total, 256)), dim3(256), 0, s, d_job, d_spins); break;
    }
    return hipGetLastError();
}


}  // namespace ea
