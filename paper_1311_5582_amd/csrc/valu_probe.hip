// Issue-rate probe for the integer vector instructions the sweep kernel is
// priced in: v_bitop3_b32 (the three-input xor of a Philox round and of the
// bond words), v_xor_b32 / v_min_u32 (two-operand instructions), v_xad_u32,
// v_mad_u64_u32 (the 32x32->64 multiplies of a Philox round; the compiler
// pairs each with a v_mov_b32 of the 64-bit addend here) and v_mul_hi_u32,
// plus whole Philox4x32-10 blocks.  Each kernel runs eight dependency chains
// per lane; the logic chains mix a non-linear truth table in so that the
// compiler cannot fold them (an all-xor chain is linear and gets folded).
// Every wave also reads the shader clock (s_memtime) and the 100 MHz
// real-time counter around its loop, which gives the clock the kernel ran at.
// Built as its own small library (not part of the simulation ABI) and driven
// by bench.py --valu-rate.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 16;

// OP 0: v_bitop3_b32 (xor3 and a ^ (b | c) alternately), 1 per step
// OP 1: v_xor_b32 then v_min_u32, 2 per step (two-operand instructions)
// OP 2: v_xad_u32 (xor then add), 1 per step
// OP 3: v_mad_u64_u32 (multiply-with-carry step), 1 per step
// OP 4: v_mul_hi_u32, 1 per step (and a v_xor_b32)
template <int OP>
__global__ void __launch_bounds__(1024) chain_kernel(uint32_t *out, uint64_t *clk, int iters, uint32_t m)
{
    uint32_t x[kChains + 2];
#pragma unroll
    for (int c = 0; c < kChains + 2; ++c) x[c] = (threadIdx.x * 2654435761u) ^ (m * (c + 1)) ^ blockIdx.x;
    uint64_t r[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) r[c] = x[c];
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    const uint64_t rt0 = __builtin_amdgcn_s_memrealtime();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                if (OP == 0)
                    x[c] = (u & 1) ? __builtin_amdgcn_bitop3_b32(x[c], x[(c + 1) % kChains], x[kChains + 1], 0x96)
                                   : __builtin_amdgcn_bitop3_b32(x[c], x[(c + 1) % kChains], x[kChains], 0x1E);
                if (OP == 1) x[c] = min(x[c] ^ x[(c + 1) % kChains], x[kChains + (u & 1)]);
                if (OP == 2) x[c] = (x[c] ^ x[(c + 1) % kChains]) + x[kChains + (u & 1)];
                if (OP == 3) r[c] = (uint64_t)(uint32_t)r[c] * m + (r[c] >> 32);
                if (OP == 4) x[c] = __umulhi(x[c], m) ^ x[(c + 1) % kChains];
            }
    }
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    const uint64_t rt1 = __builtin_amdgcn_s_memrealtime();
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= x[c] ^ (uint32_t)r[c] ^ (uint32_t)(r[c] >> 32);
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    out[gid] = acc;
    if ((threadIdx.x & 63) == 0) {
        clk[2 * (gid >> 6)] = t1 - t0;
        clk[2 * (gid >> 6) + 1] = rt1 - rt0;
    }
}

// Philox4x32-10 (Salmon et al., SC'11) on per-lane counters, two blocks in flight per lane.
__global__ void __launch_bounds__(1024) philox_kernel(uint32_t *out, uint64_t *clk, int iters, uint32_t key)
{
    uint32_t acc = 0;
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t t0 = __builtin_amdgcn_s_memtime();
    const uint64_t rt0 = __builtin_amdgcn_s_memrealtime();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            uint32_t c0 = gid, c1 = (uint32_t)it, c2 = (uint32_t)b, c3 = acc;
            uint32_t k0 = key, k1 = key ^ 0x5bd1e995u;
#pragma unroll
            for (int rd = 0; rd < 10; ++rd) {
                const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
                const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
                const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
                const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
                c1 = (uint32_t)p1;
                c3 = (uint32_t)p0;
                c0 = n0;
                c2 = n2;
                k0 += 0x9E3779B9u;
                k1 += 0xBB67AE85u;
            }
            acc ^= c0 ^ c1 ^ c2 ^ c3;
        }
    }
    const uint64_t t1 = __builtin_amdgcn_s_memtime();
    const uint64_t rt1 = __builtin_amdgcn_s_memrealtime();
    out[gid] = acc;
    if ((threadIdx.x & 63) == 0) {
        clk[2 * (gid >> 6)] = t1 - t0;
        clk[2 * (gid >> 6) + 1] = rt1 - rt0;
    }
}

}  // namespace

extern "C" {

// Runs each probe (grid workgroups of 1024 threads, `iters` loop iterations)
// twice and reports the second run: rates[k] = lane-operations per second of
// probe k counted as the instructions named above (Philox: blocks per second),
// ms[k] = its duration from HIP events, ghz[k] = the shader clock over the
// waves' loops (s_memtime ticks / real-time ticks x 100 MHz).  Probes: 0
// bitop3, 1 xor+min, 2 xad, 3 mad_u64_u32 (+ mov), 4 mul_hi (+ xor), 5 Philox.
// Returns 0, or the first HIP error code.
int ea_probe_valu_rates(int grid, int iters, double *rates, double *ms, double *ghz)
{
    constexpr int kBlock = 1024;
    constexpr int kProbes = 6;
    const size_t threads = (size_t)grid * kBlock, waves = threads / 64;
    uint32_t *out = nullptr;
    uint64_t *clk = nullptr;
    hipError_t e = hipMalloc(&out, threads * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&clk, waves * 2 * sizeof(uint64_t));
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    // instructions per lane and loop iteration, counted in the probe's assembly
    const double per_iter[kProbes] = {kUnroll * kChains, 2.0 * kUnroll * kChains, kUnroll * kChains,
                                      kUnroll * kChains, kUnroll * kChains, 2.0};
    uint64_t *hclk = new uint64_t[waves * 2];
    for (int k = 0; k < kProbes && e == hipSuccess; ++k) {
        const int n_iter = k == 5 ? iters / 8 : iters;
        float t = 0.0f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            e = hipEventRecord(a, nullptr);
            if (e != hipSuccess) break;
            switch (k) {
                case 0: hipLaunchKernelGGL(chain_kernel<0>, dim3(grid), dim3(kBlock), 0, nullptr, out, clk, n_iter, 0x9E3779B9u); break;
                case 1: hipLaunchKernelGGL(chain_kernel<1>, dim3(grid), dim3(kBlock), 0, nullptr, out, clk, n_iter, 0x9E3779B9u); break;
                case 2: hipLaunchKernelGGL(chain_kernel<2>, dim3(grid), dim3(kBlock), 0, nullptr, out, clk, n_iter, 0x9E3779B9u); break;
                case 3: hipLaunchKernelGGL(chain_kernel<3>, dim3(grid), dim3(kBlock), 0, nullptr, out, clk, n_iter, 0xD2511F53u); break;
                case 4: hipLaunchKernelGGL(chain_kernel<4>, dim3(grid), dim3(kBlock), 0, nullptr, out, clk, n_iter, 0xCD9E8D57u); break;
                default: hipLaunchKernelGGL(philox_kernel, dim3(grid), dim3(kBlock), 0, nullptr, out, clk, n_iter, 0x1234567u); break;
            }
            e = hipGetLastError();
            if (e == hipSuccess) e = hipEventRecord(b, nullptr);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        }
        if (e == hipSuccess) e = hipMemcpy(hclk, clk, waves * 2 * sizeof(uint64_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) break;
        double cyc = 0.0, rt = 0.0;
        for (size_t w = 0; w < waves; ++w) {
            cyc += (double)hclk[2 * w];
            rt += (double)hclk[2 * w + 1];
        }
        if (ms) ms[k] = t;
        if (ghz) ghz[k] = rt > 0.0 ? cyc / rt * 0.1 : 0.0;
        rates[k] = (double)threads * n_iter * per_iter[k] / (t * 1e-3);
    }
    delete[] hclk;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (out) (void)hipFree(out);
    if (clk) (void)hipFree(clk);
    return (int)e;
}

}  // extern "C"
