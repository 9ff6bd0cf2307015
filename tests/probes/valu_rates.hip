// valu_rates.hip -- issue rate of the vector instructions the sweep kernel's
// operation count is made of, relative to a plain 32-bit XOR, on gfx950.
//
// Each lane runs CHAINS independent dependency chains of one instruction kind
// for ITERS iterations, so that with WAVES wavefronts per SIMD neither latency
// nor memory limits the issue; the result of every chain is stored, so no
// chain can be dropped. Rates are lane-instructions per second over the whole
// launch (HIP events), and each kind's rate is also given as a fraction of
// the 32-bit add rate measured in the same process (a full-rate instruction). The instruction counts per
// chain step are checked in the device assembly (hipcc -S) of this file:
//   kind 0 (add):     v_add_u32
//   kind 1 (bitop3):  v_bitop3_b32
//   kind 2 (mul_lo):  v_mul_lo_u32
//   kind 3 (mad_u64): v_mad_u64_u32
//
// Build and run:
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         tests/probes/valu_rates.hip -o valu_rates && ./valu_rates

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

constexpr int CHAINS = 8;
constexpr int ITERS = 4096;
constexpr int THREADS = 256;

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

template <int KIND>
__global__ void __launch_bounds__(THREADS) chains(uint32_t *out, uint32_t seed) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a[CHAINS], b[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
        a[c] = tid * 2654435761u + seed + c;
        b[c] = tid ^ (0x9E3779B9u * (c + 1));
    }
    for (int i = 0; i < ITERS; ++i) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) {
            if constexpr (KIND == 0) {
                a[c] = a[c] + b[c];
                b[c] = b[c] + a[c];
            } else if constexpr (KIND == 1) {
                a[c] = __builtin_amdgcn_bitop3_b32(a[c], b[c], seed, 0x96);
                b[c] = __builtin_amdgcn_bitop3_b32(b[c], a[c], seed, 0x96);
            } else if constexpr (KIND == 2) {
                a[c] = a[c] * b[c];
                b[c] = b[c] * a[c];
            } else {
                // (a:b) = lo32 * K + (a:b): the 64-bit accumulator is the pair itself
                uint64_t x = (static_cast<uint64_t>(a[c]) << 32) | b[c];
                x = static_cast<uint64_t>(static_cast<uint32_t>(x)) * 0xD2511F53u + x;
                x = static_cast<uint64_t>(static_cast<uint32_t>(x)) * 0xCD9E8D57u + x;
                a[c] = static_cast<uint32_t>(x >> 32);
                b[c] = static_cast<uint32_t>(x);
            }
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s ^= a[c] + b[c];
    out[tid] = s;
}

template <int KIND>
double rate(uint32_t *out, int blocks, hipEvent_t e0, hipEvent_t e1) {
    // warm-up, then one timed launch; 2 instructions per chain step
    hipLaunchKernelGGL(chains<KIND>, dim3(blocks), dim3(THREADS), 0, 0, out, 1u);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(chains<KIND>, dim3(blocks), dim3(THREADS), 0, 0, out, 2u);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double ops = 2.0 * CHAINS * ITERS * static_cast<double>(blocks) * THREADS;
    return ops / (ms * 1e-3);
}

int main() {
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    // 16 wavefronts per SIMD: 4 SIMDs x 16 x 64 lanes per CU
    const int blocks = cus * 4 * 16 * 64 / THREADS;
    uint32_t *out = nullptr;
    CHECK(hipMalloc(&out, static_cast<size_t>(blocks) * THREADS * sizeof(uint32_t)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const char *names[4] = {"v_add_u32", "v_bitop3_b32", "v_mul_lo_u32", "v_mad_u64_u32"};
    double r[4];
    r[0] = rate<0>(out, blocks, e0, e1);
    r[1] = rate<1>(out, blocks, e0, e1);
    r[2] = rate<2>(out, blocks, e0, e1);
    r[3] = rate<3>(out, blocks, e0, e1);
    // peak of full-rate 32-bit VALU issue: CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    // = CUs x 64 lanes x 2.4e9 lane-ops/s
    const double full = static_cast<double>(cus) * 64.0 * 2.4e9;
    std::printf("device %s, %d CUs, %d blocks of %d threads (16 waves/SIMD)\n", prop.gcnArchName,
                cus, blocks, THREADS);
    std::printf("%-15s %14s %10s %12s\n", "instruction", "lane-ops/s", "vs add", "vs 2.4GHz peak");
    for (int k = 0; k < 4; ++k)
        std::printf("%-15s %14.4e %10.3f %12.3f\n", names[k], r[k], r[k] / r[0], r[k] / full);
    CHECK(hipFree(out));
    return 0;
}
