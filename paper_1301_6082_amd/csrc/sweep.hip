// sweep.hip -- gfx950 kernels around the sweep: lattice fill, density
// reduction, device clock; and the dispatch of a phase launch to the phase
// kernel of the model (compiled per model in phase_n1.hip .. phase_n4.hip).

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pcpd_internal.h"

namespace pcpd {
namespace {

__global__ void fill_words(uint64_t *__restrict__ dst, uint64_t n, uint64_t value) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = value;
}

// Counts of one chunk of one ring: per-lane popcounts, a wavefront reduction
// through cross-lane shuffles, then one atomic per wavefront.
__global__ void __launch_bounds__(256)
density_chunks(const uint64_t *__restrict__ buf, const LatDesc *__restrict__ lats,
               const DenChunk *__restrict__ chunks, Counts *__restrict__ out) {
    const DenChunk ch = chunks[blockIdx.x];
    const LatDesc ld = lats[ch.lat];
    const uint64_t *ring = buf + ld.base;
    unsigned long long n = 0, np = 0, alive = 0;
    for (uint32_t i = threadIdx.x; i < ch.nw; i += blockDim.x) {
        const uint64_t j = ch.w0 + i;
        const uint64_t jn = (j + 1 == ld.L) ? 0 : j + 1;
        const uint64_t w = ring[j];
        uint64_t wn = ring[jn];
        // connected layout: after the last word of bit b comes the first word
        // of bit b+1 (site b*L + L-1 pairs with (b+1)*L)
        if (ld.connected && jn == 0) wn = (wn >> 1) | (wn << 63);
        n += __popcll(w);
        np += __popcll(w & wn);
        alive |= w;
    }
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) {
        n += __shfl_xor(n, sh);
        np += __shfl_xor(np, sh);
        alive |= __shfl_xor(alive, sh);
    }
    if ((threadIdx.x & 63u) == 0u) {
        atomicAdd(&out[ch.lat].n, n);
        atomicAdd(&out[ch.lat].n_pair, np);
        atomicOr(&out[ch.lat].alive, alive);
    }
}

__global__ void advance_clock(uint64_t *__restrict__ clock, uint64_t delta) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *clock += delta;
}

__global__ void zero_counts(Counts *__restrict__ out, uint32_t nlat) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nlat) {
        out[i].n = 0;
        out[i].n_pair = 0;
        out[i].alive = 0;
    }
}

}  // namespace


size_t phase_lds_bytes(uint32_t B, uint32_t ldw, uint32_t S) {
    (void)S;
    // the tile, one word for the empty-tile flag, and the shared local sites
    // and run indices of two batches of 64 substeps (four teams)
    return (static_cast<size_t>(B) * ldw + 1) * sizeof(uint64_t) + 2u * 2u * 64u * sizeof(uint32_t);
}

hipError_t launch_phase(int n, const uint64_t *src, uint64_t *dst, const LatDesc *lats,
                        const TileDesc *tiles, uint32_t ntiles, const uint64_t *clock,
                        uint64_t s_off, uint32_t S, uint32_t B, const PhaseShape &shape,
                        hipStream_t stream) {
    if (ntiles == 0 || S == 0) return hipSuccess;
    switch (n) {
        case 1: return launch_phase_model1(src, dst, lats, tiles, ntiles, clock, s_off, S, B, shape, stream);
        case 2: return launch_phase_model2(src, dst, lats, tiles, ntiles, clock, s_off, S, B, shape, stream);
        case 3: return launch_phase_model3(src, dst, lats, tiles, ntiles, clock, s_off, S, B, shape, stream);
        case 4: return launch_phase_model4(src, dst, lats, tiles, ntiles, clock, s_off, S, B, shape, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_persist(int n, const PersistLaunch &a, const PhaseShape &shape,
                          hipStream_t stream) {
    switch (n) {
        case 1: return launch_persist_model1(a, shape, stream);
        case 2: return launch_persist_model2(a, shape, stream);
        case 3: return launch_persist_model3(a, shape, stream);
        case 4: return launch_persist_model4(a, shape, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_advance_clock(uint64_t *clock, uint64_t delta, hipStream_t stream) {
    hipLaunchKernelGGL(advance_clock, dim3(1), dim3(64), 0, stream, clock, delta);
    return hipGetLastError();
}

hipError_t launch_fill(uint64_t *dst, uint64_t nwords, uint64_t value, hipStream_t stream) {
    if (nwords == 0) return hipSuccess;
    uint64_t blocks = (nwords + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_words, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, dst,
                       nwords, value);
    return hipGetLastError();
}

hipError_t launch_density(const uint64_t *buf, const LatDesc *lats, const DenChunk *chunks,
                          uint32_t nchunks, Counts *out, uint32_t nlat, hipStream_t stream) {
    hipLaunchKernelGGL(zero_counts, dim3((nlat + 255) / 256), dim3(256), 0, stream, out, nlat);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nchunks == 0) return e;
    hipLaunchKernelGGL(density_chunks, dim3(nchunks), dim3(256), 0, stream, buf, lats, chunks, out);
    return hipGetLastError();
}

}  // namespace pcpd
