// sweep.hip -- gfx950 kernels of the multispin block-synchronous sweep.
//
// Data layout in HBM: one uint64 word per site, bit b = sample b; each
// (instance, plane) is a ring of L consecutive words (natural site order);
// two copies of the whole lattice alternate as source and destination.
//
// brs_phase: one workgroup owns one tile of a ring: `kint` interior blocks of
// B sites plus `hb` halo blocks on each side. It loads the tile into LDS,
// runs S consecutive substeps there, and writes the interior back. Within a
// substep every block is attempted at the same local site o (paper Sec. 3),
// one lane per block. After S substeps a halo of (n+1)*S sites per side has
// absorbed every influence from outside the tile, because one attempt reads
// and writes only sites j-1..j+n; halo windows are computed redundantly with
// the same counter-based draws as their owners, so the interior is exact.
//
// LDS layout: offset-major, word (block c, local site o) at o*ldw + c. All
// lanes of a substep touch the same row o, consecutive columns: no bank
// conflicts. ldw is odd so the row-major HBM<->LDS copies spread over banks.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pcpd_internal.h"

namespace pcpd {
namespace {

// --------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). One round maps
// (c0, c1, c2, c3) to (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
// lo(M0*c0)); the key advances by the Weyl constants between rounds. The
// 32x32->64 products compile to v_mad_u64_u32.
// --------------------------------------------------------------------------
constexpr uint32_t kMulA = 0xD2511F53u;
constexpr uint32_t kMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u;
constexpr uint32_t kWeylB = 0xBB67AE85u;

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t ka, uint32_t kb) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = static_cast<uint64_t>(c.x) * kMulA;
        const uint64_t pb = static_cast<uint64_t>(c.z) * kMulB;
        U4 nx;
        nx.x = static_cast<uint32_t>(pb >> 32) ^ c.y ^ ka;
        nx.y = static_cast<uint32_t>(pb);
        nx.z = static_cast<uint32_t>(pa >> 32) ^ c.w ^ kb;
        nx.w = static_cast<uint32_t>(pa);
        c = nx;
        ka += kWeylA;
        kb += kWeylB;
    }
    return c;
}

// Local site of substep s (uniform across the workgroup: it runs on SALU).
__device__ __forceinline__ uint32_t substep_site(const LatDesc &ld, uint64_t s, uint32_t B) {
    const U4 x = philox10(U4{0u, (ld.plane << 3) | 7u, static_cast<uint32_t>(s),
                             static_cast<uint32_t>(s >> 32)},
                          ld.key0, ld.key1);
    return static_cast<uint32_t>((static_cast<uint64_t>(x.x) * B) >> 32);
}

// Probability-q decision mask on one 32-bit half: sample b fires iff
// (2*a_b + b_b) * 2^32 + g < kh * 2^32 + kl, a = X1 half, b = X2 half.
// f_u is the outcome for prefix u = 2a + b: all-ones below kh, the shared
// comparison g < kl at kh, zero above. Selecting f_u by the two bits takes
// three bitfield inserts.
struct Sel {
    uint32_t f0, f1, f2, f3;
};

__device__ __forceinline__ Sel make_sel(uint32_t g, uint32_t kh, uint32_t kl) {
    const uint32_t tail = (g < kl) ? 0xFFFFFFFFu : 0u;
    Sel s;
    s.f0 = (kh > 0u) ? 0xFFFFFFFFu : tail;  // kh == 0 -> tail
    s.f1 = (kh > 1u) ? 0xFFFFFFFFu : ((kh == 1u) ? tail : 0u);
    s.f2 = (kh > 2u) ? 0xFFFFFFFFu : ((kh == 2u) ? tail : 0u);
    s.f3 = (kh > 3u) ? 0xFFFFFFFFu : ((kh == 3u) ? tail : 0u);
    return s;
}

__device__ __forceinline__ uint32_t pick(uint32_t a, uint32_t b, const Sel &s) {
    const uint32_t lo = (b & s.f1) | (~b & s.f0);  // a = 0
    const uint32_t hi = (b & s.f3) | (~b & s.f2);  // a = 1
    return (a & hi) | (~a & lo);
}

struct W2 {
    uint32_t lo, hi;
};

// The three draws of window k in substep s, reduced to the decision masks
// D (diffusion), Am (annihilation, before conditioning on the tuple) and R
// (fission direction, 1 = high).
struct Masks {
    W2 D, Am, R;
};

__device__ __forceinline__ Masks window_masks(const LatDesc &ld, uint32_t k, uint64_t s) {
    const uint32_t slo = static_cast<uint32_t>(s), shi = static_cast<uint32_t>(s >> 32);
    const uint32_t q8 = ld.plane << 3;
    const U4 d = philox10(U4{k, q8 | 0u, slo, shi}, ld.key0, ld.key1);
    const U4 a = philox10(U4{k, q8 | 1u, slo, shi}, ld.key0, ld.key1);
    const U4 r = philox10(U4{k, q8 | 2u, slo, shi}, ld.key0, ld.key1);
    Masks m;
    const Sel sd = make_sel(r.z, ld.kd_hi, ld.kd_lo);
    const Sel sa = make_sel(r.w, ld.kp_hi, ld.kp_lo);
    // X1 = (x | y << 32), X2 = (z | w << 32): low halves x/z, high halves y/w
    m.D.lo = pick(d.x, d.z, sd);
    m.D.hi = pick(d.y, d.w, sd);
    m.Am.lo = pick(a.x, a.z, sa);
    m.Am.hi = pick(a.y, a.w, sa);
    m.R.lo = r.x;
    m.R.hi = r.y;
    return m;
}

// Bit-sliced attempt on one 32-bit half of a window; w[0] = site j-1,
// w[1..N] = the tuple j..j+N-1, w[N+1] = site j+N.
template <int N>
__device__ __forceinline__ void attempt(uint32_t (&w)[N + 2], uint32_t D, uint32_t Am, uint32_t R) {
    uint32_t P = w[1];
#pragma unroll
    for (int i = 2; i <= N; ++i) P &= w[i];
    const uint32_t a = w[1], b = w[2];
    w[1] = (D & b) | (~D & a);  // diffusion: swap j, j+1 where D
    w[2] = (D & a) | (~D & b);
    const uint32_t nP = ~D & P;       // tuple present, no diffusion
    const uint32_t A = nP & Am;       // annihilation
    const uint32_t F = nP & ~Am;      // fission
#pragma unroll
    for (int i = 1; i <= N; ++i) w[i] &= ~A;
    w[N + 1] |= F & R;   // high: site j+N
    w[0] |= F & ~R;      // low: site j-1
}

template <int N>
__global__ void __launch_bounds__(256)
brs_phase(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
          const LatDesc *__restrict__ lats, const TileDesc *__restrict__ tiles, uint64_t s0,
          uint32_t S, uint32_t B, uint32_t hb, uint32_t ldw) {
    extern __shared__ uint64_t lds[];  // [B][ldw]
    const TileDesc td = tiles[blockIdx.x];
    const LatDesc ld = lats[td.lat];
    const uint32_t nb = ld.nblocks;
    const uint32_t ncols = td.kint + 2u * hb;
    const uint32_t tid = threadIdx.x;
    const uint32_t nthr = blockDim.x;
    // first loaded block: (k0 - hb) mod nb, without going negative
    const uint32_t kfirst = static_cast<uint32_t>(
        (static_cast<uint64_t>(td.k0) + static_cast<uint64_t>(nb) * ((hb + nb - 1u) / nb) - hb) %
        nb);

    // ---- load tile + halo: consecutive lanes read consecutive words
    {
        const uint64_t *ring = src + ld.base;
        const uint32_t total = ncols * B;
        const uint32_t cstep = nthr / B, ostep = nthr - cstep * B;
        uint32_t c = tid / B, o = tid - c * B;
        for (uint32_t i = tid; i < total; i += nthr) {
            uint32_t kg = kfirst + c;
            if (kg >= nb) kg %= nb;
            lds[o * ldw + c] = ring[static_cast<uint64_t>(kg) * B + o];
            c += cstep;
            o += ostep;
            if (o >= B) {
                o -= B;
                ++c;
            }
        }
    }
    __syncthreads();

    // ---- S substeps in LDS, one window (block) per lane
    const uint32_t c = tid;
    const bool active = c < ncols;
    uint32_t kg = kfirst + c;
    if (kg >= nb) kg %= nb;
    for (uint32_t it = 0; it < S; ++it) {
        const uint64_t s = s0 + it;
        const uint32_t o = substep_site(ld, s, B);
        const Masks mk = window_masks(ld, kg, s);
        // window sites o-1 .. o+N of block c; they spill into block c-1 when
        // o == 0 and into block c+1 when o+N >= B
        const bool ok = active && (o > 0u || c > 0u) && (o + N < B || c + 1u < ncols);
        if (ok) {
            int off[N + 2];
#pragma unroll
            for (int m = 0; m < N + 2; ++m) {
                const int r = static_cast<int>(o) - 1 + m;
                const int row = r < 0 ? r + static_cast<int>(B) : (r >= static_cast<int>(B) ? r - static_cast<int>(B) : r);
                const int sh = r < 0 ? -1 : (r >= static_cast<int>(B) ? 1 : 0);
                off[m] = row * static_cast<int>(ldw) + sh + static_cast<int>(c);
            }
            uint32_t wl[N + 2], wh[N + 2];
#pragma unroll
            for (int m = 0; m < N + 2; ++m) {
                const uint64_t v = lds[off[m]];
                wl[m] = static_cast<uint32_t>(v);
                wh[m] = static_cast<uint32_t>(v >> 32);
            }
            attempt<N>(wl, mk.D.lo, mk.Am.lo, mk.R.lo);
            attempt<N>(wh, mk.D.hi, mk.Am.hi, mk.R.hi);
#pragma unroll
            for (int m = 0; m < N + 2; ++m)
                lds[off[m]] = static_cast<uint64_t>(wl[m]) | (static_cast<uint64_t>(wh[m]) << 32);
        }
        __syncthreads();
    }

    // ---- write the interior back; it is contiguous in the ring
    {
        uint64_t *out = dst + ld.base + static_cast<uint64_t>(td.k0) * B;
        const uint32_t total = td.kint * B;
        const uint32_t cstep = nthr / B, ostep = nthr - cstep * B;
        uint32_t cc = tid / B, o = tid - cc * B;
        for (uint32_t i = tid; i < total; i += nthr) {
            out[i] = lds[o * ldw + hb + cc];
            cc += cstep;
            o += ostep;
            if (o >= B) {
                o -= B;
                ++cc;
            }
        }
    }
}

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
        const uint64_t wn = ring[jn];
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

__global__ void zero_counts(Counts *__restrict__ out, uint32_t nlat) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nlat) {
        out[i].n = 0;
        out[i].n_pair = 0;
        out[i].alive = 0;
    }
}

template <int N>
hipError_t launch_phase_n(const uint64_t *src, uint64_t *dst, const LatDesc *lats,
                          const TileDesc *tiles, uint32_t ntiles, uint64_t s0, uint32_t S,
                          uint32_t B, const PhaseShape &sh, hipStream_t stream) {
    const size_t lds = phase_lds_bytes(B, sh.ldw);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&brs_phase<N>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(kMaxLdsBytes));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(brs_phase<N>, dim3(ntiles), dim3(sh.threads), lds, stream, src, dst, lats,
                       tiles, s0, S, B, sh.hb, sh.ldw);
    return hipGetLastError();
}

}  // namespace

size_t phase_lds_bytes(uint32_t B, uint32_t ldw) {
    return static_cast<size_t>(B) * ldw * sizeof(uint64_t);
}

hipError_t launch_phase(int n, const uint64_t *src, uint64_t *dst, const LatDesc *lats,
                        const TileDesc *tiles, uint32_t ntiles, uint64_t s0, uint32_t S,
                        uint32_t B, const PhaseShape &shape, hipStream_t stream) {
    if (ntiles == 0 || S == 0) return hipSuccess;
    switch (n) {
        case 1: return launch_phase_n<1>(src, dst, lats, tiles, ntiles, s0, S, B, shape, stream);
        case 2: return launch_phase_n<2>(src, dst, lats, tiles, ntiles, s0, S, B, shape, stream);
        case 3: return launch_phase_n<3>(src, dst, lats, tiles, ntiles, s0, S, B, shape, stream);
        default: return hipErrorInvalidValue;
    }
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
