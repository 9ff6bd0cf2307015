// pcpd_internal.h -- device-side tables and kernel launchers shared by the
// two translation units of libpcpd (kernels in sweep.hip, host runtime in
// pcpd_api.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcpd {

// One (instance, plane): a ring of nblocks*B words at word offset `base` of
// each lattice copy. 56 bytes, read once per workgroup into SGPRs.
struct LatDesc {
    uint64_t base;     // word offset of site 0
    uint64_t L;        // sites (words) in the ring
    uint32_t nblocks;  // L / B
    uint32_t plane;    // plane index q: Philox counter word 1 is 8q + draw
    uint32_t key0;     // Philox key word 0 (seed)
    uint32_t key1;     // Philox key word 1 (stream id)
    uint32_t kd_hi;    // diffusion threshold K_d = kd_hi * 2^32 + kd_lo
    uint32_t kd_lo;
    uint32_t kp_hi;    // annihilation threshold K_p
    uint32_t kp_lo;
    uint32_t connected;  // 1: the 64 bits form one joined ring of 64 L sites
    uint32_t mbits;      // decorrelation bits m of every decision: 2 or 4
};

// One workgroup's tile: interior blocks [k0, k0 + kint) of lattice `lat`.
struct TileDesc {
    uint32_t lat;
    uint32_t k0;
    uint32_t kint;
    uint32_t pad;
};

// The tiles a tile's phase depends on in a persistent launch: the tiles
// local - lo .. local + hi (cyclic) of its ring, whose tiles are
// first .. first + count - 1; all of them when lo + hi + 1 >= count.
struct TileDeps {
    uint32_t first;  // index of the ring's first tile in the tile table
    uint32_t count;  // tiles of the ring
    uint32_t local;  // this tile's index within the ring
    uint32_t lohi;   // lo | hi << 16
};

// Ticket counter and abort word of a persistent launch.
struct PersistState {
    uint32_t ticket;
    uint32_t abort;
};

// One persistent launch: phases 0 .. nphases-1 of S substeps (the last one
// S_last) starting at substep *clock + s_off; phase f reads buf0 if f is even
// (buf1 if odd) and writes the other copy.
struct PersistLaunch {
    uint64_t *buf0, *buf1;
    const LatDesc *lats;
    const TileDesc *tiles;
    const TileDeps *deps;
    uint32_t ntiles, nphases;
    const uint64_t *clock;
    uint64_t s_off;
    uint32_t S, S_last, B;
    PersistState *state;
    uint32_t *done;      // [ntiles] completed phases per tile
    uint32_t spin_limit; // polls of one wait before the launch gives up
};

// One workgroup's share of a density reduction: words [w0, w0 + nw) of `lat`.
struct DenChunk {
    uint32_t lat;
    uint32_t nw;
    uint64_t w0;
};

// Counts of one (instance, plane); layout identical to pcpd_counts.
struct Counts {
    unsigned long long n;
    unsigned long long n_pair;
    unsigned long long alive;
};

// Largest LDS allocation of one workgroup on gfx950.
constexpr uint32_t kMaxLdsBytes = 160u * 1024u;
// Statically allocated LDS of the persistent phase kernel (its item words),
// which the tile's dynamic LDS must leave free.
constexpr uint32_t kPersistStaticLds = 64u;

// Kernel shape of one phase launch.
struct PhaseShape {
    uint32_t cols;     // blocks held in LDS per workgroup (interior + 2*halo)
    uint32_t threads;  // workgroup size: `teams` teams of a multiple of 64 >= cols lanes
    uint32_t ldw;      // LDS row pitch in words (>= cols + 3, odd)
    uint32_t hb;       // halo blocks on each side
    uint32_t teams;    // lanes per block (2 or 4), each applying every teams-th substep
    uint32_t skip_empty = 0;  // 1: tiles with no particle in their loaded range skip the substeps
    uint32_t general = 0;     // 1: run the kernel copy with the connected layout and the skip
};

// One phase: S substeps starting at substep *clock + s_off.
hipError_t launch_phase(int n, const uint64_t *src, uint64_t *dst, const LatDesc *lats,
                        const TileDesc *tiles, uint32_t ntiles, const uint64_t *clock,
                        uint64_t s_off, uint32_t S, uint32_t B, const PhaseShape &shape,
                        hipStream_t stream);

// The phase launch of one model (n = 1..4), each in its own translation unit.
#define PCPD_PHASE_LAUNCHER(name)                                                             \
    hipError_t name(const uint64_t *src, uint64_t *dst, const LatDesc *lats,                  \
                    const TileDesc *tiles, uint32_t ntiles, const uint64_t *clock,            \
                    uint64_t s_off, uint32_t S, uint32_t B, const PhaseShape &shape,          \
                    hipStream_t stream)
PCPD_PHASE_LAUNCHER(launch_phase_model1);
PCPD_PHASE_LAUNCHER(launch_phase_model2);
PCPD_PHASE_LAUNCHER(launch_phase_model3);
PCPD_PHASE_LAUNCHER(launch_phase_model4);
#undef PCPD_PHASE_LAUNCHER

// The persistent launch of one model (n = 1..4).
hipError_t launch_persist_model1(const PersistLaunch &a, const PhaseShape &shape, hipStream_t stream);
hipError_t launch_persist_model2(const PersistLaunch &a, const PhaseShape &shape, hipStream_t stream);
hipError_t launch_persist_model3(const PersistLaunch &a, const PhaseShape &shape, hipStream_t stream);
hipError_t launch_persist_model4(const PersistLaunch &a, const PhaseShape &shape, hipStream_t stream);
hipError_t launch_persist(int n, const PersistLaunch &a, const PhaseShape &shape, hipStream_t stream);

// *clock += delta, on the device.
hipError_t launch_advance_clock(uint64_t *clock, uint64_t delta, hipStream_t stream);

hipError_t launch_fill(uint64_t *dst, uint64_t nwords, uint64_t value, hipStream_t stream);

hipError_t launch_density(const uint64_t *buf, const LatDesc *lats, const DenChunk *chunks,
                          uint32_t nchunks, Counts *out, uint32_t nlat, hipStream_t stream);

// LDS of one phase workgroup: B x ldw lattice words, the empty-tile flag word
// and the shared substep sites of the four-team loop (1 KB).
size_t phase_lds_bytes(uint32_t B, uint32_t ldw, uint32_t S);

}  // namespace pcpd
