// brs_phase.h -- gfx950 phase kernel of the multispin block-synchronous sweep,
// included by one translation unit per model (phase_n1.hip .. phase_n4.hip).
//
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
// Two consecutive substeps whose windows touch disjoint sites commute; such
// pairs are applied in one interval between workgroup barriers.
//
// LDS layout: offset-major, word (block c, local site o) at o*ldw + c. All
// lanes of a substep touch the same row o, consecutive columns: no bank
// conflicts. ldw is odd so the row-major HBM<->LDS copies spread over banks,
// and leaves three spare columns past the tile.

#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pcpd_internal.h"
#include "philox.h"

namespace pcpd {
namespace {

// Local site of substep s: o = floor(x0 * B / 2^32) of draw 7, window 0.
__device__ __forceinline__ uint32_t substep_site(const LatDesc &ld, uint64_t s, uint32_t B) {
    const U4 x = philox10(U4{0u, (ld.plane << 3) | 7u, static_cast<uint32_t>(s),
                             static_cast<uint32_t>(s >> 32)},
                          ld.key0, ld.key1);
    return static_cast<uint32_t>((static_cast<uint64_t>(x.x) * B) >> 32);
}

// Truth table of a three-input bitwise function for v_bitop3_b32: bit
// (4*a + 2*b + c) of the table is f(a, b, c). Evaluated on the canonical
// operand patterns a = 0xF0, b = 0xCC, c = 0xAA.
template <typename F>
constexpr uint32_t lut3(F f) {
    return f(0xF0u, 0xCCu, 0xAAu) & 0xFFu;
}

// Probability-q decision, one 32-bit half: sample bit fires iff
// (2*a + b) * 2^32 + g < KH * 2^32 + kl, a = bit of X1, b = bit of X2,
// t = all-ones iff the shared tail g < kl. For each integer part KH of the
// threshold the decision is a fixed function of (a, b, t):
//   KH=0: u == 0 and t;  KH=1: u == 0, or u == 1 and t;  KH=2: u <= 1, or u == 2 and t;
//   KH=3: u <= 2, or t;  KH=4: always (q = 1).
template <int KH>
struct Decide {
    static constexpr uint32_t lut() {
        if constexpr (KH == 0) return lut3([](uint32_t a, uint32_t b, uint32_t t) { return ~a & ~b & t; });
        else if constexpr (KH == 1) return lut3([](uint32_t a, uint32_t b, uint32_t t) { return ~a & (~b | t); });
        else if constexpr (KH == 2) return lut3([](uint32_t a, uint32_t b, uint32_t t) { return ~a | (~b & t); });
        else if constexpr (KH == 3) return lut3([](uint32_t a, uint32_t b, uint32_t t) { return ~a | ~b | t; });
        else return 0xFFu;
    }
    __device__ static __forceinline__ uint32_t half(uint32_t a, uint32_t b, uint32_t t) {
        if constexpr (KH >= 4) return 0xFFFFFFFFu;
        else return __builtin_amdgcn_bitop3_b32(a, b, t, lut());
    }
};

struct W2 {
    uint32_t lo, hi;
};

// Decision masks of one window: D (diffusion), Am (annihilation, before the
// tuple condition) and R (fission direction, 1 = high), as 32-bit halves.
struct Masks {
    W2 D, Am, R;
};

// The ten rounds of the draws of one window (three; five with four
// decorrelation bits), advanced round by round together: two independent
// 32x32->64 products per draw and round. The first round's products are
// identical for all the draws (they differ only in counter word 1) and are
// computed once by the compiler.
template <int ND>
__device__ __forceinline__ void philox10_xn(U4 (&c)[ND], uint32_t ka, uint32_t kb) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            const uint64_t pa = static_cast<uint64_t>(c[j].x) * kMulA;
            const uint64_t pb = static_cast<uint64_t>(c[j].z) * kMulB;
            U4 nx;
            if (r < 2) {
                // the first two rounds have operands that are uniform across the
                // wavefront (counter words 1-3 and the key); plain XORs let the
                // compiler keep those on the scalar unit, which the vector-only
                // three-input XOR cannot
                nx.x = static_cast<uint32_t>(pb >> 32) ^ c[j].y ^ ka;
                nx.z = static_cast<uint32_t>(pa >> 32) ^ c[j].w ^ kb;
            } else {
                nx.x = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pb >> 32), c[j].y, ka, 0x96);
                nx.z = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pa >> 32), c[j].w, kb, 0x96);
            }
            nx.y = static_cast<uint32_t>(pb);
            nx.w = static_cast<uint32_t>(pa);
            c[j] = nx;
        }
        ka += kWeylA;
        kb += kWeylB;
    }
}

// Draw identity of a lane's window: its block k. In the connected layout a
// tile with columns past the ends of the word ring runs with a lapped window
// type, which also carries the lap of the lane's column (a right rotation by
// rot = lap mod 64; zero for columns inside the ring); every other tile runs
// with PlainWin, whose code has no trace of the rotation. WIDE: decisions
// with four decorrelation bits instead of two (two more draws per window).
template <bool LAP, bool WIDE>
struct WinT {
    static constexpr bool kLapped = LAP;
    static constexpr bool kWide = WIDE;
    uint32_t k;
    uint32_t rot;  // used when LAP
};
using PlainWin = WinT<false, false>;
using LapWin = WinT<true, false>;

// Right rotation of a 64-bit mask held as two halves, by r in 0..63.
__device__ __forceinline__ W2 rotr_w2(W2 x, uint32_t r) {
    const bool sw = (r & 32u) != 0u;
    const uint32_t lo = sw ? x.hi : x.lo, hi = sw ? x.lo : x.hi;
    return W2{__builtin_amdgcn_alignbit(hi, lo, r & 31u), __builtin_amdgcn_alignbit(lo, hi, r & 31u)};
}

// Probability decision with four decorrelation bits, one 32-bit half: bit i
// fires iff u_i < kh or (u_i == kh and t_i), u_i the 4-bit number of bit i of
// (a, b, c, d), a most significant; kh (0..16) is uniform across the wave.
__device__ __forceinline__ uint32_t decide_wide(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                                uint32_t t, uint32_t kh) {
    if (kh >= 16u) return 0xFFFFFFFFu;
    const uint32_t x[4] = {a, b, c, d};
    uint32_t lt = 0u, eq = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if ((kh >> (3 - i)) & 1u) {
            lt |= eq & ~x[i];
            eq &= x[i];
        } else {
            eq &= ~x[i];
        }
    }
    return lt | (eq & t);
}

template <int KDH, int KPH, typename Win>
__device__ __forceinline__ Masks window_masks(const LatDesc &ld, Win w, uint64_t s) {
    const uint32_t slo = static_cast<uint32_t>(s), shi = static_cast<uint32_t>(s >> 32);
    const uint32_t q8 = ld.plane << 3;
    const uint32_t k = w.k;
    if constexpr (Win::kWide) {
        // m = 4: X1, X2 from draws 0 (D) and 1 (A), X3, X4 from draws 3 (D)
        // and 4 (A); draw 2 as for m = 2. Sample b fires iff its four bits,
        // X1 most significant, read below the threshold's integer part, or
        // equal to it with the shared tail below its low word.
        U4 x[5] = {U4{k, q8 | 0u, slo, shi}, U4{k, q8 | 1u, slo, shi}, U4{k, q8 | 2u, slo, shi},
                   U4{k, q8 | 3u, slo, shi}, U4{k, q8 | 4u, slo, shi}};
        philox10_xn<5>(x, ld.key0, ld.key1);
        const U4 &d = x[0], &a = x[1], &r = x[2], &d2 = x[3], &a2 = x[4];
        const uint32_t td = (r.z < ld.kd_lo) ? 0xFFFFFFFFu : 0u;
        const uint32_t ta = (r.w < ld.kp_lo) ? 0xFFFFFFFFu : 0u;
        Masks m;
        m.D.lo = decide_wide(d.x, d.z, d2.x, d2.z, td, ld.kd_hi);
        m.D.hi = decide_wide(d.y, d.w, d2.y, d2.w, td, ld.kd_hi);
        m.Am.lo = decide_wide(a.x, a.z, a2.x, a2.z, ta, ld.kp_hi);
        m.Am.hi = decide_wide(a.y, a.w, a2.y, a2.w, ta, ld.kp_hi);
        m.R.lo = r.x;
        m.R.hi = r.y;
        if constexpr (Win::kLapped) {
            m.D = rotr_w2(m.D, w.rot);
            m.Am = rotr_w2(m.Am, w.rot);
            m.R = rotr_w2(m.R, w.rot);
        }
        return m;
    }
    U4 x[3] = {U4{k, q8 | 0u, slo, shi}, U4{k, q8 | 1u, slo, shi}, U4{k, q8 | 2u, slo, shi}};
    philox10_xn<3>(x, ld.key0, ld.key1);
    const U4 &d = x[0], &a = x[1], &r = x[2];
    const uint32_t td = (r.z < ld.kd_lo) ? 0xFFFFFFFFu : 0u;  // shared tails gD, gA
    const uint32_t ta = (r.w < ld.kp_lo) ? 0xFFFFFFFFu : 0u;
    Masks m;
    // X1 = x | y << 32, X2 = z | w << 32
    m.D.lo = Decide<KDH>::half(d.x, d.z, td);
    m.D.hi = Decide<KDH>::half(d.y, d.w, td);
    m.Am.lo = Decide<KPH>::half(a.x, a.z, ta);
    m.Am.hi = Decide<KPH>::half(a.y, a.w, ta);
    m.R.lo = r.x;
    m.R.hi = r.y;
    if constexpr (Win::kLapped) {
        // bit b of a lapped column holds the site of bit b + lap of its block:
        // its decisions are that bit's, moved like the column's words
        m.D = rotr_w2(m.D, w.rot);
        m.Am = rotr_w2(m.Am, w.rot);
        m.R = rotr_w2(m.R, w.rot);
    }
    return m;
}

// Pin the masks in registers at this point of the program. Before a barrier,
// the arithmetic that produces them cannot sink into the next interval, where
// it would no longer overlap the LDS latency of this interval's update.
__device__ __forceinline__ void pin(Masks &m) {
    asm volatile("" : "+v"(m.D.lo), "+v"(m.D.hi), "+v"(m.Am.lo), "+v"(m.Am.hi), "+v"(m.R.lo),
                      "+v"(m.R.hi));
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

// LDS word offsets (in words) of the window of substep site o, relative to
// the lane's column: site o-1+m sits in row (o-1+m) mod B of column c-1, c or
// c+1. Integer arithmetic only, so that it stays on the scalar unit.
template <int N>
__device__ __forceinline__ void window_offsets(uint32_t o, uint32_t B, uint32_t ldw,
                                               int (&base)[N + 2]) {
    const int W = static_cast<int>(B * ldw) - 1;  // one row-block back plus one column
#pragma unroll
    for (int m = 0; m < N + 2; ++m) {
        const int r = static_cast<int>(o) - 1 + m;
        const int below = static_cast<int>(static_cast<uint32_t>(r) >> 31);            // r < 0
        const int above = 1 - static_cast<int>(static_cast<uint32_t>(r - static_cast<int>(B)) >> 31);  // r >= B
        base[m] = r * static_cast<int>(ldw) + (below - above) * W;
    }
}

// Apply the attempt of substep site o to the lane's window in LDS (see
// run_substeps for the two addressing cases). mid() runs after the window's
// loads are issued and before their values are used: arithmetic placed there
// fills the LDS latency.
template <int N, typename Mid>
__device__ __forceinline__ void apply_window(uint64_t *lds, const Masks &m, uint32_t o,
                                             uint32_t c, uint32_t col_in, bool ok_lo,
                                             bool ok_hi, uint32_t trash, uint32_t B,
                                             uint32_t ldw, Mid &&mid) {
    uint32_t wl[N + 2], wh[N + 2];
    if (o - 1u < B - 1u - N) {
        // window rows o-1 .. o+N inside the lane's own column: one address
        // plus multiples of the pitch (all but (N+1)/B of the substeps)
        uint64_t *w = lds + ((o - 1u) * ldw + col_in);
#pragma unroll
        for (int k = 0; k < N + 2; ++k) {
            const uint64_t v = w[k * ldw];
            wl[k] = static_cast<uint32_t>(v);
            wh[k] = static_cast<uint32_t>(v >> 32);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of mid()
        mid();
        attempt<N>(wl, m.D.lo, m.Am.lo, m.R.lo);
        attempt<N>(wh, m.D.hi, m.Am.hi, m.R.hi);
#pragma unroll
        for (int k = 0; k < N + 2; ++k)
            w[k * ldw] = static_cast<uint64_t>(wl[k]) | (static_cast<uint64_t>(wh[k]) << 32);
    } else {
        // window sites o-1 .. o+N of block c spill into block c-1 when o == 0
        // and into block c+1 when o+N >= B
        const bool ok = !(o == 0u && !ok_lo) && !(o + N >= B && !ok_hi);
        const int col = static_cast<int>(ok ? c : trash);
        int base[N + 2];
        window_offsets<N>(o, B, ldw, base);
#pragma unroll
        for (int k = 0; k < N + 2; ++k) {
            const uint64_t v = lds[base[k] + col];
            wl[k] = static_cast<uint32_t>(v);
            wh[k] = static_cast<uint32_t>(v >> 32);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of mid()
        mid();
        attempt<N>(wl, m.D.lo, m.Am.lo, m.R.lo);
        attempt<N>(wh, m.D.hi, m.Am.hi, m.R.hi);
#pragma unroll
        for (int k = 0; k < N + 2; ++k)
            lds[base[k] + col] = static_cast<uint64_t>(wl[k]) | (static_cast<uint64_t>(wh[k]) << 32);
    }
}

// True when the windows of two substeps with local sites oa and ob touch
// disjoint sites: the cyclic distance of oa and ob within a block is at least
// N+2, the window length. Every block uses the same local site, so the two
// substeps then commute and may be applied in either order or together.
template <int N>
__device__ __forceinline__ bool windows_disjoint(uint32_t oa, uint32_t ob, uint32_t B) {
    uint32_t d = ob - oa;
    if (static_cast<int32_t>(d) < 0) d += B;  // (ob - oa) mod B, with oa, ob < B
    const uint32_t e = B - d;                 // (oa - ob) mod B, or B when d == 0
    return d >= N + 2u && e >= N + 2u;
}

// S substeps of one tile held in LDS (see the file comment), by two teams
// of lanes, each with one lane per block; team t applies the substeps
// it = t, t+2, t+4, ... Substeps are taken in pairs (it, it+1), it even:
// when their windows are disjoint (windows_disjoint; at B = 64 and N = 2
// all but 7 of 64 pairs) both teams apply their substep in the same interval
// between two barriers; otherwise team 0 applies its substep in one interval
// and team 1 in the next. Each team then draws the masks of its next
// substep between the loads and the arithmetic of its update, which fills
// the LDS latency. The two teams run their own loops (no register copies
// between the branches) and pass the same number of barriers. Draws past
// the phase end are computed and dropped.
// Each wavefront draws the local sites of 64 substeps at a time, one per
// lane, and reads them back with v_readlane.
// Window rows o-1 .. o+N lie inside the lane's own column when
// 1 <= o <= B-1-N; otherwise (a uniform branch, (N+1)/B of the substeps) the
// window spills into a neighbouring column and each word has its own
// address. Lanes whose window would leave the loaded columns (block 0 when
// o == 0, the last block when o+N >= B, lanes past the tile) work on the
// spare columns trash-1 .. trash+1 instead, so no branch depends on the lane.
template <int N, int KDH, int KPH, typename Win>
__device__ __forceinline__ void run_substeps(uint64_t *lds, const LatDesc &ld, Win kg,
                                             uint32_t c, uint32_t team, uint32_t ncols,
                                             uint32_t trash, uint64_t s0, uint32_t S, uint32_t B,
                                             uint32_t ldw) {
    const uint32_t lane = __lane_id();
    const bool active = c < ncols;
    const bool ok_lo = active && c != 0u;          // a spill into block c-1 stays in the tile
    const bool ok_hi = active && c + 1u != ncols;  // a spill into block c+1 stays in the tile
    const uint32_t col_in = active ? c : trash;    // column of a window inside one column
    // The masks alternate between two register sets (m0, m1) over a pair of
    // pairs, so that no register copies are needed inside the loop.
    Masks m0 = window_masks<KDH, KPH>(ld, kg, s0 + team), m1{};
    if (team == 0u) {
        // one pair: apply substep it0+j, draw substep it0+j+2
        auto step = [&](uint32_t sites, uint32_t it0, uint32_t n, uint32_t j, const Masks &use,
                        Masks &make) {
            const uint32_t oa = __builtin_amdgcn_readlane(sites, j);
            const bool split = j + 1u < n &&
                               !windows_disjoint<N>(oa, __builtin_amdgcn_readlane(sites, j + 1u), B);
            auto draw = [&] {
                make = window_masks<KDH, KPH>(ld, kg, s0 + it0 + j + 2u);
                pin(make);
            };
            apply_window<N>(lds, use, oa, c, col_in, ok_lo, ok_hi, trash, B, ldw, draw);
            __syncthreads();
            if (split) __syncthreads();  // team 1 applies its substep alone
        };
        for (uint32_t it0 = 0; it0 < S; it0 += 64u) {
            const uint32_t sites = substep_site(ld, s0 + it0 + lane, B);  // lane i: substep it0 + i
            const uint32_t n = (S - it0 < 64u) ? S - it0 : 64u;
            uint32_t j = 0;
            for (; j + 2u < n; j += 4u) {
                step(sites, it0, n, j, m0, m1);
                step(sites, it0, n, j + 2u, m1, m0);
            }
            if (j < n) {
                step(sites, it0, n, j, m0, m1);
                m0 = m1;
            }
        }
    } else {
        // one pair: apply substep it0+j+1 (if any), draw substep it0+j+3
        auto step = [&](uint32_t sites, uint32_t it0, uint32_t n, uint32_t j, const Masks &use,
                        Masks &make) {
            const bool has_b = j + 1u < n;
            const uint32_t ob = __builtin_amdgcn_readlane(sites, has_b ? j + 1u : j);
            const bool split =
                has_b && !windows_disjoint<N>(__builtin_amdgcn_readlane(sites, j), ob, B);
            if (split) __syncthreads();  // after team 0's substep
            auto draw = [&] {
                make = window_masks<KDH, KPH>(ld, kg, s0 + it0 + j + 3u);
                pin(make);
            };
            if (has_b)
                apply_window<N>(lds, use, ob, c, col_in, ok_lo, ok_hi, trash, B, ldw, draw);
            else
                draw();
            __syncthreads();
        };
        for (uint32_t it0 = 0; it0 < S; it0 += 64u) {
            const uint32_t sites = substep_site(ld, s0 + it0 + lane, B);
            const uint32_t n = (S - it0 < 64u) ? S - it0 : 64u;
            uint32_t j = 0;
            for (; j + 2u < n; j += 4u) {
                step(sites, it0, n, j, m0, m1);
                step(sites, it0, n, j + 2u, m1, m0);
            }
            if (j < n) {
                step(sites, it0, n, j, m0, m1);
                m0 = m1;
            }
        }
    }
}

// Greedy cut of the groups of T consecutive substeps of a batch of 64 into
// runs of substeps whose windows are pairwise disjoint. Lane i holds the local
// site of substep i of the batch; it returns the run index of substep i within
// its group (lanes i & ~(T-1) .. i | (T-1)). The greedy cut of a prefix of a
// group is the prefix of the group's cut, so a group cut short by the end of
// a phase takes the run indices of its members as they are.
template <int N, int T>
__device__ __forceinline__ uint32_t group_run_index(uint32_t sites, uint32_t B) {
    const uint32_t lane = __lane_id();
    const uint32_t base = lane & ~static_cast<uint32_t>(T - 1);
    const uint32_t pos = lane - base;
    uint32_t o[T];
#pragma unroll
    for (int j = 0; j < T; ++j) o[j] = __shfl(sites, static_cast<int>(base) + j, 64);
    uint32_t seg = 0, start = 0, mine = 0;
#pragma unroll
    for (int j = 1; j < T; ++j) {
        bool ok = true;
#pragma unroll
        for (int i = 0; i < j; ++i)
            if (static_cast<uint32_t>(i) >= start) ok = ok && windows_disjoint<N>(o[i], o[j], B);
        if (!ok) {
            ++seg;
            start = j;
        }
        if (static_cast<uint32_t>(j) == pos) mine = seg;
    }
    return mine;
}

// run_substeps for T teams (T divides 64): team t applies the substeps
// t, t+T, t+2T, ... Substeps are taken in groups of T consecutive ones; a
// group is cut into runs of pairwise commuting substeps (group_run_index), and
// each run is applied in one interval between workgroup barriers, every team
// of the run at once. A team draws the masks of its next substep (T later)
// between the loads and the arithmetic of its update. Every wavefront passes
// the same barriers: each computes the same cut from the same local sites.
// Local sites and run indices of the batches of 64 substeps, shared by the
// wavefronts of a four-team workgroup: two slots of (sites, runs) x 64 words
// in LDS after the tile and its flag word. Batch 0 is written by wavefront 0
// before the barrier that ends the tile load; batch b+1 by wavefront
// (b+1) mod (wavefronts) at the start of batch b, and read at the start of
// batch b+1, after the barriers of batch b. The slot it overwrites was last
// read at the start of batch b-1, before those barriers.
__device__ __forceinline__ uint32_t *batch_share(uint64_t *lds, uint32_t B, uint32_t ldw) {
    return reinterpret_cast<uint32_t *>(lds + static_cast<size_t>(B) * ldw + 1u);
}

template <int N, int T>
__device__ __forceinline__ void write_batch(uint32_t *slot, const LatDesc &ld, uint64_t s,
                                            uint32_t B) {
    const uint32_t lane = __lane_id();
    const uint32_t sites = substep_site(ld, s + lane, B);  // lane i: substep s + i
    slot[lane] = sites;
    slot[64u + lane] = group_run_index<N, T>(sites, B);
}

template <int N, int KDH, int KPH, int T, typename Win>
__device__ __forceinline__ void run_substeps_teams(uint64_t *lds, const LatDesc &ld, Win kg,
                                                   uint32_t c, uint32_t team, uint32_t ncols,
                                                   uint32_t trash, uint64_t s0, uint32_t S,
                                                   uint32_t B, uint32_t ldw) {
    static_assert(64 % T == 0, "a group must not straddle a batch of 64 local sites");
    const uint32_t lane = __lane_id();
    const bool active = c < ncols;
    const bool ok_lo = active && c != 0u;
    const bool ok_hi = active && c + 1u != ncols;
    const uint32_t col_in = active ? c : trash;
    Masks m0 = window_masks<KDH, KPH>(ld, kg, s0 + team), m1{};
    auto group = [&](uint32_t sites, uint32_t runs, uint32_t it0, uint32_t n, uint32_t g,
                     const Masks &use, Masks &make) {
        const uint32_t k = (n - g < static_cast<uint32_t>(T)) ? n - g : static_cast<uint32_t>(T);
        const uint32_t nseg = __builtin_amdgcn_readlane(runs, g + k - 1u) + 1u;
        const bool mine = team < k;
        const uint32_t myseg = __builtin_amdgcn_readlane(runs, g + (mine ? team : 0u));
        if (mine) {
            // the runs before this team's run, its own run, the runs after it
            for (uint32_t e = 0; e < myseg; ++e) __syncthreads();
            const uint32_t o = __builtin_amdgcn_readlane(sites, g + team);
            auto draw = [&] {
                make = window_masks<KDH, KPH>(ld, kg, s0 + it0 + g + team + T);
                pin(make);
            };
            apply_window<N>(lds, use, o, c, col_in, ok_lo, ok_hi, trash, B, ldw, draw);
            for (uint32_t e = myseg; e < nseg; ++e) __syncthreads();
        } else {
            // no substep of this team in a group cut short by the phase end
            for (uint32_t e = 0; e < nseg; ++e) __syncthreads();
        }
    };
    uint32_t *share = batch_share(lds, B, ldw);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nwaves = blockDim.x >> 6;
    uint32_t b = 0;
    for (uint32_t it0 = 0; it0 < S; it0 += 64u, ++b) {
        const uint32_t *slot = share + (b & 1u) * 128u;
        const uint32_t sites = slot[lane];        // lane i: local site of substep it0 + i
        const uint32_t runs = slot[64u + lane];   // its run index within its group
        if (it0 + 64u < S && wave == (b + 1u) % nwaves)
            write_batch<N, T>(share + ((b + 1u) & 1u) * 128u, ld, s0 + it0 + 64u, B);
        const uint32_t n = (S - it0 < 64u) ? S - it0 : 64u;
        uint32_t g = 0;
        for (; g + T < n; g += 2u * T) {
            group(sites, runs, it0, n, g, m0, m1);
            group(sites, runs, it0, n, g + T, m1, m0);
        }
        if (g < n) {
            group(sites, runs, it0, n, g, m0, m1);
            m0 = m1;
        }
    }
}

// T = 2 runs the two-team loop above; T = 4 the general one.
template <int N, int KDH, int KPH, int T, typename Win>
__device__ __forceinline__ void run_team_loop(uint64_t *lds, const LatDesc &ld, Win kg,
                                              uint32_t c, uint32_t team, uint32_t ncols,
                                              uint32_t trash, uint64_t s0, uint32_t S, uint32_t B,
                                              uint32_t ldw) {
    if constexpr (T == 2)
        run_substeps<N, KDH, KPH>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw);
    else
        run_substeps_teams<N, KDH, KPH, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw);
}

template <int N, int KDH, int T, typename Win>
__device__ __forceinline__ void dispatch_kp(uint64_t *lds, const LatDesc &ld,
                                            Win kg, uint32_t c, uint32_t team, uint32_t ncols,
                                            uint32_t trash,
                                            uint64_t s0, uint32_t S, uint32_t B, uint32_t ldw) {
    switch (ld.kp_hi) {
        case 0: run_team_loop<N, KDH, 0, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
        case 1: run_team_loop<N, KDH, 1, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
        case 2: run_team_loop<N, KDH, 2, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
        case 3: run_team_loop<N, KDH, 3, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
        default: run_team_loop<N, KDH, 4, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
    }
}

template <int N, int T, typename Win>
__device__ __forceinline__ void dispatch_kd(uint64_t *lds, const LatDesc &ld, Win kg, uint32_t c,
                                            uint32_t team, uint32_t ncols, uint32_t trash,
                                            uint64_t s0, uint32_t S, uint32_t B, uint32_t ldw) {
    switch (ld.kd_hi) {
        case 0: dispatch_kp<N, 0, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
        case 1: dispatch_kp<N, 1, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
        case 2: dispatch_kp<N, 2, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
        case 3: dispatch_kp<N, 3, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
        default: dispatch_kp<N, 4, T>(lds, ld, kg, c, team, ncols, trash, s0, S, B, ldw); break;
    }
}

// Connected layout (the 64 bits of a plane joined into one ring of 64 L
// sites, bit b of word j = site b*L + j): the tile's column of virtual block
// v (v < 0 or v >= nb past the ends of the word ring) holds the words of
// block v mod nb moved by m = floor(v / nb) laps, i.e. with every site m*L
// further on, which is bit b+m of the stored word: a right rotation by m.
__device__ __forceinline__ int32_t ring_lap(int64_t v, uint32_t nb) {
    if (v >= 0 && v < static_cast<int64_t>(nb)) return 0;
    if (v >= 0) return static_cast<int32_t>(v / nb);
    return -static_cast<int32_t>((-v + nb - 1) / nb);
}

__device__ __forceinline__ uint64_t rotr64(uint64_t x, int32_t m) {
    const uint32_t r = static_cast<uint32_t>(m) & 63u;
    return r ? (x >> r) | (x << (64u - r)) : x;
}

// Words moved per lane per batch between HBM and LDS: independent loads in
// flight hide the memory latency.
constexpr int kCopyBatch = 16;

// Two consecutive sites of one block, moved as one 16-byte access.
struct alignas(16) WordPair {
    uint64_t a, b;
};

// Copy `total` words of a tile, ring blocks kfirst, kfirst+1, ... (mod nb),
// from HBM (natural order) into LDS column-per-block. Lane i handles words
// i, i+nthr, ...; (column, row, ring block) advance incrementally.
template <bool OR>
__device__ __forceinline__ void load_tile(uint64_t *lds, const uint64_t *__restrict__ ring,
                                          uint32_t kfirst, uint32_t nb, uint32_t total, uint32_t B,
                                          uint32_t ldw, uint32_t tid, uint32_t nthr, uint64_t &any) {
    const uint32_t cstep = nthr / B, ostep = nthr - cstep * B, kstep = cstep % nb;
    uint32_t c = tid / B, o = tid - c * B;
    uint32_t kg = (kfirst + c) % nb;
    for (uint32_t i0 = tid; i0 < total; i0 += kCopyBatch * nthr) {
        uint64_t v[kCopyBatch];
        uint32_t a[kCopyBatch];
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u) {
            a[u] = o * ldw + c;
            v[u] = (i0 + u * nthr < total) ? ring[static_cast<uint64_t>(kg) * B + o] : 0ull;
            c += cstep;
            o += ostep;
            kg += kstep;
            if (o >= B) {
                o -= B;
                ++c;
                ++kg;
            }
            if (kg >= nb) kg -= nb;
        }
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u)
            if (i0 + u * nthr < total) {
                lds[a[u]] = v[u];
                if constexpr (OR) any |= v[u];
            }
    }
}

// load_tile for an even B and a 16-byte aligned ring: lane i handles the
// site pairs (2i, 2i+1), (2i+2*nthr, ...), ..., so a tile of up to
// 2*kCopyBatch*nthr words arrives in one round trip. FIXED_ROW: 2*nthr is a
// multiple of B, so every pair of a lane lies in the same row (the default
// shapes); the row-wrap test then drops out of the loop.
template <bool FIXED_ROW, bool OR>
__device__ __forceinline__ void load_tile_pairs(uint64_t *lds, const uint64_t *__restrict__ ring,
                                                uint32_t kfirst, uint32_t nb, uint32_t total,
                                                uint32_t B, uint32_t ldw, uint32_t tid,
                                                uint32_t nthr, uint64_t &any) {
    const WordPair *rp = reinterpret_cast<const WordPair *>(ring);
    const uint32_t step = 2u * nthr;
    const uint32_t cstep = step / B, ostep = step - cstep * B, kstep = cstep % nb;
    uint32_t c = (2u * tid) / B, o = 2u * tid - c * B;
    uint32_t kg = (kfirst + c) % nb;
    const uint32_t half = B >> 1;
    for (uint32_t i0 = 2u * tid; i0 < total; i0 += kCopyBatch * step) {
        WordPair v[kCopyBatch];
        uint32_t a[kCopyBatch];
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u) {
            a[u] = o * ldw + c;
            if (i0 + u * step < total) v[u] = rp[static_cast<uint64_t>(kg) * half + (o >> 1)];
            c += cstep;
            kg += kstep;
            if constexpr (!FIXED_ROW) {
                o += ostep;
                if (o >= B) {
                    o -= B;
                    ++c;
                    ++kg;
                }
            }
            if (kg >= nb) kg -= nb;
        }
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u)
            if (i0 + u * step < total) {
                lds[a[u]] = v[u].a;
                lds[a[u] + ldw] = v[u].b;
                if constexpr (OR) any |= v[u].a | v[u].b;
            }
    }
}

// The tile loaders by case; with OR, `any` collects the OR of every word
// loaded by this lane.
template <bool OR>
__device__ __forceinline__ void load_tile_any(uint64_t *lds, const uint64_t *__restrict__ ring,
                                              bool pairs, bool fixed_row, uint32_t kfirst,
                                              uint32_t nb, uint32_t total, uint32_t B, uint32_t ldw,
                                              uint32_t tid, uint32_t nthr, uint64_t &any) {
    if (pairs && fixed_row)
        load_tile_pairs<true, OR>(lds, ring, kfirst, nb, total, B, ldw, tid, nthr, any);
    else if (pairs)
        load_tile_pairs<false, OR>(lds, ring, kfirst, nb, total, B, ldw, tid, nthr, any);
    else
        load_tile<OR>(lds, ring, kfirst, nb, total, B, ldw, tid, nthr, any);
}

// Copy the interior columns hb .. hb+total/B-1 of the tile back to HBM, where
// they are `total` consecutive words starting at `out`.
__device__ __forceinline__ void store_interior(uint64_t *__restrict__ out, const uint64_t *lds,
                                               uint32_t hb, uint32_t total, uint32_t B, uint32_t ldw,
                                               uint32_t tid, uint32_t nthr) {
    const uint32_t cstep = nthr / B, ostep = nthr - cstep * B;
    uint32_t c = tid / B, o = tid - c * B;
    for (uint32_t i0 = tid; i0 < total; i0 += kCopyBatch * nthr) {
        uint64_t v[kCopyBatch];
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u) {
            v[u] = (i0 + u * nthr < total) ? lds[o * ldw + hb + c] : 0ull;
            c += cstep;
            o += ostep;
            if (o >= B) {
                o -= B;
                ++c;
            }
        }
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u)
            if (i0 + u * nthr < total) out[i0 + u * nthr] = v[u];
    }
}

// store_interior for an even B and a 16-byte aligned destination, one site
// pair per lane and access; FIXED_ROW as for load_tile_pairs.
template <bool FIXED_ROW>
__device__ __forceinline__ void store_interior_pairs(uint64_t *__restrict__ out,
                                                     const uint64_t *lds, uint32_t hb,
                                                     uint32_t total, uint32_t B, uint32_t ldw,
                                                     uint32_t tid, uint32_t nthr) {
    WordPair *op = reinterpret_cast<WordPair *>(out);
    const uint32_t step = 2u * nthr;
    const uint32_t cstep = step / B, ostep = step - cstep * B;
    uint32_t c = (2u * tid) / B, o = 2u * tid - c * B;
    for (uint32_t i0 = 2u * tid; i0 < total; i0 += kCopyBatch * step) {
        WordPair v[kCopyBatch];
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u) {
            if (i0 + u * step < total) {
                v[u].a = lds[o * ldw + hb + c];
                v[u].b = lds[(o + 1u) * ldw + hb + c];
            }
            c += cstep;
            if constexpr (!FIXED_ROW) {
                o += ostep;
                if (o >= B) {
                    o -= B;
                    ++c;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kCopyBatch; ++u)
            if (i0 + u * step < total) op[(i0 + u * step) >> 1] = v[u];
    }
}

// LDS row pitch of the default tile (128 columns plus three spare, odd).
constexpr uint32_t kDefaultPitch = 131;

// One tile for one phase: load the tile and its halo from `src` into LDS,
// run S substeps starting at substep s0, write the interior to `dst`. T
// lanes per block (the T teams).
// GENERAL: the copy of the kernel that also handles the connected layout and
// the empty-tile skip; the other copy (the default) compiles the classical
// path alone, so that neither feature costs it anything.
template <int N, uint32_t PITCH, int T, bool GENERAL>
__device__ __forceinline__ void tile_phase(uint64_t *lds, const uint64_t *__restrict__ src,
                                           uint64_t *__restrict__ dst, const LatDesc &ld,
                                           const TileDesc &td, uint64_t s0, uint32_t S,
                                           uint32_t B, uint32_t hb, uint32_t cols,
                                           uint32_t ldw_arg, bool skip_empty) {
    const uint32_t ldw = PITCH ? PITCH : ldw_arg;
    const uint32_t nb = ld.nblocks;
    const uint32_t ncols = td.kint + 2u * hb;
    const uint32_t tid = threadIdx.x;
    const uint32_t nthr = blockDim.x;
    // first loaded block: (k0 - hb) mod nb, without going negative
    const uint32_t kfirst = static_cast<uint32_t>(
        (static_cast<uint64_t>(td.k0) + static_cast<uint64_t>(nb) * ((hb + nb - 1u) / nb) - hb) %
        nb);

    // even B and 16-byte aligned buffers: tile copies move site pairs
    const bool pairs = (B & 1u) == 0u &&
                       ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) == 0u;

    // ---- load tile + halo: consecutive lanes read consecutive words
    const bool fixed_row = (2u * nthr) % B == 0u;
    uint64_t any = 0;
    // Empty-tile skip: no rule of the models creates a particle next to an
    // empty window, so a tile whose loaded range (interior and halo) holds
    // no particle in any of the 64 samples ends the phase empty as well; it
    // writes its (zero) interior back without running the substeps. Exact:
    // the draws of windows that meet no particle change nothing.
    // The flag word after the tile says whether some wavefront loaded a
    // particle: cleared before the loads, set after the first barrier, read
    // after the second (no substep writes it).
    bool empty = false;
    // four teams: wavefront 0 writes the shared sites of the first batch
    // while the tile's loads are in flight (read after the barrier below)
    if (GENERAL && skip_empty) {
        uint32_t *flag = reinterpret_cast<uint32_t *>(lds + static_cast<size_t>(B) * ldw);
        if (tid == 0) *flag = 0u;
        load_tile_any<true>(lds, src + ld.base, pairs, fixed_row, kfirst, nb, ncols * B, B, ldw,
                            tid, nthr, any);
        if constexpr (T != 2) {
            if (tid < 64u) write_batch<N, T>(batch_share(lds, B, ldw), ld, s0, B);
        }
        __syncthreads();
        if (__ballot(any != 0ull) != 0ull && (tid & 63u) == 0u) *flag = 1u;
        __syncthreads();
        empty = __builtin_amdgcn_readfirstlane(*flag) == 0u;
    } else {
        load_tile_any<false>(lds, src + ld.base, pairs, fixed_row, kfirst, nb, ncols * B, B, ldw,
                             tid, nthr, any);
        if constexpr (T != 2) {
            if (tid < 64u) write_batch<N, T>(batch_share(lds, B, ldw), ld, s0, B);
        }
        __syncthreads();
    }

    // ---- connected layout: rotate the columns loaded from past the ends of
    // the word ring (only at a ring's first and last tiles, or in rings
    // shorter than the tile): front columns [0, lo_end), back [hi_start, ncols)
    if constexpr (GENERAL) {
        if (ld.connected && !empty) {
            const int64_t v0 = static_cast<int64_t>(td.k0) - hb;  // virtual block of column 0
            const uint32_t lo_end =
                v0 < 0 ? static_cast<uint32_t>(-v0 < static_cast<int64_t>(ncols) ? -v0 : ncols) : 0u;
            const int64_t hs = static_cast<int64_t>(nb) - v0;
            const uint32_t hi_start = hs <= 0 ? 0u : (hs >= ncols ? ncols : static_cast<uint32_t>(hs));
            const uint32_t nout = lo_end >= hi_start ? ncols : lo_end + (ncols - hi_start);
            if (nout > 0u) {
                for (uint32_t i = tid; i < nout * B; i += nthr) {
                    const uint32_t idx = i / B, o = i - idx * B;
                    const uint32_t c =
                        lo_end >= hi_start ? idx : (idx < lo_end ? idx : hi_start + idx - lo_end);
                    const int32_t m = ring_lap(v0 + c, nb);
                    if (m != 0) lds[o * ldw + c] = rotr64(lds[o * ldw + c], m);
                }
                __syncthreads();
            }
        }
    }

    // ---- S substeps in LDS, one window (block) per lane
    if (!empty) {
        // per is a multiple of the wavefront size, so the team is uniform
        // per wavefront and its branches stay on the scalar unit
        const uint32_t per = nthr / T;
        const uint32_t team = __builtin_amdgcn_readfirstlane(tid / per);
        const uint32_t c = tid - team * per;
        const uint32_t trash = cols + 1u;  // spare columns cols .. cols+2
        uint32_t kb = kfirst + c;
        if (kb >= nb) kb %= nb;
        if constexpr (GENERAL) {
            const int64_t v0 = static_cast<int64_t>(td.k0) - hb;
            const bool lapped =
                ld.connected && (v0 < 0 || v0 + static_cast<int64_t>(ncols) > static_cast<int64_t>(nb));
            const uint32_t rot =
                lapped && c < ncols ? static_cast<uint32_t>(ring_lap(v0 + c, nb)) & 63u : 0u;
            if (ld.mbits == 4u) {
                // the decision reads the thresholds at run time: one loop copy
                if (lapped)
                    run_team_loop<N, 0, 0, T>(lds, ld, WinT<true, true>{kb, rot}, c, team, ncols,
                                              trash, s0, S, B, ldw);
                else
                    run_team_loop<N, 0, 0, T>(lds, ld, WinT<false, true>{kb, 0u}, c, team, ncols,
                                              trash, s0, S, B, ldw);
            } else if (lapped) {
                dispatch_kd<N, T>(lds, ld, LapWin{kb, rot}, c, team, ncols, trash, s0, S, B, ldw);
            } else {
                dispatch_kd<N, T>(lds, ld, PlainWin{kb, 0u}, c, team, ncols, trash, s0, S, B, ldw);
            }
        } else {
            dispatch_kd<N, T>(lds, ld, PlainWin{kb, 0u}, c, team, ncols, trash, s0, S, B, ldw);
        }
    }

    // ---- write the interior back; it is contiguous in the ring
    uint64_t *out = dst + ld.base + static_cast<uint64_t>(td.k0) * B;
    if (pairs && fixed_row)
        store_interior_pairs<true>(out, lds, hb, td.kint * B, B, ldw, tid, nthr);
    else if (pairs)
        store_interior_pairs<false>(out, lds, hb, td.kint * B, B, ldw, tid, nthr);
    else
        store_interior(out, lds, hb, td.kint * B, B, ldw, tid, nthr);
}

// One workgroup per tile, one phase per launch. With 128-block tiles two
// workgroups share a CU, with 256-block tiles one does: T wavefronts per
// SIMD. PITCH is the LDS row pitch as a compile-time constant (0: the ldw_arg
// argument); with a constant pitch the rows of a window are immediate offsets
// from one address.
template <int N, uint32_t PITCH, int T, bool GENERAL>
__global__ void __launch_bounds__(256 * T) __attribute__((amdgpu_waves_per_eu(T, T)))
brs_phase(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
          const LatDesc *__restrict__ lats, const TileDesc *__restrict__ tiles,
          const uint64_t *__restrict__ clock, uint64_t s_off, uint32_t S, uint32_t B, uint32_t hb,
          uint32_t cols, uint32_t ldw_arg, uint32_t skip_empty) {
    // first substep of the phase: the context's device clock plus this
    // launch's offset, so that a captured sequence of launches is valid at
    // any starting time
    const uint64_t s0 = *clock + s_off;
    extern __shared__ uint64_t lds[];  // [B][ldw] lattice words
    const TileDesc td = tiles[blockIdx.x];
    const LatDesc ld = lats[td.lat];
    tile_phase<N, PITCH, T, GENERAL>(lds, src, dst, ld, td, s0, S, B, hb, cols, ldw_arg,
                                     skip_empty != 0u);
}

// ---- persistent sweep: every phase of a stretch in one launch --------------
//
// Work items (phase f, tile k) are handed out in order by an atomic ticket,
// phase-major, to a grid of resident workgroups, each of which loops until the
// tickets run out. Item (f, k) reads copy f % 2 and writes copy (f + 1) % 2.
// Before it starts it waits until every tile j in deps(k) -- the tiles whose
// interiors meet tile k's loaded range, which are also the tiles whose loaded
// ranges meet tile k's interior -- has finished phase f - 1: then what it
// reads is written (phase f - 1 of those tiles) and what it overwrites (tile
// k's interior in copy (f + 1) % 2) is no longer read (phase f - 1 of those
// tiles read it). Items only wait on items with smaller tickets, which were
// taken by running workgroups, so the oldest unfinished item can always
// proceed. Results are those of one launch per phase.
//
// Completion flags count finished phases per tile. Every wavefront of a
// finished item waits for its stores to reach the L2; after a barrier, one
// lane releases at agent scope (the L2 written back, visible to other XCDs)
// and sets the flag. Wavefront 0 of a waiting item polls the flags and then
// acquires at agent scope (L1 and L2 invalidated) before a barrier releases
// the workgroup to load the tile. One release and one acquire per item: with
// one per wavefront the L2 write-backs cost half the sweep's rate. A wait
// is bounded: past `spin_limit` polls the launch sets *abort and every
// workgroup stops (the host reports a device error); a correct schedule never
// comes near the limit.

template <int N, uint32_t PITCH, int T, bool GENERAL>
__global__ void __launch_bounds__(256 * T) __attribute__((amdgpu_waves_per_eu(T, T)))
brs_persistent(uint64_t *__restrict__ buf0, uint64_t *__restrict__ buf1,
               const LatDesc *__restrict__ lats, const TileDesc *__restrict__ tiles,
               const TileDeps *__restrict__ deps, uint32_t ntiles, uint32_t nphases,
               const uint64_t *__restrict__ clock, uint64_t s_off, uint32_t S, uint32_t S_last,
               uint32_t B, uint32_t hb, uint32_t cols, uint32_t ldw_arg,
               PersistState *__restrict__ state, uint32_t *__restrict__ done,
               uint32_t spin_limit, uint32_t skip_empty) {
    extern __shared__ uint64_t lds[];  // [B][ldw] lattice words
    __shared__ uint32_t sh_item, sh_stop;
    const uint64_t clk = *clock;
    const uint32_t tid = threadIdx.x;
    const bool wave0 = __builtin_amdgcn_readfirstlane(tid) < 64u;  // uniform per wavefront
    const uint32_t items = ntiles * nphases;
    uint32_t prev = items;  // the item finished last, not yet published (none)
    for (;;) {
        // One lane publishes the item just finished (every wavefront released
        // its stores at agent scope before the barrier that ended the item)
        // and takes the next ticket. No barrier and no loop inside this
        // branch: it is the only code that depends on the lane.
        if (tid == 0) {
            if (prev < items) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(done + (prev % ntiles), prev / ntiles + 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            uint32_t t = __hip_atomic_fetch_add(&state->ticket, 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_load(&state->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                t = items;
            sh_item = t;
        }
        __syncthreads();
        // every wavefront reads the same word: they all leave together
        const uint32_t t = __builtin_amdgcn_readfirstlane(sh_item);
        if (t >= items) break;
        const uint32_t f = t / ntiles, k = t - f * ntiles;
        if (wave0) {
          bool ok = true;
          if (f > 0u) {
            // wavefront 0 waits for phase f - 1 of the tiles k depends on:
            // deps(k) are the tiles local - lo .. local + hi of k's ring
            // (cyclic), or all of them when that span covers the ring
            const TileDeps dp = deps[k];
            const uint32_t lo = dp.lohi & 0xFFFFu, hi = dp.lohi >> 16;
            const uint32_t span = lo + hi + 1u;
            const bool all = span >= dp.count;
            const uint32_t nd = all ? dp.count : span;
            const uint32_t j0 = all ? 0u : dp.local + dp.count - lo;  // lo < count here
            uint32_t polls = 0;
            for (uint32_t d = 0; d < nd && ok; ++d) {
                const uint32_t *flag = done + dp.first + (j0 + d) % dp.count;
                while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(
                           flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < f) {
                    if (++polls > spin_limit ||
                        __builtin_amdgcn_readfirstlane(__hip_atomic_load(
                            &state->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                        __hip_atomic_store(&state->abort, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        ok = false;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
            }
            // one agent-scope acquire invalidates the CU's L1 and the XCD's L2
            // for every wavefront of the workgroup; it has completed before
            // the barrier below, so no later load of the tile sees stale lines
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_s_waitcnt(0);
          }
          sh_stop = ok ? 0u : 1u;  // the same value from every lane of wavefront 0
        }
        __syncthreads();  // the whole workgroup waits for wavefront 0's wait
        if (__builtin_amdgcn_readfirstlane(sh_stop)) break;
        const TileDesc td = tiles[k];
        const LatDesc ld = lats[td.lat];
        const uint64_t s0 = clk + s_off + static_cast<uint64_t>(f) * S;
        const uint32_t Sf = (f + 1u == nphases) ? S_last : S;
        tile_phase<N, PITCH, T, GENERAL>(lds, (f & 1u) ? buf1 : buf0, (f & 1u) ? buf0 : buf1, ld, td, s0,
                                Sf, B, hb, cols, ldw_arg, skip_empty != 0u);
        // Every wavefront waits until its own stores have reached the L2 (a
        // workgroup barrier alone does not wait for global stores); the lane
        // that publishes the item then writes the L2 back with one
        // agent-scope release, which covers the stores of every wavefront.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();  // all stores in L2; LDS free for the next item
        prev = t;
    }
}

// Clear the ticket, the abort word and the completion flags of a persistent
// launch (a kernel, not a memset, so that it can be captured in a graph).
__global__ void persist_reset(PersistState *__restrict__ state, uint32_t *__restrict__ done,
                              uint32_t ntiles) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        state->ticket = 0u;
        state->abort = 0u;
    }
    for (uint32_t j = i; j < ntiles; j += gridDim.x * blockDim.x) done[j] = 0u;
}

template <int N, uint32_t PITCH, int T, bool GENERAL>
hipError_t launch_kernel(const uint64_t *src, uint64_t *dst, const LatDesc *lats,
                         const TileDesc *tiles, uint32_t ntiles, const uint64_t *clock,
                         uint64_t s_off, uint32_t S, uint32_t B, const PhaseShape &sh,
                         hipStream_t stream) {
    const size_t lds = phase_lds_bytes(B, sh.ldw, S);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&brs_phase<N, PITCH, T, GENERAL>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(kMaxLdsBytes));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((brs_phase<N, PITCH, T, GENERAL>), dim3(ntiles), dim3(sh.threads), lds, stream,
                       src, dst, lats, tiles, clock, s_off, S, B, sh.hb, sh.cols, sh.ldw,
                       sh.skip_empty);
    return hipGetLastError();
}

template <int N, int T>
hipError_t launch_teams(const uint64_t *src, uint64_t *dst, const LatDesc *lats,
                        const TileDesc *tiles, uint32_t ntiles, const uint64_t *clock,
                        uint64_t s_off, uint32_t S, uint32_t B, const PhaseShape &sh,
                        hipStream_t stream) {
    if (sh.general)
        return launch_kernel<N, 0, T, true>(src, dst, lats, tiles, ntiles, clock, s_off, S, B, sh,
                                            stream);
    if constexpr (N == 2) {
        if (sh.ldw == kDefaultPitch)
            return launch_kernel<N, kDefaultPitch, T, false>(src, dst, lats, tiles, ntiles, clock,
                                                             s_off, S, B, sh, stream);
    }
    return launch_kernel<N, 0, T, false>(src, dst, lats, tiles, ntiles, clock, s_off, S, B, sh,
                                         stream);
}

template <int N, uint32_t PITCH, int T, bool GENERAL>
hipError_t launch_persist_kernel(const PersistLaunch &a, const PhaseShape &sh,
                                 hipStream_t stream) {
    auto kernel = &brs_persistent<N, PITCH, T, GENERAL>;
    const size_t lds = phase_lds_bytes(a.B, sh.ldw, a.S);
    if (lds + kPersistStaticLds > kMaxLdsBytes) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        // the kernel's own shared words come out of the same 160 KB
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(kMaxLdsBytes - kPersistStaticLds));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    // as many workgroups as are resident at once, at most one per item; the
    // count bounds only the grid (workgroups that are not resident yet take
    // no ticket), so the LDS bound stands in if the occupancy query fails
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel),
                                                     static_cast<int>(sh.threads),
                                                     lds) != hipSuccess ||
        per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = static_cast<int>(kMaxLdsBytes / (lds + 64));
    }
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const uint64_t items = static_cast<uint64_t>(a.ntiles) * a.nphases;
    uint64_t grid = static_cast<uint64_t>(per_cu > 0 ? per_cu : 1) * static_cast<uint64_t>(cus);
    if (grid > items) grid = items;
    hipLaunchKernelGGL(persist_reset, dim3((a.ntiles + 255u) / 256u), dim3(256), 0, stream,
                       a.state, a.done, a.ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(kernel, dim3(static_cast<uint32_t>(grid)), dim3(sh.threads), lds, stream,
                       a.buf0, a.buf1, a.lats, a.tiles, a.deps, a.ntiles, a.nphases, a.clock,
                       a.s_off, a.S, a.S_last, a.B, sh.hb, sh.cols, sh.ldw, a.state, a.done,
                       a.spin_limit, sh.skip_empty);
    return hipGetLastError();
}

template <int N, int T>
hipError_t launch_persist_teams(const PersistLaunch &a, const PhaseShape &sh, hipStream_t stream) {
    if (sh.general) return launch_persist_kernel<N, 0, T, true>(a, sh, stream);
    if constexpr (N == 2) {
        if (sh.ldw == kDefaultPitch)
            return launch_persist_kernel<N, kDefaultPitch, T, false>(a, sh, stream);
    }
    return launch_persist_kernel<N, 0, T, false>(a, sh, stream);
}

template <int N>
hipError_t launch_persist_n(const PersistLaunch &a, const PhaseShape &sh, hipStream_t stream) {
    if (a.ntiles == 0 || a.nphases == 0) return hipSuccess;
    switch (sh.teams) {
        case 2: return launch_persist_teams<N, 2>(a, sh, stream);
        case 4: return launch_persist_teams<N, 4>(a, sh, stream);
        default: return hipErrorInvalidValue;
    }
}

// The default PCPD tile runs a copy of the kernel compiled for its pitch;
// every other model and shape takes the pitch as an argument. Two or four
// teams per tile. Contexts with the connected layout or the empty-tile skip
// run the general copy (pitch as an argument).
template <int N>
hipError_t launch_phase_n(const uint64_t *src, uint64_t *dst, const LatDesc *lats,
                          const TileDesc *tiles, uint32_t ntiles, const uint64_t *clock,
                          uint64_t s_off, uint32_t S, uint32_t B, const PhaseShape &sh,
                          hipStream_t stream) {
    switch (sh.teams) {
        case 2: return launch_teams<N, 2>(src, dst, lats, tiles, ntiles, clock, s_off, S, B, sh, stream);
        case 4: return launch_teams<N, 4>(src, dst, lats, tiles, ntiles, clock, s_off, S, B, sh, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace pcpd
