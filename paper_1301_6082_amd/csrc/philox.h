// philox.h -- Philox-4x32-10 for device code (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11). One round maps
// (c0, c1, c2, c3) to (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
// lo(M0*c0)); the key advances by the Weyl constants between rounds. The
// 32x32->64 products compile to v_mad_u64_u32, the three-input XORs to one
// v_bitop3_b32 each.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pcpd {

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
        nx.x = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pb >> 32), c.y, ka, 0x96);
        nx.y = static_cast<uint32_t>(pb);
        nx.z = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pa >> 32), c.w, kb, 0x96);
        nx.w = static_cast<uint32_t>(pa);
        c = nx;
        ka += kWeylA;
        kb += kWeylB;
    }
    return c;
}

}  // namespace pcpd
