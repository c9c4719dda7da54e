// philox.hpp -- device Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
//
// Counter-based: the output is a pure function of (counter, key), so every
// 64-site word draws its own random words from (g, t, 2j + parity, 0) with no
// per-thread generator state to load or store (the paper keeps a TinyMT
// state per thread, Sec. II-B).  The key is a kernel argument and stays in
// scalar registers; the first round's product of the uniform counter word is
// scalar work as well.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sca {

struct u32x4 {
    uint32_t v0, v1, v2, v3;
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u;
    constexpr uint32_t kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u;
    constexpr uint32_t kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // One 32x32->64 product gives both halves (v_mad_u64_u32, full rate on
        // gfx950, where separate mul_hi and mul_lo take two instructions), and
        // each three-way xor is one v_bitop3_b32 (truth table 0x96).
        const uint64_t pA = (uint64_t)kMulA * c0;
        const uint64_t pB = (uint64_t)kMulB * c2;
        const uint32_t hiA = (uint32_t)(pA >> 32), loA = (uint32_t)pA;
        const uint32_t hiB = (uint32_t)(pB >> 32), loB = (uint32_t)pB;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hiB, c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hiA, c3, k1, 0x96);
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return {c0, c1, c2, c3};
}

}  // namespace sca
