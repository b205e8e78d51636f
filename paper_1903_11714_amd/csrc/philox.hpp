// philox.hpp — Philox4x32-10 for gfx950 device code.
//
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11, "Parallel random numbers:
// as easy as 1, 2, 3"): ten rounds of two 32x32 -> 64-bit products (M0 * x0, M1 * x2) mixed
// with the other two words and the key; the key advances by the Weyl increments (W0, W1)
// between rounds.  The whole key schedule is uniform across a launch, so it lives in scalar
// registers and costs no vector instructions; each round is two v_mad_u64_u32 and two three-input xors.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

// P0 / P2: the number of leading rounds whose new word 0 / word 2 is formed with plain xors instead of
// v_bitop3_b32.  A plain xor lets the compiler keep a round whose inputs are uniform on the scalar
// unit, and it folds two uniform operands into one before a single vector xor; v_bitop3_b32 is the
// better form once two of the three inputs vary by lane.  The defaults suit a counter of a
// lane-varying group and row with a uniform sweep and colour word; a caller whose row is uniform
// passes <2, 3>.  Every choice computes the same function.
template <int P0 = 2, int P2 = 1>
__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t a = (uint64_t)kPhiloxM0 * c0;
        const uint64_t b = (uint64_t)kPhiloxM1 * c2;
        // three-input xor in one gfx950 v_bitop3_b32 (truth table 0x96)
        const uint32_t n0 = round < P0 ? (uint32_t)(b >> 32) ^ (c1 ^ k0)
                                       : __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), c1, k0, 0x96);
        const uint32_t n2 = round < P2 ? (uint32_t)(a >> 32) ^ (c3 ^ k1)
                                       : __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), c3, k1, 0x96);
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return Words4{c0, c1, c2, c3};
}

}  // namespace ising
