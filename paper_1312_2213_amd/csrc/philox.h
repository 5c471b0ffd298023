// philox.h -- Philox4x32-10 counter-based generator for gfx950 device code.
//
// Definition: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3" (SC'11), Philox4x32 with 10 rounds: per round
//   (hi0, lo0) = M0 * x0,  (hi1, lo1) = M1 * x2,
//   x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0),
// and the key advances by the Weyl increments between rounds.
//
// Stream layout used by every kernel: counter = (chain, sweep, block, tag),
// key = (seed low 32 bits, seed high 32 bits).  With the chain in x0 and the
// block in x2, the first two rounds split into a per-lane constant part
// (chain) and a wave-uniform part (sweep, block), which the compiler keeps
// in scalar registers; only rounds 3..10 cost vector multiplies.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muca {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

constexpr uint32_t kTagSweep = 0u;
constexpr uint32_t kTagInit = 1u;
constexpr uint32_t kTagRotate = 2u; // polymer spherical rotations
constexpr uint32_t kTagBridge = 3u; // polymer double bridging

struct Words4 {
    uint32_t w[4];
};

// Rounds 0 and 1 keep plain XORs so that wave-uniform inputs can stay on
// the scalar unit; later rounds use one gfx950 three-input bitop3 (truth
// table 0x96 = a ^ b ^ c) per output word.
template <int R>
__device__ __forceinline__ void philox_round(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3,
                                             uint32_t k0, uint32_t k1)
{
    const uint64_t p0 = (uint64_t)kPhiloxM0 * x0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * x2;
    uint32_t n0, n2;
    if constexpr (R < 2) {
        n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    } else {
        n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), x1, k0, 0x96);
        n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), x3, k1, 0x96);
    }
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = n0;
    x2 = n2;
}

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
    philox_round<0>(c0, c1, c2, c3, k0, k1);
    philox_round<1>(c0, c1, c2, c3, k0 + 1u * kPhiloxW0, k1 + 1u * kPhiloxW1);
    philox_round<2>(c0, c1, c2, c3, k0 + 2u * kPhiloxW0, k1 + 2u * kPhiloxW1);
    philox_round<3>(c0, c1, c2, c3, k0 + 3u * kPhiloxW0, k1 + 3u * kPhiloxW1);
    philox_round<4>(c0, c1, c2, c3, k0 + 4u * kPhiloxW0, k1 + 4u * kPhiloxW1);
    philox_round<5>(c0, c1, c2, c3, k0 + 5u * kPhiloxW0, k1 + 5u * kPhiloxW1);
    philox_round<6>(c0, c1, c2, c3, k0 + 6u * kPhiloxW0, k1 + 6u * kPhiloxW1);
    philox_round<7>(c0, c1, c2, c3, k0 + 7u * kPhiloxW0, k1 + 7u * kPhiloxW1);
    philox_round<8>(c0, c1, c2, c3, k0 + 8u * kPhiloxW0, k1 + 8u * kPhiloxW1);
    philox_round<9>(c0, c1, c2, c3, k0 + 9u * kPhiloxW0, k1 + 9u * kPhiloxW1);
    Words4 o;
    o.w[0] = c0;
    o.w[1] = c1;
    o.w[2] = c2;
    o.w[3] = c3;
    return o;
}

} // namespace muca
