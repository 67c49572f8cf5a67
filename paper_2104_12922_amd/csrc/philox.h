// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel Random Numbers: As Easy as 1, 2, 3", SC 2011), device side.
//
// The paper renders its corpus from deterministic random numbers, the noise
// oscillators included (Section 2.1).  Both the parameter draw and the noise
// oscillator use this bijection: key = 64-bit seed, counter = (voice id lo,
// voice id hi, block index, stream), stream 0 for parameters, 1 for noise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace synth {

// In-place: c[0..3] <- Philox4x32-10(c, (k0, k1)).  Each round forms the two
// 64-bit products of words 0 and 2 with the round multipliers, mixes their
// high halves with words 1 and 3 and the key, and the key advances by the Weyl
// increments between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    // three-input XORs: one v_bitop3_b32 each (truth table 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c[1], k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c[3], k1, 0x96);
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

}  // namespace synth
