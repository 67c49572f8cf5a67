// Deterministic parameter draw (Sections 2.1 and 3.3): u[i][p] in [0, 1) from
// Philox4x32-10, key = seed, counter = (g lo, g hi, p >> 2, tag), word p & 3,
// u = top 24 bits * 2^-24 (exact in float32); tag names the synth
// architecture (0: the default Voice, 1: the FM voice).  One thread per
// (voice, block of four parameters).
#include "philox.h"
#include "synth_internal.h"

namespace synth {
namespace {

__global__ void __launch_bounds__(256) sample_params_kernel(uint64_t seed, uint64_t first_g,
                                                            int64_t batch, const uint64_t* ids,
                                                            int n_params, uint32_t tag,
                                                            float* out) {
  const int blocks_per_voice = (n_params + 3) / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = t / blocks_per_voice;
  const int blk = (int)(t - b * blocks_per_voice);
  if (b >= batch) return;
  const uint64_t g = ids ? ids[b] : first_g + (uint64_t)b;
  uint32_t w[4] = {(uint32_t)g, (uint32_t)(g >> 32), (uint32_t)blk, tag};
  philox4x32_10(w, (uint32_t)seed, (uint32_t)(seed >> 32));
  float* row = out + b * n_params;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int p = 4 * blk + e;
    if (p < n_params) row[p] = (float)(w[e] >> 8) * (1.0f / 16777216.0f);
  }
}

// is_test[i] = 1 if voice g = ids[i] (or first_g + i) lies in a test block:
// (g div 1024) mod 10 == 9 (the corpus's 9:1 split in blocks of 1024).
__global__ void __launch_bounds__(256) is_test_kernel(uint64_t first_g, int64_t batch,
                                                      const uint64_t* ids, uint8_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch) return;
  const uint64_t g = ids ? ids[i] : first_g + (uint64_t)i;
  out[i] = (uint8_t)(((g >> 10) % 10u) == 9u);
}

}  // namespace

hipError_t launch_is_test(uint64_t first_g, int64_t batch, const uint64_t* voice_ids,
                          uint8_t* is_test, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(is_test_kernel, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s,
                     first_g, batch, voice_ids, is_test);
  return hipGetLastError();
}

hipError_t launch_sample_params(uint64_t seed, uint64_t first_g, int64_t batch,
                                const uint64_t* voice_ids, float* params, hipStream_t s,
                                int n_params, uint32_t tag) {
  if (batch == 0) return hipSuccess;
  const int64_t threads = batch * ((n_params + 3) / 4);
  const int64_t blocks = (threads + 255) / 256;
  hipLaunchKernelGGL(sample_params_kernel, dim3((unsigned)blocks), dim3(256), 0, s, seed,
                     first_g, batch, voice_ids, n_params, tag, params);
  return hipGetLastError();
}

}  // namespace synth
