// Internal launch interfaces between the C ABI (api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace synth {

constexpr int kNumParams = 78;

// Per-parameter range hyperparameters (Section 3.3), passed by value in the
// kernel argument block (1.9 KB, below the 4 KB kernarg limit).
struct NebulaArgs {
  double lo[kNumParams];
  double hi[kNumParams];
  double inv_curve[kNumParams];   // 1 / curve
  uint32_t sym[3];                // bit p: parameter p is symmetric
  uint32_t linear[3];             // bit p: curve == 1 (no warp)
};

struct RenderArgs {
  const float* params;       // [B][78]
  const uint64_t* voice_ids; // [B] or null
  const int64_t* offsets;    // [B+1] or null
  float* audio;
  uint64_t first_g;
  int64_t n_uniform;
  int64_t batch;
  double sr;                 // sample rate
  double rc;                 // control rate
  double nyq_midi;           // pitch (MIDI) above which f > sr / 2
  int q;                     // audio samples per control sample
  uint32_t q_magic;          // ceil(2^32 / q): x / q == umulhi(x, q_magic) for x < 2^16
  int slices;                // workgroups per voice (uniform lengths only)
  int persistent_grid;       // >0: workgroup w renders voices w, w+grid, ...
  int mix_mode;
  uint32_t nk0, nk1;         // noise key
  NebulaArgs neb;
};

hipError_t launch_sample_params(uint64_t seed, uint64_t first_g, int64_t batch,
                                const uint64_t* voice_ids, float* params, hipStream_t s);

// runs_per_segment in {1, 2, 4}; clamp: some pitch can exceed sr / 2.
hipError_t launch_render(const RenderArgs& a, int runs_per_segment, bool clamp, int grid,
                         hipStream_t s);

hipError_t launch_peak_normalise(const RenderArgs& a, hipStream_t s);

size_t adjoint_workspace_bytes(int64_t batch, int64_t n_samples, int q);
int64_t adjoint_max_chunks();
hipError_t launch_render_backward(const RenderArgs& a, const float* grad_audio, double* ws,
                                  float* grad_params, int runs_per_segment, hipStream_t s);

hipError_t launch_mrstft(const float* x, const float* target, int64_t batch, int64_t n_samples,
                         double* loss, float* grad, hipStream_t s);

}  // namespace synth
