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

// Voice b's sample range [start, start + len) in a packed batch with
// offsets[0 .. batch] (int64, required non-decreasing with offsets[0] = 0, so
// that the buffer holds offsets[batch] samples).  The range is cut to
// [0, offsets[batch]) (empty if nothing is left), so a malformed offsets
// array cannot make a kernel read or write outside the caller's buffer; for
// valid offsets it is offsets[b] .. offsets[b + 1].
__device__ __forceinline__ void packed_range(const int64_t* offsets, int64_t batch, int64_t b,
                                             int64_t& start, int64_t& len) {
  const int64_t total = offsets[batch];
  int64_t s = offsets[b], e = offsets[b + 1];
  if (s < 0) s = 0;
  if (e > total) e = total;
  start = s;
  len = e > s ? e - s : 0;
}

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
  const int32_t* order;      // null, or the voices in the order workgroups take them
  const double* carries;     // null, or [B][carry_stride][4] chunk-start carries
  int64_t carry_stride;      // chunks per voice in carries
};

// ---------------------------------------------------------------------------
// bf16 MFMA GEMM (gemm.hip): C[M x N] = alpha * A[M x K] B[K x N] (+ bias, epilogue)
// ---------------------------------------------------------------------------
enum {
  kEpiNone = 0,        // store x
  kEpiGelu = 1,        // store gelu(x) (erf form); pre-activation to pre if given
  kEpiSigmoid = 2,     // store 1 / (1 + exp(-x))
  kEpiGeluGrad = 3,    // store x * gelu'(aux[row][col])
  kEpiPowerPairs = 4,  // columns (2f, 2f+1) = (Re, Im): store Re^2 + Im^2 at column f
  kEpiLogMelT = 5      // store log(x + 1e-6) at feature[(row / 64) * 8192 + col * 64 + row % 64]
};
enum { kOpKMajor = 0, kOpRowMajorMN = 1 };

struct GemmArgs {
  int64_t M, N, K;
  const void* A;       // bf16
  int64_t lda;
  const void* B;       // bf16
  int64_t ldb;
  void* C;
  int64_t ldc;
  int c_bf16;          // output dtype: 1 bf16, 0 float32
  const float* bias;   // [N] or null
  int epilogue;
  const float* aux;    // kEpiGeluGrad operand, same layout as C
  float* pre;          // optional float32 pre-activation output (layout of C)
  float alpha, beta;   // beta != 0: C = epi(...) + beta * C
  int split;           // > 1: split K over that many workgroups per tile (epilogues 0-3)
  float* partial;      // split > 1: float32 workspace [split][M][N]
};

hipError_t launch_gemm_bf16(const GemmArgs& g, int a_op, int b_op, hipStream_t s);
// Split that fills the chip for a GEMM of this shape (1: none), and its
// workspace bytes.
int gemm_split_for(int64_t M, int64_t N, int64_t K);
size_t gemm_split_bytes(int64_t M, int64_t N, int split);

// elementwise / reduction helpers of the learned proposal (mlp.hip)
hipError_t launch_f32_to_bf16(const float* x, void* y, int64_t n, hipStream_t s);
hipError_t launch_diff_reduce(int kind, int axis, const float* a, const float* b, int64_t rows,
                              int64_t cols, int64_t lda, int64_t ldb, double scale, int accumulate,
                              double* out, hipStream_t s);
hipError_t launch_sum_f64(const double* x, int64_t n, double scale, double* out, hipStream_t s);
hipError_t launch_scale_rows(const float* g, const double* sc, int64_t rows, int64_t cols,
                             float* out, hipStream_t s);
size_t l1_pair_sum_workspace(int64_t n, int64_t m, int64_t dim);
hipError_t launch_l1_pair_sum(const float* A, int64_t lda, int64_t n, const float* B, int64_t ldb,
                              int64_t m, int64_t dim, double* partial, double* out, hipStream_t s);
hipError_t launch_mmd_combine(double* out, int64_t n, int64_t m, hipStream_t s);
hipError_t launch_fm_render(const float* params, const int64_t* offsets, int64_t batch,
                            int64_t n_samples, float* audio, double sr, double rc, int q,
                            const NebulaArgs& neb, const int32_t* order, hipStream_t s);
int64_t vcf_chunks(int64_t max_samples, int q);
hipError_t launch_vcf_forward(const float* x, const int64_t* offsets, int64_t batch,
                              int64_t n_samples, const float* env, int64_t env_ld,
                              const float* params, int q, double sr, float* y, double* states,
                              int64_t state_ld, const int32_t* order, hipStream_t s);
hipError_t launch_vcf_backward(const float* x, const float* g, const int64_t* offsets,
                               int64_t batch, int64_t n_samples, const float* env, int64_t env_ld,
                               const float* params, int q, double sr, const double* states,
                               int64_t state_ld, float* g_x, float* g_params, float* g_env,
                               const int32_t* order, hipStream_t s);
hipError_t launch_colsum(const void* x, int x_bf16, int64_t rows, int64_t cols, int64_t ld,
                         float* sum, float* sumsq, hipStream_t s);
// Column sums of a bf16 matrix (bias gradients) in two deterministic passes
// through a float64 workspace of colsum_ws_bytes(rows, cols) bytes (falls
// back to launch_colsum when the workspace is missing or too small).
size_t colsum_ws_bytes(int64_t rows, int64_t cols);
hipError_t launch_colsum_bf16_ws(const void* x, int64_t rows, int64_t cols, int64_t ld, float* sum,
                                 void* ws, size_t ws_bytes, hipStream_t s);
hipError_t launch_feature_stats(const float* x, int64_t rows, int64_t cols, float min_var,
                                float* mean, float* inv_std, hipStream_t s);
hipError_t launch_standardize(const float* x, const float* mean, const float* inv_std,
                              int64_t rows, int64_t cols, void* y_bf16, hipStream_t s);
hipError_t launch_mse_sigmoid_grad(const float* out, const float* target, int64_t rows,
                                   int64_t cols, void* dz_bf16, double* loss_rows,
                                   hipStream_t s);
hipError_t launch_adam(int64_t n, float* w, void* w_bf16, const float* g, float* m, float* v,
                       float lr, float b1, float b2, float eps, int step, hipStream_t s);
// log-mel power spectrum (dft.hip): basis bf16 [2048][2048]; power bf16 [batch * 64][ldp]
hipError_t launch_dft_basis(void* basis_bf16, hipStream_t s);
hipError_t launch_dft_power(const float* audio, const int64_t* offsets, int64_t n_uniform,
                            int64_t batch, const void* basis, void* power, int64_t ldp,
                            hipStream_t s);
hipError_t launch_logit_init(const float* u, float* z, float* u_out, int64_t n, float eps,
                             hipStream_t s);
hipError_t launch_logit_adam(int64_t n, float* z, float* u, const float* grad_u, float* m,
                             float* v, float lr, float b1, float b2, float eps, int step,
                             hipStream_t s);
hipError_t launch_best_update(const double* loss, int64_t rows, int64_t cols, int64_t row_stride,
                              int64_t col_stride, int64_t col_base, const float* params,
                              int64_t param_dim, double* best, int64_t* best_idx,
                              float* best_params, hipStream_t s);

hipError_t launch_is_test(uint64_t first_g, int64_t batch, const uint64_t* voice_ids,
                          uint8_t* is_test, hipStream_t s);
hipError_t launch_sample_params(uint64_t seed, uint64_t first_g, int64_t batch,
                                const uint64_t* voice_ids, float* params, hipStream_t s,
                                int n_params = kNumParams, uint32_t tag = 0);

// runs_per_segment in {1, 2, 4}; clamp: some pitch can exceed sr / 2.
hipError_t launch_render(const RenderArgs& a, int runs_per_segment, bool clamp, int grid,
                         hipStream_t s);
// Chunk-start phase carries of every voice for a render split over
// workgroups (render.hip): [B][stride][4] doubles (LFO 1, LFO 2, VCO 1,
// VCO 2), stride = chunks of the longest voice.
hipError_t launch_voice_carries(const RenderArgs& a, int runs_per_segment, bool clamp,
                                double* carries, int64_t stride, hipStream_t s);

hipError_t launch_peak_normalise(const RenderArgs& a, hipStream_t s);

size_t adjoint_workspace_bytes(int64_t batch, int64_t n_samples, int q);
// where the chunk-start carries begin in an adjoint workspace
double* adjoint_carries(double* ws, int64_t batch, int64_t n_samples, int q);
int64_t adjoint_max_chunks();
hipError_t launch_render_backward(const RenderArgs& a, const float* grad_audio, double* ws,
                                  float* grad_params, int runs_per_segment, hipStream_t s);

// log-mel features by FFT (spectral.hip): mel_basis bf16 [128][ldm] with each
// band's first and last nonzero bin in columns 1025 and 1026; features float32
// [batch][128][64].
constexpr int kMelBands = 128;
constexpr int kMelWeightsMax = 2304;   // nonzero mel weights over all bands
hipError_t launch_logmel_fft(const float* audio, const int64_t* offsets, int64_t n_uniform,
                             int64_t batch, const void* mel_basis, int64_t ldm, float* features,
                             hipStream_t s);
// The same features standardised and rounded to bf16 (see MelStd in spectral.hip).
hipError_t launch_logmel_fft_std(const float* audio, const int64_t* offsets, int64_t n_uniform,
                                 int64_t batch, const void* mel_basis, int64_t ldm,
                                 const float* mean, const float* inv_std, const int64_t* row_map,
                                 void* out_bf16, hipStream_t s);
size_t mrstft_workspace_bytes(int64_t batch, int64_t n_samples, bool with_grad);
// tlog: NULL (target frames transformed every call) or the target's log
// magnitudes from launch_mrstft_target (target then unused).
hipError_t launch_mrstft(const float* x, const float* target, const float* tlog, int64_t batch,
                         int64_t n_samples, double* loss, float* grad, void* workspace,
                         hipStream_t s);
size_t mrstft_target_bytes(int64_t batch, int64_t n_samples);
hipError_t launch_mrstft_target(const float* target, int64_t batch, int64_t n_samples, float* tlog,
                                hipStream_t s);

}  // namespace synth
