/*
 * synth.h - C ABI of the MI355X modular-synthesizer voice renderer.
 *
 * Implements the hot path of "One Billion Audio Sounds from GPU-enabled Modular
 * Synthesis" (Turian et al., DAFx 2021, arXiv 2104.12922): batched rendering of
 * the default Voice (Section 3.2) from normalised parameters (Section 3.3),
 * with deterministic counter-based random numbers for both the parameters and
 * the noise oscillator (Section 2.1).
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status (synth_status); none throws.
 *   - "dev" pointers are HIP device pointers owned by the caller; "host" pointers
 *     are read during the call only.  The library keeps no reference to either.
 *   - Calls are stream-ordered and asynchronous on the given HIP stream
 *     (hipStream_t passed as void*; NULL = the default stream).  The library
 *     never synchronises; a device fault surfaces at the caller's next sync.
 *   - Argument errors are detected on the host before any launch and return
 *     SYNTH_EINVAL / SYNTH_EUNSUPPORTED with nothing written.
 *   - The library allocates no device memory on these paths.
 *   - Results are bitwise deterministic for fixed inputs and independent of the
 *     batch composition (a voice's output depends only on its parameters, its
 *     voice id and the config).
 */
#ifndef SYNTH_H_
#define SYNTH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SYNTH_OK = 0,
    SYNTH_EINVAL = -1,        /* bad pointer, size or value */
    SYNTH_ENOMEM = -2,        /* caller-provided buffer too small */
    SYNTH_EDEVICE = -3,       /* HIP launch/runtime error */
    SYNTH_EUNSUPPORTED = -4   /* valid but not implemented configuration */
} synth_status;

#define SYNTH_NUM_PARAMS 78

/* Render configuration.
 *   sample_rate  audio rate in Hz (44100 by default, Section 2.2); must be an
 *                integer multiple q of control_rate with q % 4 == 0, q <= 1024.
 *   control_rate rate of the control modules (ADSR, LFO) in Hz (441 by
 *                default, Section 3.1).
 *   noise_seed   64-bit key of the noise oscillator's counter-based generator.
 *   mix_mode     0: audio mixer output is the plain sum of the three levelled
 *                VCA outputs; 1: additionally each voice is divided by
 *                max(1, peak |y|) (peak-normalise only when clipping).
 *   nebula       host pointer to [78][4] doubles, row p = (min, max, curve,
 *                symmetric) of parameter p (Section 3.3; symmetric is 0 or 1,
 *                curve > 0).  Required. */
typedef struct synth_config {
    double sample_rate;
    double control_rate;
    uint64_t noise_seed;
    int32_t mix_mode;
    int32_t reserved;        /* must be 0 */
    const double* nebula;
} synth_config;

/* Number of normalised parameters of the Voice: 78 (Section 1.1). */
int synth_num_params(void);

/* Parameter p (0 <= p < 78) of the default Voice in canonical order: its
 * name ("module.parameter", static string), and the default nebula's min,
 * max, curve and symmetric flag (Section 3.3).  Any output pointer may be
 * NULL.  SYNTH_EINVAL for p out of range. */
int synth_param_info(int p, const char** name, double* min, double* max, double* curve,
                     int* symmetric);

/* Static, NUL-terminated description of a status code. */
const char* synth_status_string(int status);

/* Train/test split of the corpus (Section 2.2): 9*1024 train voices, then 1024
 * test voices, repeating.  Returns 1 if global voice index g is a test voice. */
int synth_is_test(uint64_t g);

/* Deterministic parameter draw (Sections 2.1 and 3.3).
 *   params[i][p] = (w >> 8) * 2^-24, w = word (p & 3) of Philox4x32-10 with
 *   key (seed lo, seed hi) and counter (g lo, g hi, p >> 2, 0), where
 *   g = voice_ids[i] if voice_ids != NULL else first_g + i.
 *   voice_ids  dev uint64 [batch] or NULL.
 *   params     dev float32 [batch][78], written; values in [0, 1 - 2^-24].
 *   batch >= 0 (0 is a no-op). */
int synth_sample_params(uint64_t seed, uint64_t first_g, int64_t batch,
                        const uint64_t* voice_ids, float* params, void* stream);

/* Render a batch of voices (Sections 3.1-3.3).
 *   params     dev float32 [batch][78], normalised parameters in [0, 1].
 *   voice_ids  dev uint64 [batch] or NULL (=> first_g + i); addresses the
 *              noise oscillator's counter.
 *   offsets    dev int64 [batch + 1] or NULL.  If given, voice i is written to
 *              audio[offsets[i] .. offsets[i+1]) (ragged lengths, packed); the
 *              offsets must be non-decreasing from offsets[0] = 0.  They are
 *              read on the device (not checked on the host); every kernel cuts
 *              a voice's range to [0, offsets[batch]), so malformed offsets
 *              give undefined audio but no access outside audio[0 ..
 *              offsets[batch]).  If NULL every voice has n_samples samples
 *              and voice i starts at audio[i * n_samples].
 *   n_samples  uniform length when offsets == NULL (> 0); ignored otherwise.
 *   audio      dev float32, written: batch * n_samples floats, or offsets[batch].
 *   Output: y(n) = L1 * sine(n) * a1(n) + L2 * squaresaw(n) * a2(n)
 *                  + L3 * noise(n) * a3(n) (mix_mode 0).
 * Float32 audio; the phase of both oscillators is accumulated in float64. */
int synth_render(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                 uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                 float* audio, void* stream);

/* synth_render with a workspace: small uniform batches then split each voice
 * over more workgroups, with the chunk-start phase carries computed first
 * (see synth_render_plan_ws); the audio is bit-identical to synth_render's.
 * synth_render_workspace returns the bytes it needs (0: the default plan does
 * not split this batch, and synth_render_ws is synth_render).  workspace ==
 * NULL or offsets != NULL: exactly synth_render. */
size_t synth_render_workspace(const synth_config* cfg, int64_t batch, int64_t n_samples);
int synth_render_ws(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                    uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                    float* audio, void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * synth_render_ws with its workspace taken from a buffer the library holds,
 * a static device array of SYNTH_NOALLOC_SCRATCH_BYTES (16 MiB) on each device
 * it runs on, kept until the process ends.  Same arguments and bit-identical
 * audio as synth_render_ws / synth_render; allocates nothing.  Returns
 * SYNTH_ENOMEM when the batch needs more workspace than the array holds
 * (synth_render_workspace(cfg, batch, n_samples) > SYNTH_NOALLOC_SCRATCH_BYTES:
 * batch * ceil(ceil(n_samples / q) / 62) * 32 bytes for a split batch), and
 * SYNTH_EDEVICE if the array's device address cannot be obtained.  Every call
 * on one device shares that device's array: calls that overlap on a device
 * (concurrent streams or threads) race and must be serialised by the caller. */
#define SYNTH_NOALLOC_SCRATCH_BYTES (16 << 20)
int synth_render_noalloc(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                         uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                         float* audio, void* stream);

/* Corpus generator (Section 2.1: every sound of the corpus is addressed by
 * its index and reproduced from the seed alone, parameters and noise alike;
 * Section 2.2: a 9:1 train/test split in blocks of 1024).  For voices
 * g = voice_ids[i] (dev uint64 [batch]) or first_g + i (voice_ids NULL):
 *   params   dev float32 [batch][78]: synth_sample_params(seed, g)
 *   audio    dev float32 [batch][n_samples]: synth_render of those
 *            parameters with the noise keyed by seed (cfg->noise_seed is
 *            not used; the rest of cfg as for synth_render)
 *   is_test  dev uint8 [batch]: synth_is_test(g)
 * workspace as synth_render_ws (synth_render_workspace(cfg, batch,
 * n_samples) bytes, or NULL).  A voice's outputs depend only on (seed, g),
 * so the corpus shards over devices and processes by ranges of g with no
 * communication.  Errors as synth_sample_params and synth_render_ws. */
int synth_generate(const synth_config* cfg, uint64_t seed, const uint64_t* voice_ids,
                   uint64_t first_g, int64_t batch, int64_t n_samples, float* params, float* audio,
                   uint8_t* is_test, void* workspace, size_t workspace_bytes, void* stream);

/* Same as synth_render with an explicit launch plan (used by the autotuner and
 * by tests): runs_per_segment in {1, 2, 4} splits each control period into
 * that many per-lane runs; slices_per_voice >= 1 splits each voice over that
 * many workgroups (each takes a contiguous share of the voice's 62-period
 * chunks; uniform lengths must have at least that many chunks); persistent != 0 launches
 * grid_blocks workgroups (0 => chosen by the library) of which workgroup w
 * renders voices w, w + grid_blocks, w + 2 * grid_blocks, ... (no device
 * state).  Fails with SYNTH_EUNSUPPORTED for a plan the configuration cannot
 * use, SYNTH_EINVAL for out-of-range plan values. */
int synth_render_plan(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                      uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                      float* audio, int runs_per_segment, int slices_per_voice,
                      int persistent, int grid_blocks, void* stream);

/* synth_render_plan with a voice order and a workspace for split voices.  With
 * slices_per_voice > 1 a workgroup that starts inside a voice needs the
 * phase carries (LFOs, VCOs) at its first chunk; synth_render_plan walks the
 * earlier chunks' control stages for them, this entry computes every chunk's
 * carries first, in parallel over chunks (the chunks' own sums, then the
 * per-voice carry updates in chunk order: the same float64 operations, so the
 * audio is bit-identical to synth_render_plan's).
 *   max_samples  longest voice with offsets (ignored without): sizes the
 *                carries; a longer voice still renders correctly (its later
 *                chunks walk as in synth_render_plan).
 *   order        dev int32 [batch], a permutation of 0 .. batch - 1, or NULL:
 *                workgroups take the voices in this order (e.g. longest
 *                first, so that short voices fill the end of the launch);
 *                the output does not depend on it.  Entries outside
 *                0 .. batch - 1 are skipped.
 *   workspace    dev, >= synth_render_plan_workspace(cfg, batch, max_samples)
 *                bytes (SYNTH_ENOMEM otherwise), contents clobbered; NULL or
 *                slices_per_voice == 1: no carries are precomputed.
 *   batch <= 65535 with a workspace and slices > 1 (SYNTH_EUNSUPPORTED). */
size_t synth_render_plan_workspace(const synth_config* cfg, int64_t batch, int64_t max_samples);
int synth_render_plan_ws(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                         uint64_t first_g, int64_t batch, const int64_t* offsets,
                         int64_t n_samples, int64_t max_samples, float* audio,
                         int runs_per_segment, int slices_per_voice, int persistent,
                         int grid_blocks, const int32_t* order, void* workspace,
                         size_t workspace_bytes, void* stream);

/* Workspace (bytes of device memory) that synth_render_backward needs for a
 * batch of uniform-length voices: batch * (ceil(n_samples / q) * 21 +
 * chunks * 88) doubles (per-segment sums; the chunk-start phase carries of
 * voices split over workgroups; per-chunk totals of the chunk-parallel
 * control-rate adjoint: 4 sums, 2 LFO phase adjoints, 78 parameter
 * adjoints; chunks = ceil(ceil(n_samples / q) / 62)).  Returns 0 for an
 * invalid cfg. */
size_t synth_render_backward_workspace(const synth_config* cfg, int64_t batch, int64_t n_samples);

/* Adjoint of synth_render (uniform lengths): grad_params[i][p] =
 * sum_n grad_audio[i][n] * d audio[i][n] / d params[i][p], the exact
 * derivative of the render's definition almost everywhere (hard LFO square
 * and saw wraps, ramp kinks and the noise contribute their one-sided /
 * zero derivatives).  Envelopes and oscillators are recomputed, not stored.
 *   params, voice_ids, first_g, batch, n_samples  as for synth_render.
 *   grad_audio   dev float32 [batch][n_samples].
 *   grad_params  dev float32 [batch][78], written.
 *   workspace    dev buffer of >= synth_render_backward_workspace() bytes,
 *                caller-owned, contents clobbered.
 * Returns SYNTH_EUNSUPPORTED for mix_mode 1, for nebulas whose pitch can exceed
 * sample_rate / 2, for voices longer than 512 * 62 control samples and for
 * batch * chunks > 2^31 - 1; SYNTH_ENOMEM if workspace_bytes is too small.
 * Bitwise deterministic. */
int synth_render_backward(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                          uint64_t first_g, int64_t batch, int64_t n_samples,
                          const float* grad_audio, float* grad_params, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Multi-resolution log-magnitude STFT L1 loss (Section 4: the multi-scale
 * spectrogram distance, L1), per voice, and optionally its gradient.
 *   For voice b: loss[b] = sum over n in (512, 1024, 2048), hop n/4, of the mean
 *   over frames t < F_n = floor((N - n) / hop) + 1 and bins k <= n/2 of
 *   |log(|X_tk| + 1e-5) - log(|T_tk| + 1e-5)|, X and T the periodic-Hann STFTs
 *   (frames start at t * hop, no padding) of x and target; a resolution with
 *   no complete frame (n_samples < n) contributes 0.
 *   x, target  dev float32 [batch][n_samples].
 *   loss       dev float64 [batch], written.
 *   grad_x     dev float32 [batch][n_samples] or NULL; if given it receives
 *              d loss[b] / d x[b][.] (float32 FFT arithmetic).
 *   workspace  dev buffer, 16-byte aligned (SYNTH_EINVAL otherwise), of >=
 *              synth_mrstft_workspace(batch, n_samples, grad_x != NULL)
 *              bytes, caller-owned, contents clobbered (with a gradient: each
 *              workgroup's overlap-added segment of 19 hops per 16 frames,
 *              about 14 bytes per input sample).
 *   0 < n_samples <= 2^31, batch <= 65535 (SYNTH_EUNSUPPORTED above).
 *   Bitwise deterministic. */
size_t synth_mrstft_workspace(int64_t batch, int64_t n_samples, int with_grad);
int synth_mrstft_loss(const float* x, const float* target, int64_t batch, int64_t n_samples,
                      double* loss, float* grad_x, void* workspace, size_t workspace_bytes,
                      void* stream);

/* The same loss against a fixed target whose spectra are computed once:
 * synth_mrstft_target writes, for every frame of every resolution, the
 * target's log2(|T_k| + 1e-5) for bins k <= n/2 (float32, exactly the values
 * synth_mrstft_loss computes inside) to tlog, dev, of tlog_bytes >=
 * synth_mrstft_target_bytes(batch, n_samples) bytes (about 24 bytes per
 * input sample; SYNTH_ENOMEM otherwise).  synth_mrstft_loss_cached then
 * transforms only the render's frames: loss and gradient are bitwise those of
 * synth_mrstft_loss with that target.  tlog must come from
 * synth_mrstft_target with the same batch and n_samples (a smaller tlog_bytes
 * is SYNTH_ENOMEM).  Same sizes, limits and workspace as synth_mrstft_loss. */
size_t synth_mrstft_target_bytes(int64_t batch, int64_t n_samples);
int synth_mrstft_target(const float* target, int64_t batch, int64_t n_samples, float* tlog,
                        size_t tlog_bytes, void* stream);
int synth_mrstft_loss_cached(const float* x, const float* tlog, size_t tlog_bytes, int64_t batch,
                             int64_t n_samples, double* loss, float* grad_x, void* workspace,
                             size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Learned proposal: log-mel features and an MLP mapping them to parameters
 * (inverse synthesis, audio -> parameters, Section 2).  bf16 operands with
 * float32 accumulation on the MFMA units.  "bf16" pointers hold raw bfloat16
 * (uint16) values.  All pointers are dev unless stated; all calls are
 * stream-ordered, deterministic, and write only the outputs named.
 * ------------------------------------------------------------------------- */

/* C[M][N] (row stride ldc) = epi(alpha * A B + bias) (+ beta * C).
 *   a_layout 0: A[m * lda + k] (K contiguous); 1: A[k * lda + m].
 *   b_layout 0: B[n * ldb + k] (K contiguous); 1: B[k * ldb + n].
 *   c_bf16 1: C is bf16, 0: float32.  bias float32 [N] or NULL.
 *   epilogue 0 none, 1 GELU (erf form), 2 sigmoid, 3 multiply by GELU'(aux)
 *   with aux float32 laid out like C.  pre: optional float32 copy of the
 *   pre-epilogue value (layout of C).  Operands need not be aligned; 16-byte
 *   aligned rows take the vector path. */
int synth_gemm_bf16(int a_layout, int b_layout, int64_t M, int64_t N, int64_t K, const void* A,
                    int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, int c_bf16,
                    const float* bias, int epilogue, const float* aux, float* pre, float alpha,
                    float beta, void* stream);

/* Log-mel features: 64 frames of 2048 samples at hop 2756 (no padding),
 * periodic Hann window, power spectrum, 128 HTK mel triangles from 0 to
 * sample_rate / 2 (no area normalisation), log(x + 1e-6).
 *   synth_logmel_init fills the tables once: mel_basis bf16 [128][1032]
 *   (columns 0-1024 the weights; columns 1025 and 1026 of band b hold, as
 *   uint16, its first and last nonzero bin) and, if dft_basis != NULL,
 *   dft_basis bf16 [2048][2048] for synth_logmel_mfma (row 0: w(k), row 1:
 *   w(k)(-1)^k - the real bins 0 and 1024 - then rows 2f, 2f+1:
 *   w(k) cos(2 pi f k / 2048), -w(k) sin(...) for f = 1..1023); it
 *   synchronises the stream.  SYNTH_EUNSUPPORTED if a band's nonzero bins
 *   are not one run or there are more than 2304 nonzero weights.
 *   synth_logmel: power spectrum by float32 FFT of the windowed frames,
 *   rounded to bf16; each band summed over its nonzero bins in float32; one
 *   kernel, workspace unused (may be NULL).
 *   synth_logmel_mfma: the power spectrum as one bf16 MFMA GEMM of the frames
 *   (rounded to bf16) with dft_basis (window folded in) - more arithmetic,
 *   bf16 inputs - and the mel projection as a bf16 MFMA GEMM with float32
 *   accumulation; workspace >= synth_logmel_workspace(batch) bytes.
 *   audio: float32, voice b = audio[b * n_samples ..] of n_samples samples
 *   (offsets == NULL, n_samples > 0) or the ragged range
 *   audio[offsets[b] .. offsets[b+1]) (offsets dev int64 [batch + 1]); samples
 *   past a voice's end count as 0 (a render shorter than the 175676 samples
 *   the frames span is featurised as if zero-padded).  features float32
 *   [batch][128][64] (mel bin major, frame minor). */
size_t synth_logmel_workspace(int64_t batch);
int synth_logmel_init(double sample_rate, void* dft_basis, void* mel_basis, void* stream);
int synth_logmel(const float* audio, const int64_t* offsets, int64_t batch, int64_t n_samples,
                 const void* mel_basis, void* workspace, size_t workspace_bytes, float* features,
                 void* stream);
/* synth_logmel's features standardised and rounded to bf16 in the same
 * kernel: features_bf16[r][c] = bf16((x[c] - mean[c]) * inv_std[c]) (float32
 * arithmetic, round to nearest even: bitwise what synth_standardize gives for
 * synth_logmel's output) for the features x of voice b, written to row
 * r = row_index[b] (row_index dev int64 [batch], or NULL for r = b; a row
 * outside [0, batch) is not written).  mean, inv_std: dev float32 [8192];
 * features_bf16: dev bf16 [batch][8192].  No workspace. */
int synth_logmel_standardized(const float* audio, const int64_t* offsets, int64_t batch,
                              int64_t n_samples, const void* mel_basis, const float* mean,
                              const float* inv_std, const int64_t* row_index,
                              void* features_bf16, void* stream);
int synth_logmel_mfma(const float* audio, const int64_t* offsets, int64_t batch,
                      int64_t n_samples, const void* dft_basis, const void* mel_basis,
                      void* workspace, size_t workspace_bytes, float* features, void* stream);

/* Column sums (and sums of squares if sumsq != NULL) of a rows x cols matrix
 * (row stride ld; bf16 if x_bf16 else float32), float32 outputs [cols]. */
int synth_colstats(const void* x, int x_bf16, int64_t rows, int64_t cols, int64_t ld, float* sum,
                   float* sumsq, void* stream);
/* Feature standardisation statistics of a rows x cols float32 matrix (rows
 * > 0): mean[c] and inv_std[c] = 1 / sqrt(max(var_c, min_var)) with the
 * population variance, both float32 [cols], accumulated in float64. */
int synth_feature_stats(const float* x, int64_t rows, int64_t cols, float min_var, float* mean,
                        float* inv_std, void* stream);
/* y (bf16) = (x - mean[col]) * inv_std[col] for a rows x cols float32 matrix. */
int synth_standardize(const float* x, const float* mean, const float* inv_std, int64_t rows,
                      int64_t cols, void* y_bf16, void* stream);
/* y (bf16) = round-to-nearest-even(x), n elements. */
int synth_to_bf16(const float* x, void* y, int64_t n, void* stream);

/* Bytes of the optional MLP workspace (0 for invalid sizes).  With it, a
 * GEMM whose output has too few tiles to fill the chip splits K over
 * several workgroups, writes float32 partial sums there and adds them in a
 * fixed order, and the backward's bias gradients are summed over row
 * slices there (float64) and then over the slices in order: results stay
 * deterministic.  Without it (NULL) the same sums run unsplit. */
size_t synth_mlp_workspace(int64_t batch, int64_t d_in, int64_t d_h, int64_t d_out);

/* MLP forward, d_in -> d_h -> d_h -> d_out: h1 = gelu(x W1 + b1),
 * h2 = gelu(h1 W2 + b2), out = sigmoid(h2 W3 + b3).  Weights are stored
 * transposed and K-major: w1t [d_h][d_in], w2t [d_h][d_h], w3t [d_out][d_h]
 * (bf16); biases float32.  x, h1, h2 bf16 [batch][.]; h1pre, h2pre float32
 * pre-activations (may be NULL when no backward follows); out float32.
 * workspace: NULL (no split reductions) or synth_mlp_workspace() bytes,
 * else SYNTH_ENOMEM; calls sharing one workspace must be stream-ordered. */
int synth_mlp_forward(int64_t batch, int64_t d_in, int64_t d_h, int64_t d_out, const void* x,
                      const void* w1t, const float* b1, const void* w2t, const float* b2,
                      const void* w3t, const float* b3, float* h1pre, void* h1, float* h2pre,
                      void* h2, float* out, void* workspace, size_t workspace_bytes,
                      void* stream);
/* MLP backward of the loss mean((out - target)^2) over batch x d_out:
 * loss_rows (float64 [batch]) receives each row's sum of squared errors;
 * gw*t (float32, layouts of w*t) and gb* (float32) receive the gradients;
 * dz3 bf16 [batch][d_out], dh2 / dh1 bf16 [batch][d_h] are scratch;
 * workspace as for synth_mlp_forward. */
int synth_mlp_backward(int64_t batch, int64_t d_in, int64_t d_h, int64_t d_out, const void* x,
                       const void* w2t, const void* w3t, const float* h1pre, const void* h1,
                       const float* h2pre, const void* h2, const float* out, const float* target,
                       float* gw1t, float* gb1, float* gw2t, float* gb2, float* gw3t, float* gb3,
                       void* dz3, void* dh2, void* dh1, double* loss_rows, void* workspace,
                       size_t workspace_bytes, void* stream);
/* Bias-corrected Adam step `step` (>= 1) on float32 w with moments m, v; if
 * w_bf16 != NULL it receives the updated weights rounded to bf16. */
int synth_adam(int64_t n, float* w, void* w_bf16, const float* grad, float* m, float* v, float lr,
               float beta1, float beta2, float eps, int step, void* stream);

/* ---------------------------------------------------------------------------
 * Sound matching (inverse synthesis by gradient descent through the render,
 * Sections 2 and 2.3: estimating the parameters of a given sound).  The
 * parameters are optimised as logits z with u = sigmoid(z), so every step
 * stays inside [0, 1].
 * ------------------------------------------------------------------------- */

/* z = log(u' / (1 - u')) with u' = clamp(u, eps, 1 - eps), and
 * u_out = sigmoid(z) (u_out may alias u).  0 < eps < 1/2; n floats. */
int synth_logit_init(const float* u, float* z, float* u_out, int64_t n, float eps, void* stream);

/* One Adam step (bias-corrected, step >= 1) on logits z given dL/du at the
 * current u = sigmoid(z): dL/dz = dL/du * u (1 - u); then u <- sigmoid(z).
 * z, u, m, v updated in place; grad_u read; n floats each. */
int synth_logit_adam(int64_t n, float* z, float* u, const float* grad_u, float* m, float* v,
                     float lr, float beta1, float beta2, float eps, int step, void* stream);

/* Best-so-far tracking.  For each row r < rows, over columns c < cols, the
 * loss of element e = r * row_stride + c * col_stride is loss[e]; the
 * smallest (first on ties) replaces best[r] if strictly smaller, and then
 * best_idx[r] = col_base + c (if best_idx != NULL) and best_params[r][.] =
 * params[e][.] (param_dim floats; both NULL or both given).  loss float64,
 * best float64 [rows] (initialise to +inf), best_idx int64 [rows]. */
int synth_best_update(const double* loss, int64_t rows, int64_t cols, int64_t row_stride,
                      int64_t col_stride, int64_t col_base, const float* params, int64_t param_dim,
                      double* best, int64_t* best_idx, float* best_params, void* stream);

/* -------------------------------------------------------------------------
 * Fixed-order float64 reductions closing the learned and matching paths on
 * the device (the proposal's mean squared error, the spectral loss's chain
 * rule, and the distances the paper scores sounds with: L1 between log-mel
 * spectrograms, Section 4, and the squared error of estimated parameters).
 * Bitwise reproducible: every sum runs in a fixed order.
 * ------------------------------------------------------------------------- */

/* Sums of f(a - b) with f = |.| (kind 0) or (.)^2 (kind 1), a and b float32
 * rows x cols matrices (row strides lda, ldb >= cols; b NULL reads as 0).
 * axis 1: out[r] = scale * sum_c f(a[r][c] - b[r][c]) for r < rows (rows
 * < 2^31); axis 0: out[c] = scale * sum_r f(...) for c < cols.  With
 * accumulate != 0 the result is added to out's previous value.  out: dev
 * float64.  SYNTH_EINVAL on a bad kind, axis, size, stride or NULL pointer. */
int synth_diff_reduce(int kind, int axis, const float* a, const float* b, int64_t rows,
                      int64_t cols, int64_t lda, int64_t ldb, double scale, int accumulate,
                      double* out, void* stream);

/* out[0] = scale * sum_i x[i] (x dev float64 [n], out dev float64 [1]). */
int synth_sum_f64(const double* x, int64_t n, double scale, double* out, void* stream);

/* out[r][c] = g[r][c] * float(s[r]) (g, out dev float32 rows x cols, may
 * alias; s dev float64 [rows]): a per-row chain-rule factor. */
int synth_scale_rows(const float* g, const double* s, int64_t rows, int64_t cols, float* out,
                     void* stream);

/* -------------------------------------------------------------------------
 * Maximum mean discrepancy between two sets of sounds (Section 5, equation
 * "mmd"), with the L1 distance between embeddings (float32 log-mel
 * spectrograms, flattened) as the auditory distance d: the biased
 * (V-statistic) estimate over all pairs, self-pairs included,
 *   MMD(X, Y) = 2 S(X, Y) / (n m) - S(X, X) / n^2 - S(Y, Y) / m^2,
 *   S(A, B)   = sum_{i, j} sum_k |A[i][k] - B[j][k]|.
 * Each sum accumulates a pair's distance in float32 over runs of 256
 * dimensions and everything else in float64, in a fixed order, so results
 * are bitwise reproducible.
 * ------------------------------------------------------------------------- */

/* Bytes of device workspace synth_l1_pair_sum needs for sets of n and m
 * embeddings of dim floats (0 for an empty set or n, m above 2^17). */
size_t synth_l1_pair_sum_workspace(int64_t n, int64_t m, int64_t dim);

/* Bytes of device workspace synth_mmd_l1 needs: the largest of the three
 * pair sums' (n, m), (n, n), (m, m). */
size_t synth_mmd_l1_workspace(int64_t n, int64_t m, int64_t dim);

/* out[0] = S(A, B) (dev float64) for A dev float32 [n][dim] (row stride lda
 * >= dim), B dev float32 [m][dim] (ldb >= dim); 0 <= n, m <= 2^17, dim >= 0
 * (an empty set or dim 0 gives 0).  workspace: dev, 8-byte aligned, at least
 * synth_l1_pair_sum_workspace(n, m, dim) bytes, overwritten.  SYNTH_EINVAL
 * on a bad size, stride or NULL pointer, SYNTH_ENOMEM on a short workspace. */
int synth_l1_pair_sum(const float* A, int64_t lda, int64_t n, const float* B, int64_t ldb,
                      int64_t m, int64_t dim, void* workspace, size_t workspace_bytes,
                      double* out, void* stream);

/* out[0..3] = {MMD(X, Y), S(X, Y), S(X, X), S(Y, Y)} (dev float64 [4]) for X
 * dev float32 [n][dim], Y dev float32 [m][dim] (dense rows), 1 <= n, m <=
 * 2^17.  MMD(X, X) is exactly 0: S(X, X) is computed as S(X, Y) would be for
 * Y = X.  workspace >= synth_mmd_l1_workspace(n, m, dim) bytes.  Errors as
 * synth_l1_pair_sum. */
int synth_mmd_l1(const float* X, int64_t n, const float* Y, int64_t m, int64_t dim,
                 void* workspace, size_t workspace_bytes, double* out, void* stream);

/* -------------------------------------------------------------------------
 * Resonant low-pass filter module (a subtractive filter, one of the modules
 * Section 7 lists to add) and its adjoint.  Per voice b, control period j
 * (samples [j period, (j + 1) period)) has the cutoff
 *   f = clamp(440 * 2^((cutoff + depth * env[b][j] - 69) / 12), 10 Hz, 0.45 sample_rate)
 * and R. Bristow-Johnson's cookbook second-order low-pass at f and Q
 * (w = 2 pi f / sample_rate, alpha = sin w / (2 Q), b0 = b2 = (1 - cos w) /
 * 2 / (1 + alpha), b1 = (1 - cos w) / (1 + alpha), a1 = -2 cos w / (1 +
 * alpha), a2 = (1 - alpha) / (1 + alpha)), run as the direct-form-I
 * recurrence y[n] = b0 x[n] + b1 x[n-1] + b2 x[n-2] - a1 y[n-1] - a2 y[n-2]
 * from a zero state with the coefficients switched at period boundaries
 * (float64 state and coefficients, float32 samples).  Unit gain at DC, gain Q
 * at the cutoff.
 *   x, y        dev float32, [batch][n_samples] (offsets NULL) or packed with
 *               offsets (dev int64 [batch + 1], as synth_render); y may be x.
 *   max_samples with offsets: the longest voice (sizes env and states);
 *               ignored without.
 *   env         dev float32 [batch][env_ld], env_ld >= ceil(longest / period):
 *               the control signal (for instance an ADSR) per period.
 *   params      dev float32 [batch][3]: cutoff (MIDI note number), depth
 *               (semitones per unit of env), Q (> 0).
 *   period      4 .. 256 samples (SYNTH_EUNSUPPORTED otherwise).
 *   states      dev float64 [batch][state_ld][2] or NULL: the recurrence
 *               state at every 64-period chunk start, which the backward
 *               pass needs; state_ld >= synth_vcf_state_chunks(longest, period).
 *   order       NULL, or dev int32 [batch], a permutation of 0 .. batch - 1:
 *               the order in which workgroups take the voices (for ragged
 *               batches, longest first shortens the tail); results do not
 *               depend on it.  batch <= 2^31 - 1 with an order; an entry
 *               outside 0 .. batch - 1 is skipped (that workgroup does
 *               nothing).
 * SYNTH_EINVAL on a bad size, stride or NULL pointer.
 * ------------------------------------------------------------------------- */

/* Number of 64-period chunks of a voice of max_samples samples (0 for
 * out-of-range arguments). */
int64_t synth_vcf_state_chunks(int64_t max_samples, int period);

int synth_vcf_lowpass(const float* x, const int64_t* offsets, int64_t batch, int64_t n_samples,
                      int64_t max_samples, const float* env, int64_t env_ld, const float* params,
                      int period, double sample_rate, float* y, double* states, int64_t state_ld,
                      const int32_t* order, void* stream);

/* Adjoint of synth_vcf_lowpass for the same inputs, given grad_y = dL/dy and
 * the states its forward call wrote: grad_x = dL/dx (dev float32, layout of
 * x; may be grad_y), grad_params = dL/d(cutoff, depth, Q) (dev float32
 * [batch][3]), grad_env = dL/denv (dev float32 [batch][env_ld], rows written
 * for the voice's periods; may be NULL).  The clamp passes the gradient
 * where 10 Hz <= f <= 0.45 sample_rate and blocks it outside.  order as
 * synth_vcf_lowpass. */
int synth_vcf_lowpass_backward(const float* x, const float* grad_y, const int64_t* offsets,
                               int64_t batch, int64_t n_samples, int64_t max_samples,
                               const float* env, int64_t env_ld, const float* params, int period,
                               double sample_rate, const double* states, int64_t state_ld,
                               float* grad_x, float* grad_params, float* grad_env,
                               const int32_t* order, void* stream);

/* -------------------------------------------------------------------------
 * Four-operator FM voice (the FM architecture Sections 3.2 and 7 announce).
 * 44 normalised parameters per voice: 0 midi_f0, 1 note duration (s);
 * 2 + 8i for operator i = 0..3: ratio, detune (cents), level, attack (s),
 * decay (s), sustain, release (s), envelope curve exponent; 34..39 the
 * modulation indices M[0][1], M[0][2], M[0][3], M[1][2], M[1][3], M[2][3]
 * (cycles; operator j modulates the phase of operator i < j); 40..43 the
 * mix weights.  Operator i: f_i = 440 2^((midi_f0 - 69) / 12) ratio_i
 * 2^(detune_i / 1200) (at most sr / 2), o_i(n) = level_i env_i(n)
 * sin(2 pi (n f_i / sr + sum_{j > i} M[i][j] o_j(n))), env_i the Voice's
 * ADSR at the control rate upsampled linearly; y = sum_i w_i o_i /
 * max(1, sum_i w_i).  No operator feedback.  Indices above about 64 cycles
 * lose the hardware sine's accuracy.
 * ------------------------------------------------------------------------- */
typedef struct synth_fm_config {
    double sample_rate;      /* as synth_config: an integer multiple q of */
    double control_rate;     /* control_rate, q % 4 == 0, 4 <= q <= 1024 */
    const double* nebula;    /* host [44][4] doubles: (min, max, curve, symmetric) */
} synth_fm_config;

/* Normalised FM parameters [batch][44] float32 (dev): the draw of
 * synth_sample_params with counter word 3 = 1 (the FM voice's stream), so
 * the FM and default voices of one (seed, g) are independent. */
int synth_fm_sample_params(uint64_t seed, uint64_t first_g, int64_t batch,
                           const uint64_t* voice_ids, float* params, void* stream);

/* Render batch FM voices from params (dev float32 [batch][44]) into audio
 * (dev float32): uniform [batch][n_samples] when offsets is NULL, else
 * packed with offsets (dev int64 [batch + 1], as synth_render).  SYNTH_EINVAL
 * for a bad nebula (min > max, curve <= 0, symmetric not 0/1, envelope
 * curve minimum <= 0), size or pointer; SYNTH_EUNSUPPORTED for rates whose
 * ratio is not a multiple of 4 in 4 .. 1024.  order: NULL, or dev int32
 * [batch], a permutation of 0 .. batch - 1, the order in which workgroups
 * take the voices (results do not depend on it; an entry outside
 * 0 .. batch - 1 is skipped). */
int synth_fm_render(const synth_fm_config* cfg, const float* params, int64_t batch,
                    const int64_t* offsets, int64_t n_samples, float* audio,
                    const int32_t* order, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SYNTH_H_ */
