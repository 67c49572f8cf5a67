// C ABI of the voice renderer: host-side argument checks, launch planning and
// dispatch to the HIP kernels.  See include/synth.h for the contract.
#include <math.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "synth.h"
#include "synth_internal.h"

using synth::NebulaArgs;
using synth::RenderArgs;

namespace {

constexpr int kSegsPerChunk = 62;   // must match render.hip

int to_status(hipError_t e) { return e == hipSuccess ? SYNTH_OK : SYNTH_EDEVICE; }

// Validates cfg and fills the render arguments that do not depend on the batch.
int prepare(const synth_config* cfg, RenderArgs* a, bool* clamp) {
  if (!cfg || !cfg->nebula) return SYNTH_EINVAL;
  if (cfg->reserved != 0) return SYNTH_EINVAL;
  if (cfg->mix_mode != 0 && cfg->mix_mode != 1) return SYNTH_EINVAL;
  const double sr = cfg->sample_rate, rc = cfg->control_rate;
  if (!(sr > 0.0) || !(rc > 0.0) || !isfinite(sr) || !isfinite(rc)) return SYNTH_EINVAL;
  const double qf = sr / rc;
  const double qr = nearbyint(qf);
  if (fabs(qr - qf) > 1e-9 * qf || qr < 4.0 || qr > 1024.0) return SYNTH_EUNSUPPORTED;
  const int q = (int)qr;
  if (q % 4 != 0) return SYNTH_EUNSUPPORTED;

  memset(a, 0, sizeof(*a));
  NebulaArgs& nb = a->neb;
  const double* t = cfg->nebula;
  for (int p = 0; p < synth::kNumParams; ++p) {
    const double lo = t[4 * p + 0], hi = t[4 * p + 1], c = t[4 * p + 2], s = t[4 * p + 3];
    if (!isfinite(lo) || !isfinite(hi) || !(lo <= hi) || !(c > 0.0) || !isfinite(c))
      return SYNTH_EINVAL;
    if (s != 0.0 && s != 1.0) return SYNTH_EINVAL;
    nb.lo[p] = lo;
    nb.hi[p] = hi;
    nb.inv_curve[p] = 1.0 / c;
    if (s == 1.0) nb.sym[p >> 5] |= 1u << (p & 31);
    if (c == 1.0) nb.linear[p >> 5] |= 1u << (p & 31);
  }
  // ADSR curve exponents must be positive (pow of a [0,1] ramp)
  for (int k = 0; k < 6; ++k)
    if (!(nb.lo[2 + 5 * k + 4] > 0.0)) return SYNTH_EINVAL;

  a->sr = sr;
  a->rc = rc;
  a->q = q;
  a->q_magic = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)q - 1) / (uint64_t)q);
  a->mix_mode = cfg->mix_mode;
  a->nk0 = (uint32_t)cfg->noise_seed;
  a->nk1 = (uint32_t)(cfg->noise_seed >> 32);
  // Highest pitch any voice of this nebula can reach: midi + tuning + max(0, depth).
  double m_max = -1e300;
  const int tune[2] = {68, 71};
  for (int v = 0; v < 2; ++v) {
    const int tb = tune[v];
    const double m = nb.hi[0] + nb.hi[tb] + fmax(0.0, nb.hi[tb + 1]);
    m_max = fmax(m_max, m);
  }
  a->nyq_midi = 69.0 + 12.0 * log2(sr / 2.0 / 440.0);
  *clamp = m_max >= a->nyq_midi - 1e-9;
  return SYNTH_OK;
}

}  // namespace

extern "C" {

int synth_num_params(void) { return SYNTH_NUM_PARAMS; }

const char* synth_status_string(int status) {
  switch (status) {
    case SYNTH_OK: return "ok";
    case SYNTH_EINVAL: return "invalid argument";
    case SYNTH_ENOMEM: return "buffer too small";
    case SYNTH_EDEVICE: return "HIP device error";
    case SYNTH_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

int synth_is_test(uint64_t g) { return (g / 1024u) % 10u == 9u; }

int synth_sample_params(uint64_t seed, uint64_t first_g, int64_t batch, const uint64_t* voice_ids,
                        float* params, void* stream) {
  if (batch < 0) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!params) return SYNTH_EINVAL;
  if (batch > ((int64_t)1 << 31) * 256 / 20) return SYNTH_EINVAL;
  return to_status(synth::launch_sample_params(seed, first_g, batch, voice_ids, params,
                                               (hipStream_t)stream));
}

int synth_render_plan(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                      uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                      float* audio, int runs_per_segment, int slices_per_voice, int persistent,
                      int grid_blocks, void* stream) {
  if (batch < 0) return SYNTH_EINVAL;
  RenderArgs a;
  bool clamp = false;
  const int st = prepare(cfg, &a, &clamp);
  if (st != SYNTH_OK) return st;
  if (batch == 0) return SYNTH_OK;
  if (!params || !audio) return SYNTH_EINVAL;
  if (!offsets && n_samples <= 0) return SYNTH_EINVAL;
  if (!offsets && n_samples > ((int64_t)1 << 40)) return SYNTH_EINVAL;
  if (runs_per_segment != 1 && runs_per_segment != 2 && runs_per_segment != 4) return SYNTH_EINVAL;
  if (a.q % runs_per_segment != 0) return SYNTH_EUNSUPPORTED;
  if (a.q / runs_per_segment > 192) return SYNTH_EUNSUPPORTED;   // LDS tile <= 48 KB
  if (slices_per_voice < 1 || grid_blocks < 0) return SYNTH_EINVAL;
  if (offsets && slices_per_voice != 1) return SYNTH_EUNSUPPORTED;
  if (!offsets) {
    const int64_t J = (n_samples + a.q - 1) / a.q;
    const int64_t nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
    if (slices_per_voice > nchunks) return SYNTH_EUNSUPPORTED;
  }
  const int64_t items = batch * (int64_t)slices_per_voice;
  if (items > 0x7FFFFFFF) return SYNTH_EINVAL;

  a.params = params;
  a.voice_ids = voice_ids;
  a.offsets = offsets;
  a.audio = audio;
  a.first_g = first_g;
  a.n_uniform = offsets ? 0 : n_samples;
  a.batch = batch;
  a.slices = slices_per_voice;
  int grid = (int)items;
  if (persistent) {
    grid = grid_blocks > 0 ? grid_blocks : 256 * 12;
    if ((int64_t)grid > items) grid = (int)items;
    a.persistent_grid = grid;
  }
  hipError_t e = synth::launch_render(a, runs_per_segment, clamp, grid, (hipStream_t)stream);
  if (e != hipSuccess) return SYNTH_EDEVICE;
  if (a.mix_mode == 1) {
    a.slices = 1;
    e = synth::launch_peak_normalise(a, (hipStream_t)stream);
  }
  return to_status(e);
}

int synth_render(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                 uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                 float* audio, void* stream) {
  int slices = 1;
  if (!offsets && cfg && n_samples > 0 && batch > 0 && cfg->control_rate > 0.0) {
    // Small uniform batches: split voices so that the grid covers the chip.
    const double q = nearbyint(cfg->sample_rate / cfg->control_rate);
    if (q >= 4.0) {
      const int64_t J = (n_samples + (int64_t)q - 1) / (int64_t)q;
      const int64_t nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
      int64_t want = (2048 + batch - 1) / batch;
      if (want > nchunks / 4) want = nchunks / 4;
      if (want > 1) slices = (int)want;
    }
  }
  int rps = 4;
  if (cfg && cfg->control_rate > 0.0) {
    const double q = nearbyint(cfg->sample_rate / cfg->control_rate);
    if (fmod(q, 4.0) != 0.0) rps = 1;
  }
  return synth_render_plan(cfg, params, voice_ids, first_g, batch, offsets, n_samples, audio, rps,
                           slices, 0, 0, stream);
}

size_t synth_render_backward_workspace(const synth_config* cfg, int64_t batch, int64_t n_samples) {
  RenderArgs a;
  bool clamp = false;
  if (prepare(cfg, &a, &clamp) != SYNTH_OK || batch < 0 || n_samples <= 0) return 0;
  return synth::adjoint_workspace_bytes(batch, n_samples, a.q);
}

int synth_render_backward(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                          uint64_t first_g, int64_t batch, int64_t n_samples,
                          const float* grad_audio, float* grad_params, void* workspace,
                          size_t workspace_bytes, void* stream) {
  if (batch < 0) return SYNTH_EINVAL;
  RenderArgs a;
  bool clamp = false;
  const int st = prepare(cfg, &a, &clamp);
  if (st != SYNTH_OK) return st;
  if (batch == 0) return SYNTH_OK;
  if (!params || !grad_audio || !grad_params || !workspace) return SYNTH_EINVAL;
  if (n_samples <= 0 || n_samples > ((int64_t)1 << 40) || batch > 0x7FFFFFFF) return SYNTH_EINVAL;
  if (a.mix_mode != 0 || clamp) return SYNTH_EUNSUPPORTED;
  const int64_t J = (n_samples + a.q - 1) / a.q;
  if ((J + kSegsPerChunk - 1) / kSegsPerChunk > synth::adjoint_max_chunks()) return SYNTH_EUNSUPPORTED;
  if (workspace_bytes < synth::adjoint_workspace_bytes(batch, n_samples, a.q)) return SYNTH_ENOMEM;
  const int rps = (a.q % 4 == 0 && a.q / 4 <= 192) ? 4 : 1;
  a.params = params;
  a.voice_ids = voice_ids;
  a.first_g = first_g;
  a.batch = batch;
  a.n_uniform = n_samples;
  a.slices = 1;
  return to_status(synth::launch_render_backward(a, grad_audio, (double*)workspace, grad_params,
                                                 rps, (hipStream_t)stream));
}

int synth_mrstft_loss(const float* x, const float* target, int64_t batch, int64_t n_samples,
                      double* loss, float* grad_x, void* stream) {
  if (batch < 0 || n_samples <= 0 || n_samples > ((int64_t)1 << 31)) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!x || !target || !loss) return SYNTH_EINVAL;
  if (batch > 0x7FFFFFFF) return SYNTH_EINVAL;
  return to_status(synth::launch_mrstft(x, target, batch, n_samples, loss, grad_x,
                                        (hipStream_t)stream));
}

}  // extern "C"
