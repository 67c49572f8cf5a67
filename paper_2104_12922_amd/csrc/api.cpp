// C ABI of the voice renderer: host-side argument checks, launch planning and
// dispatch to the HIP kernels.  See include/synth.h for the contract.
#include <math.h>
#include <string.h>

#include <atomic>
#include <mutex>

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

constexpr int64_t kMaxSet = (int64_t)1 << 17;   // sounds per set for the MMD sums
constexpr int kFmNumParams = 44;
constexpr uint32_t kFmArchTag = 1;             // the FM voice's parameter-draw stream

extern "C" {

int synth_num_params(void) { return SYNTH_NUM_PARAMS; }

namespace {
// Default Voice parameters in canonical order (Section 3.3 and the Voice's
// module list, Section 3.2): name, min, max, curve, symmetric.  Ranges are
// those of the default nebula (note duration from 0 s).
constexpr double kPi = 3.14159265358979323846;
struct ParamInfo {
  const char* name;
  double lo, hi, curve;
  int sym;
};
const ParamInfo kParamInfo[SYNTH_NUM_PARAMS] = {
    {"keyboard.midi_f0", 24.0, 84.0, 1.0, 0},
    {"keyboard.duration", 0.0, 4.0, 1.0, 0},
    {"adsr_1.attack", 0.0, 2.0, 1.0, 0},
    {"adsr_1.decay", 0.0, 2.0, 1.0, 0},
    {"adsr_1.sustain", 0.0, 1.0, 1.0, 0},
    {"adsr_1.release", 0.0, 2.0, 1.0, 0},
    {"adsr_1.alpha", 0.1, 6.0, 1.0, 0},
    {"adsr_2.attack", 0.0, 2.0, 1.0, 0},
    {"adsr_2.decay", 0.0, 2.0, 1.0, 0},
    {"adsr_2.sustain", 0.0, 1.0, 1.0, 0},
    {"adsr_2.release", 0.0, 2.0, 1.0, 0},
    {"adsr_2.alpha", 0.1, 6.0, 1.0, 0},
    {"lfo_1_rate_adsr.attack", 0.0, 2.0, 1.0, 0},
    {"lfo_1_rate_adsr.decay", 0.0, 2.0, 1.0, 0},
    {"lfo_1_rate_adsr.sustain", 0.0, 1.0, 1.0, 0},
    {"lfo_1_rate_adsr.release", 0.0, 2.0, 1.0, 0},
    {"lfo_1_rate_adsr.alpha", 0.1, 6.0, 1.0, 0},
    {"lfo_1_amp_adsr.attack", 0.0, 2.0, 1.0, 0},
    {"lfo_1_amp_adsr.decay", 0.0, 2.0, 1.0, 0},
    {"lfo_1_amp_adsr.sustain", 0.0, 1.0, 1.0, 0},
    {"lfo_1_amp_adsr.release", 0.0, 2.0, 1.0, 0},
    {"lfo_1_amp_adsr.alpha", 0.1, 6.0, 1.0, 0},
    {"lfo_2_rate_adsr.attack", 0.0, 2.0, 1.0, 0},
    {"lfo_2_rate_adsr.decay", 0.0, 2.0, 1.0, 0},
    {"lfo_2_rate_adsr.sustain", 0.0, 1.0, 1.0, 0},
    {"lfo_2_rate_adsr.release", 0.0, 2.0, 1.0, 0},
    {"lfo_2_rate_adsr.alpha", 0.1, 6.0, 1.0, 0},
    {"lfo_2_amp_adsr.attack", 0.0, 2.0, 1.0, 0},
    {"lfo_2_amp_adsr.decay", 0.0, 2.0, 1.0, 0},
    {"lfo_2_amp_adsr.sustain", 0.0, 1.0, 1.0, 0},
    {"lfo_2_amp_adsr.release", 0.0, 2.0, 1.0, 0},
    {"lfo_2_amp_adsr.alpha", 0.1, 6.0, 1.0, 0},
    {"lfo_1.rate", 0.0, 20.0, 1.0, 0},
    {"lfo_1.mod_depth", -10.0, 20.0, 1.0, 0},
    {"lfo_1.initial_phase", -kPi, kPi, 1.0, 0},
    {"lfo_1.w_sin", 0.0, 1.0, 1.0, 0},
    {"lfo_1.w_tri", 0.0, 1.0, 1.0, 0},
    {"lfo_1.w_saw", 0.0, 1.0, 1.0, 0},
    {"lfo_1.w_rsaw", 0.0, 1.0, 1.0, 0},
    {"lfo_1.w_sqr", 0.0, 1.0, 1.0, 0},
    {"lfo_2.rate", 0.0, 20.0, 1.0, 0},
    {"lfo_2.mod_depth", -10.0, 20.0, 1.0, 0},
    {"lfo_2.initial_phase", -kPi, kPi, 1.0, 0},
    {"lfo_2.w_sin", 0.0, 1.0, 1.0, 0},
    {"lfo_2.w_tri", 0.0, 1.0, 1.0, 0},
    {"lfo_2.w_saw", 0.0, 1.0, 1.0, 0},
    {"lfo_2.w_rsaw", 0.0, 1.0, 1.0, 0},
    {"lfo_2.w_sqr", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_1_pitch<-adsr_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_1_pitch<-adsr_2", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_1_pitch<-lfo_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_1_pitch<-lfo_2", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_1_amp<-adsr_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_1_amp<-adsr_2", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_1_amp<-lfo_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_1_amp<-lfo_2", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_2_pitch<-adsr_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_2_pitch<-adsr_2", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_2_pitch<-lfo_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_2_pitch<-lfo_2", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_2_amp<-adsr_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_2_amp<-adsr_2", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_2_amp<-lfo_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.vco_2_amp<-lfo_2", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.noise_amp<-adsr_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.noise_amp<-adsr_2", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.noise_amp<-lfo_1", 0.0, 1.0, 1.0, 0},
    {"mod_matrix.noise_amp<-lfo_2", 0.0, 1.0, 1.0, 0},
    {"vco_1.tuning", -24.0, 24.0, 1.0, 1},
    {"vco_1.mod_depth", -12.0, 12.0, 1.0, 1},
    {"vco_1.initial_phase", -kPi, kPi, 1.0, 0},
    {"vco_2.tuning", -24.0, 24.0, 1.0, 1},
    {"vco_2.mod_depth", -12.0, 12.0, 1.0, 1},
    {"vco_2.initial_phase", -kPi, kPi, 1.0, 0},
    {"vco_2.shape", 0.0, 1.0, 1.0, 0},
    {"mixer.level_sine", 0.0, 1.0, 1.0, 0},
    {"mixer.level_squaresaw", 0.0, 1.0, 1.0, 0},
    {"mixer.level_noise", 0.0, 1.0, 1.0, 0},
};
}  // namespace

int synth_param_info(int p, const char** name, double* min, double* max, double* curve,
                     int* symmetric) {
  if (p < 0 || p >= SYNTH_NUM_PARAMS) return SYNTH_EINVAL;
  const ParamInfo& q = kParamInfo[p];
  if (name) *name = q.name;
  if (min) *min = q.lo;
  if (max) *max = q.hi;
  if (curve) *curve = q.curve;
  if (symmetric) *symmetric = q.sym;
  return SYNTH_OK;
}

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

int synth_fm_sample_params(uint64_t seed, uint64_t first_g, int64_t batch,
                           const uint64_t* voice_ids, float* params, void* stream) {
  if (batch < 0) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!params) return SYNTH_EINVAL;
  if (batch > ((int64_t)1 << 31) * 256 / 11) return SYNTH_EINVAL;
  return to_status(synth::launch_sample_params(seed, first_g, batch, voice_ids, params,
                                               (hipStream_t)stream, kFmNumParams, kFmArchTag));
}

int synth_fm_render(const synth_fm_config* cfg, const float* params, int64_t batch,
                    const int64_t* offsets, int64_t n_samples, float* audio,
                    const int32_t* order, void* stream) {
  if (!cfg || !cfg->nebula || batch < 0) return SYNTH_EINVAL;
  const double sr = cfg->sample_rate, rc = cfg->control_rate;
  if (!(sr > 0.0) || !(rc > 0.0) || !isfinite(sr) || !isfinite(rc)) return SYNTH_EINVAL;
  const double qf = sr / rc, qr = nearbyint(qf);
  if (fabs(qr - qf) > 1e-9 * qf || qr < 4.0 || qr > 1024.0) return SYNTH_EUNSUPPORTED;
  if ((int)qr % 4 != 0) return SYNTH_EUNSUPPORTED;
  NebulaArgs nb;
  memset(&nb, 0, sizeof(nb));
  const double* t = cfg->nebula;
  for (int p = 0; p < kFmNumParams; ++p) {
    const double lo = t[4 * p + 0], hi = t[4 * p + 1], c = t[4 * p + 2], sy = t[4 * p + 3];
    if (!isfinite(lo) || !isfinite(hi) || !(lo <= hi) || !(c > 0.0) || !isfinite(c))
      return SYNTH_EINVAL;
    if (sy != 0.0 && sy != 1.0) return SYNTH_EINVAL;
    nb.lo[p] = lo;
    nb.hi[p] = hi;
    nb.inv_curve[p] = 1.0 / c;
    if (sy == 1.0) nb.sym[p >> 5] |= 1u << (p & 31);
    if (c == 1.0) nb.linear[p >> 5] |= 1u << (p & 31);
  }
  for (int k = 0; k < 4; ++k)              // envelope curve exponents must be positive
    if (!(nb.lo[2 + 8 * k + 7] > 0.0)) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!params || !audio || batch > 0x7FFFFFFF) return SYNTH_EINVAL;
  if (!offsets && (n_samples <= 0 || n_samples > ((int64_t)1 << 40))) return SYNTH_EINVAL;
  return to_status(synth::launch_fm_render(params, offsets, batch, offsets ? 0 : n_samples, audio,
                                           sr, rc, (int)qr, nb, order, (hipStream_t)stream));
}

namespace {
int64_t chunks_of(int64_t n_samples, int q) {
  const int64_t J = (n_samples + q - 1) / q;
  return (J + kSegsPerChunk - 1) / kSegsPerChunk;
}

int render_plan_impl(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                     uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                     int64_t max_samples, float* audio, int runs_per_segment,
                     int slices_per_voice, int persistent, int grid_blocks, const int32_t* order,
                     void* workspace, size_t workspace_bytes, void* stream) {
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
  a.order = order;
  if (order && batch > 0x7FFFFFFF) return SYNTH_EINVAL;
  int grid = (int)items;
  if (persistent) {
    grid = grid_blocks > 0 ? grid_blocks : 256 * 12;
    if ((int64_t)grid > items) grid = (int)items;
    a.persistent_grid = grid;
  }
  hipError_t e;
  if (workspace && slices_per_voice > 1) {
    const int64_t lmax = offsets ? max_samples : n_samples;
    if (lmax <= 0) return SYNTH_EINVAL;
    const int64_t stride = chunks_of(lmax, a.q);
    if (workspace_bytes < (size_t)(batch * stride) * 4 * sizeof(double)) return SYNTH_ENOMEM;
    if (batch > 65535 || stride > 0x7FFFFFFF) return SYNTH_EUNSUPPORTED;
    e = synth::launch_voice_carries(a, runs_per_segment, clamp, (double*)workspace, stride,
                                    (hipStream_t)stream);
    if (e != hipSuccess) return SYNTH_EDEVICE;
    a.carries = (const double*)workspace;
    a.carry_stride = stride;
  }
  e = synth::launch_render(a, runs_per_segment, clamp, grid, (hipStream_t)stream);
  if (e != hipSuccess) return SYNTH_EDEVICE;
  if (a.mix_mode == 1) {
    a.slices = 1;
    e = synth::launch_peak_normalise(a, (hipStream_t)stream);
  }
  return to_status(e);
}
}  // namespace

int synth_render_plan(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                      uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                      float* audio, int runs_per_segment, int slices_per_voice, int persistent,
                      int grid_blocks, void* stream) {
  return render_plan_impl(cfg, params, voice_ids, first_g, batch, offsets, n_samples, 0, audio,
                          runs_per_segment, slices_per_voice, persistent, grid_blocks, nullptr,
                          nullptr, 0, stream);
}

size_t synth_render_plan_workspace(const synth_config* cfg, int64_t batch, int64_t max_samples) {
  RenderArgs a;
  bool clamp = false;
  if (batch <= 0 || max_samples <= 0 || prepare(cfg, &a, &clamp) != SYNTH_OK) return 0;
  return (size_t)(batch * chunks_of(max_samples, a.q)) * 4 * sizeof(double);
}

int synth_render_plan_ws(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                         uint64_t first_g, int64_t batch, const int64_t* offsets,
                         int64_t n_samples, int64_t max_samples, float* audio,
                         int runs_per_segment, int slices_per_voice, int persistent,
                         int grid_blocks, const int32_t* order, void* workspace,
                         size_t workspace_bytes, void* stream) {
  return render_plan_impl(cfg, params, voice_ids, first_g, batch, offsets, n_samples, max_samples,
                          audio, runs_per_segment, slices_per_voice, persistent, grid_blocks, order,
                          workspace, workspace_bytes, stream);
}

namespace {
// The library's default plan: runs per segment 4 (1 if q is not a multiple
// of 4); small uniform batches split each voice over workgroups so that the
// grid covers the chip - at most a quarter of its chunks when the slices
// walk the earlier chunks for their carries, up to all of them when the
// carries are computed first.
void default_plan(const synth_config* cfg, int64_t batch, const int64_t* offsets,
                  int64_t n_samples, bool carried, int* rps, int* slices) {
  *slices = 1;
  *rps = 4;
  if (!cfg || !(cfg->control_rate > 0.0)) return;
  const double q = nearbyint(cfg->sample_rate / cfg->control_rate);
  if (fmod(q, 4.0) != 0.0) *rps = 1;
  if (!offsets && n_samples > 0 && batch > 0 && q >= 4.0) {
    const int64_t nchunks = chunks_of(n_samples, (int)q);
    int64_t want = (2048 + batch - 1) / batch;
    const int64_t cap = carried ? nchunks : nchunks / 4;
    if (want > cap) want = cap;
    if (want > 1) *slices = (int)want;
  }
}
}  // namespace

int synth_render(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                 uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                 float* audio, void* stream) {
  int rps, slices;
  default_plan(cfg, batch, offsets, n_samples, false, &rps, &slices);
  return synth_render_plan(cfg, params, voice_ids, first_g, batch, offsets, n_samples, audio, rps,
                           slices, 0, 0, stream);
}

size_t synth_render_workspace(const synth_config* cfg, int64_t batch, int64_t n_samples) {
  int rps, slices;
  default_plan(cfg, batch, nullptr, n_samples, true, &rps, &slices);
  if (slices <= 1 || batch > 65535) return 0;
  return synth_render_plan_workspace(cfg, batch, n_samples);
}

int synth_render_ws(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                    uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                    float* audio, void* workspace, size_t workspace_bytes, void* stream) {
  if (!workspace || offsets) {
    return synth_render(cfg, params, voice_ids, first_g, batch, offsets, n_samples, audio, stream);
  }
  int rps, slices;
  default_plan(cfg, batch, offsets, n_samples, true, &rps, &slices);
  return render_plan_impl(cfg, params, voice_ids, first_g, batch, offsets, n_samples, n_samples,
                          audio, rps, slices, 0, 0, nullptr, workspace, workspace_bytes, stream);
}

// ---------------------------------------------------------------------------
// Allocation-free render.  The chunk-carry workspace of synth_render_ws comes
// from a static device array, `scratch`: each device the library runs on holds
// its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory, so its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is passed to kernels.  Every call on a device shares its array:
// calls that overlap on one device (concurrent streams or threads) race.  The
// carry kernels write every entry the render reads in the same call, so
// nothing needs clearing between calls.
// ---------------------------------------------------------------------------
namespace {
static __device__ __align__(256) unsigned char scratch[SYNTH_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::atomic<void*> g_scratch_ptr[kMaxDevices];

// This device's address of `scratch`, or nullptr if it cannot be looked up.
void* device_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
  if (p) return p;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
  if (!p) {
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev].store(p, std::memory_order_release);
  }
  return p;
}
}  // namespace

int synth_render_noalloc(const synth_config* cfg, const float* params, const uint64_t* voice_ids,
                         uint64_t first_g, int64_t batch, const int64_t* offsets, int64_t n_samples,
                         float* audio, void* stream) {
  const size_t need = offsets ? 0 : synth_render_workspace(cfg, batch, n_samples);
  if (need == 0)      // the default plan needs no workspace: this is synth_render
    return synth_render(cfg, params, voice_ids, first_g, batch, offsets, n_samples, audio, stream);
  if (need > (size_t)SYNTH_NOALLOC_SCRATCH_BYTES) return SYNTH_ENOMEM;
  void* ws = device_scratch();
  if (!ws) return SYNTH_EDEVICE;
  return synth_render_ws(cfg, params, voice_ids, first_g, batch, offsets, n_samples, audio, ws,
                         (size_t)SYNTH_NOALLOC_SCRATCH_BYTES, stream);
}

int synth_generate(const synth_config* cfg, uint64_t seed, const uint64_t* voice_ids,
                   uint64_t first_g, int64_t batch, int64_t n_samples, float* params, float* audio,
                   uint8_t* is_test, void* workspace, size_t workspace_bytes, void* stream) {
  if (!cfg || batch < 0 || n_samples <= 0) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!params || !audio || !is_test) return SYNTH_EINVAL;
  synth_config c = *cfg;
  c.noise_seed = seed;               // the corpus's noise is keyed by its seed
  int st = synth_sample_params(seed, first_g, batch, voice_ids, params, stream);
  if (st != SYNTH_OK) return st;
  st = synth_render_ws(&c, params, voice_ids, first_g, batch, nullptr, n_samples, audio, workspace,
                       workspace_bytes, stream);
  if (st != SYNTH_OK) return st;
  return to_status(synth::launch_is_test(first_g, batch, voice_ids, is_test, (hipStream_t)stream));
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
  if (batch * ((J + kSegsPerChunk - 1) / kSegsPerChunk) > 0x7FFFFFFF) return SYNTH_EUNSUPPORTED;
  if (workspace_bytes < synth::adjoint_workspace_bytes(batch, n_samples, a.q)) return SYNTH_ENOMEM;
  const int rps = (a.q % 4 == 0 && a.q / 4 <= 192) ? 4 : 1;
  a.params = params;
  a.voice_ids = voice_ids;
  a.first_g = first_g;
  a.batch = batch;
  a.n_uniform = n_samples;
  const int64_t nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
  const bool carried = batch <= 65535;
  {
    // Small batches: split each voice's audio-rate pass over several
    // workgroups so that the grid covers the chip (as the render does),
    // starting from precomputed chunk carries: up to 8192 workgroups, i.e.
    // every chunk its own workgroup for 256 voices of 4 s (5% faster than
    // 2048 workgroups there; the pass holds 2 wavefronts per SIMD).
    int64_t want = (8192 + batch - 1) / batch;
    const int64_t cap = carried ? nchunks : nchunks / 4;
    if (want > cap) want = cap;
    a.slices = want > 1 ? (int)want : 1;
    if (batch * (int64_t)a.slices > 0x7FFFFFFF) a.slices = 1;
  }
  if (carried && a.slices > 1) {
    double* carries = synth::adjoint_carries((double*)workspace, batch, n_samples, a.q);
    if (synth::launch_voice_carries(a, rps, false, carries, nchunks, (hipStream_t)stream) !=
        hipSuccess)
      return SYNTH_EDEVICE;
    a.carries = carries;
    a.carry_stride = nchunks;
  }
  return to_status(synth::launch_render_backward(a, grad_audio, (double*)workspace, grad_params,
                                                 rps, (hipStream_t)stream));
}

size_t synth_mrstft_workspace(int64_t batch, int64_t n_samples, int with_grad) {
  if (batch < 0 || n_samples <= 0 || n_samples > ((int64_t)1 << 31)) return 0;
  return synth::mrstft_workspace_bytes(batch, n_samples, with_grad != 0);
}

int synth_mrstft_loss(const float* x, const float* target, int64_t batch, int64_t n_samples,
                      double* loss, float* grad_x, void* workspace, size_t workspace_bytes,
                      void* stream) {
  if (batch < 0 || n_samples <= 0 || n_samples > ((int64_t)1 << 31)) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!x || !target || !loss || !workspace) return SYNTH_EINVAL;
  if (reinterpret_cast<uintptr_t>(workspace) & 15) return SYNTH_EINVAL;
  if (batch > 65535) return SYNTH_EUNSUPPORTED;
  if (workspace_bytes < synth::mrstft_workspace_bytes(batch, n_samples, grad_x != nullptr))
    return SYNTH_ENOMEM;
  return to_status(synth::launch_mrstft(x, target, nullptr, batch, n_samples, loss, grad_x,
                                        workspace, (hipStream_t)stream));
}

size_t synth_mrstft_target_bytes(int64_t batch, int64_t n_samples) {
  if (batch < 0 || n_samples <= 0 || n_samples > ((int64_t)1 << 31)) return 0;
  return synth::mrstft_target_bytes(batch, n_samples);
}

int synth_mrstft_target(const float* target, int64_t batch, int64_t n_samples, float* tlog,
                        size_t tlog_bytes, void* stream) {
  if (batch < 0 || n_samples <= 0 || n_samples > ((int64_t)1 << 31)) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (batch > 65535) return SYNTH_EUNSUPPORTED;
  const size_t need = synth::mrstft_target_bytes(batch, n_samples);
  if (need == 0) return SYNTH_OK;                    // no complete frame
  if (!target || !tlog) return SYNTH_EINVAL;
  if (tlog_bytes < need) return SYNTH_ENOMEM;
  return to_status(synth::launch_mrstft_target(target, batch, n_samples, tlog, (hipStream_t)stream));
}

int synth_mrstft_loss_cached(const float* x, const float* tlog, size_t tlog_bytes, int64_t batch,
                             int64_t n_samples, double* loss, float* grad_x, void* workspace,
                             size_t workspace_bytes, void* stream) {
  if (batch < 0 || n_samples <= 0 || n_samples > ((int64_t)1 << 31)) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!x || !loss || !workspace) return SYNTH_EINVAL;
  if (!tlog && synth::mrstft_target_bytes(batch, n_samples) > 0) return SYNTH_EINVAL;
  if (tlog_bytes < synth::mrstft_target_bytes(batch, n_samples)) return SYNTH_ENOMEM;
  if (reinterpret_cast<uintptr_t>(workspace) & 15) return SYNTH_EINVAL;
  if (batch > 65535) return SYNTH_EUNSUPPORTED;
  if (workspace_bytes < synth::mrstft_workspace_bytes(batch, n_samples, grad_x != nullptr))
    return SYNTH_ENOMEM;
  return to_status(synth::launch_mrstft(x, nullptr, tlog, batch, n_samples, loss, grad_x,
                                        workspace, (hipStream_t)stream));
}

// ---------------------------------------------------------------------------
// bf16 MFMA GEMM, log-mel features, learned proposal (MLP) and Adam
// ---------------------------------------------------------------------------
int synth_gemm_bf16(int a_layout, int b_layout, int64_t M, int64_t N, int64_t K, const void* A,
                    int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, int c_bf16,
                    const float* bias, int epilogue, const float* aux, float* pre, float alpha,
                    float beta, void* stream) {
  if (M < 0 || N < 0 || K < 0) return SYNTH_EINVAL;
  if (M == 0 || N == 0) return SYNTH_OK;
  if (!A || !B || !C) return SYNTH_EINVAL;
  if ((a_layout != synth::kOpKMajor && a_layout != synth::kOpRowMajorMN) ||
      (b_layout != synth::kOpKMajor && b_layout != synth::kOpRowMajorMN))
    return SYNTH_EINVAL;
  if (epilogue < synth::kEpiNone || epilogue > synth::kEpiGeluGrad) return SYNTH_EINVAL;
  if (epilogue == synth::kEpiGeluGrad && !aux) return SYNTH_EINVAL;
  if (lda < (a_layout == synth::kOpKMajor ? K : M) || ldb < (b_layout == synth::kOpKMajor ? K : N) ||
      ldc < N)
    return SYNTH_EINVAL;
  synth::GemmArgs g = {};
  g.M = M; g.N = N; g.K = K; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.c_bf16 = c_bf16 ? 1 : 0; g.bias = bias; g.epilogue = epilogue; g.aux = aux; g.pre = pre;
  g.alpha = alpha; g.beta = beta;
  return to_status(synth::launch_gemm_bf16(g, a_layout, b_layout, (hipStream_t)stream));
}

namespace {
constexpr int kMelNfft = 2048, kMelHop = 2756, kMelFrames = 64, kMelBins = 128, kMelLd = 1032;

uint16_t host_f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
}  // namespace

size_t synth_logmel_workspace(int64_t batch) {
  return batch < 0 ? 0 : (size_t)batch * kMelFrames * kMelLd * sizeof(uint16_t);
}

int synth_logmel_init(double sample_rate, void* dft_basis, void* mel_basis, void* stream) {
  if (!mel_basis || !(sample_rate > 0.0)) return SYNTH_EINVAL;
  hipError_t e = hipSuccess;
  if (dft_basis) {
    e = synth::launch_dft_basis(dft_basis, (hipStream_t)stream);
    if (e != hipSuccess) return SYNTH_EDEVICE;
  }
  // HTK mel triangles (mel = 2595 log10(1 + f / 700)), 130 edges from 0 to sr/2,
  // peak 1, no area normalisation; stored K-major [128][1032] in bf16.
  static thread_local uint16_t table[kMelBins * kMelLd];
  auto hz2mel = [](double f) { return 2595.0 * log10(1.0 + f / 700.0); };
  auto mel2hz = [](double m) { return 700.0 * (pow(10.0, m / 2595.0) - 1.0); };
  const double mtop = hz2mel(sample_rate / 2.0);
  double edges[kMelBins + 2];
  for (int i = 0; i < kMelBins + 2; ++i) edges[i] = mel2hz(mtop * i / (kMelBins + 1));
  for (int b = 0; b < kMelBins; ++b)
    for (int k = 0; k < kMelLd; ++k) {
      double w = 0.0;
      if (k <= kMelNfft / 2) {
        const double f = k * sample_rate / kMelNfft;
        const double up = (f - edges[b]) / (edges[b + 1] - edges[b]);
        const double down = (edges[b + 2] - f) / (edges[b + 2] - edges[b + 1]);
        w = fmax(0.0, fmin(up, down));
      }
      table[b * kMelLd + k] = host_f2bf((float)w);
    }
  // padding columns 1025, 1026 of band b: its first and last nonzero bin
  // (first > last when the band has none), read by the FFT path
  int total = 0;
  for (int b = 0; b < kMelBins; ++b) {
    int lo = kMelNfft / 2 + 1, hi = -1;
    for (int k = 0; k <= kMelNfft / 2; ++k)
      if (table[b * kMelLd + k] != 0) {
        lo = k < lo ? k : lo;
        hi = k;
      }
    if (hi < 0) lo = 1, hi = 0;
    for (int k = lo; k <= hi; ++k)       // triangles: nonzero on one run of bins
      if (table[b * kMelLd + k] == 0) return SYNTH_EUNSUPPORTED;
    total += hi - lo + 1;
    table[b * kMelLd + kMelNfft / 2 + 1] = (uint16_t)lo;
    table[b * kMelLd + kMelNfft / 2 + 2] = (uint16_t)hi;
  }
  if (total > synth::kMelWeightsMax) return SYNTH_EUNSUPPORTED;
  e = hipMemcpyAsync(mel_basis, table, sizeof(table), hipMemcpyHostToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return SYNTH_EDEVICE;
  return to_status(hipStreamSynchronize((hipStream_t)stream));
}

namespace {
int logmel_common(bool fft, const float* audio, const int64_t* offsets, int64_t batch,
                  int64_t n_samples, const void* dft_basis, const void* mel_basis,
                  void* workspace, size_t workspace_bytes, float* features, void* stream) {
  if (batch < 0) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!audio || !mel_basis || !features) return SYNTH_EINVAL;
  if (!offsets && n_samples <= 0) return SYNTH_EINVAL;
  const hipStream_t s = (hipStream_t)stream;
  const int64_t n = offsets ? 0 : n_samples;
  if (fft)
    return to_status(synth::launch_logmel_fft(audio, offsets, n, batch, mel_basis, kMelLd,
                                              features, s));
  if (!dft_basis || !workspace) return SYNTH_EINVAL;
  if (workspace_bytes < synth_logmel_workspace(batch)) return SYNTH_ENOMEM;
  hipError_t e = synth::launch_dft_power(audio, offsets, n, batch, dft_basis, workspace, kMelLd, s);
  if (e != hipSuccess) return SYNTH_EDEVICE;
  synth::GemmArgs h = {};
  h.M = batch * kMelFrames; h.N = kMelBins; h.K = kMelNfft / 2 + 1;
  h.A = workspace; h.lda = kMelLd; h.B = mel_basis; h.ldb = kMelLd;
  h.C = features; h.ldc = kMelBins; h.c_bf16 = 0; h.epilogue = synth::kEpiLogMelT; h.alpha = 1.0f;
  return to_status(synth::launch_gemm_bf16(h, synth::kOpKMajor, synth::kOpKMajor, s));
}
}  // namespace

int synth_logmel(const float* audio, const int64_t* offsets, int64_t batch, int64_t n_samples,
                 const void* mel_basis, void* workspace, size_t workspace_bytes, float* features,
                 void* stream) {
  return logmel_common(true, audio, offsets, batch, n_samples, nullptr, mel_basis, workspace,
                       workspace_bytes, features, stream);
}

int synth_logmel_standardized(const float* audio, const int64_t* offsets, int64_t batch,
                              int64_t n_samples, const void* mel_basis, const float* mean,
                              const float* inv_std, const int64_t* row_index,
                              void* features_bf16, void* stream) {
  if (batch < 0) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!audio || !mel_basis || !mean || !inv_std || !features_bf16) return SYNTH_EINVAL;
  if (!offsets && n_samples <= 0) return SYNTH_EINVAL;
  return to_status(synth::launch_logmel_fft_std(audio, offsets, offsets ? 0 : n_samples, batch,
                                                mel_basis, kMelLd, mean, inv_std, row_index,
                                                features_bf16, (hipStream_t)stream));
}

int synth_logmel_mfma(const float* audio, const int64_t* offsets, int64_t batch,
                      int64_t n_samples, const void* dft_basis, const void* mel_basis,
                      void* workspace, size_t workspace_bytes, float* features, void* stream) {
  return logmel_common(false, audio, offsets, batch, n_samples, dft_basis, mel_basis, workspace,
                       workspace_bytes, features, stream);
}

int synth_diff_reduce(int kind, int axis, const float* a, const float* b, int64_t rows,
                      int64_t cols, int64_t lda, int64_t ldb, double scale, int accumulate,
                      double* out, void* stream) {
  if ((kind != 0 && kind != 1) || (axis != 0 && axis != 1) || rows < 0 || cols < 0) return SYNTH_EINVAL;
  if (lda < cols || (b && ldb < cols)) return SYNTH_EINVAL;
  if ((axis == 1 ? rows : cols) > 0 && !out) return SYNTH_EINVAL;
  if (rows > 0 && cols > 0 && !a) return SYNTH_EINVAL;
  if (axis == 1 && rows > 0x7FFFFFFF) return SYNTH_EINVAL;
  return to_status(synth::launch_diff_reduce(kind, axis, a, b, rows, cols, lda, ldb, scale,
                                             accumulate, out, (hipStream_t)stream));
}

int synth_sum_f64(const double* x, int64_t n, double scale, double* out, void* stream) {
  if (n < 0 || !out || (n > 0 && !x)) return SYNTH_EINVAL;
  return to_status(synth::launch_sum_f64(x, n, scale, out, (hipStream_t)stream));
}

int synth_scale_rows(const float* g, const double* s, int64_t rows, int64_t cols, float* out,
                     void* stream) {
  if (rows < 0 || cols < 0) return SYNTH_EINVAL;
  if (rows * cols > 0 && (!g || !s || !out)) return SYNTH_EINVAL;
  return to_status(synth::launch_scale_rows(g, s, rows, cols, out, (hipStream_t)stream));
}

size_t synth_l1_pair_sum_workspace(int64_t n, int64_t m, int64_t dim) {
  if (n <= 0 || m <= 0 || dim < 0 || n > kMaxSet || m > kMaxSet) return 0;
  return synth::l1_pair_sum_workspace(n, m, dim);
}

size_t synth_mmd_l1_workspace(int64_t n, int64_t m, int64_t dim) {
  size_t need = synth_l1_pair_sum_workspace(n, m, dim);
  const size_t xx = synth_l1_pair_sum_workspace(n, n, dim);
  const size_t yy = synth_l1_pair_sum_workspace(m, m, dim);
  need = xx > need ? xx : need;
  return yy > need ? yy : need;
}

int synth_l1_pair_sum(const float* A, int64_t lda, int64_t n, const float* B, int64_t ldb,
                      int64_t m, int64_t dim, void* workspace, size_t workspace_bytes,
                      double* out, void* stream) {
  if (n < 0 || m < 0 || dim < 0 || n > kMaxSet || m > kMaxSet || !out) return SYNTH_EINVAL;
  if (lda < dim || ldb < dim) return SYNTH_EINVAL;
  if (n > 0 && m > 0 && dim > 0 && (!A || !B)) return SYNTH_EINVAL;
  const size_t need = synth_l1_pair_sum_workspace(n, m, dim);
  if (need > 0 && (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 7))) return SYNTH_EINVAL;
  if (workspace_bytes < need) return SYNTH_ENOMEM;
  return to_status(synth::launch_l1_pair_sum(A, lda, n, B, ldb, m, dim, (double*)workspace, out,
                                             (hipStream_t)stream));
}

int synth_mmd_l1(const float* X, int64_t n, const float* Y, int64_t m, int64_t dim,
                 void* workspace, size_t workspace_bytes, double* out, void* stream) {
  if (n < 1 || m < 1 || dim < 0 || n > kMaxSet || m > kMaxSet || !out) return SYNTH_EINVAL;
  if (dim > 0 && (!X || !Y)) return SYNTH_EINVAL;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 7)) return SYNTH_EINVAL;
  if (workspace_bytes < synth_mmd_l1_workspace(n, m, dim)) return SYNTH_ENOMEM;
  const hipStream_t s = (hipStream_t)stream;
  double* ws = (double*)workspace;
  // the three sums reuse the workspace in stream order
  hipError_t e = synth::launch_l1_pair_sum(X, dim, n, Y, dim, m, dim, ws, out + 1, s);
  if (e == hipSuccess) e = synth::launch_l1_pair_sum(X, dim, n, X, dim, n, dim, ws, out + 2, s);
  if (e == hipSuccess) e = synth::launch_l1_pair_sum(Y, dim, m, Y, dim, m, dim, ws, out + 3, s);
  if (e == hipSuccess) e = synth::launch_mmd_combine(out, n, m, s);
  return to_status(e);
}

int64_t synth_vcf_state_chunks(int64_t max_samples, int period) {
  if (max_samples <= 0 || period < 4 || period > 256) return 0;
  return synth::vcf_chunks(max_samples, period);
}

namespace {
int vcf_check(const float* x, const int64_t* offsets, int64_t batch, int64_t n_samples,
              const float* env, int64_t env_ld, const float* params, int period,
              double sample_rate, const float* out, const double* states, int64_t state_ld,
              int64_t max_samples) {
  if (batch < 0 || batch > 0x7FFFFFFF) return SYNTH_EINVAL;
  if (period < 4 || period > 256) return SYNTH_EUNSUPPORTED;
  if (!(sample_rate > 0.0) || !isfinite(sample_rate)) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!x || !env || !params || !out) return SYNTH_EINVAL;
  if (!offsets && n_samples <= 0) return SYNTH_EINVAL;
  if (max_samples <= 0 || max_samples > ((int64_t)1 << 40)) return SYNTH_EINVAL;
  if (env_ld < (max_samples + period - 1) / period) return SYNTH_EINVAL;
  if (states && state_ld < synth::vcf_chunks(max_samples, period)) return SYNTH_EINVAL;
  return SYNTH_OK;
}
}  // namespace

int synth_vcf_lowpass(const float* x, const int64_t* offsets, int64_t batch, int64_t n_samples,
                      int64_t max_samples, const float* env, int64_t env_ld, const float* params,
                      int period, double sample_rate, float* y, double* states, int64_t state_ld,
                      const int32_t* order, void* stream) {
  const int64_t lmax = offsets ? max_samples : n_samples;
  const int st = vcf_check(x, offsets, batch, n_samples, env, env_ld, params, period, sample_rate,
                           y, states, state_ld, batch > 0 ? lmax : 1);
  if (st != SYNTH_OK || batch == 0) return st;
  if (order && batch > 0x7FFFFFFF) return SYNTH_EINVAL;
  return to_status(synth::launch_vcf_forward(x, offsets, batch, offsets ? 0 : n_samples, env,
                                             env_ld, params, period, sample_rate, y, states,
                                             state_ld, order, (hipStream_t)stream));
}

int synth_vcf_lowpass_backward(const float* x, const float* grad_y, const int64_t* offsets,
                               int64_t batch, int64_t n_samples, int64_t max_samples,
                               const float* env, int64_t env_ld, const float* params, int period,
                               double sample_rate, const double* states, int64_t state_ld,
                               float* grad_x, float* grad_params, float* grad_env,
                               const int32_t* order, void* stream) {
  const int64_t lmax = offsets ? max_samples : n_samples;
  const int st = vcf_check(x, offsets, batch, n_samples, env, env_ld, params, period, sample_rate,
                           grad_x, states, state_ld, batch > 0 ? lmax : 1);
  if (st != SYNTH_OK || batch == 0) return st;
  if (!grad_y || !states || !grad_params) return SYNTH_EINVAL;
  if (order && batch > 0x7FFFFFFF) return SYNTH_EINVAL;
  return to_status(synth::launch_vcf_backward(x, grad_y, offsets, batch, offsets ? 0 : n_samples,
                                              env, env_ld, params, period, sample_rate, states,
                                              state_ld, grad_x, grad_params, grad_env, order,
                                              (hipStream_t)stream));
}

int synth_colstats(const void* x, int x_bf16, int64_t rows, int64_t cols, int64_t ld, float* sum,
                   float* sumsq, void* stream) {
  if (rows < 0 || cols < 0 || ld < cols || (cols > 0 && (!x || !sum))) return SYNTH_EINVAL;
  return to_status(synth::launch_colsum(x, x_bf16, rows, cols, ld, sum, sumsq, (hipStream_t)stream));
}

int synth_feature_stats(const float* x, int64_t rows, int64_t cols, float min_var, float* mean,
                        float* inv_std, void* stream) {
  if (rows <= 0 || cols < 0 || !(min_var > 0.0f)) return SYNTH_EINVAL;
  if (cols > 0 && (!x || !mean || !inv_std)) return SYNTH_EINVAL;
  return to_status(synth::launch_feature_stats(x, rows, cols, min_var, mean, inv_std,
                                               (hipStream_t)stream));
}

int synth_standardize(const float* x, const float* mean, const float* inv_std, int64_t rows,
                      int64_t cols, void* y_bf16, void* stream) {
  if (rows < 0 || cols < 0) return SYNTH_EINVAL;
  if (rows * cols > 0 && (!x || !mean || !inv_std || !y_bf16)) return SYNTH_EINVAL;
  return to_status(synth::launch_standardize(x, mean, inv_std, rows, cols, y_bf16, (hipStream_t)stream));
}

int synth_to_bf16(const float* x, void* y, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!x || !y))) return SYNTH_EINVAL;
  return to_status(synth::launch_f32_to_bf16(x, y, n, (hipStream_t)stream));
}

namespace {
// The MLP's GEMMs as (M, N, K); forward: 0-2, backward: 3-7.
void mlp_shapes(int64_t batch, int64_t d_in, int64_t d_h, int64_t d_out, int64_t sh[8][3]) {
  const int64_t v[8][3] = {{batch, d_h, d_in}, {batch, d_h, d_h},  {batch, d_out, d_h},
                           {d_out, d_h, batch}, {batch, d_h, d_out}, {d_h, d_h, batch},
                           {batch, d_h, d_h},  {d_h, d_in, batch}};
  memcpy(sh, v, sizeof(v));
}

// Runs g with K split over workgroups when its output tiles alone would leave
// CUs idle and the caller gave a workspace for the partial sums.
hipError_t gemm_maybe_split(synth::GemmArgs g, int a_op, int b_op, void* workspace,
                            hipStream_t s) {
  if (workspace) {
    g.split = synth::gemm_split_for(g.M, g.N, g.K);
    g.partial = static_cast<float*>(workspace);
  }
  return synth::launch_gemm_bf16(g, a_op, b_op, s);
}
}  // namespace

size_t synth_mlp_workspace(int64_t batch, int64_t d_in, int64_t d_h, int64_t d_out) {
  if (batch <= 0 || d_in <= 0 || d_h <= 0 || d_out <= 0) return 0;
  int64_t sh[8][3];
  mlp_shapes(batch, d_in, d_h, d_out, sh);
  // the bias gradients' column sums use it too (between the GEMMs)
  size_t b = synth::colsum_ws_bytes(batch, d_h > d_out ? d_h : d_out);
  for (auto& m : sh) {
    const size_t x = synth::gemm_split_bytes(m[0], m[1], synth::gemm_split_for(m[0], m[1], m[2]));
    b = x > b ? x : b;
  }
  return b;
}

int synth_mlp_forward(int64_t batch, int64_t d_in, int64_t d_h, int64_t d_out, const void* x,
                      const void* w1t, const float* b1, const void* w2t, const float* b2,
                      const void* w3t, const float* b3, float* h1pre, void* h1, float* h2pre,
                      void* h2, float* out, void* workspace, size_t workspace_bytes,
                      void* stream) {
  if (batch < 0 || d_in <= 0 || d_h <= 0 || d_out <= 0) return SYNTH_EINVAL;
  if (batch == 0) return SYNTH_OK;
  if (!x || !w1t || !b1 || !w2t || !b2 || !w3t || !b3 || !h1 || !h2 || !out) return SYNTH_EINVAL;
  if (workspace && workspace_bytes < synth_mlp_workspace(batch, d_in, d_h, d_out))
    return SYNTH_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  synth::GemmArgs g = {};
  g.alpha = 1.0f;
  // h1 = gelu(x W1 + b1): A = x [batch][d_in], B = W1^T [d_h][d_in] (K-major)
  g.M = batch; g.N = d_h; g.K = d_in; g.A = x; g.lda = d_in; g.B = w1t; g.ldb = d_in;
  g.C = h1; g.ldc = d_h; g.c_bf16 = 1; g.bias = b1; g.epilogue = synth::kEpiGelu; g.pre = h1pre;
  hipError_t e = gemm_maybe_split(g, synth::kOpKMajor, synth::kOpKMajor, workspace, s);
  if (e != hipSuccess) return SYNTH_EDEVICE;
  g.K = d_h; g.A = h1; g.lda = d_h; g.B = w2t; g.ldb = d_h; g.C = h2; g.bias = b2; g.pre = h2pre;
  e = gemm_maybe_split(g, synth::kOpKMajor, synth::kOpKMajor, workspace, s);
  if (e != hipSuccess) return SYNTH_EDEVICE;
  g.N = d_out; g.A = h2; g.B = w3t; g.C = out; g.ldc = d_out; g.c_bf16 = 0; g.bias = b3;
  g.epilogue = synth::kEpiSigmoid; g.pre = nullptr;
  return to_status(gemm_maybe_split(g, synth::kOpKMajor, synth::kOpKMajor, workspace, s));
}

int synth_mlp_backward(int64_t batch, int64_t d_in, int64_t d_h, int64_t d_out, const void* x,
                       const void* w2t, const void* w3t, const float* h1pre, const void* h1,
                       const float* h2pre, const void* h2, const float* out, const float* target,
                       float* gw1t, float* gb1, float* gw2t, float* gb2, float* gw3t, float* gb3,
                       void* dz3, void* dh2, void* dh1, double* loss_rows, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (batch <= 0 || d_in <= 0 || d_h <= 0 || d_out <= 0) return SYNTH_EINVAL;
  if (!x || !w2t || !w3t || !h1pre || !h1 || !h2pre || !h2 || !out || !target || !gw1t || !gb1 ||
      !gw2t || !gb2 || !gw3t || !gb3 || !dz3 || !dh2 || !dh1 || !loss_rows)
    return SYNTH_EINVAL;
  if (workspace && workspace_bytes < synth_mlp_workspace(batch, d_in, d_h, d_out))
    return SYNTH_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  using synth::kOpKMajor;
  using synth::kOpRowMajorMN;
  hipError_t e = synth::launch_mse_sigmoid_grad(out, target, batch, d_out, dz3, loss_rows, s);
  if (e != hipSuccess) return SYNTH_EDEVICE;
  synth::GemmArgs g = {};
  g.alpha = 1.0f;
  // dW3^T [d_out][d_h] = dz3^T h2
  g.M = d_out; g.N = d_h; g.K = batch; g.A = dz3; g.lda = d_out; g.B = h2; g.ldb = d_h;
  g.C = gw3t; g.ldc = d_h; g.c_bf16 = 0;
  if ((e = gemm_maybe_split(g, kOpRowMajorMN, kOpRowMajorMN, workspace, s)) != hipSuccess) return SYNTH_EDEVICE;
  if ((e = synth::launch_colsum_bf16_ws(dz3, batch, d_out, d_out, gb3, workspace, workspace_bytes, s)) != hipSuccess) return SYNTH_EDEVICE;
  // dh2 = (dz3 W3^T^T) * gelu'(h2pre): A = dz3 [batch][d_out], B[k][n] = W3^T[k][n]
  g = {}; g.alpha = 1.0f;
  g.M = batch; g.N = d_h; g.K = d_out; g.A = dz3; g.lda = d_out; g.B = w3t; g.ldb = d_h;
  g.C = dh2; g.ldc = d_h; g.c_bf16 = 1; g.epilogue = synth::kEpiGeluGrad; g.aux = h2pre;
  if ((e = gemm_maybe_split(g, kOpKMajor, kOpRowMajorMN, workspace, s)) != hipSuccess) return SYNTH_EDEVICE;
  // dW2^T = dh2^T h1, db2
  g = {}; g.alpha = 1.0f;
  g.M = d_h; g.N = d_h; g.K = batch; g.A = dh2; g.lda = d_h; g.B = h1; g.ldb = d_h;
  g.C = gw2t; g.ldc = d_h;
  if ((e = gemm_maybe_split(g, kOpRowMajorMN, kOpRowMajorMN, workspace, s)) != hipSuccess) return SYNTH_EDEVICE;
  if ((e = synth::launch_colsum_bf16_ws(dh2, batch, d_h, d_h, gb2, workspace, workspace_bytes, s)) != hipSuccess) return SYNTH_EDEVICE;
  // dh1 = (dh2 W2^T^T) * gelu'(h1pre)
  g = {}; g.alpha = 1.0f;
  g.M = batch; g.N = d_h; g.K = d_h; g.A = dh2; g.lda = d_h; g.B = w2t; g.ldb = d_h;
  g.C = dh1; g.ldc = d_h; g.c_bf16 = 1; g.epilogue = synth::kEpiGeluGrad; g.aux = h1pre;
  if ((e = gemm_maybe_split(g, kOpKMajor, kOpRowMajorMN, workspace, s)) != hipSuccess) return SYNTH_EDEVICE;
  // dW1^T = dh1^T x, db1
  g = {}; g.alpha = 1.0f;
  g.M = d_h; g.N = d_in; g.K = batch; g.A = dh1; g.lda = d_h; g.B = x; g.ldb = d_in;
  g.C = gw1t; g.ldc = d_in;
  if ((e = gemm_maybe_split(g, kOpRowMajorMN, kOpRowMajorMN, workspace, s)) != hipSuccess) return SYNTH_EDEVICE;
  return to_status(synth::launch_colsum_bf16_ws(dh1, batch, d_h, d_h, gb1, workspace, workspace_bytes, s));
}

int synth_logit_init(const float* u, float* z, float* u_out, int64_t n, float eps, void* stream) {
  if (n < 0 || !(eps > 0.0f && eps < 0.5f)) return SYNTH_EINVAL;
  if (n > 0 && (!u || !z || !u_out)) return SYNTH_EINVAL;
  return to_status(synth::launch_logit_init(u, z, u_out, n, eps, (hipStream_t)stream));
}

int synth_logit_adam(int64_t n, float* z, float* u, const float* grad_u, float* m, float* v,
                     float lr, float beta1, float beta2, float eps, int step, void* stream) {
  if (n < 0 || step < 1) return SYNTH_EINVAL;
  if (n > 0 && (!z || !u || !grad_u || !m || !v)) return SYNTH_EINVAL;
  return to_status(synth::launch_logit_adam(n, z, u, grad_u, m, v, lr, beta1, beta2, eps, step,
                                            (hipStream_t)stream));
}

int synth_best_update(const double* loss, int64_t rows, int64_t cols, int64_t row_stride,
                      int64_t col_stride, int64_t col_base, const float* params, int64_t param_dim,
                      double* best, int64_t* best_idx, float* best_params, void* stream) {
  if (rows < 0 || cols < 0 || row_stride < 0 || col_stride < 0 || param_dim < 0) return SYNTH_EINVAL;
  if (rows == 0) return SYNTH_OK;
  if (!loss || !best || (cols > 0 && rows > 1 && row_stride == 0)) return SYNTH_EINVAL;
  if ((params != nullptr) != (best_params != nullptr)) return SYNTH_EINVAL;
  if (params && param_dim == 0) return SYNTH_EINVAL;
  return to_status(synth::launch_best_update(loss, rows, cols, row_stride, col_stride, col_base,
                                             params, param_dim, best, best_idx, best_params,
                                             (hipStream_t)stream));
}

int synth_adam(int64_t n, float* w, void* w_bf16, const float* grad, float* m, float* v, float lr,
               float beta1, float beta2, float eps, int step, void* stream) {
  if (n < 0 || step < 1) return SYNTH_EINVAL;
  if (n > 0 && (!w || !grad || !m || !v)) return SYNTH_EINVAL;
  return to_status(synth::launch_adam(n, w, w_bf16, grad, m, v, lr, beta1, beta2, eps, step,
                                      (hipStream_t)stream));
}

}  // extern "C"
