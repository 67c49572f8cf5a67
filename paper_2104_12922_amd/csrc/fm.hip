// Four-operator FM voice (the FM architecture Sections 3.2 and 7 announce).
// Four sine operators on the keyboard pitch, operator i at f_i = 440
// 2^((midi_f0 - 69) / 12) ratio_i 2^(detune_i / 1200) (at most sr / 2), each
// scaled by its level and its own ADSR (the Voice's envelope at the control
// rate, upsampled linearly, holding the last control value); operator j
// modulates operator i < j's phase with index M[i][j] cycles:
//   o_i(n) = level_i env_i(n) sin(2 pi (n f_i / sr + sum_{j > i} M[i][j] o_j(n)))
// for i = 3, 2, 1, 0, and y(n) = sum_i w_i o_i(n) / max(1, sum_i w_i).
//
// No operator feeds back on itself, so every sample is a closed-form
// function of n: one wavefront per voice takes 64 control periods (a chunk)
// at a time; lane l evaluates the four envelopes at control sample
// 64c + l + 1 (float64, the Voice's ADSR code; 64c is the previous chunk's
// last) into LDS, then every lane renders four
// consecutive samples per step (lanes on consecutive 16-byte groups, so each
// store instruction writes 1 KB of contiguous audio).  The four samples share
// a control period; the phase n f_i / sr of the first is formed in float64
// and reduced to [0, 1), the next three add f_i / sr in float32 (within
// 2e-7 cycles), and the float32 hardware sine takes revolutions.  Periods
// after every envelope has reached 0 are zero-filled without computation.
// Bound by VALU issue: four sines and four modulated phases per sample.
#include "voice_device.h"

namespace synth {
namespace {

using voice::adsr_value;
using voice::kEnvA;
using voice::kEnvAlpha;
using voice::kEnvD;
using voice::kEnvInvA;
using voice::kEnvInvD;
using voice::kEnvInvR;
using voice::kEnvR;
using voice::kEnvS;
using voice::kDerived;
using voice::map_param;

constexpr int kFmParams = 44;
constexpr int kOpBase[4] = {2, 10, 18, 26};
constexpr int kModBase = 34, kMixBase = 40;

struct FmArgs {
  const float* params;       // [B][44] normalised
  const int64_t* offsets;    // [B + 1] or null
  int64_t n_uniform;
  int64_t batch;
  float* audio;
  double sr, rc;
  int q;
  uint32_t q_magic;          // x / q == umulhi(x, q_magic) for x < 2^16
  NebulaArgs neb;            // first 44 entries used
  const int32_t* order;      // null, or the voices in the order workgroups take them
};

__global__ void __launch_bounds__(64) fm_render_kernel(FmArgs a) {
  __shared__ double v[kFmParams];
  __shared__ double dv[kDerived];
  __shared__ float envs[4][65];
  const int lane = threadIdx.x;
  const int64_t b = a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
  if (b < 0 || b >= a.batch) return;         // an order entry out of range renders nothing
  int64_t start, L;
  if (a.offsets) {
    packed_range(a.offsets, a.batch, b, start, L);
  } else {
    start = b * a.n_uniform;
    L = a.n_uniform;
  }
  if (L <= 0) return;
  float* out = a.audio + start;
  if (lane < kFmParams) v[lane] = map_param((double)a.params[b * kFmParams + lane], lane, a.neb);
  __syncthreads();
  const double rc = a.rc;
  if (lane < 4) {                          // envelope of operator `lane`, in control samples
    const int pb = kOpBase[lane] + 3;
    const double A = v[pb] * rc, D = v[pb + 1] * rc, R = v[pb + 3] * rc;
    dv[kEnvA + lane] = A;
    dv[kEnvInvA + lane] = 1.0 / A;
    dv[kEnvD + lane] = D;
    dv[kEnvInvD + lane] = 1.0 / D;
    dv[kEnvR + lane] = R;
    dv[kEnvInvR + lane] = 1.0 / R;
    dv[kEnvS + lane] = v[pb + 2];
    dv[kEnvAlpha + lane] = v[pb + 4];
  }
  __syncthreads();
  const double note_off = v[1] * rc;
  // operator constants (uniform)
  double inc[4];
  float lvl[4], incf[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int pb = kOpBase[i];
    const double f = 440.0 * voice::exp2_f64((v[0] - 69.0) / 12.0) * v[pb] *
                     voice::exp2_f64(v[pb + 1] / 1200.0);
    inc[i] = fmin(f, a.sr / 2.0) / a.sr;
    incf[i] = (float)inc[i];
    lvl[i] = (float)v[pb + 2];
  }
  const float m01 = (float)v[kModBase], m02 = (float)v[kModBase + 1], m03 = (float)v[kModBase + 2];
  const float m12 = (float)v[kModBase + 3], m13 = (float)v[kModBase + 4];
  const float m23 = (float)v[kModBase + 5];
  const double wsum = v[kMixBase] + v[kMixBase + 1] + v[kMixBase + 2] + v[kMixBase + 3];
  const double wn = 1.0 / fmax(1.0, wsum);
  const float w0 = (float)(v[kMixBase] * wn), w1 = (float)(v[kMixBase + 1] * wn);
  const float w2 = (float)(v[kMixBase + 2] * wn), w3 = (float)(v[kMixBase + 3] * wn);
  // every envelope is exactly 0 from control sample note_off + R_i on; a
  // period whose two control values are 0 is silent
  double rel_end = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) rel_end = fmax(rel_end, note_off + dv[kEnvR + i]);
  const int64_t J = (L + a.q - 1) / a.q;
  const int64_t j_silent = (int64_t)fmin((double)J, floor(rel_end) + 2.0);
  const float inv_q = 1.0f / (float)a.q;
  const bool vec = ((start & 3) == 0);
  for (int64_t j0 = 0; j0 < J; j0 += 64) {
    const int64_t c0 = j0 * a.q;
    const int cnt = (int)min((int64_t)64 * a.q, L - c0);
    if (j0 >= j_silent) {                  // silent from here on: zero-fill the rest
      for (int64_t p = c0 + 4 * lane; p < L; p += 256) {
        if (vec && p + 4 <= L) {
          *reinterpret_cast<float4*>(out + p) = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
          for (int e = 0; e < 4 && p + e < L; ++e) out[p + e] = 0.0f;
        }
      }
      break;
    }
    // control values at j0 + 0 .. 64 (the last period holds its value): lane
    // l evaluates j0 + l + 1; the value at j0 is the previous chunk's last
    // one (the same control sample), so every lane works on each evaluation
    {
      float carry[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) carry[i] = envs[i][64];
      if (j0 == 0 && lane == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) carry[i] = lvl[i] * (float)adsr_value(dv, i, 0.0, note_off);
      }
      const double jd = (double)min(j0 + lane + 1, J - 1);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float e = lvl[i] * (float)adsr_value(dv, i, jd, note_off);
        if (lane == 0) envs[i][0] = carry[i];
        envs[i][lane + 1] = e;
      }
    }
    __syncthreads();
    for (int p = 4 * lane; p < cnt; p += 256) {
      // samples p .. p + 3 lie in one control period (q and p are multiples
      // of 4): one period index, one float64 phase per operator, the other
      // three phases and envelope values by float32 steps from it
      const int seg = (int)__umulhi((uint32_t)p, a.q_magic);
      const float t0 = (float)(p - seg * a.q) * inv_q;
      const double n0d = (double)(c0 + p);
      float ph0[4], e0[4], de[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double th = n0d * inc[i];
        ph0[i] = (float)(th - floor(th));
        e0[i] = envs[i][seg];
        de[i] = envs[i][seg + 1] - e0[i];
      }
      float y[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float t = fmaf((float)e, inv_q, t0);
        float ph[4], en[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ph[i] = fmaf((float)e, incf[i], ph0[i]);
          en[i] = fmaf(t, de[i], e0[i]);
        }
        const float o3 = en[3] * __builtin_amdgcn_sinf(ph[3]);
        const float o2 = en[2] * __builtin_amdgcn_sinf(fmaf(m23, o3, ph[2]));
        const float o1 = en[1] * __builtin_amdgcn_sinf(fmaf(m12, o2, fmaf(m13, o3, ph[1])));
        const float o0 =
            en[0] * __builtin_amdgcn_sinf(fmaf(m01, o1, fmaf(m02, o2, fmaf(m03, o3, ph[0]))));
        y[e] = fmaf(w0, o0, fmaf(w1, o1, fmaf(w2, o2, w3 * o3)));
      }
      const int64_t n0 = c0 + p;
      if (vec && p + 4 <= cnt) {
        *reinterpret_cast<float4*>(out + n0) = make_float4(y[0], y[1], y[2], y[3]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (p + e < cnt) out[n0 + e] = y[e];
      }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_fm_render(const float* params, const int64_t* offsets, int64_t batch,
                            int64_t n_samples, float* audio, double sr, double rc, int q,
                            const NebulaArgs& neb, const int32_t* order, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  FmArgs a;
  a.params = params;
  a.offsets = offsets;
  a.n_uniform = offsets ? 0 : n_samples;
  a.batch = batch;
  a.audio = audio;
  a.sr = sr;
  a.rc = rc;
  a.q = q;
  a.q_magic = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)q - 1) / (uint64_t)q);
  a.neb = neb;
  a.order = order;
  hipLaunchKernelGGL(fm_render_kernel, dim3((unsigned)batch), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace synth
