// Fused Voice render for gfx950 (CDNA4): one 64-lane wavefront per voice.
//
// The Voice (Section 3.2): keyboard -> six ADSRs -> two rate-modulated LFOs
// scaled by their amplitude ADSRs -> modulation mixer -> (upsampled to the audio
// rate) sine VCO, square-saw VCO, noise -> VCAs -> audio mixer.  Control modules
// run at the control rate (Section 3.1): one control sample per q audio samples.
//
// Work decomposition (per voice, 62 control periods - "segments" - per chunk):
//   control stage   lane l evaluates control sample j = 62c + l (l <= 62) in
//                   float64: the six envelopes, both LFOs (their phase is a
//                   wavefront exclusive scan of the rate plus a carry), the
//                   modulation mixer, and per segment the pitch-glide
//                   increment, its geometric ratio and the segment's phase
//                   advance; a second float64 scan gives each segment's start
//                   phase.  Nothing is written to HBM.
//   oscillator pass each lane renders one run of h = q / RPS consecutive
//                   samples of one segment: float64 phase recurrence, half-cycle
//                   range reduction, float32 sine, tanh-waveshaped square-saw,
//                   VCAs, mixer; the result goes to an LDS tile.
//   store pass      each lane takes 4 consecutive tile samples, adds the noise
//                   oscillator (one Philox call gives 8 16-bit noise samples)
//                   through its VCA, and writes them with one 16-byte store, so
//                   each store instruction covers 1 KB of contiguous audio.
// Segments at or after the end of the longest release are exactly silent
// (every envelope is 0 there): they are zero-filled without computation.
#include <math.h>

#include "philox.h"
#include "synth_internal.h"

namespace synth {
namespace {

constexpr int kWave = 64;
constexpr int kSegsPerChunk = 62;
constexpr int kPointsPerChunk = kSegsPerChunk + 1;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kLn2 = 0.693147180559945309417232121458;

// ---------------------------------------------------------------------------
// float64 control-rate helpers
// ---------------------------------------------------------------------------
// x^e for x in [0, 1] (0^e = 0, 1^e = 1 without evaluating exp2/log2).
__device__ __forceinline__ double pow01(double x, double e) {
  return x <= 0.0 ? 0.0 : (x >= 1.0 ? 1.0 : exp2(e * log2(x)));
}

// clamp((j - start) / len, 0, 1); len == 0 is the step [j >= start].
__device__ __forceinline__ double ramp(double j, double start, double len, double inv_len) {
  return len > 0.0 ? fmin(fmax((j - start) * inv_len, 0.0), 1.0) : (j >= start ? 1.0 : 0.0);
}

__device__ __forceinline__ bool bit(const uint32_t* w, int p) { return (w[p >> 5] >> (p & 31)) & 1u; }

// Normalised u -> human-readable value (Section 3.3): u^(1/curve) on [min, max],
// or for symmetric parameters sign(d)|d|^(1/curve), d = 2u - 1, centred.
__device__ double map_param(double u, int p, const NebulaArgs& nb) {
  const double lo = nb.lo[p], span = nb.hi[p] - nb.lo[p];
  const bool lin = bit(nb.linear, p);
  if (!bit(nb.sym, p)) return lo + span * (lin ? u : pow(u, nb.inv_curve[p]));
  const double d = 2.0 * u - 1.0;
  const double ad = fabs(d);
  const double w = lin ? ad : pow(ad, nb.inv_curve[p]);
  const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
  return lo + span * (1.0 + sg * w) / 2.0;
}

// Exclusive prefix sum across the 64 lanes (lane 0 gets 0).
__device__ __forceinline__ double wave_excl_scan(double x, int lane) {
  double incl = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const double t = __shfl_up(incl, d);
    if (lane >= d) incl += t;
  }
  const double ex = __shfl_up(incl, 1);
  return lane == 0 ? 0.0 : ex;
}

// ---------------------------------------------------------------------------
// float32 audio-rate helpers
// ---------------------------------------------------------------------------
// sin(2 pi th) for the sine VCO: th (cycles, float64) is reduced to the
// nearest integer in float64, r = th - rint(th) in [-1/2, 1/2], and the
// hardware sine (input in revolutions, absolute error ~1.3e-7 on [-1/2, 1/2])
// is evaluated on float(r).
__device__ __forceinline__ float sin_cycles(double th) {
  const float r = (float)(th - rint(th));
  return __builtin_amdgcn_sinf(r);
}

// sin and cos of 2 pi th for the square-saw.  Its tanh edge multiplies the
// sine by K (up to ~1600) at every zero crossing, so the sine must be
// relatively accurate there, at th = 0 and th = 1/2 alike: th is reduced to
// the nearest half cycle in float64, r = th - n/2 in [-1/4, 1/4] (exact),
// sin(2 pi th) = (-1)^n sin(2 pi r), cos(2 pi th) = (-1)^n cos(2 pi r).  The
// hardware sine has ~9e-7 relative error near 0, which moves tanh(K sin) by
// at most ~4e-7.
__device__ __forceinline__ void sincos_cycles(double th, float& s, float& c) {
  const double n = rint(2.0 * th);
  const float r = (float)fma(-0.5, n, th);
  const uint32_t flip = ((uint32_t)(int)n) << 31;     // sign bit of (-1)^n
  s = __uint_as_float(__float_as_uint(__builtin_amdgcn_sinf(r)) ^ flip);
  c = __uint_as_float(__float_as_uint(__builtin_amdgcn_cosf(r)) ^ flip);
}

// tanh(z) = 1 - 2 / (exp(2z) + 1) from z2 = 2 log2(e) z; saturates to +-1
// through exp2 overflow or underflow, absolute error ~1e-7.
__device__ __forceinline__ float tanh_from_log2(float z2) {
  const float e = __builtin_amdgcn_exp2f(z2);
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

// Square-saw: (1 - s/2) tanh(K sin 2 pi th) (1 + s cos 2 pi th); K2 = 2 log2(e) K.
__device__ __forceinline__ float squaresaw(double th, float K2, float shape, float gain) {
  float s, c;
  sincos_cycles(th, s, c);
  return gain * tanh_from_log2(K2 * s) * fmaf(shape, c, 1.0f);
}

// expm1(x) in float64: Taylor series for |x| <= 1/4 (terms to x^15, relative
// truncation < 1e-19), the library routine otherwise.
__device__ __forceinline__ double expm1_f64(double x) {
  if (fabs(x) > 0.25) return expm1(x);
  double p = 1.0 / 1307674368000.0;          // 1/15!
  p = fma(p, x, 1.0 / 87178291200.0);
  p = fma(p, x, 1.0 / 6227020800.0);
  p = fma(p, x, 1.0 / 479001600.0);
  p = fma(p, x, 1.0 / 39916800.0);
  p = fma(p, x, 1.0 / 3628800.0);
  p = fma(p, x, 1.0 / 362880.0);
  p = fma(p, x, 1.0 / 40320.0);
  p = fma(p, x, 1.0 / 5040.0);
  p = fma(p, x, 1.0 / 720.0);
  p = fma(p, x, 1.0 / 120.0);
  p = fma(p, x, 1.0 / 24.0);
  p = fma(p, x, 1.0 / 6.0);
  p = fma(p, x, 0.5);
  p = fma(p, x, 1.0);
  return p * x;
}

// Zero out[z0, z1) with all 64 lanes (z0 a multiple of 4).
__device__ void zero_fill(float* out, int64_t z0, int64_t z1, int lane, bool aligned) {
  if (z1 <= z0) return;
  if (aligned) {
    const int64_t n4 = (z1 - z0) / 4;
    float4* d4 = reinterpret_cast<float4*>(out + z0);
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t i = lane; i < n4; i += kWave) d4[i] = zero;
    for (int64_t i = z0 + 4 * n4 + lane; i < z1; i += kWave) out[i] = 0.0f;
  } else {
    for (int64_t i = z0 + lane; i < z1; i += kWave) out[i] = 0.0f;
  }
}

// Per-voice constants derived once from the parameters (LDS, read by every lane).
enum {
  kEnvA = 0, kEnvInvA = 6, kEnvD = 12, kEnvInvD = 18, kEnvR = 24, kEnvInvR = 30, kEnvS = 36,
  kEnvAlpha = 42, kLfoInvW = 48, kMixInvNorm = 50, kDerived = 56
};

// Per-segment oscillator data of a chunk, one row per VCO.
enum { kSegTheta = 0, kSegInc = 1, kSegRatio = 2, kSegRunSum = 3, kSegRunRatio = 4, kSegFields = 5 };

struct VoiceShared {
  double v[kNumParams];        // human-readable parameter values
  double d[kDerived];          // derived per-voice constants (enum above)
  double seg[2][kSegFields][kWave];   // per VCO and segment: start phase (cycles, in [0,1)),
                                      // start increment, per-sample ratio, first-run sum,
                                      // per-run ratio
  double carry[4];             // phase carries (cycles): LFO 1, LFO 2, VCO 1, VCO 2
  float2 namp[kWave];          // per segment of the chunk: noise VCA (start, slope) * level * 2^-15
};

template <int RPS, bool CLAMP>
__device__ void render_item(const RenderArgs& a, int64_t b, int slice, VoiceShared& sh,
                            float* tile) {
  const int lane = threadIdx.x;
  const int q = a.q;
  const int h = q / RPS;             // samples per run
  const double qd = (double)q;
  const double hd = (double)h;

  int64_t off0, N;
  if (a.offsets) {
    off0 = a.offsets[b];
    N = a.offsets[b + 1] - off0;
  } else {
    off0 = b * a.n_uniform;
    N = a.n_uniform;
  }
  if (N <= 0) return;
  const uint64_t g = a.voice_ids ? a.voice_ids[b] : a.first_g + (uint64_t)b;
  float* out = a.audio + off0;
  const bool aligned = (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
  const double rc = a.rc, sr = a.sr;

  __syncthreads();
  for (int p = lane; p < kNumParams; p += kWave)
    sh.v[p] = map_param((double)a.params[b * kNumParams + p], p, a.neb);
  __syncthreads();
  const double* v = sh.v;
  if (lane < 6) {                    // envelope k: durations in control samples
    const int pb = 2 + 5 * lane;
    const double A = v[pb] * rc, D = v[pb + 1] * rc, R = v[pb + 3] * rc;
    sh.d[kEnvA + lane] = A;
    sh.d[kEnvInvA + lane] = 1.0 / A;
    sh.d[kEnvD + lane] = D;
    sh.d[kEnvInvD + lane] = 1.0 / D;
    sh.d[kEnvR + lane] = R;
    sh.d[kEnvInvR + lane] = 1.0 / R;
    sh.d[kEnvS + lane] = v[pb + 2];
    sh.d[kEnvAlpha + lane] = v[pb + 4];
  } else if (lane < 8) {             // LFO: 1 / sum of shape weights (0 if none)
    const int pb = 32 + 8 * (lane - 6);
    const double ws = v[pb + 3] + v[pb + 4] + v[pb + 5] + v[pb + 6] + v[pb + 7];
    sh.d[kLfoInvW + lane - 6] = ws > 0.0 ? 1.0 / ws : 0.0;
  } else if (lane < 13) {            // modulation mixer row: 1 / max(1, sum of gains)
    const int pb = 48 + 4 * (lane - 8);
    sh.d[kMixInvNorm + lane - 8] = 1.0 / fmax(1.0, v[pb] + v[pb + 1] + v[pb + 2] + v[pb + 3]);
  }
  __syncthreads();
  const double* dv = sh.d;

  const int64_t J = (N + q - 1) / q;     // control samples == segments
  const int64_t nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
  const int64_t c_lo = nchunks * slice / a.slices;
  const int64_t c_hi = nchunks * (slice + 1) / a.slices;

  const double note_off = v[1] * rc;
  // Every envelope is exactly 0 from control sample js on: the release ramp
  // has reached 1 (at least one control sample past note-off + release).
  double jsil = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) jsil = fmax(jsil, note_off + v[2 + 5 * k + 3] * rc);
  jsil = fmin(jsil, 9.0e15);
  const int64_t js = (int64_t)floor(jsil) + 2;
  const int64_t c_sil = (js + kSegsPerChunk - 1) / kSegsPerChunk;

  // square-saw constants: K from the highest reachable pitch
  const double midi = v[0];
  const double m_hi = fmax(0.0, midi + v[71] + fmax(0.0, v[72]));
  const double f_hi = fmin(440.0 * exp2((m_hi - 69.0) / 12.0), sr / 2.0);
  const float K2 = (float)(2.0 * 1.4426950408889634 * 12000.0 / (f_hi * log10(f_hi)));
  const float shape = (float)v[74];
  const float sq_gain = (float)(1.0 - v[74] / 2.0);
  const double L1 = v[75], L2 = v[76], L3 = v[77];

  // phase carries in cycles, reduced mod 1 at every chunk boundary
  if (lane < 4) {
    const double ph0 = v[lane == 0 ? 34 : lane == 1 ? 42 : lane == 2 ? 70 : 73] / kTwoPi;
    sh.carry[lane] = ph0 - floor(ph0);
  }
  __syncthreads();
  const uint32_t glo = (uint32_t)g, ghi = (uint32_t)(g >> 32);

  for (int64_t c = 0; c < c_hi; ++c) {
    if (c >= c_sil) {
      const int64_t z0 = (c > c_lo ? c : c_lo) * (int64_t)kSegsPerChunk * q;
      const int64_t z1 = c_hi * (int64_t)kSegsPerChunk * q < N ? c_hi * (int64_t)kSegsPerChunk * q : N;
      zero_fill(out, z0, z1, lane, aligned);
      break;
    }
    // ---------------- control stage: lane = control sample j ----------------
    const int64_t j = c * kSegsPerChunk + lane;
    const double jd = (double)j;
    // Envelopes go through LDS (the tile is idle during the control stage), one
    // at a time, which keeps the float64 exp2/log2 chains from being interleaved.
    double* envs = reinterpret_cast<double*>(tile);
#pragma unroll 1
    for (int k = 0; k < 6; ++k) {
      // ADSR: attack rise, decay fall towards sustain, release fall from note-off,
      // each ramp raised to the curve exponent alpha.
      const double A = dv[kEnvA + k], D = dv[kEnvD + k], R = dv[kEnvR + k];
      const double S = dv[kEnvS + k], al = dv[kEnvAlpha + k];
      const double att = ramp(jd, 0.0, A, dv[kEnvInvA + k]);
      const double dec = ramp(jd, A, D, dv[kEnvInvD + k]);
      const double rel = ramp(jd, note_off, R, dv[kEnvInvR + k]);
      envs[k * kWave + lane] =
          pow01(att, al) * (S + (1.0 - S) * pow01(1.0 - dec, al)) * pow01(1.0 - rel, al);
    }
    // LFOs (rate ADSR modulates the rate; amp ADSR is a control-rate VCA),
    // written next to the envelopes: lfo'_i at envs[(6 + i) * 64 + lane].
#pragma unroll 1
    for (int i = 0; i < 2; ++i) {
      const int pb = 32 + 8 * i;
      const double f = fmax(0.0, v[pb] + v[pb + 1] * envs[(2 + 2 * i) * kWave + lane]);
      const double inc = lane < kPointsPerChunk - 1 ? f / rc : 0.0;
      const double th = sh.carry[i] + wave_excl_scan(inc, lane);
      const double ph = th - floor(th);
      const double num = v[pb + 3] * ((1.0 + sinpi(2.0 * ph)) / 2.0) +
                         v[pb + 4] * (1.0 - fabs(2.0 * ph - 1.0)) + v[pb + 5] * ph +
                         v[pb + 6] * (1.0 - ph) + v[pb + 7] * (ph < 0.5 ? 1.0 : 0.0);
      envs[(6 + i) * kWave + lane] = (num * dv[kLfoInvW + i]) * envs[(3 + 2 * i) * kWave + lane];
      const double nc = __shfl(th, kSegsPerChunk);            // phase at the next chunk's first point
      __syncthreads();
      if (lane == 0) sh.carry[i] = nc - floor(nc);
    }
    // modulation mixer: inputs adsr_1, adsr_2, lfo'_1, lfo'_2
    const double x0 = envs[lane], x1 = envs[kWave + lane];
    const double x2 = envs[6 * kWave + lane], x3 = envs[7 * kWave + lane];
    double y[5], yn[5];
    const bool last = (j + 1 >= J);                  // right end held at the last control sample
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const int pb = 48 + 4 * o;
      const double acc = v[pb] * x0 + v[pb + 1] * x1 + v[pb + 2] * x2 + v[pb + 3] * x3;
      y[o] = acc * dv[kMixInvNorm + o];
    }
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const double t = __shfl_down(y[o], 1);
      yn[o] = last ? y[o] : t;
    }
    // per segment (lane < 62): pitch glide, phase advance; one VCO at a time
#pragma unroll 1
    for (int vc = 0; vc < 2; ++vc) {
      const int tb = vc ? 71 : 68;
      const double ya = vc ? y[2] : y[0];
      const double yb = vc ? yn[2] : yn[0];
      const double base = midi + v[tb];
      const double m0 = base + v[tb + 1] * ya;
      const double m1 = base + v[tb + 1] * yb;
      const double i0 = 440.0 * exp2((m0 - 69.0) / 12.0) / sr;
      const double Lr = (m1 - m0) * (kLn2 / (12.0 * qd));   // log of the per-sample ratio
      const double e1 = expm1_f64(Lr);
      const double eh = expm1_f64(Lr * hd);
      const double rr = 1.0 + e1;
      const double Rh = 1.0 + eh;
      const double Sh = (e1 == 0.0) ? i0 * hd : i0 * (eh / e1);
      double S;
      if constexpr (CLAMP) {
        // some increments may exceed 1/2 cycle (f > sr/2): sum them one by one
        S = 0.0;
        double inc = i0;
        for (int k = 0; k < q; ++k) {
          S += fmin(inc, 0.5);
          inc *= rr;
        }
      } else {
        S = Sh;
        double t = Sh;
#pragma unroll
        for (int m = 1; m < RPS; ++m) {
          t *= Rh;
          S += t;
        }
      }
      const double th = sh.carry[2 + vc] + wave_excl_scan(lane < kSegsPerChunk ? S : 0.0, lane);
      sh.seg[vc][kSegTheta][lane] = th - floor(th);
      sh.seg[vc][kSegInc][lane] = i0;
      sh.seg[vc][kSegRatio][lane] = rr;
      sh.seg[vc][kSegRunSum][lane] = Sh;
      sh.seg[vc][kSegRunRatio][lane] = Rh;
      const double nc = __shfl(th, kSegsPerChunk);
      __syncthreads();
      if (lane == 0) sh.carry[2 + vc] = nc - floor(nc);
    }
    if (c < c_lo) continue;                      // slice starts later: only carries needed

    const float a10 = (float)(L1 * y[1]), a1d = (float)(L1 * (yn[1] - y[1]) / qd);
    const float a20 = (float)(L2 * y[3]), a2d = (float)(L2 * (yn[3] - y[3]) / qd);
    __syncthreads();                             // previous chunk's readers of namp are done
    if (lane < kSegsPerChunk)                    // noise VCA ramp, pre-scaled by the 2^-15 of the noise map
      sh.namp[lane] = make_float2((float)(L3 * y[4]) * (1.0f / 32768.0f),
                                  (float)(L3 * (yn[4] - y[4]) / qd) * (1.0f / 32768.0f));
    __syncthreads();

    // ---------------- oscillator and store passes ----------------
    constexpr int segs_pp = kWave / RPS;
    const int nseg = (int)((J - c * kSegsPerChunk) < kSegsPerChunk ? (J - c * kSegsPerChunk)
                                                                    : kSegsPerChunk);
    const int npass = (nseg + segs_pp - 1) / segs_pp;
    for (int p = 0; p < npass; ++p) {
      const int ls = p * segs_pp + lane / RPS;   // chunk-local segment of this lane's run
      const int m = lane % RPS;                  // run within the segment
      const int src = ls < kWave ? ls : kWave - 1;
      double t1 = sh.seg[0][kSegTheta][src], i1 = sh.seg[0][kSegInc][src];
      double t2 = sh.seg[1][kSegTheta][src], i2 = sh.seg[1][kSegInc][src];
      const double r1 = sh.seg[0][kSegRatio][src], r2 = sh.seg[1][kSegRatio][src];
      const float A10 = __shfl(a10, src), A1d = __shfl(a1d, src);
      const float A20 = __shfl(a20, src), A2d = __shfl(a2d, src);
      if constexpr (CLAMP) {
        for (int k = 0; k < m * h; ++k) {
          t1 += fmin(i1, 0.5); i1 *= r1;
          t2 += fmin(i2, 0.5); i2 *= r2;
        }
      } else {
        double s1 = sh.seg[0][kSegRunSum][src], R1 = sh.seg[0][kSegRunRatio][src];
        double s2 = sh.seg[1][kSegRunSum][src], R2 = sh.seg[1][kSegRunRatio][src];
        for (int t = 0; t < m; ++t) {
          t1 += s1; s1 *= R1; i1 *= R1;
          t2 += s2; s2 *= R2; i2 *= R2;
        }
      }
      float kf = (float)(m * h);
      float* trow = tile + lane * h;
      for (int k = 0; k < h; ++k) {
        const float x1 = sin_cycles(t1);
        const float x2 = squaresaw(t2, K2, shape, sq_gain);
        const float A1 = fmaf(kf, A1d, A10);
        const float A2 = fmaf(kf, A2d, A20);
        trow[k] = fmaf(A2, x2, A1 * x1);
        if constexpr (CLAMP) {
          t1 += fmin(i1, 0.5); t2 += fmin(i2, 0.5);
        } else {
          t1 += i1; t2 += i2;
        }
        i1 *= r1;
        i2 *= r2;
        kf += 1.0f;
      }
      __syncthreads();
      // Store pass: noise + VCA, 4 consecutive samples per lane per 16-byte store.
      // Every lane computes one Philox call (8 noise samples) per 512 samples;
      // lane l's 4 samples of each 256-sample half take two of its group's
      // words from the lane that drew them.  4 samples never straddle a
      // segment because q is a multiple of 4.
      const int64_t pbase = (c * kSegsPerChunk + (int64_t)p * segs_pp) * q;
      int64_t cnt64 = (int64_t)((nseg - p * segs_pp) < segs_pp ? (nseg - p * segs_pp) : segs_pp) * q;
      if (cnt64 > N - pbase) cnt64 = N - pbase;
      const int cnt = (int)cnt64;
      const uint32_t grp0 = (uint32_t)(pbase >> 3);
      const int seg0 = p * segs_pp;
      for (int base = 0; base < cnt; base += 512) {
        uint32_t w[4] = {glo, ghi, grp0 + (uint32_t)(base >> 3) + (uint32_t)lane, 1u};
        philox4x32_10(w, a.nk0, a.nk1);
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
          const int src_l = sub * 32 + (lane >> 1);
          const uint32_t w0 = __shfl(w[0], src_l), w1 = __shfl(w[1], src_l);
          const uint32_t w2 = __shfl(w[2], src_l), w3 = __shfl(w[3], src_l);
          const uint32_t wa = (lane & 1) ? w2 : w0;
          const uint32_t wb = (lane & 1) ? w3 : w1;
          const int li = base + sub * 256 + 4 * lane;   // pass-local sample
          if (li < cnt) {
            const int lsg = (int)__umulhi((uint32_t)li, a.q_magic);   // li / q
            const float2 na = sh.namp[seg0 + lsg];
            const float a0 = fmaf((float)(li - lsg * q), na.y, na.x);   // noise VCA at li
            const float4 t4 = *reinterpret_cast<const float4*>(tile + li);
            float o[4];
            o[0] = fmaf((float)(wa & 0xFFFFu) - 32767.5f, a0, t4.x);
            o[1] = fmaf((float)(wa >> 16) - 32767.5f, fmaf(1.0f, na.y, a0), t4.y);
            o[2] = fmaf((float)(wb & 0xFFFFu) - 32767.5f, fmaf(2.0f, na.y, a0), t4.z);
            o[3] = fmaf((float)(wb >> 16) - 32767.5f, fmaf(3.0f, na.y, a0), t4.w);
            float* dst = out + pbase + li;
            if (aligned && li + 4 <= cnt) {
              *reinterpret_cast<float4*>(dst) = make_float4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (li + e < cnt) dst[e] = o[e];
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

template <int RPS, bool CLAMP>
__global__ void __launch_bounds__(kWave) render_kernel(const RenderArgs a) {
  __shared__ VoiceShared sh;
  extern __shared__ __align__(16) float tile[];
  const int64_t nitems = a.batch * a.slices;
  for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x)
    render_item<RPS, CLAMP>(a, item / a.slices, (int)(item % a.slices), sh, tile);
}

// Mix mode 1: y <- y / max(1, max |y|) per voice.  One 256-thread workgroup per voice.
__global__ void __launch_bounds__(256) peak_normalise_kernel(const RenderArgs a) {
  __shared__ float red[256];
  const int64_t b = blockIdx.x;
  int64_t off0, N;
  if (a.offsets) {
    off0 = a.offsets[b];
    N = a.offsets[b + 1] - off0;
  } else {
    off0 = b * a.n_uniform;
    N = a.n_uniform;
  }
  float* y = a.audio + off0;
  float m = 0.0f;
  for (int64_t i = threadIdx.x; i < N; i += 256) m = fmaxf(m, fabsf(y[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const float peak = red[0];
  if (peak <= 1.0f) return;
  const float inv = 1.0f / peak;
  for (int64_t i = threadIdx.x; i < N; i += 256) y[i] = y[i] * inv;
}

template <int RPS>
hipError_t launch_rps(const RenderArgs& a, bool clamp, int grid, hipStream_t s) {
  // LDS tile: one run of q / RPS floats per lane; it also holds the six
  // float64 envelopes and two LFO outputs of the control stage.
  size_t shmem = (size_t)kWave * (a.q / RPS) * sizeof(float);
  if (shmem < 8 * kWave * sizeof(double)) shmem = 8 * kWave * sizeof(double);
  if (clamp)
    hipLaunchKernelGGL((render_kernel<RPS, true>), dim3(grid), dim3(kWave), shmem, s, a);
  else
    hipLaunchKernelGGL((render_kernel<RPS, false>), dim3(grid), dim3(kWave), shmem, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_render(const RenderArgs& a, int runs_per_segment, bool clamp, int grid,
                         hipStream_t s) {
  if (a.batch == 0) return hipSuccess;
  switch (runs_per_segment) {
    case 1: return launch_rps<1>(a, clamp, grid, s);
    case 2: return launch_rps<2>(a, clamp, grid, s);
    case 4: return launch_rps<4>(a, clamp, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_peak_normalise(const RenderArgs& a, hipStream_t s) {
  if (a.batch == 0) return hipSuccess;
  hipLaunchKernelGGL(peak_normalise_kernel, dim3((unsigned)a.batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace synth
