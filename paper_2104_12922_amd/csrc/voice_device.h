// Device-side building blocks of the Voice shared by the render and its
// adjoint: parameter mapping (Section 3.3), control-rate float64 helpers,
// wavefront scans, and the float32 oscillator evaluations.
#pragma once

#include <math.h>

#include "series_tables.h"
#include "synth_internal.h"

namespace synth {
namespace voice {

constexpr int kWave = 64;
constexpr int kSegsPerChunk = 62;
constexpr int kPointsPerChunk = kSegsPerChunk + 1;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kLn2 = 0.693147180559945309417232121458;

// Series coefficients in device memory.  Machine LICM is off (see build.py),
// so a float64 constant used in a loop is rematerialised with two VALU moves
// at every use; read from memory the compiler cannot fold, uniform addresses
// become scalar loads into SGPRs, which the float64 FMAs take as operands.
enum {
  kExpC3 = 0, kExpC4, kExpC5,                              // 1/3!, 1/4!, 1/5!
  kLogC3, kLogC4, kLogC5, kLogC6, kLogC7,                  // 1/3, -1/4, 1/5, -1/6, 1/7
  kSin3, kSin5, kSin7, kSin9, kSin11, kSin13, kSin15, kSin17, kSin19, kSin21, kSin23,
  kCos2, kCos4, kCos6, kCos8, kCos10, kCos12, kCos14, kCos16, kCos18, kCos20, kCos22,
  kEm3, kEm4, kEm5, kEm6, kEm7, kEm8, kEm9, kEm10, kEm11, kEm12, kEm13, kEm14, kEm15,
  kNumSeriesC
};
static __device__ double kSeriesC[kNumSeriesC] = {
    1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0,
    1.0 / 3.0, -0.25, 1.0 / 5.0, -1.0 / 6.0, 1.0 / 7.0,
    // (-1)^k / (2k + 1)!, k = 1 .. 11
    -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0, -1.0 / 39916800.0,
    1.0 / 6227020800.0, -1.0 / 1307674368000.0, 1.0 / 355687428096000.0,
    -1.0 / 121645100408832000.0, 1.0 / 51090942171709440000.0, -1.0 / 25852016738884976640000.0,
    // (-1)^k / (2k)!, k = 1 .. 11
    -0.5, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0, -1.0 / 3628800.0, 1.0 / 479001600.0,
    -1.0 / 87178291200.0, 1.0 / 20922789888000.0, -1.0 / 6402373705728000.0,
    1.0 / 2432902008176640000.0, -1.0 / 1124000727777607680000.0,
    // 1 / k!, k = 3 .. 15
    1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0, 1.0 / 40320.0,
    1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0,
    1.0 / 6227020800.0, 1.0 / 87178291200.0, 1.0 / 1307674368000.0};

// ---------------------------------------------------------------------------
// float64 control-rate helpers
// ---------------------------------------------------------------------------
// 2^y in float64 by Tang's table-driven method (ACM TOMS 15(2), 1989): with
// n = rint(256 y), y = e + j/256 + r, j = n mod 256, e = floor(n / 256) and
// r = y - n/256 exact (|r| <= 1/512), 2^y = 2^e 2^(j/256) exp(r ln 2); the
// table entry is correctly rounded and exp(z), |z| <= 0.0014, its Taylor
// series to degree 5 (truncation below 1e-20 relative).  y is clamped to
// [-1100, 1023] (below -1075 the result is 0).
__device__ __forceinline__ double exp2_f64(double y) {
  y = fmin(fmax(y, -1100.0), 1023.0);
  const double nd = rint(y * 256.0);
  const int n = (int)nd;
  const double z = fma(nd, -1.0 / 256.0, y) * kLn2;
  double p = fma(z, kSeriesC[kExpC5], kSeriesC[kExpC4]);
  p = fma(p, z, kSeriesC[kExpC3]);
  p = fma(p, z, 0.5);
  p = fma(p, z, 1.0);
  p = fma(p, z, 1.0);
  return ldexp(kExp2T[n & 255] * p, n >> 8);
}

// log2(x) for finite x > 0 in float64 by the table-driven method (Tang, ACM
// TOMS 16(4), 1990): x = m 2^e with m in [1/sqrt 2, sqrt 2), c = 1 + j/256 the
// table point nearest m (j = rint(256 (m - 1)) in -75 .. 106), u = m/c - 1
// formed as m (1/c) - 1 with the correctly rounded 1/c (|u| <= 0.0028,
// absolute error ~1e-16), log2 x = (e + log2 c) + log1p(u) / ln 2 with log1p
// by its series to degree 7 (truncation below 1e-21); near x = 1 both c = 1
// and log2 c = 0, so the result stays relatively accurate there.
__device__ __forceinline__ double log2_f64(double x) {
  int e;
  double m = frexp(x, &e);                    // m in [1/2, 1)
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  const int j = (int)rint((m - 1.0) * 256.0) + kLogJ0;
  const double u = fma(m, kInvC[j], -1.0);
  double p = fma(u, kSeriesC[kLogC7], kSeriesC[kLogC6]);
  p = fma(p, u, kSeriesC[kLogC5]);
  p = fma(p, u, kSeriesC[kLogC4]);
  p = fma(p, u, kSeriesC[kLogC3]);
  p = fma(p, u, -0.5);
  p = fma(p, u, 1.0);
  return fma(p * u, 1.0 / kLn2, kLog2T[j] + (double)e);
}

// sin(2 pi p) in float64 for a phase p in cycles: r = p - rint(p) in
// [-1/2, 1/2] (exact), folded to |r| <= 1/4 by sin(pi - a) = sin(a), then the
// Taylor series of sin(2 pi r) to degree 23 (|2 pi r| <= pi/2: truncation
// below 1e-20).
__device__ __forceinline__ double sin_cycles_f64(double p) {
  double r = p - rint(p);
  if (r > 0.25) r = 0.5 - r;
  if (r < -0.25) r = -0.5 - r;
  const double a = r * kTwoPi, a2 = a * a;
  double s = kSeriesC[kSin23];
#pragma unroll
  for (int k = kSin21; k >= kSin3; --k) s = fma(s, a2, kSeriesC[k]);
  s = fma(s, a2, 1.0);
  return s * a;
}

// sin(2 pi th) and cos(2 pi th) in float64: th is reduced to the nearest half
// cycle, r = th - n/2 in [-1/4, 1/4] (exact), a = 2 pi r, and the Taylor
// series of sin a to degree 23 and cos a to degree 22 (|a| <= pi/2:
// truncation below 4e-18) give sin(2 pi th) = (-1)^n sin a, cos(2 pi th) =
// (-1)^n cos a.
__device__ __forceinline__ void sincos_cycles_f64(double th, double& s, double& c) {
  const double n = rint(2.0 * th);
  const double a = fma(-0.5, n, th) * kTwoPi, a2 = a * a;
  double ps = kSeriesC[kSin23];
#pragma unroll
  for (int k = kSin21; k >= kSin3; --k) ps = fma(ps, a2, kSeriesC[k]);
  ps = fma(ps, a2, 1.0);
  double pc = kSeriesC[kCos22];
#pragma unroll
  for (int k = kCos20; k >= kCos2; --k) pc = fma(pc, a2, kSeriesC[k]);
  pc = fma(pc, a2, 1.0);
  const double sg = (((int)n) & 1) ? -1.0 : 1.0;
  s = sg * (ps * a);
  c = sg * pc;
}

// cos(2 pi th) in float64 by the reduction and series of sincos_cycles_f64.
__device__ __forceinline__ double cos_cycles_f64(double th) {
  const double n = rint(2.0 * th);
  const double a = fma(-0.5, n, th) * kTwoPi, a2 = a * a;
  double pc = kSeriesC[kCos22];
#pragma unroll
  for (int k = kCos20; k >= kCos2; --k) pc = fma(pc, a2, kSeriesC[k]);
  pc = fma(pc, a2, 1.0);
  return (((int)n) & 1) ? -pc : pc;
}

// x^e for x in [0, 1] (0^e = 0, 1^e = 1 without evaluating exp2/log2); in
// (0, 1) within about 1e-13 relative of the correctly rounded power.
__device__ __forceinline__ double pow01(double x, double e) {
  return x <= 0.0 ? 0.0 : (x >= 1.0 ? 1.0 : exp2_f64(e * log2_f64(x)));
}

// clamp((j - start) / len, 0, 1); len == 0 is the step [j >= start].
__device__ __forceinline__ double ramp(double j, double start, double len, double inv_len) {
  return len > 0.0 ? fmin(fmax((j - start) * inv_len, 0.0), 1.0) : (j >= start ? 1.0 : 0.0);
}

__device__ __forceinline__ bool bit(const uint32_t* w, int p) { return (w[p >> 5] >> (p & 31)) & 1u; }

// Normalised u -> human-readable value (Section 3.3): u^(1/curve) on [min, max],
// or for symmetric parameters sign(d)|d|^(1/curve), d = 2u - 1, centred.
__device__ inline double map_param(double u, int p, const NebulaArgs& nb) {
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
// sin(2 pi th) for the sine VCO within one run of samples: the caller
// reduces th to [-1/2, 1/2] in float64 at the run's start, so within a run
// of at most 192 samples of at most 1/2 cycle each |th| < 97 and float(th)
// is within 2^-18 cycles of it (sine error < 2.5e-5, typically far less: the
// per-sample increment is f / sr); the hardware sine takes revolutions and
// reduces its input itself (valid for |x| < 256).  The square-saw, whose
// tanh edge amplifies phase error, keeps the exact half-cycle reduction.
__device__ __forceinline__ float sin_cycles_run(double th) {
  return __builtin_amdgcn_sinf((float)th);
}

// Square-saw without its gain (1 - s/2), which the caller folds into the VCA:
// tanh(K sin 2 pi th) (1 + shape cos 2 pi th), K2 = 2 log2(e) K.  Its tanh
// edge multiplies the sine by K (up to ~1600) at every zero crossing, so the
// sine must be relatively accurate there, at th = 0 and th = 1/2 alike: th is
// reduced to the nearest half cycle in float64, r = th - n/2 in [-1/4, 1/4]
// (exact), and with s = sin 2 pi r, c = cos 2 pi r (hardware, ~9e-7 relative
// near 0, moving tanh(K s) by at most ~4e-7) and sigma = (-1)^n,
// sin 2 pi th = sigma s and cos 2 pi th = sigma c; tanh is odd, so the value
// is tanh(K s) (sigma + shape c).  tanh(z) = 1 - 2 / (exp(2z) + 1) from
// z2 = 2 log2(e) z saturates to +-1 through exp2 overflow or underflow
// (absolute error ~1e-7).
__device__ __forceinline__ float squaresaw_unit(double th, float K2, float shape) {
  const double n = rint(2.0 * th);
  const float r = (float)fma(-0.5, n, th);
  const float s = __builtin_amdgcn_sinf(r), c = __builtin_amdgcn_cosf(r);
  const float sigma = __uint_as_float((((uint32_t)(int)n) << 31) | 0x3F800000u);   // (-1)^n
  const float e = __builtin_amdgcn_exp2f(K2 * s);
  const float t = fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
  return t * fmaf(shape, c, sigma);
}

// expm1(x) in float64: Taylor series to x^8 for |x| <= 1/64 (relative
// truncation < 1e-19; the usual case, a pitch glide of under a semitone per
// control sample), to x^15 for |x| <= 1/4 (< 1e-19), the library routine
// otherwise.
__device__ __forceinline__ double expm1_f64(double x) {
  if (fabs(x) <= 0.015625) {
    double p = kSeriesC[kEm8];
#pragma unroll
    for (int k = kEm7; k >= kEm3; --k) p = fma(p, x, kSeriesC[k]);
    p = fma(p, x, 0.5);
    p = fma(p, x, 1.0);
    return p * x;
  }
  if (fabs(x) > 0.25) return expm1(x);
  double p = kSeriesC[kEm15];
#pragma unroll
  for (int k = kEm14; k >= kEm3; --k) p = fma(p, x, kSeriesC[k]);
  p = fma(p, x, 0.5);
  p = fma(p, x, 1.0);
  return p * x;
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

// Maps voice b's parameters into sh.v, fills the derived constants sh.d and
// the initial phase carries (LFOs and VCOs, cycles reduced mod 1).  All 64
// lanes call it; it ends with a barrier.
__device__ inline void voice_setup(const RenderArgs& a, int64_t b, VoiceShared& sh, int lane) {
  const double rc = a.rc;
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
  // phase carries in cycles, reduced mod 1 at every chunk boundary
  if (lane < 4) {
    const double ph0 = v[lane == 0 ? 34 : lane == 1 ? 42 : lane == 2 ? 70 : 73] / kTwoPi;
    sh.carry[lane] = ph0 - floor(ph0);
  }
  __syncthreads();
}

// ADSR k at control sample jd: attack rise, decay fall towards sustain,
// release fall from note-off, each ramp raised to the curve exponent alpha.
__device__ __forceinline__ double adsr_value(const double* dv, int k, double jd, double note_off) {
  const double A = dv[kEnvA + k], D = dv[kEnvD + k], R = dv[kEnvR + k];
  const double S = dv[kEnvS + k], al = dv[kEnvAlpha + k];
  const double att = ramp(jd, 0.0, A, dv[kEnvInvA + k]);
  const double dec = ramp(jd, A, D, dv[kEnvInvD + k]);
  const double rel = ramp(jd, note_off, R, dv[kEnvInvR + k]);
  return pow01(att, al) * (S + (1.0 - S) * pow01(1.0 - dec, al)) * pow01(1.0 - rel, al);
}

// The raw LFO chunk sums of control_stage (tl[0], tl[1]) alone: the rate
// ADSRs and the rate scan, with the same float64 operations.
__device__ inline void lfo_chunk_sums(const RenderArgs& a, const VoiceShared& sh, int64_t c,
                                      int lane, double* tl) {
  const double* v = sh.v;
  const double* dv = sh.d;
  const double rc = a.rc;
  const double note_off = v[1] * rc;
  const double jd = (double)(c * kSegsPerChunk + lane);
#pragma unroll 1
  for (int i = 0; i < 2; ++i) {
    const int pb = 32 + 8 * i;
    const double f = fmax(0.0, v[pb] + v[pb + 1] * adsr_value(dv, 2 + 2 * i, jd, note_off));
    const double inc = lane < kPointsPerChunk - 1 ? f / rc : 0.0;
    const double sc = wave_excl_scan(inc, lane);
    const double s62 = __shfl(sc, kSegsPerChunk);
    if (lane == 0) tl[i] = s62;
  }
}

// Control stage of chunk c (control samples j = 62c + lane): the six ADSRs
// (to envs[k * 64 + lane], float64 LDS scratch of 8 * 64 doubles), both LFOs
// after their amplitude ADSR (envs[(6 + i) * 64 + lane]), the modulation mixer
// outputs y[o] at j and yn[o] at j + 1 (held at J - 1), and per segment
// (lane < 62) the oscillator data sh.seg; advances the LFO and VCO phase
// carries to the next chunk.  All 64 lanes call it.
template <int RPS, bool CLAMP>
//   tl (optional): receives the four raw chunk sums the carries advance by
//   (LFO 1, LFO 2, VCO 1, VCO 2: the exclusive scans at lane 62), so that
//   carry' = (carry + tl) - floor(carry + tl) reproduces this chunk's update.
__device__ inline void control_stage(const RenderArgs& a, VoiceShared& sh, double* envs, int64_t c,
                                     int64_t J, int h, int lane, double y[5], double yn[5],
                                     double* tl = nullptr) {
  const double* v = sh.v;
  const double* dv = sh.d;
  const double rc = a.rc, sr = a.sr;
  const int q = a.q;
  const double qd = (double)q, hd = (double)h;
  const double note_off = v[1] * rc;
  const double midi = v[0];
  const int64_t j = c * kSegsPerChunk + lane;
  const double jd = (double)j;
  // Envelopes go through LDS (the tile is idle during the control stage), one
  // at a time, which keeps the float64 exp2/log2 chains from being interleaved.
#pragma unroll 1
  for (int k = 0; k < 6; ++k) envs[k * kWave + lane] = adsr_value(dv, k, jd, note_off);
  // LFOs (rate ADSR modulates the rate; amp ADSR is a control-rate VCA),
  // written next to the envelopes: lfo'_i at envs[(6 + i) * 64 + lane].
#pragma unroll 1
  for (int i = 0; i < 2; ++i) {
    const int pb = 32 + 8 * i;
    const double f = fmax(0.0, v[pb] + v[pb + 1] * envs[(2 + 2 * i) * kWave + lane]);
    const double inc = lane < kPointsPerChunk - 1 ? f / rc : 0.0;
    const double sc = wave_excl_scan(inc, lane);
    const double th = sh.carry[i] + sc;
    if (tl) {
      const double s62 = __shfl(sc, kSegsPerChunk);
      if (lane == 0) tl[i] = s62;
    }
    const double ph = th - floor(th);
    const double num = v[pb + 3] * ((1.0 + sin_cycles_f64(ph)) / 2.0) +
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
    const double i0 = 440.0 * exp2_f64((m0 - 69.0) * (1.0 / 12.0)) / sr;
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
    const double sc = wave_excl_scan(lane < kSegsPerChunk ? S : 0.0, lane);
    const double th = sh.carry[2 + vc] + sc;
    if (tl) {
      const double s62 = __shfl(sc, kSegsPerChunk);
      if (lane == 0) tl[2 + vc] = s62;
    }
    sh.seg[vc][kSegTheta][lane] = th - floor(th);
    sh.seg[vc][kSegInc][lane] = i0;
    sh.seg[vc][kSegRatio][lane] = rr;
    sh.seg[vc][kSegRunSum][lane] = Sh;
    sh.seg[vc][kSegRunRatio][lane] = Rh;
    const double nc = __shfl(th, kSegsPerChunk);
    __syncthreads();
    if (lane == 0) sh.carry[2 + vc] = nc - floor(nc);
  }
}

}  // namespace voice
}  // namespace synth
