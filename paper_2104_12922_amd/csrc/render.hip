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
//   store pass      each lane takes 8 consecutive tile samples, adds the noise
//                   oscillator (one Philox call gives 8 16-bit noise samples)
//                   through its VCA, and writes them with two 16-byte stores,
//                   so each store instruction covers 2 KB of contiguous audio.
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
__device__ __forceinline__ double pow01(double x, double e) {
  return x <= 0.0 ? 0.0 : (x >= 1.0 ? 1.0 : pow(x, e));
}

__device__ __forceinline__ double ramp(double j, double start, double len) {
  return len > 0.0 ? fmin(fmax((j - start) / len, 0.0), 1.0) : (j >= start ? 1.0 : 0.0);
}

// ADSR (attack, decay, release and note-off in control samples): product of
// the attack rise, the decay fall towards sustain and the release fall, each
// ramp raised to the curve exponent alpha.
__device__ __forceinline__ double adsr(double j, double A, double D, double S, double R,
                                       double alpha, double O) {
  const double att = ramp(j, 0.0, A);
  const double dec = ramp(j, A, D);
  const double rel = ramp(j, O, R);
  return pow01(att, alpha) * (S + (1.0 - S) * pow01(1.0 - dec, alpha)) * pow01(1.0 - rel, alpha);
}

__device__ __forceinline__ bool bit(const uint32_t* w, int p) { return (w[p >> 5] >> (p & 31)) & 1u; }

// Normalised u -> human-readable value (Section 3.3): u^(1/curve) on [min, max],
// or for symmetric parameters sign(d)|d|^(1/curve), d = 2u - 1, centred.
__device__ double map_param(double u, int p, const NebulaArgs& nb) {
  const double lo = nb.lo[p], span = nb.hi[p] - nb.lo[p];
  const bool lin = bit(nb.linear, p);
  if (!bit(nb.sym, p)) return lo + span * (lin ? u : pow01(u, nb.inv_curve[p]));
  const double d = 2.0 * u - 1.0;
  const double ad = fabs(d);
  const double w = lin ? ad : pow01(ad, nb.inv_curve[p]);
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
// sin and cos of 2*pi*th.  th (cycles, float64) is reduced to the nearest half
// cycle in float64, r = th - n/2 in [-1/4, 1/4] (exact), so sin(2 pi th) =
// (-1)^n sin(2 pi r) is evaluated with a relative (not only absolute) error of
// ~1e-7 near every zero crossing - the square-saw's tanh edge amplifies the
// sine by up to ~1600 there.  Taylor polynomials of sin x (to x^11) and cos x
// (to x^12) on |x| <= pi/2: truncation below 6e-8.
__device__ __forceinline__ void sincos_cycles(double th, float& s, float& c) {
  const double n = rint(2.0 * th);
  const float r = (float)fma(-0.5, n, th);
  const float x = r * 6.28318530717958647692f;
  const float x2 = x * x;
  float ps = fmaf(x2, -2.50521083854417187751e-8f, 2.75573192239858906526e-6f);
  ps = fmaf(x2, ps, -1.98412698412698412698e-4f);
  ps = fmaf(x2, ps, 8.33333333333333333333e-3f);
  ps = fmaf(x2, ps, -1.66666666666666666667e-1f);
  float pc = fmaf(x2, 2.08767569878680989792e-9f, -2.75573192239858906526e-7f);
  pc = fmaf(x2, pc, 2.48015873015873015873e-5f);
  pc = fmaf(x2, pc, -1.38888888888888888889e-3f);
  pc = fmaf(x2, pc, 4.16666666666666666667e-2f);
  pc = fmaf(x2, pc, -0.5f);
  const float sn = fmaf(x * x2, ps, x);
  const float cs = fmaf(x2, pc, 1.0f);
  const bool odd = ((long long)n) & 1;
  s = odd ? -sn : sn;
  c = odd ? -cs : cs;
}

__device__ __forceinline__ float sin_cycles(double th) {
  const double n = rint(2.0 * th);
  const float r = (float)fma(-0.5, n, th);
  const float x = r * 6.28318530717958647692f;
  const float x2 = x * x;
  float ps = fmaf(x2, -2.50521083854417187751e-8f, 2.75573192239858906526e-6f);
  ps = fmaf(x2, ps, -1.98412698412698412698e-4f);
  ps = fmaf(x2, ps, 8.33333333333333333333e-3f);
  ps = fmaf(x2, ps, -1.66666666666666666667e-1f);
  const float sn = fmaf(x * x2, ps, x);
  return (((long long)n) & 1) ? -sn : sn;
}

// tanh(z) = sign(z) (1 - e) / (1 + e), e = exp(-2|z|) = 2^(-2 log2(e) |z|).
__device__ __forceinline__ float tanh_f(float z) {
  const float e = __builtin_amdgcn_exp2f(-2.88539008177792681472f * fabsf(z));
  const float t = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
  return copysignf(t, z);
}

// Square-saw: (1 - s/2) tanh(K sin 2 pi th) (1 + s cos 2 pi th).
__device__ __forceinline__ float squaresaw(double th, float K, float shape, float gain) {
  float s, c;
  sincos_cycles(th, s, c);
  return gain * tanh_f(K * s) * fmaf(shape, c, 1.0f);
}

__device__ __forceinline__ void store8(float* dst, const float* o, int64_t valid, bool aligned) {
  if (valid >= 8 && aligned) {
    float4* d4 = reinterpret_cast<float4*>(dst);
    d4[0] = make_float4(o[0], o[1], o[2], o[3]);
    d4[1] = make_float4(o[4], o[5], o[6], o[7]);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (e < valid) dst[e] = o[e];
  }
}

// Zero out[z0, z1) with all 64 lanes (z0 a multiple of 8).
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

struct VoiceShared {
  double v[kNumParams];        // human-readable parameter values
  float2 namp[kWave];          // per segment of the chunk: noise VCA (start, slope) * level
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

  __syncthreads();
  for (int p = lane; p < kNumParams; p += kWave)
    sh.v[p] = map_param((double)a.params[b * kNumParams + p], p, a.neb);
  __syncthreads();
  const double* v = sh.v;

  const int64_t J = (N + q - 1) / q;     // control samples == segments
  const int64_t nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
  const int64_t c_lo = nchunks * slice / a.slices;
  const int64_t c_hi = nchunks * (slice + 1) / a.slices;

  const double rc = a.rc, sr = a.sr;
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
  const float K = (float)(12000.0 / (f_hi * log10(f_hi)));
  const float shape = (float)v[74];
  const float sq_gain = (float)(1.0 - v[74] / 2.0);
  const double L1 = v[75], L2 = v[76], L3 = v[77];

  // phase carries in cycles, reduced mod 1 at every chunk boundary
  double lfo_carry[2] = {v[34] / kTwoPi, v[42] / kTwoPi};
  double vco_carry[2] = {v[70] / kTwoPi, v[73] / kTwoPi};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    lfo_carry[i] -= floor(lfo_carry[i]);
    vco_carry[i] -= floor(vco_carry[i]);
  }

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
    double env[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int pb = 2 + 5 * k;
      env[k] = adsr(jd, v[pb] * rc, v[pb + 1] * rc, v[pb + 2], v[pb + 3] * rc, v[pb + 4], note_off);
    }
    double x[4] = {env[0], env[1], 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int pb = 32 + 8 * i;
      const double f = fmax(0.0, v[pb] + v[pb + 1] * env[2 + 2 * i]);
      const double inc = lane < kPointsPerChunk - 1 ? f / rc : 0.0;
      const double th = lfo_carry[i] + wave_excl_scan(inc, lane);
      const double ph = th - floor(th);
      const double w0 = v[pb + 3], w1 = v[pb + 4], w2 = v[pb + 5], w3 = v[pb + 6], w4 = v[pb + 7];
      const double wsum = w0 + w1 + w2 + w3 + w4;
      const double num = w0 * ((1.0 + sin(kTwoPi * ph)) / 2.0) + w1 * (1.0 - fabs(2.0 * ph - 1.0)) +
                         w2 * ph + w3 * (1.0 - ph) + w4 * (ph < 0.5 ? 1.0 : 0.0);
      const double l = wsum > 0.0 ? num / wsum : 0.0;
      x[2 + i] = l * env[3 + 2 * i];                 // control-rate VCA (amp ADSR)
      const double nc = __shfl(th, kSegsPerChunk);   // phase at the next chunk's first point
      lfo_carry[i] = nc - floor(nc);
    }
    double y[5], yn[5];
    const bool last = (j + 1 >= J);                  // right end held at the last control sample
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const int pb = 48 + 4 * o;
      const double gs = v[pb] + v[pb + 1] + v[pb + 2] + v[pb + 3];
      const double acc = v[pb] * x[0] + v[pb + 1] * x[1] + v[pb + 2] * x[2] + v[pb + 3] * x[3];
      y[o] = acc / fmax(1.0, gs);
    }
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      const double t = __shfl_down(y[o], 1);
      yn[o] = last ? y[o] : t;
    }
    // per segment (lane < 62): pitch glide, phase advance, VCA ramps
    double thS[2], inc0[2], rr[2], Sh[2], Rh[2];
#pragma unroll
    for (int vc = 0; vc < 2; ++vc) {
      const int tb = vc ? 71 : 68;
      const int yo = vc ? 2 : 0;
      const double base = midi + v[tb];
      const double m0 = base + v[tb + 1] * y[yo];
      const double m1 = base + v[tb + 1] * yn[yo];
      const double i0 = 440.0 * exp2((m0 - 69.0) / 12.0) / sr;
      const double Lr = (m1 - m0) * (kLn2 / (12.0 * qd));   // log of the per-sample ratio
      const double e1 = expm1(Lr);
      const double eh = expm1(Lr * hd);
      inc0[vc] = i0;
      rr[vc] = 1.0 + e1;
      Rh[vc] = 1.0 + eh;
      Sh[vc] = (e1 == 0.0) ? i0 * hd : i0 * (eh / e1);
      double S;
      if constexpr (CLAMP) {
        // some increments may exceed 1/2 cycle (f > sr/2): sum them one by one
        S = 0.0;
        double inc = i0;
        for (int k = 0; k < q; ++k) {
          S += fmin(inc, 0.5);
          inc *= rr[vc];
        }
      } else {
        S = Sh[vc];
        double t = Sh[vc];
#pragma unroll
        for (int m = 1; m < RPS; ++m) {
          t *= Rh[vc];
          S += t;
        }
      }
      const double th = vco_carry[vc] + wave_excl_scan(lane < kSegsPerChunk ? S : 0.0, lane);
      thS[vc] = th - floor(th);
      const double nc = __shfl(th, kSegsPerChunk);
      vco_carry[vc] = nc - floor(nc);
    }
    if (c < c_lo) continue;                      // slice starts later: only carries needed

    const float a10 = (float)(L1 * y[1]), a1d = (float)(L1 * (yn[1] - y[1]) / qd);
    const float a20 = (float)(L2 * y[3]), a2d = (float)(L2 * (yn[3] - y[3]) / qd);
    __syncthreads();                             // previous chunk's readers of namp are done
    if (lane < kSegsPerChunk)
      sh.namp[lane] = make_float2((float)(L3 * y[4]), (float)(L3 * (yn[4] - y[4]) / qd));
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
      double t1 = __shfl(thS[0], src), i1 = __shfl(inc0[0], src), r1 = __shfl(rr[0], src);
      double t2 = __shfl(thS[1], src), i2 = __shfl(inc0[1], src), r2 = __shfl(rr[1], src);
      const float A10 = __shfl(a10, src), A1d = __shfl(a1d, src);
      const float A20 = __shfl(a20, src), A2d = __shfl(a2d, src);
      if constexpr (CLAMP) {
        for (int k = 0; k < m * h; ++k) {
          t1 += fmin(i1, 0.5); i1 *= r1;
          t2 += fmin(i2, 0.5); i2 *= r2;
        }
      } else {
        double s1 = __shfl(Sh[0], src), R1 = __shfl(Rh[0], src);
        double s2 = __shfl(Sh[1], src), R2 = __shfl(Rh[1], src);
        for (int t = 0; t < m; ++t) {
          t1 += s1; s1 *= R1; i1 *= R1;
          t2 += s2; s2 *= R2; i2 *= R2;
        }
      }
      float kf = (float)(m * h);
      float* trow = tile + lane * h;
      for (int k = 0; k < h; ++k) {
        const float x1 = sin_cycles(t1);
        const float x2 = squaresaw(t2, K, shape, sq_gain);
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
      const int64_t pbase = (c * kSegsPerChunk + (int64_t)p * segs_pp) * q;
      int64_t cnt = (int64_t)((nseg - p * segs_pp) < segs_pp ? (nseg - p * segs_pp) : segs_pp) * q;
      if (cnt > N - pbase) cnt = N - pbase;
      const int ngroups = (int)((cnt + 7) / 8);
      for (int gi = lane; gi < ngroups; gi += kWave) {
        const int64_t n = pbase + 8 * (int64_t)gi;
        uint32_t w[4] = {(uint32_t)g, (uint32_t)(g >> 32), (uint32_t)(n >> 3), 1u};
        philox4x32_10(w, a.nk0, a.nk1);
        const int cl = p * segs_pp * q + 8 * gi;     // chunk-local sample
        int sg = cl / q;
        int kk = cl - sg * q;
        float2 na = sh.namp[sg];
        float o[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (kk == q) {
            kk = 0;
            ++sg;
            na = sh.namp[sg < kWave ? sg : kWave - 1];
          }
          const uint32_t hw = (w[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
          const float x3 = ((float)hw - 32767.5f) * (1.0f / 32768.0f);
          const float an = fmaf((float)kk, na.y, na.x);
          o[e] = fmaf(an, x3, tile[8 * gi + e]);
          ++kk;
        }
        store8(out + n, o, cnt - 8 * (int64_t)gi, aligned);
      }
      __syncthreads();
    }
  }
}

template <int RPS, bool CLAMP>
__global__ void __launch_bounds__(kWave) render_kernel(const RenderArgs a) {
  __shared__ VoiceShared sh;
  extern __shared__ float tile[];
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
  const size_t shmem = (size_t)kWave * (a.q / RPS) * sizeof(float);
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
