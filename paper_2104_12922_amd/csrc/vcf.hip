// Resonant low-pass filter module and its adjoint: the subtractive filter
// Section 7 lists as a module to add.  Per voice, control period j (samples
// [j q, (j + 1) q)) has the cutoff
//   f_j = clamp(440 * 2^((cutoff + depth * env[j] - 69) / 12), 10 Hz, 0.45 sr)
// and the second-order low-pass section of R. Bristow-Johnson's "Audio EQ
// Cookbook" at f_j and the voice's Q (c = cos w, s = sin w, w = 2 pi f / sr,
// alpha = s / (2 Q)):
//   b0 = b2 = (1 - c) / 2 / (1 + alpha), b1 = (1 - c) / (1 + alpha),
//   a1 = -2 c / (1 + alpha), a2 = (1 - alpha) / (1 + alpha),
// run as the direct-form-I recurrence
//   y[n] = b0 x[n] + b1 x[n-1] + b2 x[n-2] - a1 y[n-1] - a2 y[n-2]
// from a zero state, coefficients switched at period boundaries.
//
// The recurrence is linear in the state v[n] = (y[n-1], y[n-2]): a run of L
// samples with constant coefficients maps v to A^L v + z, A = [[-a1, -a2],
// [1, 0]], z its zero-state response.  Each period is cut into S lane
// segments of h = q / S samples (S = 4 or 2 when that leaves h >= 32), and
// one wavefront takes one voice, 64 segments (a chunk) at a time: the
// chunk's samples are staged in LDS as they lie in HBM by direct
// global-to-LDS loads (segment s at s h: an even h gives the lanes' sweep
// reads bank conflicts, 2-way for h = 50, cheaper than a padded layout's
// index arithmetic), lane s
// runs segment s from a zero state (z) and raises A to its length by
// squaring, an inclusive scan of the affine maps (M, z) over the lanes gives
// every segment's entry state from the chunk's, and each lane runs its
// segment again from that state, writing y over x in LDS; the chunk is then
// stored with coalesced writes.  Small chunks keep the LDS per workgroup
// small, so that several wavefronts share a SIMD and hide the sequential
// sweeps' latency.  State and coefficients are float64; samples are float32
// in HBM, read and written once each (8 bytes per sample).
//
// The adjoint: with lambda[n] = dL/dy[n] (through all later samples),
//   lambda[n] = g[n] - a1(n+1) lambda[n+1] - a2(n+2) lambda[n+2],
//   dL/dx[m]  = b0(m) lambda[m] + b1(m+1) lambda[m+1] + b2(m+2) lambda[m+2],
//   dL/db_k(j) = sum_{n in j} lambda[n] x[n-k], dL/da_k(j) = -sum_{n in j} lambda[n] y[n-k],
// (coef(m): the coefficient of the period holding sample m), then through
// the cookbook formulas to w and Q, and through f to the cutoff, the depth
// and env[j].  It walks the chunks last to first; per chunk it recomputes
// the forward entry states from the chunk-start state the forward pass saved
// (same scan as the forward), runs the lambda recurrence backward per lane
// from a zero state, scans the lanes' affine maps in reverse, runs lambda
// again from the true entry states (lambda over g in LDS), then a forward
// sweep per period rebuilds y, sums the coefficient gradients and forms
// dL/dx over x in LDS.
#include <type_traits>

#include "voice_device.h"

namespace synth {
namespace {

using voice::kLn2;
using voice::kTwoPi;
using voice::sincos_cycles_f64;

constexpr double kVcfFMin = 10.0;
constexpr double kVcfFMaxFrac = 0.45;

// Lane segments per control period: each lane takes a quarter (or half)
// period when that leaves at least 32 samples, so a chunk of 64 segments is
// small in LDS and more wavefronts share a CU, while the per-segment work
// (coefficients, the matrix power, the lane scan) stays small per sample.
// Segments hold at least 4 samples (the period is at least 4).
int vcf_segments(int q) {
  if (q % 4 == 0 && q / 4 >= 32) return 4;
  if (q % 2 == 0 && q / 2 >= 32) return 2;
  return 1;
}

struct VcfArgs {
  const float* x;
  const float* g;            // backward: dL/dy
  const int64_t* offsets;    // [B + 1] or null
  int64_t n_uniform;
  int64_t batch;
  const float* env;          // [B][env_ld]
  int64_t env_ld;
  const float* params;       // [B][3]: cutoff (MIDI note), depth (semitones), Q
  int q;                     // samples per control period
  int S;                     // lane segments per period (1, 2 or 4)
  int h;                     // samples per lane segment, q / S (>= 4)
  double sr;
  float* y;                  // forward output / backward dL/dx
  double* states;            // [B][state_ld][2]: (y[c0 - 1], y[c0 - 2]) at chunk starts
  int64_t state_ld;
  float* g_params;           // backward: [B][3]
  float* g_env;              // backward: [B][env_ld] or null
  const int32_t* order;      // null, or the voices in the order workgroups take them
};

struct Coef {
  double b0, b1, a1, a2;     // b2 = b0
};

struct CoefGrad {
  Coef k;
  double dw[4];              // d(b0, b1, a1, a2) / dw
  double dq[4];              // d(b0, b1, a1, a2) / dQ
  double dmdw;               // dw / dm (m: cutoff + depth env), 0 when clamped
};

// 2^y in float64 without a table lookup (the filter's cutoff is formed once
// per lane segment, after a load of its control value; a second, dependent
// load would double the latency): y = n + r with n = rint(y), |r| <= 1/2, and
// 2^r = exp(z), z = r ln 2, |z| <= 0.347, by its Taylor series to degree 13
// (truncation below 5e-18 relative).  y is clamped to [-1100, 1023].
__device__ __forceinline__ double exp2_series_f64(double y) {
  y = fmin(fmax(y, -1100.0), 1023.0);
  const double n = rint(y);
  const double z = (y - n) * kLn2;
  double p = 1.0 / 6227020800.0;                   // 1 / 13!
  p = fma(p, z, 1.0 / 479001600.0);
  p = fma(p, z, 1.0 / 39916800.0);
  p = fma(p, z, 1.0 / 3628800.0);
  p = fma(p, z, 1.0 / 362880.0);
  p = fma(p, z, 1.0 / 40320.0);
  p = fma(p, z, 1.0 / 5040.0);
  p = fma(p, z, 1.0 / 720.0);
  p = fma(p, z, 1.0 / 120.0);
  p = fma(p, z, 1.0 / 24.0);
  p = fma(p, z, 1.0 / 6.0);
  p = fma(p, z, 0.5);
  p = fma(p, z, 1.0);
  p = fma(p, z, 1.0);
  return ldexp(p, (int)n);
}

__device__ __forceinline__ double vcf_cutoff(double m, double sr, bool& live) {
  const double f = 440.0 * exp2_series_f64((m - 69.0) / 12.0);
  live = f >= kVcfFMin && f <= kVcfFMaxFrac * sr;
  return fmin(fmax(f, kVcfFMin), kVcfFMaxFrac * sr);
}

__device__ __forceinline__ Coef vcf_coef(const VcfArgs& a, double cutoff, double depth, double Q,
                                         double env) {
  bool live;
  const double f = vcf_cutoff(fma(depth, env, cutoff), a.sr, live);
  double s, c;
  sincos_cycles_f64(f / a.sr, s, c);
  const double alpha = s / (2.0 * Q);
  const double ia0 = 1.0 / (1.0 + alpha);
  Coef k;
  k.b0 = (1.0 - c) * 0.5 * ia0;
  k.b1 = (1.0 - c) * ia0;
  k.a1 = -2.0 * c * ia0;
  k.a2 = (1.0 - alpha) * ia0;
  return k;
}

__device__ __forceinline__ CoefGrad vcf_coef_grad(const VcfArgs& a, double cutoff, double depth,
                                                  double Q, double env) {
  bool live;
  const double f = vcf_cutoff(fma(depth, env, cutoff), a.sr, live);
  double s, c;
  sincos_cycles_f64(f / a.sr, s, c);
  const double alpha = s / (2.0 * Q);
  const double ia0 = 1.0 / (1.0 + alpha);
  CoefGrad r;
  r.k.b0 = (1.0 - c) * 0.5 * ia0;
  r.k.b1 = (1.0 - c) * ia0;
  r.k.a1 = -2.0 * c * ia0;
  r.k.a2 = (1.0 - alpha) * ia0;
  const double dal_w = c / (2.0 * Q), dal_q = -alpha / Q;
  // coefficient = N / (1 + alpha): d = (dN - coefficient * dalpha) / (1 + alpha)
  r.dw[0] = (0.5 * s - r.k.b0 * dal_w) * ia0;
  r.dw[1] = (s - r.k.b1 * dal_w) * ia0;
  r.dw[2] = (2.0 * s - r.k.a1 * dal_w) * ia0;
  r.dw[3] = -(1.0 + r.k.a2) * dal_w * ia0;
  r.dq[0] = -r.k.b0 * dal_q * ia0;
  r.dq[1] = -r.k.b1 * dal_q * ia0;
  r.dq[2] = -r.k.a1 * dal_q * ia0;
  r.dq[3] = -(1.0 + r.k.a2) * dal_q * ia0;
  // w = 2 pi f / sr, f = 440 2^((m - 69) / 12): dw/dm = w ln 2 / 12
  r.dmdw = live ? kTwoPi * f / a.sr * (kLn2 / 12.0) : 0.0;
  return r;
}

struct Mat2 {
  double m00, m01, m10, m11;
};

__device__ __forceinline__ Mat2 mat_mul(const Mat2& p, const Mat2& r) {   // p r
  Mat2 o;
  o.m00 = fma(p.m00, r.m00, p.m01 * r.m10);
  o.m01 = fma(p.m00, r.m01, p.m01 * r.m11);
  o.m10 = fma(p.m10, r.m00, p.m11 * r.m10);
  o.m11 = fma(p.m10, r.m01, p.m11 * r.m11);
  return o;
}

__device__ __forceinline__ Mat2 mat_pow(Mat2 p, int e) {
  Mat2 r = {1.0, 0.0, 0.0, 1.0};
  while (e > 0) {
    if (e & 1) r = mat_mul(r, p);
    e >>= 1;
    if (e) p = mat_mul(p, p);
  }
  return r;
}

__device__ __forceinline__ void voice_range(const VcfArgs& a, int64_t b, int64_t& start,
                                            int64_t& len) {
  if (a.offsets) {
    packed_range(a.offsets, a.batch, b, start, len);
  } else {
    start = b * a.n_uniform;
    len = a.n_uniform;
  }
}

// Stage samples [c0, c0 + cnt) of src (voice base pointer) into LDS
// (chunk-relative sample p at lds[p]) with direct global-to-LDS loads: each
// wave instruction moves 64 consecutive 16-byte groups (1 KB; 4-byte words
// when the voice's samples are not 16-byte aligned or cnt is not a multiple
// of 4) into LDS without passing through registers, so the whole chunk is in
// flight at once.  Addresses are clamped into [0, cnt): positions past cnt
// hold copies of earlier samples, which no sweep uses.  The loads complete
// asynchronously: stage_wait() must run before the LDS is read.
__device__ __forceinline__ void lds_dma(const float* src, float* dst, int bytes) {
  auto* d = (__attribute__((address_space(3))) void*)dst;
  if (bytes == 16)
    __builtin_amdgcn_global_load_lds(src, d, 16, 0, 0);
  else
    __builtin_amdgcn_global_load_lds(src, d, 4, 0, 0);
}

__device__ __forceinline__ void stage_in(float* lds, const float* __restrict__ src, int64_t c0,
                                         int cnt, const VcfArgs& a, bool vec) {
  const int lane = threadIdx.x, span = 64 * a.h;            // LDS floats of a chunk
  const float* base = src + c0;
  if (vec && (cnt & 3) == 0) {
    const int full = span / 256;                              // groups of 64 x 16 bytes
#pragma unroll 4
    for (int k = 0; k < full; ++k) lds_dma(base + min(256 * k + 4 * lane, cnt - 4), lds + 256 * k, 16);
    const int p = 256 * full + 4 * lane;
    if (p < span) lds_dma(base + min(p, cnt - 4), lds + 256 * full, 16);
  } else {
    for (int k = 0; 64 * k < span; ++k)
      lds_dma(base + min(64 * k + lane, cnt - 1), lds + 64 * k, 4);
  }
}

// Waits for this wave's outstanding global loads, the staging ones included
// (s_waitcnt vmcnt(0); the other counters left free).
__device__ __forceinline__ void stage_wait() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Store samples [c0, c0 + cnt) of the chunk in LDS to dst (voice base
// pointer): lane l takes 16-byte groups l, l + 64, ...; with 16-byte aligned
// samples and cnt a multiple of 4, batches of four groups' LDS reads are
// issued before their stores, else 4-byte stores.
constexpr int kOutBatch = 4;

__device__ __forceinline__ void stage_out(const float* lds, float* __restrict__ dst, int64_t c0,
                                          int cnt, bool vec) {
  const int lane = threadIdx.x;
  float* base = dst + c0;
  if (vec && (cnt & 3) == 0) {
    int p0 = 0;
    for (; p0 + 256 * kOutBatch <= cnt; p0 += 256 * kOutBatch) {
      float4 v[kOutBatch];
#pragma unroll
      for (int k = 0; k < kOutBatch; ++k)
        v[k] = *reinterpret_cast<const float4*>(lds + p0 + 256 * k + 4 * lane);
#pragma unroll
      for (int k = 0; k < kOutBatch; ++k)
        *reinterpret_cast<float4*>(base + p0 + 256 * k + 4 * lane) = v[k];
    }
    for (int p = p0 + 4 * lane; p < cnt; p += 256)
      *reinterpret_cast<float4*>(base + p) = *reinterpret_cast<const float4*>(lds + p);
    return;
  }
  for (int p = 4 * lane; p < cnt; p += 256) {
    const float4 v = *reinterpret_cast<const float4*>(lds + p);
    base[p] = v.x;
    if (p + 1 < cnt) base[p + 1] = v.y;
    if (p + 2 < cnt) base[p + 2] = v.z;
    if (p + 3 < cnt) base[p + 3] = v.w;
  }
}

// Inclusive scan over lanes of the affine maps v -> M v + z, earlier lanes
// applied first (dir = +1: lane - d is earlier; dir = -1: lane + d is).
template <int DIR>
__device__ __forceinline__ void scan_affine(Mat2& M, double& z0, double& z1) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    Mat2 P;
    double p0, p1;
    if (DIR > 0) {
      P.m00 = __shfl_up(M.m00, d); P.m01 = __shfl_up(M.m01, d);
      P.m10 = __shfl_up(M.m10, d); P.m11 = __shfl_up(M.m11, d);
      p0 = __shfl_up(z0, d); p1 = __shfl_up(z1, d);
    } else {
      P.m00 = __shfl_down(M.m00, d); P.m01 = __shfl_down(M.m01, d);
      P.m10 = __shfl_down(M.m10, d); P.m11 = __shfl_down(M.m11, d);
      p0 = __shfl_down(z0, d); p1 = __shfl_down(z1, d);
    }
    const bool has = DIR > 0 ? lane >= d : lane + d < 64;
    if (has) {
      const double n0 = fma(M.m00, p0, fma(M.m01, p1, z0));
      const double n1 = fma(M.m10, p0, fma(M.m11, p1, z1));
      M = mat_mul(M, P);
      z0 = n0;
      z1 = n1;
    }
  }
}

// Walks a lane's segment in LDS: f(i, x[i]) for i = 0 .. len - 1 in order
// (sweep) or len - 1 .. 0 (sweep_rev), the next block of eight LDS reads in
// flight while the current block runs.  The block reads are unconditional:
// they may run up to eight floats past either end of the segment, which the
// LDS pads (kLdsPad floats before and after the staged samples) keep inside
// the allocation; values read past the segment are never used.  f may write
// x[i] (in place).
constexpr int kSweep = 8;
constexpr int kLdsPad = 8;

template <class F>
__device__ __forceinline__ void sweep(const float* xs, int len, F&& f) {
  const int full = len & ~(kSweep - 1);
  float cur[kSweep], nxt[kSweep];
#pragma unroll
  for (int e = 0; e < kSweep; ++e) cur[e] = xs[e];
  for (int i = 0; i < full; i += kSweep) {
#pragma unroll
    for (int e = 0; e < kSweep; ++e) nxt[e] = xs[i + kSweep + e];
#pragma unroll
    for (int e = 0; e < kSweep; ++e) f(i + e, cur[e]);
#pragma unroll
    for (int e = 0; e < kSweep; ++e) cur[e] = nxt[e];
  }
  for (int i = full; i < len; ++i) f(i, xs[i]);
}

template <class F>
__device__ __forceinline__ void sweep_rev(const float* xs, int len, F&& f) {
  const int full = len & ~(kSweep - 1);
  for (int i = len - 1; i >= full; --i) f(i, xs[i]);
  float cur[kSweep], nxt[kSweep];
#pragma unroll
  for (int e = 0; e < kSweep; ++e) cur[e] = xs[full - kSweep + e];
  for (int i = full - kSweep; i >= 0; i -= kSweep) {
#pragma unroll
    for (int e = 0; e < kSweep; ++e) nxt[e] = xs[i - kSweep + e];
#pragma unroll
    for (int e = kSweep - 1; e >= 0; --e) f(i + e, cur[e]);
#pragma unroll
    for (int e = 0; e < kSweep; ++e) cur[e] = nxt[e];
  }
}

template <class F>
__device__ __forceinline__ void sweep2(const float* xs, const float* gs, int len, F&& f) {
  const int full = len & ~(kSweep - 1);
  float cx[kSweep], cg[kSweep], nx[kSweep], ng[kSweep];
#pragma unroll
  for (int e = 0; e < kSweep; ++e) {
    cx[e] = xs[e];
    cg[e] = gs[e];
  }
  for (int i = 0; i < full; i += kSweep) {
#pragma unroll
    for (int e = 0; e < kSweep; ++e) {
      nx[e] = xs[i + kSweep + e];
      ng[e] = gs[i + kSweep + e];
    }
#pragma unroll
    for (int e = 0; e < kSweep; ++e) f(i + e, cx[e], cg[e]);
#pragma unroll
    for (int e = 0; e < kSweep; ++e) {
      cx[e] = nx[e];
      cg[e] = ng[e];
    }
  }
  for (int i = full; i < len; ++i) f(i, xs[i], gs[i]);
}

// Forward recompute of one chunk: each active lane's entry state (y[s-1],
// y[s-2]) from the chunk-start state (v0, v1); returns the chunk's exit
// state via (e0, e1) (uniform).  xa: staged x; xh1, xh2: x[c0-1], x[c0-2].
__device__ __forceinline__ void forward_entry_states(const float* xa, const VcfArgs& a,
                                                     const Coef& k, int len, double xh1, double xh2,
                                                     double v0, double v1, double& in0,
                                                     double& in1, double& e0, double& e1) {
  const int lane = threadIdx.x;
  const float* xs = xa + lane * a.h;
  double x1 = lane ? (double)xa[lane * a.h - 1] : xh1;
  double x2 = lane ? (double)xa[lane * a.h - 2] : xh2;
  double y1 = 0.0, y2 = 0.0;
  sweep(xs, len, [&](int, float xf) {
    const double x0 = (double)xf;
    const double ff = fma(k.b0, x0 + x2, k.b1 * x1);
    const double y0 = fma(-k.a1, y1, fma(-k.a2, y2, ff));
    x2 = x1; x1 = x0; y2 = y1; y1 = y0;
  });
  Mat2 M = {1.0, 0.0, 0.0, 1.0};
  double z0 = 0.0, z1 = 0.0;
  if (len > 0) {
    const Mat2 A = {-k.a1, -k.a2, 1.0, 0.0};
    M = mat_pow(A, len);
    z0 = y1;
    z1 = y2;
  }
  scan_affine<1>(M, z0, z1);
  const double o0 = fma(M.m00, v0, fma(M.m01, v1, z0));
  const double o1 = fma(M.m10, v0, fma(M.m11, v1, z1));
  in0 = __shfl_up(o0, 1);
  in1 = __shfl_up(o1, 1);
  if (lane == 0) {
    in0 = v0;
    in1 = v1;
  }
  e0 = __shfl(o0, 63);
  e1 = __shfl(o1, 63);
}

__global__ void __launch_bounds__(64) vcf_forward_kernel(VcfArgs a) {
  extern __shared__ float lds_raw[];          // pad, 64 h, pad, 64 control values
  float* lds = lds_raw + kLdsPad;
  const int64_t b = a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
  if (b < 0 || b >= a.batch) return;         // an order entry out of range renders nothing
  const int lane = threadIdx.x;
  int64_t start, L;
  voice_range(a, b, start, L);
  if (L <= 0) return;
  const float* xv = a.x + start;
  float* yv = a.y + start;
  const bool vec = ((reinterpret_cast<uintptr_t>(xv) | reinterpret_cast<uintptr_t>(yv)) & 15) == 0;
  const double cutoff = a.params[b * 3], depth = a.params[b * 3 + 1], Q = a.params[b * 3 + 2];
  const int64_t J = (L + a.h - 1) / a.h;          // lane segments of the voice
  const int64_t chunks = (J + 63) / 64;
  // control values of chunk c's lane segments into lds_env[lane] (loaded
  // with the chunk's samples, so the coefficients wait for no other load)
  float* lds_env = lds + 64 * a.h + kLdsPad;
  auto stage_env = [&](int64_t c) {
    const int64_t j = min(c * 64 + lane, J - 1);
    lds_dma(a.env + b * a.env_ld + j / a.S, lds_env, 4);
  };
  // Per chunk: wait for its samples and control values, form the
  // coefficients, run the chunk, store it, and start the next chunk's loads.
  double v0 = 0.0, v1 = 0.0, xh1 = 0.0, xh2 = 0.0;
  stage_env(0);
  stage_in(lds, xv, 0, (int)min((int64_t)64 * a.h, L), a, vec);
  for (int64_t c = 0; c < chunks; ++c) {
    const int64_t c0 = c * 64 * a.h;
    const int cnt = (int)min((int64_t)64 * a.h, L - c0);
    if (a.states && lane == 0) {
      a.states[(b * a.state_ld + c) * 2] = v0;
      a.states[(b * a.state_ld + c) * 2 + 1] = v1;
    }
    const int64_t j = c * 64 + lane;
    const int len = j < J ? (int)min((int64_t)a.h, L - j * a.h) : 0;
    stage_wait();
    __syncthreads();
    Coef k = {0.0, 0.0, 0.0, 0.0};
    if (len > 0) k = vcf_coef(a, cutoff, depth, Q, (double)lds_env[lane]);
    double in0, in1, e0, e1;
    forward_entry_states(lds, a, k, len, xh1, xh2, v0, v1, in0, in1, e0, e1);
    // x history for this lane's segment and for the next chunk, read before
    // any lane overwrites its segment with y
    float* xs = lds + lane * a.h;
    double x1 = lane ? (double)lds[lane * a.h - 1] : xh1;
    double x2 = lane ? (double)lds[lane * a.h - 2] : xh2;
    const double nxh1 = (double)lds[64 * a.h - 1];
    const double nxh2 = (double)lds[64 * a.h - 2];
    __syncthreads();
    double y1 = in0, y2 = in1;
    sweep(xs, len, [&](int i, float xf) {
      const double x0 = (double)xf;
      const double ff = fma(k.b0, x0 + x2, k.b1 * x1);
      const double y0 = fma(-k.a1, y1, fma(-k.a2, y2, ff));
      xs[i] = (float)y0;
      x2 = x1; x1 = x0; y2 = y1; y1 = y0;
    });
    __syncthreads();
    stage_out(lds, yv, c0, cnt, vec);
    __syncthreads();
    if (c + 1 < chunks) {
      stage_env(c + 1);
      stage_in(lds, xv, c0 + 64 * a.h, (int)min((int64_t)64 * a.h, L - c0 - 64 * a.h), a, vec);
    }
    v0 = e0;
    v1 = e1;
    xh1 = nxh1;
    xh2 = nxh2;
  }
}

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) vcf_backward_kernel(VcfArgs a) {
  extern __shared__ float lds_raw[];          // pad, x then dL/dx, pad, pad, g then lambda, pad
  float* xa = lds_raw + kLdsPad;
  float* ga = xa + 64 * a.h + 2 * kLdsPad;
  const int64_t b = a.order ? (int64_t)a.order[blockIdx.x] : (int64_t)blockIdx.x;
  if (b < 0 || b >= a.batch) return;         // an order entry out of range renders nothing
  const int lane = threadIdx.x;
  int64_t start, L;
  voice_range(a, b, start, L);
  if (L <= 0) {
    if (lane < 3) a.g_params[b * 3 + lane] = 0.0f;
    return;
  }
  const float* xv = a.x + start;
  const float* gv = a.g + start;
  float* dxv = a.y + start;
  const bool vec = ((reinterpret_cast<uintptr_t>(xv) | reinterpret_cast<uintptr_t>(gv) |
                     reinterpret_cast<uintptr_t>(dxv)) & 15) == 0;
  const double cutoff = a.params[b * 3], depth = a.params[b * 3 + 1], Q = a.params[b * 3 + 2];
  const int64_t J = (L + a.h - 1) / a.h;      // lane segments of the voice
  const int64_t chunks = (J + 63) / 64;
  // What a chunk needs from HBM besides its samples: the forward state at
  // its start, x[c0 - 1], x[c0 - 2], and the coefficients (with their
  // derivatives) of lane segment 64 c + lane and of the segment after it
  // (lane 63: the first of the next chunk; zero past the voice, where lambda
  // is 0).
  struct ChunkIn {
    double v0, v1, xh1, xh2, envj;
    CoefGrad kg;
    Coef kn;
  };
  auto chunk_in = [&](int64_t c) {
    ChunkIn r;
    const int64_t c0 = c * 64 * a.h;
    r.v0 = a.states[(b * a.state_ld + c) * 2];
    r.v1 = a.states[(b * a.state_ld + c) * 2 + 1];
    r.xh1 = c0 >= 1 ? (double)xv[c0 - 1] : 0.0;
    r.xh2 = c0 >= 2 ? (double)xv[c0 - 2] : 0.0;
    const int64_t j = c * 64 + lane;
    r.envj = j < J ? (double)a.env[b * a.env_ld + j / a.S] : 0.0;
    r.kg = {};
    if (j < J) r.kg = vcf_coef_grad(a, cutoff, depth, Q, r.envj);
    r.kn.b0 = __shfl_down(r.kg.k.b0, 1);
    r.kn.b1 = __shfl_down(r.kg.k.b1, 1);
    r.kn.a1 = __shfl_down(r.kg.k.a1, 1);
    r.kn.a2 = __shfl_down(r.kg.k.a2, 1);
    if (lane == 63) {
      r.kn = {0.0, 0.0, 0.0, 0.0};
      if (j + 1 < J) r.kn = vcf_coef(a, cutoff, depth, Q, (double)a.env[b * a.env_ld + (j + 1) / a.S]);
    }
    return r;
  };
  auto stage_chunk = [&](int64_t c) {
    const int64_t c0 = c * 64 * a.h;
    const int cnt = (int)min((int64_t)64 * a.h, L - c0);
    stage_in(xa, xv, c0, cnt, a, vec);
    stage_in(ga, gv, c0, cnt, a, vec);
  };
  // Per chunk (last to first): wait for its samples, run it, gather the
  // previous chunk's inputs (their loads then wait for no store), store
  // dL/dx, and start the previous chunk's sample loads.
  double u0 = 0.0, u1 = 0.0;                  // (lambda[c_end], lambda[c_end + 1])
  double gc = 0.0, gd = 0.0, gq = 0.0;        // this lane's share of dL/d(cutoff, depth, Q)
  ChunkIn in = chunk_in(chunks - 1);
  stage_chunk(chunks - 1);
  for (int64_t c = chunks - 1; c >= 0; --c) {
    const int64_t c0 = c * 64 * a.h;
    const int cnt = (int)min((int64_t)64 * a.h, L - c0);
    const double v0 = in.v0, v1 = in.v1, xh1 = in.xh1, xh2 = in.xh2, envj = in.envj;
    const CoefGrad kg = in.kg;
    const Coef k = kg.k, kn = in.kn;
    const int64_t j = c * 64 + lane;
    const int len = j < J ? (int)min((int64_t)a.h, L - j * a.h) : 0;
    stage_wait();
    __syncthreads();
    // forward entry states (y[s-1], y[s-2]) of every period
    double fin0, fin1, fe0, fe1;
    forward_entry_states(xa, a, k, len, xh1, xh2, v0, v1, fin0, fin1, fe0, fe1);
    // lambda over the segment, samples last to first, from the state (l1,
    // l2) = (lambda[e], lambda[e+1]) after it: the last sample takes the
    // next segment's a1 and a2, the one before it the next segment's a2, the
    // rest this segment's; with `store`, lambda is written over g.
    float* gs = ga + lane * a.h;
    auto lambda_run = [&](double& l1, double& l2, auto store) {
      int n = len;
      if (n >= 1) {
        const double l0 = fma(-kn.a1, l1, fma(-kn.a2, l2, (double)gs[n - 1]));
        if (store) gs[n - 1] = (float)l0;
        l2 = l1;
        l1 = l0;
        --n;
      }
      if (n >= 1) {
        const double l0 = fma(-k.a1, l1, fma(-kn.a2, l2, (double)gs[n - 1]));
        if (store) gs[n - 1] = (float)l0;
        l2 = l1;
        l1 = l0;
        --n;
      }
      sweep_rev(gs, n, [&](int i, float gf) {
        const double l0 = fma(-k.a1, l1, fma(-k.a2, l2, (double)gf));
        if (store) gs[i] = (float)l0;
        l2 = l1;
        l1 = l0;
      });
    };
    // from a zero state: the segment's affine map (lambda[e], lambda[e+1])
    // -> (lambda[s], lambda[s+1])
    double l1 = 0.0, l2 = 0.0;
    lambda_run(l1, l2, std::false_type{});
    Mat2 M = {1.0, 0.0, 0.0, 1.0};
    double z0 = 0.0, z1 = 0.0;
    if (len > 0) {
      M = {-kn.a1, -kn.a2, 1.0, 0.0};
      if (len >= 2) {
        const Mat2 C2 = {-k.a1, -kn.a2, 1.0, 0.0};
        M = mat_mul(C2, M);
        if (len >= 3) {
          const Mat2 Bm = {-k.a1, -k.a2, 1.0, 0.0};
          M = mat_mul(mat_pow(Bm, len - 2), M);
        }
      }
      z0 = l1;
      z1 = l2;
    }
    scan_affine<-1>(M, z0, z1);
    const double o0 = fma(M.m00, u0, fma(M.m01, u1, z0));
    const double o1 = fma(M.m10, u0, fma(M.m11, u1, z1));
    double in0 = __shfl_down(o0, 1), in1 = __shfl_down(o1, 1);   // (lambda[e], lambda[e+1])
    if (lane == 63) {
      in0 = u0;
      in1 = u1;
    }
    const double nu0 = __shfl(o0, 0), nu1 = __shfl(o1, 0);
    // lambda from the true entry state, written over g
    l1 = in0;
    l2 = in1;
    lambda_run(l1, l2, std::true_type{});
    // x history of this period, read before any lane writes dL/dx over x
    double x1 = lane ? (double)xa[lane * a.h - 1] : xh1;
    double x2 = lane ? (double)xa[lane * a.h - 2] : xh2;
    __syncthreads();
    // forward sweep: y rebuilt from the entry state, the coefficient
    // gradients, and dL/dx[n - 2] once lambda[n] is known
    float* xs = xa + lane * a.h;
    double y1 = fin0, y2 = fin1;
    double lm1 = 0.0, lm2 = 0.0;               // lambda[n-1], lambda[n-2]
    // sums of lambda[n] (x[n] + x[n-2]) (b0 = b2), lambda[n] x[n-1],
    // lambda[n] y[n-1], lambda[n] y[n-2]
    double Gb02 = 0.0, Gb1 = 0.0, Ga1 = 0.0, Ga2 = 0.0;
    auto fwd_step = [&](int i, float xf, float lf, auto write) {
      const double x0 = (double)xf;
      const double l0 = (double)lf;
      const double x02 = x0 + x2;
      Gb02 = fma(l0, x02, Gb02);
      Gb1 = fma(l0, x1, Gb1);
      Ga1 = fma(l0, y1, Ga1);
      Ga2 = fma(l0, y2, Ga2);
      const double y0 = fma(-k.a1, y1, fma(-k.a2, y2, fma(k.b0, x02, k.b1 * x1)));
      if (write) xs[i - 2] = (float)fma(k.b0, lm2 + l0, k.b1 * lm1);
      x2 = x1; x1 = x0; y2 = y1; y1 = y0;
      lm2 = lm1; lm1 = l0;
    };
    // the first two samples complete no dL/dx of this segment
    if (len >= 1) fwd_step(0, xs[0], gs[0], std::false_type{});
    if (len >= 2) fwd_step(1, xs[1], gs[1], std::false_type{});
    if (len > 2)
      sweep2(xs + 2, gs + 2, len - 2, [&](int i, float xf, float lf) {
        fwd_step(i + 2, xf, lf, std::true_type{});
      });
    if (len >= 2) xs[len - 2] = (float)fma(k.b0, lm2, fma(k.b1, lm1, kn.b0 * in0));
    if (len >= 1) xs[len - 1] = (float)fma(k.b0, lm1, fma(kn.b1, in0, kn.b0 * in1));
    double gm = 0.0;
    if (len > 0) {
      const double Gw = Gb02 * kg.dw[0] + Gb1 * kg.dw[1] - Ga1 * kg.dw[2] - Ga2 * kg.dw[3];
      const double Gq = Gb02 * kg.dq[0] + Gb1 * kg.dq[1] - Ga1 * kg.dq[2] - Ga2 * kg.dq[3];
      gm = Gw * kg.dmdw;
      gc += gm;
      gd = fma(gm, envj, gd);
      gq += Gq;
    }
    // dL/denv[period]: the S lane segments of a period are adjacent lanes
    for (int off = 1; off < a.S; off <<= 1) gm += __shfl_xor(gm, off);
    if (c > 0) in = chunk_in(c - 1);
    if (a.g_env && len > 0 && (lane & (a.S - 1)) == 0)
      a.g_env[b * a.env_ld + j / a.S] = (float)(gm * depth);
    __syncthreads();
    stage_out(xa, dxv, c0, cnt, vec);
    __syncthreads();
    if (c > 0) stage_chunk(c - 1);
    u0 = nu0;
    u1 = nu1;
  }
  // per-voice sums over lanes in a fixed order
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    gc += __shfl_down(gc, off);
    gd += __shfl_down(gd, off);
    gq += __shfl_down(gq, off);
  }
  if (lane == 0) {
    a.g_params[b * 3] = (float)gc;
    a.g_params[b * 3 + 1] = (float)gd;
    a.g_params[b * 3 + 2] = (float)gq;
  }
}

VcfArgs make_args(const float* x, const float* g, const int64_t* offsets, int64_t batch,
                  int64_t n_samples, const float* env, int64_t env_ld, const float* params,
                  int q, double sr, float* y, double* states, int64_t state_ld, float* g_params,
                  float* g_env, const int32_t* order) {
  VcfArgs a;
  a.x = x;
  a.g = g;
  a.offsets = offsets;
  a.n_uniform = offsets ? 0 : n_samples;
  a.batch = batch;
  a.env = env;
  a.env_ld = env_ld;
  a.params = params;
  a.q = q;
  a.S = vcf_segments(q);
  a.h = q / a.S;
  a.sr = sr;
  a.y = y;
  a.states = states;
  a.state_ld = state_ld;
  a.g_params = g_params;
  a.g_env = g_env;
  a.order = order;
  return a;
}

}  // namespace

int64_t vcf_chunks(int64_t max_samples, int q) {
  const int h = q / vcf_segments(q);
  const int64_t J = (max_samples + h - 1) / h;
  return (J + 63) / 64;
}

hipError_t launch_vcf_forward(const float* x, const int64_t* offsets, int64_t batch,
                              int64_t n_samples, const float* env, int64_t env_ld,
                              const float* params, int q, double sr, float* y, double* states,
                              int64_t state_ld, const int32_t* order, hipStream_t s) {
  const VcfArgs a = make_args(x, nullptr, offsets, batch, n_samples, env, env_ld, params, q, sr, y,
                              states, state_ld, nullptr, nullptr, order);
  const size_t lds = (size_t)(64 * a.h + 2 * kLdsPad + 64) * sizeof(float);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)vcf_forward_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(vcf_forward_kernel, dim3((unsigned)batch), dim3(64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_vcf_backward(const float* x, const float* g, const int64_t* offsets,
                               int64_t batch, int64_t n_samples, const float* env, int64_t env_ld,
                               const float* params, int q, double sr, const double* states,
                               int64_t state_ld, float* g_x, float* g_params, float* g_env,
                               const int32_t* order, hipStream_t s) {
  const VcfArgs a = make_args(x, g, offsets, batch, n_samples, env, env_ld, params, q, sr, g_x,
                              const_cast<double*>(states), state_ld, g_params, g_env, order);
  const size_t lds = (size_t)2 * (64 * a.h + 2 * kLdsPad) * sizeof(float);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)vcf_backward_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(vcf_backward_kernel, dim3((unsigned)batch), dim3(64), lds, s, a);
  return hipGetLastError();
}

}  // namespace synth
