// Adjoint of the Voice render: d(sum_n g(n) y(n)) / d(params), g = dL/dy given.
//
// Forward recap (per voice; q audio samples per control sample):
//   a_o(n) = (1 - t) y_o(j) + t y_o(j+1), j = n div q, t = (n mod q) / q
//   theta_v(n) = phi_v / 2pi + sum_{k<n} inc_v(k), inc_v = hz(m_v) / sr,
//   m_v = midi + tune_v + depth_v a_pitch_v
//   y = L1 sin(2 pi theta_1) a_1 + L2 x2(theta_2) a_3 + L3 noise a_4
//
// Kernel A (one wavefront per voice) recomputes the forward with the render's
// own control stage and phase recurrences and reduces, per control segment s,
//   D_v = sum dtheta_v,  C{0,1}_v = sum w{0,1} inc_v,  E{0,1}_v = sum w{0,1} inc_v P_v
// (w0 = 1 - t, w1 = t, P_v the inclusive in-segment prefix of dtheta_v), the
// VCA row sums A{0,1}_o = sum w{0,1} g L x, and the sums for the levels, the
// square-saw shape and its gain K.  With Gend_v(s) = sum of D_v over later
// segments, the upsampled pitch adjoint of segment s is
//   B{0,1}_v(s) = (Gend_v(s) + D_v(s)) C{0,1}_v(s) - E{0,1}_v(s),
// i.e. sum_k w inc Gtheta(k) with Gtheta(k) = sum_{n>k} dtheta(n): the reverse
// (suffix) scan of the phase adjoint is split into an in-segment part (here)
// and a cross-segment float64 scan (kernel B).
//
// Kernel B (one wavefront per voice) walks the control samples backward by
// chunks: segment adjoints -> dy_o(j) (transposed upsampling), modulation
// mixer, LFOs (shape weights, phase with its own suffix scan, rate clamp),
// control-rate VCAs and the six ADSRs, accumulating d(human value) per lane in
// LDS; then a fixed-order lane reduction and the curve-mapping Jacobian give
// d/d(normalised parameter).  Deterministic; no atomics.
#include <math.h>

#include "philox.h"
#include "synth_internal.h"
#include "voice_device.h"

namespace synth {
namespace {

using namespace voice;

enum {
  kRD1 = 0, kRC01, kRC11, kRE01, kRE11,           // sine VCO phase adjoint
  kRD2, kRC02, kRC12, kRE02, kRE12,               // square-saw VCO phase adjoint
  kRA01, kRA11, kRA03, kRA13, kRA04, kRA14,       // VCA rows 1, 3, 4
  kRL1, kRL2, kRL3, kRShape, kRK,                 // levels, shape, square-saw gain
  kNumRed
};

template <int RPS>
__global__ void __launch_bounds__(kWave) adjoint_audio_kernel(const RenderArgs a,
                                                              const float* __restrict__ g_audio,
                                                              double* __restrict__ red) {
  __shared__ VoiceShared sh;
  extern __shared__ __align__(16) float tile[];
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x / a.slices;
  const int slice = (int)(blockIdx.x % a.slices);
  const int q = a.q;
  const int h = q / RPS;
  const double qd = (double)q;
  const int64_t N = a.n_uniform;
  const int64_t J = (N + q - 1) / q;
  const uint64_t g = a.voice_ids ? a.voice_ids[b] : a.first_g + (uint64_t)b;
  const float* gv = g_audio + b * N;
  double* rv = red + b * J * kNumRed;
  float* tg = tile;                 // g(n) of the pass
  float* tgn = tile + kWave * h;    // g(n) * noise(n) of the pass

  voice_setup(a, b, sh, lane);
  const double* v = sh.v;
  const double rc = a.rc, sr = a.sr;
  const double note_off = v[1] * rc;
  double jsil = 0.0;
  for (int k = 0; k < 6; ++k) jsil = fmax(jsil, note_off + v[2 + 5 * k + 3] * rc);
  jsil = fmin(jsil, 9.0e15);
  const int64_t js = (int64_t)floor(jsil) + 2;
  const int64_t nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
  const int64_t c_sil = (js + kSegsPerChunk - 1) / kSegsPerChunk;
  // this workgroup's chunks (a voice may be split over several workgroups;
  // the carries at its first chunk are precomputed, or the earlier chunks
  // are walked through the control stage only)
  const int64_t c_lo = nchunks * slice / a.slices;
  const int64_t c_hi = nchunks * (slice + 1) / a.slices;

  const double midi = v[0];
  const double m_hi = fmax(0.0, midi + v[71] + fmax(0.0, v[72]));
  const double f_hi = fmin(440.0 * exp2((m_hi - 69.0) / 12.0), sr / 2.0);
  const double Kd = 12000.0 / (f_hi * log10(f_hi));
  const float shape = (float)v[74];
  const float cg = (float)(1.0 - v[74] / 2.0);
  const double shape_d = v[74], cg2pi_d = (1.0 - v[74] / 2.0) * kTwoPi, L2d = v[76];
  const double L1d_2pi = v[75] * kTwoPi;
  constexpr double kM2Log2e = -2.0 * 1.4426950408889634;   // exp(-2|z|) = 2^(kM2Log2e |z|)
  const float L1 = (float)v[75], L2 = (float)v[76], L3 = (float)v[77];
  const uint32_t glo = (uint32_t)g, ghi = (uint32_t)(g >> 32);

  int64_t c_start = 0;
  if (a.carries && c_lo > 0 && c_lo < a.carry_stride) {
    // chunk-start carries computed beforehand (as for a split render)
    if (lane < 4) sh.carry[lane] = a.carries[(b * a.carry_stride + c_lo) * 4 + lane];
    __syncthreads();
    c_start = c_lo;
  }
  for (int64_t c = c_start; c < c_hi; ++c) {
    if (c >= c_sil) {
      // exactly silent from here on: every reduction is zero (the envelopes are
      // 0 with zero derivative, so no parameter sees these samples)
      const int64_t s0 = (c > c_lo ? c : c_lo) * kSegsPerChunk;
      const int64_t s1 = c_hi * kSegsPerChunk < J ? c_hi * kSegsPerChunk : J;
      for (int64_t i = lane; i < (s1 - s0) * kNumRed; i += kWave) rv[s0 * kNumRed + i] = 0.0;
      break;
    }
    double y[5], yn[5];
    control_stage<RPS, false>(a, sh, reinterpret_cast<double*>(tile), c, J, h, lane, y, yn);
    if (c < c_lo) continue;                      // slice starts later: only carries needed
    // unscaled VCA ramps of this lane's segment
    const double a10_d = y[1], a1d_d = (yn[1] - y[1]) / qd;   // float64 ramp for the phase adjoint
    const float a10 = (float)a10_d, a1d = (float)a1d_d;
    const double a30_d = y[3], a3d_d = (yn[3] - y[3]) / qd;   // float64 ramp for the phase adjoint
    const float a30 = (float)a30_d, a3d = (float)a3d_d;
    const float a40 = (float)y[4], a4d = (float)((yn[4] - y[4]) / qd);
    __syncthreads();

    constexpr int segs_pp = kWave / RPS;
    const int nseg = (int)((J - c * kSegsPerChunk) < kSegsPerChunk ? (J - c * kSegsPerChunk)
                                                                    : kSegsPerChunk);
    const int npass = (nseg + segs_pp - 1) / segs_pp;
    for (int p = 0; p < npass; ++p) {
      // ---- load pass: g and g * noise into LDS, 4 samples per lane ----
      const int64_t pbase = (c * kSegsPerChunk + (int64_t)p * segs_pp) * q;
      int64_t cnt64 = (int64_t)((nseg - p * segs_pp) < segs_pp ? (nseg - p * segs_pp) : segs_pp) * q;
      if (cnt64 > N - pbase) cnt64 = N - pbase;
      const int cnt = (int)cnt64;
      const int tcap = kWave * h;
      const uint32_t grp0 = (uint32_t)(pbase >> 3);
      for (int base = 0; base < tcap; base += 512) {
        uint32_t w[4] = {glo, ghi, grp0 + (uint32_t)(base >> 3) + (uint32_t)lane, 1u};
        philox4x32_10(w, a.nk0, a.nk1);
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
          const int src_l = sub * 32 + (lane >> 1);
          const uint32_t w0 = __shfl(w[0], src_l), w1 = __shfl(w[1], src_l);
          const uint32_t w2 = __shfl(w[2], src_l), w3 = __shfl(w[3], src_l);
          const uint32_t wa = (lane & 1) ? w2 : w0;
          const uint32_t wb = (lane & 1) ? w3 : w1;
          const int li = base + sub * 256 + 4 * lane;
          if (li < tcap) {
            float gg[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) gg[e] = li + e < cnt ? gv[pbase + li + e] : 0.0f;
            const float n0 = ((float)(wa & 0xFFFFu) - 32767.5f) * (1.0f / 32768.0f);
            const float n1 = ((float)(wa >> 16) - 32767.5f) * (1.0f / 32768.0f);
            const float n2 = ((float)(wb & 0xFFFFu) - 32767.5f) * (1.0f / 32768.0f);
            const float n3 = ((float)(wb >> 16) - 32767.5f) * (1.0f / 32768.0f);
            *reinterpret_cast<float4*>(tg + li) = make_float4(gg[0], gg[1], gg[2], gg[3]);
            *reinterpret_cast<float4*>(tgn + li) =
                make_float4(gg[0] * n0, gg[1] * n1, gg[2] * n2, gg[3] * n3);
          }
        }
      }
      __syncthreads();
      // ---- run pass: forward recompute and per-run reductions ----
      const int ls = p * segs_pp + lane / RPS;
      const int m = lane % RPS;
      const int src = ls < kWave ? ls : kWave - 1;
      double t1 = sh.seg[0][kSegTheta][src], i1 = sh.seg[0][kSegInc][src];
      double t2 = sh.seg[1][kSegTheta][src], i2 = sh.seg[1][kSegInc][src];
      const double r1 = sh.seg[0][kSegRatio][src], r2 = sh.seg[1][kSegRatio][src];
      {
        double s1 = sh.seg[0][kSegRunSum][src], R1 = sh.seg[0][kSegRunRatio][src];
        double s2 = sh.seg[1][kSegRunSum][src], R2 = sh.seg[1][kSegRunRatio][src];
        for (int t = 0; t < m; ++t) {
          t1 += s1; s1 *= R1; i1 *= R1;
          t2 += s2; s2 *= R2; i2 *= R2;
        }
      }
      const float A10 = __shfl(a10, src), A1d = __shfl(a1d, src);
      const double A10d = __shfl(a10_d, src), A1dd = __shfl(a1d_d, src);
      const float A30 = __shfl(a30, src), A3d = __shfl(a3d, src);
      const double A30d = __shfl(a30_d, src), A3dd = __shfl(a3d_d, src);
      const float A40 = __shfl(a40, src), A4d = __shfl(a4d, src);
      double acc[kNumRed];
#pragma unroll
      for (int r = 0; r < kNumRed; ++r) acc[r] = 0.0;
      // The amplitude-side sums (VCA rows, levels, shape, K) are accumulated in
      // float32 over the run (at most q / RPS samples) and promoted once; the
      // phase-adjoint sums stay float64.
      float fa[kNumRed - kRA01];
#pragma unroll
      for (int r = 0; r < kNumRed - kRA01; ++r) fa[r] = 0.0f;
      const double inv_q = 1.0 / qd;
      double P1 = 0.0, P2 = 0.0;
      const int seg_valid = ls < nseg ? 1 : 0;
      // samples of this run that exist in the voice (the last segment may be partial)
      const int64_t run0 = (c * kSegsPerChunk + ls) * (int64_t)q + m * h;
      const int nlive = seg_valid ? (int)(N - run0 < h ? (N - run0 > 0 ? N - run0 : 0) : h) : 0;
      for (int k = 0; k < h; ++k) {
        const int ks = m * h + k;                  // sample index within the segment
        const double live = k < nlive ? 1.0 : 0.0;
        const float kf = (float)ks;
        const double wt1 = (double)ks * inv_q, wt0 = 1.0 - wt1;
        const float wt1f = (float)ks * (float)inv_q, wt0f = 1.0f - wt1f;
        const float gk = seg_valid ? tg[lane * h + k] : 0.0f;
        const float gnk = seg_valid ? tgn[lane * h + k] : 0.0f;
        const float a1 = fmaf(kf, A1d, A10), a3 = fmaf(kf, A3d, A30), a4 = fmaf(kf, A4d, A40);
        // sine VCO (its phase adjoint in float64 for the reason given below)
        const float r1f = (float)(t1 - rint(t1));
        const float x1 = __builtin_amdgcn_sinf(r1f);
        const double dth1 = (double)gk * L1d_2pi * fma((double)ks, A1dd, A10d) * cos_cycles_f64(t1);
        // square-saw VCO: T = tanh(K s), sech^2 = 4e/(1+e)^2 with e = exp(-2|K s|).
        // Its phase adjoint is a sum over the voice of terms of both signs that
        // the tanh edge scales by up to 2 pi K; for pitch parameters the sum can
        // be 1e6 times smaller than the sum of its magnitudes, so float32
        // rounding of the terms (the hardware sine and exponential, the VCA
        // ramp) would dominate it.  The term is evaluated in float64.
        double s2, c2;
        sincos_cycles_f64(t2, s2, c2);
        const double zd = Kd * s2;
        const double e = exp2_f64(kM2Log2e * fabs(zd));
        const double de = 1.0 + e;
        double ri = __builtin_amdgcn_rcp(de);
        ri = fma(fma(-de, ri, 1.0), ri, ri);
        ri = fma(fma(-de, ri, 1.0), ri, ri);
        const double Td = copysign((1.0 - e) * ri, zd);
        const double sech2 = 4.0 * e * ri * ri;
        const double Qd = fma(shape_d, c2, 1.0);
        const double gl2a3d = (double)gk * L2d * fma((double)ks, A3dd, A30d);
        const double dth2 = gl2a3d * cg2pi_d * (sech2 * Kd * c2 * Qd - Td * shape_d * s2);
        const float s2f = (float)s2, c2f = (float)c2, T = (float)Td, Q = (float)Qd;
        const float x2 = cg * T * Q;
        const float gl2a3 = gk * L2 * a3;
        // phase-adjoint reductions (float64)
        P1 += dth1;
        P2 += dth2;
        const double l1 = live * i1, l2 = live * i2;
        acc[kRC01] += wt0 * l1;
        acc[kRC11] += wt1 * l1;
        acc[kRE01] += wt0 * l1 * P1;
        acc[kRE11] += wt1 * l1 * P1;
        acc[kRC02] += wt0 * l2;
        acc[kRC12] += wt1 * l2;
        acc[kRE02] += wt0 * l2 * P2;
        acc[kRE12] += wt1 * l2 * P2;
        // VCA rows (transposed upsampling weights), levels, shape, K
        const float d1 = gk * L1 * x1, d3 = gk * L2 * x2, d4 = L3 * gnk;
        fa[kRA01 - kRA01] = fmaf(wt0f, d1, fa[kRA01 - kRA01]);
        fa[kRA11 - kRA01] = fmaf(wt1f, d1, fa[kRA11 - kRA01]);
        fa[kRA03 - kRA01] = fmaf(wt0f, d3, fa[kRA03 - kRA01]);
        fa[kRA13 - kRA01] = fmaf(wt1f, d3, fa[kRA13 - kRA01]);
        fa[kRA04 - kRA01] = fmaf(wt0f, d4, fa[kRA04 - kRA01]);
        fa[kRA14 - kRA01] = fmaf(wt1f, d4, fa[kRA14 - kRA01]);
        fa[kRL1 - kRA01] += gk * x1 * a1;
        fa[kRL2 - kRA01] += gk * x2 * a3;
        fa[kRL3 - kRA01] += gnk * a4;
        fa[kRShape - kRA01] += gl2a3 * (cg * T * c2f - 0.5f * T * Q);
        fa[kRK - kRA01] += gl2a3 * cg * (float)sech2 * s2f * Q;
        t1 += i1; i1 *= r1;
        t2 += i2; i2 *= r2;
      }
      acc[kRD1] = P1;
      acc[kRD2] = P2;
#pragma unroll
      for (int r = kRA01; r < kNumRed; ++r) acc[r] = (double)fa[r - kRA01];
      // combine the RPS runs of each segment: E += P_before * C, then sums
      if (RPS > 1) {
        const int gb = lane & ~(RPS - 1);          // first lane of this segment's group
        double pb1 = 0.0, pb2 = 0.0;
        for (int mm = 0; mm < RPS; ++mm) {
          const double d1v = __shfl(P1, gb + mm), d2v = __shfl(P2, gb + mm);
          if (mm < m) { pb1 += d1v; pb2 += d2v; }
        }
        acc[kRE01] += pb1 * acc[kRC01];
        acc[kRE11] += pb1 * acc[kRC11];
        acc[kRE02] += pb2 * acc[kRC02];
        acc[kRE12] += pb2 * acc[kRC12];
#pragma unroll
        for (int r = 0; r < kNumRed; ++r) {
          double tot = 0.0;
          for (int mm = 0; mm < RPS; ++mm) tot += __shfl(acc[r], gb + mm);
          acc[r] = tot;
        }
      }
      const int64_t sglob = c * kSegsPerChunk + ls;
      if (m == 0 && ls < nseg) {
#pragma unroll
        for (int r = 0; r < kNumRed; ++r) rv[sglob * kNumRed + r] = acc[r];
      }
      __syncthreads();
    }
  }
}

// Per-lane parameter accumulators; rows padded by one double so that the
// final per-parameter sums over lanes (lane p reads row p) hit distinct banks.
constexpr int kAccRow = kWave + 1;

// Adds x to lane's accumulator of parameter p (gradient pass only).
template <bool G>
__device__ __forceinline__ void gadd(double (*g)[kAccRow], int p, int lane, double x) {
  if constexpr (G) g[p][lane] += x;
}

// Reverse exclusive scan over lanes: sum of x over lanes l' > l.
__device__ __forceinline__ double wave_rev_excl_scan(double x, int lane) {
  double incl = x;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const double t = __shfl_down(incl, d);
    if (lane + d < kWave) incl += t;
  }
  const double ex = __shfl_down(incl, 1);
  return lane == kWave - 1 ? 0.0 : ex;
}

// float64 ADSR with the pieces its adjoint needs.
struct EnvEval {
  double att, dec, rel, Pa, Pd, Pr, M, env;
};

__device__ __forceinline__ EnvEval env_eval(const double* dv, int k, double jd, double note_off) {
  EnvEval E;
  const double A = dv[kEnvA + k], D = dv[kEnvD + k], R = dv[kEnvR + k];
  const double S = dv[kEnvS + k], al = dv[kEnvAlpha + k];
  E.att = ramp(jd, 0.0, A, dv[kEnvInvA + k]);
  E.dec = ramp(jd, A, D, dv[kEnvInvD + k]);
  E.rel = ramp(jd, note_off, R, dv[kEnvInvR + k]);
  E.Pa = pow01(E.att, al);
  E.Pd = pow01(1.0 - E.dec, al);
  E.Pr = pow01(1.0 - E.rel, al);
  E.M = S + (1.0 - S) * E.Pd;
  E.env = E.Pa * E.M * E.Pr;
  return E;
}

// d/dx x^alpha and d/dalpha x^alpha for x in (0, 1] (0 for x <= 0, as the
// oracle's masked power).
__device__ __forceinline__ void pow01_grad(double x, double al, double P, double& dx, double& dal) {
  if (x > 0.0) {
    dx = al * P / x;
    dal = P * log(x);
  } else {
    dx = 0.0;
    dal = 0.0;
  }
}

// ramp = clamp((j - s) / L, 0, 1): gradient passes inside [0, 1] (inclusive)
// for L > 0; d/ds = -1/L, d/dL = -(j - s) / L^2.
__device__ __forceinline__ bool ramp_live(double jd, double s, double L, double invL) {
  if (!(L > 0.0)) return false;
  const double r = (jd - s) * invL;
  return r >= 0.0 && r <= 1.0;
}

// Control-rate adjoint of chunk c of a voice: control samples j = 62c ..
// 62c + 61 on lanes 1..62 (lane l <-> j = 62c - 1 + l); lane 0 carries
// segment 62c - 1, whose right-end adjoint lands on lane 1.  The chunk needs
// from the others only Gend1/2 (the phase adjoints D of all later segments),
// lc (both LFO phases at control sample 62c) and, for the parameter
// adjoints, Lsuf (both LFOs' phase adjoints summed over all later control
// samples).  dph_tot receives this chunk's LFO phase-adjoint sums; with GRADS
// the chunk's parameter adjoints are added to gacc[p][lane].
template <bool GRADS>
__device__ __forceinline__ void control_chunk(const RenderArgs& a, const VoiceShared& vs,
                                              double (*gacc)[kAccRow], const double* rv, int64_t c,
                                              int64_t J, int lane, double Gend1, double Gend2,
                                              const double* lc, const double* Lsuf,
                                              double* dph_tot) {
  const double* v = vs.v;
  const double* dv = vs.d;
  const double rc = a.rc;
  const double kPitch = kLn2 / 12.0;
  const double note_off = v[1] * rc;
  const bool owned_lane = lane >= 1 && lane <= kSegsPerChunk;
  const int64_t j = c * kSegsPerChunk - 1 + lane;
  const double jd = (double)j;
  const bool inr = j >= 0 && j < J;
  const bool own = owned_lane && inr;
  double R[kNumRed];
#pragma unroll
  for (int r = 0; r < kNumRed; ++r) R[r] = inr ? rv[j * kNumRed + r] : 0.0;
  // segment phase adjoints: later segments of this chunk + those of later chunks
  const double D1 = own ? R[kRD1] : 0.0, D2 = own ? R[kRD2] : 0.0;
  const double Ge1 = Gend1 + wave_rev_excl_scan(D1, lane);
  const double Ge2 = Gend2 + wave_rev_excl_scan(D2, lane);
  // lane 0 (segment 62c - 1) needs the sum over all of this chunk's segments.
  // The shuffles run on every lane: a cross-lane read from a lane that is
  // masked off by a branch returns no data.
  const double ge1_1 = __shfl(Ge1, 1), d1_1 = __shfl(D1, 1);
  const double ge2_1 = __shfl(Ge2, 1), d2_1 = __shfl(D2, 1);
  const double G1 = lane == 0 ? ge1_1 + d1_1 : Ge1;
  const double G2 = lane == 0 ? ge2_1 + d2_1 : Ge2;
  const double B01 = (G1 + R[kRD1]) * R[kRC01] - R[kRE01];
  const double B11 = (G1 + R[kRD1]) * R[kRC11] - R[kRE11];
  const double B02 = (G2 + R[kRD2]) * R[kRC02] - R[kRE02];
  const double B12 = (G2 + R[kRD2]) * R[kRC12] - R[kRE12];
  // right-end contributions come from the previous segment (lane - 1)
  const double pB11 = __shfl_up(B11, 1), pB12 = __shfl_up(B12, 1);
  const double pA11 = __shfl_up(R[kRA11], 1), pA13 = __shfl_up(R[kRA13], 1);
  const double pA14 = __shfl_up(R[kRA14], 1);
  const bool lastj = (j == J - 1);

  // forward recompute at control sample j
  EnvEval E[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) E[k] = env_eval(dv, k, jd, note_off);
  double ph[2], shp[2][5], lfo[2], fpre[2];
  {
    // LFO phase: carry at the chunk's first owned sample + exclusive scan
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int pb = 32 + 8 * i;
      fpre[i] = v[pb] + v[pb + 1] * E[2 + 2 * i].env;
      const double inc = owned_lane ? fmax(0.0, fpre[i]) / rc : 0.0;
      double incl = inc;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const double t = __shfl_up(incl, d);
        if (lane >= d) incl += t;
      }
      const double th = lc[i] + (incl - inc);
      const double p = th - floor(th);
      ph[i] = p;
      shp[i][0] = (1.0 + sinpi(2.0 * p)) / 2.0;
      shp[i][1] = 1.0 - fabs(2.0 * p - 1.0);
      shp[i][2] = p;
      shp[i][3] = 1.0 - p;
      shp[i][4] = p < 0.5 ? 1.0 : 0.0;
      const double num = v[pb + 3] * shp[i][0] + v[pb + 4] * shp[i][1] + v[pb + 5] * shp[i][2] +
                         v[pb + 6] * shp[i][3] + v[pb + 7] * shp[i][4];
      lfo[i] = num * dv[kLfoInvW + i];
    }
  }
  const double x[4] = {E[0].env, E[1].env, lfo[0] * E[3].env, lfo[1] * E[5].env};
  double y[5];
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    const int pb = 48 + 4 * o;
    y[o] = (v[pb] * x[0] + v[pb + 1] * x[1] + v[pb + 2] * x[2] + v[pb + 3] * x[3]) *
           dv[kMixInvNorm + o];
  }
  double yn_p[2];
  {
    const double t0 = __shfl_down(y[0], 1), t2 = __shfl_down(y[2], 1);
    yn_p[0] = lastj ? y[0] : t0;
    yn_p[1] = lastj ? y[2] : t2;
  }

  // dy_o(j): transposed upsampling of the segment adjoints
  double dy[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (own) {
    const double b1 = B01 + (lane >= 1 ? pB11 : 0.0) + (lastj ? B11 : 0.0);
    const double b2 = B02 + (lane >= 1 ? pB12 : 0.0) + (lastj ? B12 : 0.0);
    dy[0] = v[69] * kPitch * b1;
    dy[2] = v[72] * kPitch * b2;
    dy[1] = R[kRA01] + pA11 + (lastj ? R[kRA11] : 0.0);
    dy[3] = R[kRA03] + pA13 + (lastj ? R[kRA13] : 0.0);
    dy[4] = R[kRA04] + pA14 + (lastj ? R[kRA14] : 0.0);
    // pitch, phase, level, shape and K contributions of segment j
    const double m1 = kPitch * (B01 + B11), m2 = kPitch * (B02 + B12);
    gadd<GRADS>(gacc, 0, lane, m1 + m2);
    gadd<GRADS>(gacc, 68, lane, m1);
    gadd<GRADS>(gacc, 71, lane, m2);
    gadd<GRADS>(gacc, 69, lane, kPitch * (y[0] * B01 + yn_p[0] * B11));
    gadd<GRADS>(gacc, 72, lane, kPitch * (y[2] * B02 + yn_p[1] * B12));
    gadd<GRADS>(gacc, 70, lane, R[kRD1] / kTwoPi);
    gadd<GRADS>(gacc, 73, lane, R[kRD2] / kTwoPi);
    gadd<GRADS>(gacc, 75, lane, R[kRL1]);
    gadd<GRADS>(gacc, 76, lane, R[kRL2]);
    gadd<GRADS>(gacc, 77, lane, R[kRL3]);
    gadd<GRADS>(gacc, 74, lane, R[kRShape]);
  }
  // the square-saw gain K = 12000 / (f_hi log10 f_hi), f_hi from the highest pitch
  const double dK = own ? R[kRK] : 0.0;
  if (dK != 0.0) {
    const double midi = v[0];
    const double mh = midi + v[71] + fmax(0.0, v[72]);
    const double m_hi = fmax(0.0, mh);
    const double fh = 440.0 * exp2((m_hi - 69.0) / 12.0);
    if (fh <= a.sr / 2.0) {
      const double Kd = 12000.0 / (fh * log10(fh));
      const double dKdf = -(Kd / fh) * (1.0 + 1.0 / log(fh));
      const double dm = dK * dKdf * fh * kPitch;
      if (mh >= 0.0) {
        gadd<GRADS>(gacc, 0, lane, dm);
        gadd<GRADS>(gacc, 71, lane, dm);
        if (v[72] >= 0.0) gadd<GRADS>(gacc, 72, lane, dm);
      }
    }
  }

  // modulation mixer: y_o = sum_i G_oi x_i / n_o, n_o = max(1, sum_i G_oi)
  double dx[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    const int pb = 48 + 4 * o;
    const double inv = dv[kMixInvNorm + o];
    const bool big = (v[pb] + v[pb + 1] + v[pb + 2] + v[pb + 3]) >= 1.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dx[i] += v[pb + i] * dy[o] * inv;
      if (own) gadd<GRADS>(gacc, pb + i, lane, dy[o] * (x[i] - (big ? y[o] : 0.0)) * inv);
    }
  }
  double denv[6] = {dx[0], dx[1], 0.0, 0.0, 0.0, 0.0};
  // LFOs
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int pb = 32 + 8 * i;
    const double dl = dx[2 + i] * E[3 + 2 * i].env;
    denv[3 + 2 * i] += dx[2 + i] * lfo[i];
    const double invW = dv[kLfoInvW + i];
    double dph = 0.0;
    if (invW > 0.0) {
      const double p = ph[i];
      const double sd = (p * 2.0 - 1.0) > 0.0 ? 1.0 : ((p * 2.0 - 1.0) < 0.0 ? -1.0 : 0.0);
      const double der = v[pb + 3] * (0.5 * kTwoPi * cospi(2.0 * p)) + v[pb + 4] * (-2.0 * sd) +
                         v[pb + 5] - v[pb + 6];
      dph = own ? dl * der * invW : 0.0;
      if (own)
#pragma unroll
        for (int k = 0; k < 5; ++k) gadd<GRADS>(gacc, pb + 3 + k, lane, dl * (shp[i][k] - lfo[i]) * invW);
    }
    // phase: d phi += dph / 2 pi; d inc(k) = sum_{j > k} dph(j)
    if (own) gadd<GRADS>(gacc, pb + 2, lane, dph / kTwoPi);
    const double later = Lsuf[i] + wave_rev_excl_scan(dph, lane);
    {
      double s = dph;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      dph_tot[i] = s;
    }
    if (own && fpre[i] >= 0.0) {
      const double df = later / rc;
      gadd<GRADS>(gacc, pb, lane, df);
      gadd<GRADS>(gacc, pb + 1, lane, df * E[2 + 2 * i].env);
      denv[2 + 2 * i] += df * v[pb + 1];
    }
  }
  // ADSRs
  if (own) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int pb = 2 + 5 * k;
      const EnvEval& e = E[k];
      const double de = denv[k];
      if (de == 0.0) continue;
      const double A = dv[kEnvA + k], D = dv[kEnvD + k], Rr = dv[kEnvR + k];
      const double Sus = dv[kEnvS + k], al = dv[kEnvAlpha + k];
      const double dPa = de * e.M * e.Pr;
      const double dM = de * e.Pa * e.Pr;
      const double dPr = de * e.Pa * e.M;
      gadd<GRADS>(gacc, pb + 2, lane, dM * (1.0 - e.Pd));
      const double dPd = dM * (1.0 - Sus);
      double gx, ga, dA = 0.0, dD = 0.0, dR = 0.0, dO = 0.0, dal = 0.0;
      pow01_grad(e.att, al, e.Pa, gx, ga);
      dal += dPa * ga;
      if (ramp_live(jd, 0.0, A, dv[kEnvInvA + k])) dA += dPa * gx * (-jd * dv[kEnvInvA + k] * dv[kEnvInvA + k]);
      pow01_grad(1.0 - e.dec, al, e.Pd, gx, ga);
      dal += dPd * ga;
      if (ramp_live(jd, A, D, dv[kEnvInvD + k])) {
        const double dd = -dPd * gx;       // d/d dec
        dA += dd * (-dv[kEnvInvD + k]);
        dD += dd * (-(jd - A) * dv[kEnvInvD + k] * dv[kEnvInvD + k]);
      }
      pow01_grad(1.0 - e.rel, al, e.Pr, gx, ga);
      dal += dPr * ga;
      if (ramp_live(jd, note_off, Rr, dv[kEnvInvR + k])) {
        const double dr = -dPr * gx;       // d/d rel
        dO += dr * (-dv[kEnvInvR + k]);
        dR += dr * (-(jd - note_off) * dv[kEnvInvR + k] * dv[kEnvInvR + k]);
      }
      gadd<GRADS>(gacc, pb + 0, lane, dA * rc);
      gadd<GRADS>(gacc, pb + 1, lane, dD * rc);
      gadd<GRADS>(gacc, pb + 3, lane, dR * rc);
      gadd<GRADS>(gacc, pb + 4, lane, dal);
      gadd<GRADS>(gacc, 1, lane, dO * rc);
    }
  }
}

// The control-rate adjoint runs chunk-parallel: one wavefront per (voice,
// chunk).  The serial dependencies between chunks (LFO phases forward, the
// phase-adjoint suffix sums backward) go through per-chunk totals stored by
// earlier passes and combined in the order a single wavefront walking the
// chunks would combine them, so every chunk sees the same inputs as in such
// a walk.
struct CtlArgs {
  double* sums;      // [batch][chunks][4]: D1, D2 over owned segments; LFO 1, 2 increments
  double* dph;       // [batch][chunks][2]: LFO 1, 2 phase-adjoint sums
  double* gpart;     // [batch][chunks][78]: parameter adjoints per chunk (human values)
  int64_t nchunks;
};

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// LFO phases at chunk c's first owned control sample and the phase-adjoint
// sums of all later chunks, from the pass-0 totals (serial order).
__device__ __forceinline__ void chunk_inputs(const VoiceShared& vs, const double* sums, int64_t c,
                                             int64_t nchunks, double* lc, double& Gend1,
                                             double& Gend2) {
  lc[0] = vs.carry[0];
  lc[1] = vs.carry[1];
  for (int64_t k = 0; k < c; ++k) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      lc[i] += sums[k * 4 + 2 + i];
      lc[i] -= floor(lc[i]);
    }
  }
  Gend1 = 0.0;
  Gend2 = 0.0;
  for (int64_t k = nchunks - 1; k > c; --k) {
    Gend1 += sums[k * 4];
    Gend2 += sums[k * 4 + 1];
  }
}

// Pass 0: per chunk, D1 and D2 summed over its owned segments and both LFO
// phase increments summed over its owned control samples.
__global__ void __launch_bounds__(kWave) adjoint_chunk_sums_kernel(const RenderArgs a,
                                                                   const double* __restrict__ red,
                                                                   CtlArgs t) {
  __shared__ VoiceShared vs;
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x / t.nchunks, c = blockIdx.x % t.nchunks;
  const int64_t J = (a.n_uniform + a.q - 1) / a.q;
  const double* rv = red + b * J * kNumRed;
  voice_setup(a, b, vs, lane);
  const double* v = vs.v;
  const double* dv = vs.d;
  const double rc = a.rc;
  const double note_off = v[1] * rc;
  const int64_t j = c * kSegsPerChunk - 1 + lane;
  const bool owned_lane = lane >= 1 && lane <= kSegsPerChunk;
  const bool own = owned_lane && j < J;            // owned lanes have j >= 0
  const double s1 = wave_sum(own ? rv[j * kNumRed + kRD1] : 0.0);
  const double s2 = wave_sum(own ? rv[j * kNumRed + kRD2] : 0.0);
  double li[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int pb = 32 + 8 * i;
    const EnvEval Er = env_eval(dv, 2 + 2 * i, (double)j, note_off);
    const double f = fmax(0.0, v[pb] + v[pb + 1] * Er.env);
    li[i] = wave_sum(own ? f / rc : 0.0);
  }
  if (lane == 0) {
    double* o = t.sums + (b * t.nchunks + c) * 4;
    o[0] = s1;
    o[1] = s2;
    o[2] = li[0];
    o[3] = li[1];
  }
}

// Pass 1: per chunk, the LFO phase-adjoint sums (they need the chunk's whole
// forward recompute and mixer adjoint, not its parameter adjoints).
__global__ void __launch_bounds__(kWave) adjoint_chunk_lfo_kernel(const RenderArgs a,
                                                                  const double* __restrict__ red,
                                                                  CtlArgs t) {
  __shared__ VoiceShared vs;
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x / t.nchunks, c = blockIdx.x % t.nchunks;
  const int64_t J = (a.n_uniform + a.q - 1) / a.q;
  voice_setup(a, b, vs, lane);
  double lc[2], G1, G2;
  chunk_inputs(vs, t.sums + b * t.nchunks * 4, c, t.nchunks, lc, G1, G2);
  const double Lsuf[2] = {0.0, 0.0};
  double tot[2];
  control_chunk<false>(a, vs, nullptr, red + b * J * kNumRed, c, J, lane, G1, G2, lc, Lsuf, tot);
  if (lane == 0) {
    t.dph[(b * t.nchunks + c) * 2] = tot[0];
    t.dph[(b * t.nchunks + c) * 2 + 1] = tot[1];
  }
}

// Pass 2: per chunk, the parameter adjoints (human values), summed over the
// lanes in lane order.
struct GradShared {
  VoiceShared vs;
  double gacc[kNumParams][kAccRow];
};

__global__ void __launch_bounds__(kWave) adjoint_chunk_grad_kernel(const RenderArgs a,
                                                                   const double* __restrict__ red,
                                                                   CtlArgs t) {
  __shared__ GradShared S;
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x / t.nchunks, c = blockIdx.x % t.nchunks;
  const int64_t J = (a.n_uniform + a.q - 1) / a.q;
  for (int p = 0; p < kNumParams; ++p) S.gacc[p][lane] = 0.0;
  voice_setup(a, b, S.vs, lane);
  double lc[2], G1, G2;
  chunk_inputs(S.vs, t.sums + b * t.nchunks * 4, c, t.nchunks, lc, G1, G2);
  double Lsuf[2] = {0.0, 0.0};
  for (int64_t k = t.nchunks - 1; k > c; --k) {
    Lsuf[0] += t.dph[(b * t.nchunks + k) * 2];
    Lsuf[1] += t.dph[(b * t.nchunks + k) * 2 + 1];
  }
  double tot[2];
  control_chunk<true>(a, S.vs, S.gacc, red + b * J * kNumRed, c, J, lane, G1, G2, lc, Lsuf, tot);
  __syncthreads();
  for (int p = lane; p < kNumParams; p += kWave) {
    double s = 0.0;
    for (int l = 0; l < kWave; ++l) s += S.gacc[p][l];
    t.gpart[(b * t.nchunks + c) * kNumParams + p] = s;
  }
}

// Pass 3: per voice, the chunks' parameter adjoints summed (last chunk
// first) and taken through the curve mapping's Jacobian to the normalised
// parameters.
__global__ void __launch_bounds__(kWave) adjoint_params_kernel(const RenderArgs a, CtlArgs t,
                                                               float* __restrict__ grad_params) {
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  for (int p = lane; p < kNumParams; p += kWave) {
    double s = 0.0;
    for (int64_t c = t.nchunks - 1; c >= 0; --c) s += t.gpart[(b * t.nchunks + c) * kNumParams + p];
    const double u = (double)a.params[b * kNumParams + p];
    const NebulaArgs& nb = a.neb;
    const double span = nb.hi[p] - nb.lo[p];
    const bool lin = bit(nb.linear, p);
    const double e = nb.inv_curve[p];
    double jac;
    if (!bit(nb.sym, p)) {
      jac = lin ? span : (u > 0.0 ? span * e * pow(u, e - 1.0) : 0.0);
    } else {
      const double d = 2.0 * u - 1.0;
      const double ad = fabs(d);
      jac = ad > 0.0 ? (lin ? span : span * e * pow(ad, e - 1.0)) : 0.0;
    }
    grad_params[b * kNumParams + p] = (float)(s * jac);
  }
}

template <int RPS>
hipError_t launch_adjoint_rps(const RenderArgs& a, const float* g, double* red, float* gp,
                              hipStream_t s) {
  size_t shmem = (size_t)2 * kWave * (a.q / RPS) * sizeof(float);
  if (shmem < 8 * kWave * sizeof(double)) shmem = 8 * kWave * sizeof(double);
  hipLaunchKernelGGL((adjoint_audio_kernel<RPS>), dim3((unsigned)(a.batch * a.slices)), dim3(kWave),
                     shmem, s, a, g, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the control-rate passes' totals follow the segment sums and the carries
  const int64_t J = (a.n_uniform + a.q - 1) / a.q;
  CtlArgs t;
  t.nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
  t.sums = red + a.batch * (J * kNumRed + t.nchunks * 4);
  t.dph = t.sums + a.batch * t.nchunks * 4;
  t.gpart = t.dph + a.batch * t.nchunks * 2;
  const dim3 chunks((unsigned)(a.batch * t.nchunks));
  hipLaunchKernelGGL(adjoint_chunk_sums_kernel, chunks, dim3(kWave), 0, s, a, red, t);
  hipLaunchKernelGGL(adjoint_chunk_lfo_kernel, chunks, dim3(kWave), 0, s, a, red, t);
  hipLaunchKernelGGL(adjoint_chunk_grad_kernel, chunks, dim3(kWave), 0, s, a, red, t);
  hipLaunchKernelGGL(adjoint_params_kernel, dim3((unsigned)a.batch), dim3(kWave), 0, s, a, t, gp);
  return hipGetLastError();
}

}  // namespace

size_t adjoint_workspace_bytes(int64_t batch, int64_t n_samples, int q) {
  // per-segment sums [batch][J][21], the chunk-start carries [batch][chunks][4],
  // then the control-rate passes' per-chunk totals [batch][chunks][4 + 2 + 78]
  const int64_t J = (n_samples + q - 1) / q;
  const int64_t nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
  return (size_t)batch * ((size_t)J * kNumRed + (size_t)nchunks * (4 + 4 + 2 + kNumParams)) *
         sizeof(double);
}

double* adjoint_carries(double* ws, int64_t batch, int64_t n_samples, int q) {
  const int64_t J = (n_samples + q - 1) / q;
  return ws + batch * J * kNumRed;
}

int64_t adjoint_max_chunks() { return 512; }

hipError_t launch_render_backward(const RenderArgs& a, const float* grad_audio, double* ws,
                                  float* grad_params, int runs_per_segment, hipStream_t s) {
  if (a.batch == 0) return hipSuccess;
  switch (runs_per_segment) {
    case 1: return launch_adjoint_rps<1>(a, grad_audio, ws, grad_params, s);
    case 2: return launch_adjoint_rps<2>(a, grad_audio, ws, grad_params, s);
    case 4: return launch_adjoint_rps<4>(a, grad_audio, ws, grad_params, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace synth
