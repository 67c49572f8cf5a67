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
#include "voice_device.h"

namespace synth {
namespace {

using namespace voice;

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

// Four consecutive samples li .. li + 3 of a pass (one segment): tile value
// plus noise through the noise VCA.  wa, wb: the Philox words of the samples
// (16-bit halves, low half first); x = (h + 0.5) / 32768 - 1 with the 2^-15
// folded into the ramp namp (per segment of the pass: value at the segment's
// first sample and slope).  The segment index li / q is formed in float32:
// (li + 1/2) / q lies at least 1/(2q) from an integer and li < 64 q, so the
// truncation is exact.
__device__ __forceinline__ void noise_vca4(float* o, uint32_t wa, uint32_t wb, float4 t, int li,
                                           int q, float inv_qf, const float2* namp) {
  const int lsg = (int)fmaf((float)li, inv_qf, 0.5f * inv_qf);
  const float2 na = namp[lsg];
  const float a0 = fmaf((float)(li - __mul24(lsg, q)), na.y, na.x);
  o[0] = fmaf((float)(wa & 0xFFFFu) - 32767.5f, a0, t.x);
  o[1] = fmaf((float)(wa >> 16) - 32767.5f, fmaf(1.0f, na.y, a0), t.y);
  o[2] = fmaf((float)(wb & 0xFFFFu) - 32767.5f, fmaf(2.0f, na.y, a0), t.z);
  o[3] = fmaf((float)(wb >> 16) - 32767.5f, fmaf(3.0f, na.y, a0), t.w);
}

// Noise group gi of a pass: samples 8 gi .. 8 gi + 7 (pass-local; the pass
// starts at a multiple of 8 samples), one Philox call whose four words hold
// their 16-bit noise in sample order, added through the noise VCA to the tile
// values and written to out[8 gi ..] (VEC: two 16-byte stores, the group
// whole and out 16-byte aligned; else element by element below cnt).  The
// tile holds a multiple of 8 floats >= cnt, so its reads stay inside it.
template <bool VEC>
__device__ __forceinline__ void noise_group(float* out, const float* tile, int gi, int cnt,
                                            uint32_t glo, uint32_t ghi, uint32_t grp0, uint32_t k0,
                                            uint32_t k1, int q, float inv_qf, const float2* namp) {
  const int li = 8 * gi;
  uint32_t w[4] = {glo, ghi, grp0 + (uint32_t)gi, 1u};
  philox4x32_10(w, k0, k1);
  const float4 ta = *reinterpret_cast<const float4*>(tile + li);
  const float4 tb = *reinterpret_cast<const float4*>(tile + li + 4);
  float o[8];
  noise_vca4(o, w[0], w[1], ta, li, q, inv_qf, namp);
  noise_vca4(o + 4, w[2], w[3], tb, li + 4, q, inv_qf, namp);
  float* dst = out + li;
  if constexpr (VEC) {
    *reinterpret_cast<float4*>(dst) = make_float4(o[0], o[1], o[2], o[3]);
    *reinterpret_cast<float4*>(dst + 4) = make_float4(o[4], o[5], o[6], o[7]);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (li + e < cnt) dst[e] = o[e];
  }
}

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
    packed_range(a.offsets, a.batch, b, off0, N);
  } else {
    off0 = b * a.n_uniform;
    N = a.n_uniform;
  }
  if (N <= 0) return;
  const uint64_t g = a.voice_ids ? a.voice_ids[b] : a.first_g + (uint64_t)b;
  float* out = a.audio + off0;
  const bool aligned = (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
  const double rc = a.rc, sr = a.sr;

  voice_setup(a, b, sh, lane);
  const double* v = sh.v;
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

  const uint32_t glo = (uint32_t)g, ghi = (uint32_t)(g >> 32);
  const float inv_qf = 1.0f / (float)q;

  int64_t c_start = 0;
  if (a.carries && c_lo > 0 && c_lo < a.carry_stride) {
    // the carries at chunk c_lo were computed beforehand: no walk over the
    // earlier chunks' control stages (a voice longer than the carries cover
    // walks as before)
    if (lane < 4) sh.carry[lane] = a.carries[(b * a.carry_stride + c_lo) * 4 + lane];
    __syncthreads();
    c_start = c_lo;
  }
  for (int64_t c = c_start; c < c_hi; ++c) {
    if (c >= c_sil) {
      const int64_t z0 = (c > c_lo ? c : c_lo) * (int64_t)kSegsPerChunk * q;
      const int64_t z1 = c_hi * (int64_t)kSegsPerChunk * q < N ? c_hi * (int64_t)kSegsPerChunk * q : N;
      zero_fill(out, z0, z1, lane, aligned);
      break;
    }
    // ---------------- control stage: lane = control sample j ----------------
    double y[5], yn[5];
    control_stage<RPS, CLAMP>(a, sh, reinterpret_cast<double*>(tile), c, J, h, lane, y, yn);
    if (c < c_lo) continue;                      // slice starts later: only carries needed

    const float a10 = (float)(L1 * y[1]), a1d = (float)(L1 * (yn[1] - y[1]) / qd);
    // VCO 2's VCA ramp carries the square-saw gain (1 - shape / 2)
    const float a20 = (float)(L2 * y[3]) * sq_gain;
    const float a2d = (float)(L2 * (yn[3] - y[3]) / qd) * sq_gain;
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
      t1 -= rint(t1);                            // exact; see sin_cycles_run
      // VCA ramps at the run's first sample, then advanced by their slopes
      // (float32; 25 additions move them by about 1e-6 relative)
      const float kf0 = (float)(m * h);
      float A1 = fmaf(kf0, A1d, A10);
      float A2 = fmaf(kf0, A2d, A20);
      float* trow = tile + lane * h;
      // Consume the LDS and cross-lane loads here, so that the loop below
      // carries no wait on them (its own LDS stores are never waited for).
      asm volatile("" ::"v"(t1), "v"(i1), "v"(t2), "v"(i2), "v"(r1), "v"(r2));
      asm volatile("" ::"v"(A1), "v"(A1d), "v"(A2), "v"(A2d));
#pragma unroll 5
      for (int k = 0; k < h; ++k) {
        const float x1 = sin_cycles_run(t1);
        const float x2 = squaresaw_unit(t2, K2, shape);   // gain (1 - s/2) is in A2
        trow[k] = fmaf(A2, x2, A1 * x1);
        if constexpr (CLAMP) {
          t1 += fmin(i1, 0.5); t2 += fmin(i2, 0.5);
        } else {
          t1 += i1; t2 += i2;
        }
        i1 *= r1;
        i2 *= r2;
        A1 += A1d;
        A2 += A2d;
      }
      __syncthreads();
      // Store pass: noise + VCA.  Lane l takes noise groups gi = l, l + 64, ...
      // of the pass: one Philox call gives the 16-bit noise of samples 8 gi ..
      // 8 gi + 7 in its four words, in sample order, so no lane needs another's
      // words; the lane adds them through the noise VCA to its 8 tile samples
      // and writes them with two 16-byte stores.  The pass starts at a sample
      // that is a multiple of 8 (16, 32 or 64 segments of q = 4k samples), and
      // 4 samples never straddle a segment because q is a multiple of 4.
      const int64_t pbase = (c * kSegsPerChunk + (int64_t)p * segs_pp) * q;
      int64_t cnt64 = (int64_t)((nseg - p * segs_pp) < segs_pp ? (nseg - p * segs_pp) : segs_pp) * q;
      if (cnt64 > N - pbase) cnt64 = N - pbase;
      const int cnt = (int)cnt64;
      const uint32_t grp0 = (uint32_t)(pbase >> 3);
      const int seg0 = p * segs_pp;
      // whole groups with vector stores (no branch in the loop body), then
      // the last partial group, or every group of an unaligned voice, element
      // by element
      const int full = aligned ? (cnt & ~7) : 0;
      for (int gi = lane; 8 * gi < full; gi += kWave)
        noise_group<true>(out + pbase, tile, gi, cnt, glo, ghi, grp0, a.nk0, a.nk1, q, inv_qf,
                          sh.namp + seg0);
      for (int gi = (full >> 3) + lane; 8 * gi < cnt; gi += kWave)
        noise_group<false>(out + pbase, tile, gi, cnt, glo, ghi, grp0, a.nk0, a.nk1, q, inv_qf,
                           sh.namp + seg0);
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
  {
    const int64_t k = item / a.slices;
    const int64_t b = a.order ? (int64_t)a.order[k] : k;
    if (b >= 0 && b < a.batch) render_item<RPS, CLAMP>(a, b, (int)(item % a.slices), sh, tile);
  }
}

// Chunk-start carries for launches that split voices over workgroups: the
// LFO and VCO phases the control stage carries from chunk to chunk, at the
// start of every chunk, without walking the chunks one after another.  Each
// chunk's raw sums come from its own control stage (one wavefront per chunk
// and voice); one wavefront per voice then applies the updates
// carry' = (carry + t) - floor(carry + t) in chunk order, the same float64
// operations the walk performs, so a split render is bit-identical to an
// unsplit one.  Pass 0 takes the LFO sums (the LFO rates depend on envelopes
// only: just those envelopes are evaluated), pass 1 the VCO sums given the
// LFO carries.
template <int RPS, bool CLAMP, int PASS>
__global__ void __launch_bounds__(kWave) carry_sums_kernel(const RenderArgs a, double* carries,
                                                           int64_t stride) {
  __shared__ VoiceShared sh;
  __shared__ double envs[8 * kWave];
  const int lane = threadIdx.x;
  const int64_t c = blockIdx.x, b = blockIdx.y;
  int64_t off0 = 0, N = a.n_uniform;
  if (a.offsets) packed_range(a.offsets, a.batch, b, off0, N);
  const int64_t J = (N + a.q - 1) / a.q;
  const int64_t nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
  if (N <= 0 || c >= nchunks) return;
  voice_setup(a, b, sh, lane);
  double* cr = carries + (b * stride + c) * 4;
  if (PASS == 1 && lane < 2) sh.carry[lane] = cr[lane];
  __syncthreads();
  double y[5], yn[5], tl[4];
  if (PASS == 0)
    lfo_chunk_sums(a, sh, c, lane, tl);
  else
    control_stage<RPS, CLAMP>(a, sh, envs, c, J, a.q / RPS, lane, y, yn, tl);
  if (lane == 0) {
    cr[2 * PASS] = tl[2 * PASS];
    cr[2 * PASS + 1] = tl[2 * PASS + 1];
  }
}

template <int PASS>
__global__ void __launch_bounds__(kWave) carry_scan_kernel(const RenderArgs a, double* carries,
                                                           int64_t stride) {
  __shared__ VoiceShared sh;
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  int64_t off0 = 0, N = a.n_uniform;
  if (a.offsets) packed_range(a.offsets, a.batch, b, off0, N);
  const int64_t J = (N + a.q - 1) / a.q;
  const int64_t nchunks = (J + kSegsPerChunk - 1) / kSegsPerChunk;
  if (N <= 0) return;
  voice_setup(a, b, sh, lane);
  if (lane < 2) {
    const int k = 2 * PASS + lane;
    double cy = sh.carry[k];
    const int64_t nc_max = nchunks < stride ? nchunks : stride;
    for (int64_t c = 0; c < nc_max; ++c) {
      double* cr = carries + (b * stride + c) * 4;
      const double t = cr[k];
      cr[k] = cy;
      const double nc = cy + t;
      cy = nc - floor(nc);
    }
  }
}

// Mix mode 1: y <- y / max(1, max |y|) per voice.  One 256-thread workgroup per voice.
__global__ void __launch_bounds__(256) peak_normalise_kernel(const RenderArgs a) {
  __shared__ float red[256];
  const int64_t b = blockIdx.x;
  int64_t off0, N;
  if (a.offsets) {
    packed_range(a.offsets, a.batch, b, off0, N);
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

template <int RPS, bool CLAMP>
hipError_t carries_rps(const RenderArgs& a, double* carries, int64_t stride, hipStream_t s) {
  const dim3 grid((unsigned)stride, (unsigned)a.batch);
  hipLaunchKernelGGL((carry_sums_kernel<RPS, CLAMP, 0>), grid, dim3(kWave), 0, s, a, carries, stride);
  hipLaunchKernelGGL((carry_scan_kernel<0>), dim3((unsigned)a.batch), dim3(kWave), 0, s, a, carries,
                     stride);
  hipLaunchKernelGGL((carry_sums_kernel<RPS, CLAMP, 1>), grid, dim3(kWave), 0, s, a, carries, stride);
  hipLaunchKernelGGL((carry_scan_kernel<1>), dim3((unsigned)a.batch), dim3(kWave), 0, s, a, carries,
                     stride);
  return hipGetLastError();
}

template <int RPS>
hipError_t carries_clamp(const RenderArgs& a, bool clamp, double* carries, int64_t stride,
                         hipStream_t s) {
  return clamp ? carries_rps<RPS, true>(a, carries, stride, s)
               : carries_rps<RPS, false>(a, carries, stride, s);
}

hipError_t launch_voice_carries(const RenderArgs& a, int runs_per_segment, bool clamp,
                                double* carries, int64_t stride, hipStream_t s) {
  if (a.batch == 0 || stride == 0) return hipSuccess;
  if (a.batch > 65535 || stride > 0x7FFFFFFF) return hipErrorInvalidValue;
  switch (runs_per_segment) {
    case 1: return carries_clamp<1>(a, clamp, carries, stride, s);
    case 2: return carries_clamp<2>(a, clamp, carries, stride, s);
    case 4: return carries_clamp<4>(a, clamp, carries, stride, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_peak_normalise(const RenderArgs& a, hipStream_t s) {
  if (a.batch == 0) return hipSuccess;
  hipLaunchKernelGGL(peak_normalise_kernel, dim3((unsigned)a.batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace synth
