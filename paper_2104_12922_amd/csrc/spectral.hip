// Multi-resolution log-magnitude STFT L1 loss and its gradient (float32 FFT).
//
// The paper scores sounds with a multi-scale spectrogram distance over several
// FFT sizes and prefers L1 (Section 4, distance evaluation).  Per voice:
//   loss = sum over n in (512, 1024, 2048), hop n/4, of
//          mean_{frame t, bin k <= n/2} |log(|X_tk| + 1e-5) - log(|T_tk| + 1e-5)|
// with X, T the periodic-Hann STFTs (no padding) of the render x and target.
//
// Frames are independent jobs.  Kernel 1 (grid = voices x frame chunks of
// every resolution) takes 16 frames of one resolution per workgroup of four
// wavefronts; wavefront w takes frames f0 + 4 i + w.  A real frame of n
// samples is transformed as a complex sequence of n/2 points (even samples
// real, odd imaginary) by a wave-level Stockham FFT, then split into the
// n/2 + 1 bins of the real spectrum.  Render and target frames get separate
// FFTs (a shared complex FFT would leak the louder signal's rounding noise
// into the quieter one's spectrum).  For the gradient,
// G_k = sign(d_k) X_k / (|X_k| (|X_k| + eps)) / (F (n/2 + 1)) is extended to a
// Hermitian spectrum H (H_0 = 2 Re G_0, H_{n/2} = 2 Re G_{n/2}), inverted by
// the same half-size complex FFT, and the frame's gradient 0.5 w(m) h(m) is
// overlap-added, four frames at a time in frame order, into the workgroup's
// segment of 19 hops.  Kernel 2 adds, for every sample, the (at most two)
// segments that cover it per resolution in a fixed order, and sums the
// per-workgroup loss partials in a fixed order: bitwise deterministic, no
// atomics.
#include <math.h>

#include "synth_internal.h"
#include "wave_fft.h"

namespace synth {
namespace {

constexpr int kMrWaves = 4;
constexpr int kMrThreads = 64 * kMrWaves;
constexpr int kFramesPerBlock = 16;
// A workgroup's frames f0 .. f0 + 15 cover hops f0 .. f0 + 18 of the voice:
// their gradient rows are overlap-added in LDS into one segment of 19 hops.
constexpr int kSegHops = kFramesPerBlock + 3;
constexpr float kEps = 1e-5f;

struct MrArgs {
  const float* x;
  const float* t;
  int64_t n;                   // samples per voice
  int64_t batch;
  int F[3];                    // frames per resolution
  int chunk_base[4];           // first block index of each resolution's chunks
  int64_t wbase[3];            // workspace float offset of each resolution's segments
  double scale[3];             // 1 / (F (n/2 + 1))
  float* wgrad;                // per-workgroup gradient segments (null: loss only)
  double* partial;             // [batch][chunk_base[3]] loss partial sums
  float* grad;                 // output gradient (null: loss only)
  double* loss;
  float* tlog;                 // target log2(|T| + eps) per frame and bin (MODE 1 writes, 2 reads)
  int64_t tbase[3];            // float offset of each resolution's rows in tlog
};

// LDS of one resolution (Nc = n / 2 complex points per transform).
template <int Nc>
struct MrShared {
  static constexpr int ola_slots = 4 * Nc;   // >= the 7 hops of four frames
  float2 buf[kMrWaves][Nc];    // one FFT buffer per wavefront
  alignas(8) float win[2 * Nc];  // periodic Hann window
  float2 rs[Nc / 2 + 1];       // exp(-2 pi i k / n), k <= n / 4 (real split)
  float2 pt[wfft::pt_size<Nc>()];   // FFT pass twiddles
  float ola[ola_slots];        // overlap-add accumulator
  double red[kMrWaves];
};

// Bins k and Nc - k (k < Nc / 2) of the real spectrum of a frame whose
// half-size complex FFT Z is in buf: X_k = E + W O, X_{Nc-k} = conj(E - W O)
// with E = (Z_k + conj Z_{Nc-k}) / 2, O = -i (Z_k - conj Z_{Nc-k}) / 2,
// W = exp(-2 pi i k / n).  k = Nc / 2 gives X_{Nc/2} in the first output.
template <int Nc>
__device__ __forceinline__ void real_pair(const float2* buf, const float2* rs, int k, float2& Xk,
                                          float2& Xm) {
  const float2 zk = buf[wfft::swz<Nc>(k)];
  const float2 zc = buf[wfft::swz<Nc>((Nc - k) & (Nc - 1))];
  const float2 E = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y - zc.y));
  const float2 O = make_float2(0.5f * (zk.y + zc.y), -0.5f * (zk.x - zc.x));
  const float2 WO = wfft::cmul(rs[k], O);
  Xk = wfft::add(E, WO);
  const float2 D = wfft::sub(E, WO);
  Xm = make_float2(D.x, -D.y);
}

// |X| of a bin without underflow (hardware sqrt, about 1 ulp).  Squaring the
// components underflows for |X| below about 1e-19 (quiet release tails reach
// that), which would drop the bin's magnitude to 0 and its gradient, whose
// size 1 / (|X| + eps) is largest there, with it: a bin below 2^-50 is
// scaled by 2^100 (exact) first.  Xs and as are the scaled bin and magnitude
// (unscaled for the other bins); the result is |X|.
__device__ __forceinline__ float bin_mag(float2 X, float2& Xs, float& as) {
  const bool tiny = fmaxf(fabsf(X.x), fabsf(X.y)) < 0x1p-50f;
  const float s = tiny ? 0x1p100f : 1.0f;
  Xs = make_float2(X.x * s, X.y * s);
  as = __builtin_amdgcn_sqrtf(Xs.x * Xs.x + Xs.y * Xs.y);
  return tiny ? as * 0x1p-100f : as;
}

// log2(|T| + eps) of a target bin (hardware log2, about 1 ulp).
__device__ __forceinline__ float target_log(float2 T) {
  float2 Ts;
  float as;
  return __builtin_amdgcn_logf(bin_mag(T, Ts, as) + kEps);
}

// One bin's loss share (added to acc) and gradient spectrum value, from the
// render bin X and the target's lt = target_log(T).
__device__ __forceinline__ float2 bin_grad(float2 X, float lt, double scale_d, float scale,
                                           bool edge, bool want_grad, double& acc) {
  // hardware log2 and reciprocal (about 1 ulp each); G = sign(d) scale
  // X / (|X| (|X| + eps)) = sign(d) scale Xs / (as (|X| + eps)), whose
  // denominator stays a normal float32 for every bin
  float2 Xs;
  float as;
  const float ax = bin_mag(X, Xs, as);
  const float d = 0.69314718055994531f * (__builtin_amdgcn_logf(ax + kEps) - lt);
  acc += scale_d * (double)fabsf(d);
  float2 G = make_float2(0.f, 0.f);
  if (want_grad && as > 0.0f && d != 0.0f) {
    const float gm = copysignf(scale, d) * __builtin_amdgcn_rcpf((ax + kEps) * as);
    G = make_float2(gm * Xs.x, gm * Xs.y);
  }
  if (edge) G = make_float2(2.0f * G.x, 0.0f);
  return G;
}

// MODE 0: loss (and gradient) from render and target frames; MODE 1: only
// the target's log magnitudes, written to a.tlog (no loss); MODE 2: loss
// (and gradient) with the target's log magnitudes read from a.tlog.
template <int RES, int MODE>
__device__ __forceinline__ void mrstft_frames(const MrArgs& a, MrShared<256 << RES>& sh, int64_t b,
                                              int blk) {
  constexpr int r = RES;
  constexpr int n = 512 << r;
  constexpr int Nc = n / 2;             // complex points per transform
  constexpr int kOlaSlots = MrShared<Nc>::ola_slots;
  constexpr int P = Nc / 64;            // points per lane
  constexpr int QB = Nc / 128;          // bin pairs per lane (k = lane + 64 q < Nc / 2)
  constexpr int hop = n / 4;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int chunk = blk - a.chunk_base[r];
  const int F = a.F[r];
  const bool want_grad = MODE != 1 && a.wgrad != nullptr;
  // The scale is applied in float32 to the gradient and in float64 to the loss.
  const double scale_d = a.scale[r];
  const float scale = (float)scale_d;

  // ---- tables of this resolution ----
  for (int k = tid; k < n; k += kMrThreads) sh.win[k] = 0.5f - 0.5f * cospif(2.0f * (float)k / (float)n);
  for (int k = tid; k <= Nc / 2; k += kMrThreads) {
    float sn, cs;
    sincospif(2.0f * (float)k / (float)n, &sn, &cs);
    sh.rs[k] = make_float2(cs, -sn);
  }
  wfft::build_pass_twiddles<Nc>(sh.pt, tid, kMrThreads);
  for (int i = tid; i < kOlaSlots; i += kMrThreads) sh.ola[i] = 0.0f;
  __syncthreads();

  const int f_begin = chunk * kFramesPerBlock;
  const int f_end = min(F, f_begin + kFramesPerBlock);
  const int nch = a.chunk_base[r + 1] - a.chunk_base[r];
  float* seg = want_grad ? a.wgrad + a.wbase[r] + ((int64_t)b * nch + chunk) * (kSegHops * hop)
                         : nullptr;
  float2* buf = sh.buf[wv];
  const float* xs = a.x + b * a.n;
  const float* ts = a.t + b * a.n;
  double acc = 0.0;

  for (int f0 = f_begin; f0 < f_end; f0 += kMrWaves) {
    const int f = f0 + wv;
    const bool live = f < f_end;        // wave-uniform
    if (live) {
      const float* fx = xs + (int64_t)f * hop;
      const float* ft = ts + (int64_t)f * hop;
      float* trow = a.tlog ? a.tlog + a.tbase[r] + ((int64_t)b * F + f) * (Nc + 1) : nullptr;
      float2 v[P];
      // ---- target frame: log magnitudes of bins k, Nc - k, Nc / 2 ----
      float Lk[QB + 1], Lm[QB + 1];
      if constexpr (MODE == 2) {
#pragma unroll
        for (int q = 0; q <= QB; ++q) {
          const int k = q < QB ? lane + 64 * q : Nc / 2;
          Lk[q] = trow[k];
          Lm[q] = trow[Nc - k];
        }
      } else {
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const int m = lane + 64 * q;
          const float2 w2 = *reinterpret_cast<const float2*>(&sh.win[2 * m]);
          v[q] = make_float2(w2.x * ft[2 * m], w2.y * ft[2 * m + 1]);
        }
        wfft::wave_fft<Nc, true>(v, buf, sh.pt, lane);
#pragma unroll
        for (int q = 0; q <= QB; ++q) {
          float2 Tk, Tm;
          real_pair<Nc>(buf, sh.rs, q < QB ? lane + 64 * q : Nc / 2, Tk, Tm);
          Lk[q] = target_log(Tk);
          Lm[q] = target_log(Tm);
        }
        if constexpr (MODE == 1) {
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            const int k = lane + 64 * q;
            trow[k] = Lk[q];
            trow[Nc - k] = Lm[q];
          }
          if (lane == 0) trow[Nc / 2] = Lk[QB];
          continue;
        }
      }
      // ---- render frame ----
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int m = lane + 64 * q;
        const float2 w2 = *reinterpret_cast<const float2*>(&sh.win[2 * m]);
        v[q] = make_float2(w2.x * fx[2 * m], w2.y * fx[2 * m + 1]);
      }
      wfft::wave_fft<Nc, true>(v, buf, sh.pt, lane);
      float2 Hk[QB + 1], Hm[QB + 1];
#pragma unroll
      for (int q = 0; q <= QB; ++q) {
        const int k = q < QB ? lane + 64 * q : Nc / 2;
        float2 Xk, Xm;
        real_pair<Nc>(buf, sh.rs, k, Xk, Xm);
        if (q < QB) {
          Hk[q] = bin_grad(Xk, Lk[q], scale_d, scale, k == 0, want_grad, acc);
          Hm[q] = bin_grad(Xm, Lm[q], scale_d, scale, k == 0, want_grad, acc);   // bin Nc - k
        } else {
          // bin Nc / 2, once per frame (lane 0)
          double a2 = 0.0;
          Hk[q] = bin_grad(Xk, Lk[q], scale_d, scale, false, want_grad, a2);
          if (lane == 0) acc += a2;
          Hm[q] = make_float2(0.f, 0.f);
        }
      }
      if (want_grad) {
        // ---- H to LDS (slot k holds H_k; slot 0 holds (H_0, H_Nc), both real) ----
        wfft::wave_fence();
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const int k = lane + 64 * q;
          if (k == 0) {
            buf[wfft::swz<Nc>(0)] = make_float2(Hk[q].x, Hm[q].x);
          } else {
            buf[wfft::swz<Nc>(k)] = Hk[q];
            buf[wfft::swz<Nc>(Nc - k)] = Hm[q];
          }
        }
        if (lane == 0) buf[wfft::swz<Nc>(Nc / 2)] = Hk[QB];
        wfft::wave_fence();
        // ---- inverse input: Y_m = (H_m + conj H_{Nc-m}) + i conj(W^m) (H_m - conj H_{Nc-m}) ----
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const int m = lane + 64 * q;
          float2 hk, hc;
          if (m == 0) {
            const float2 h0 = buf[wfft::swz<Nc>(0)];
            hk = make_float2(h0.x, 0.f);
            hc = make_float2(h0.y, 0.f);
          } else {
            hk = buf[wfft::swz<Nc>(m)];
            const float2 t2 = buf[wfft::swz<Nc>(Nc - m)];
            hc = make_float2(t2.x, -t2.y);
          }
          const float2 A = wfft::add(hk, hc), D = wfft::sub(hk, hc);
          // W^m = exp(-2 pi i m / n); for m > Nc / 2 from W^{Nc - m} = -conj(W^m)
          const float2 wm = m <= Nc / 2 ? sh.rs[m] : make_float2(-sh.rs[Nc - m].x, sh.rs[Nc - m].y);
          const float2 cd = wfft::cmulc(D, wm);        // conj(W^m) D
          v[q] = make_float2(A.x - cd.y, A.y + cd.x);   // A + i (conj(W^m) D)
        }
        wfft::wave_fft<Nc, false>(v, buf, sh.pt, lane);
      }
    }
    if (want_grad) {
      __syncthreads();                  // the four frames' rows are in the buffers
      // ---- overlap-add: frame f0 + s contributes 0.5 w(o) y(o) at o = p - s hop ----
      const int p0 = (f0 - f_begin) * hop;           // block-relative start of frame f0
      for (int p = tid; p < (kMrWaves - 1) * hop + n; p += kMrThreads) {
        float g = 0.0f;
#pragma unroll
        for (int s2 = 0; s2 < kMrWaves; ++s2) {
          const int o = p - s2 * hop;
          if (o >= 0 && o < n && f0 + s2 < f_end) {
            const float2 yy = sh.buf[s2][wfft::swz<Nc>(o >> 1)];
            g += 0.5f * sh.win[o] * ((o & 1) ? yy.y : yy.x);
          }
        }
        float* slotp = sh.ola + ((p0 + p) & (kOlaSlots - 1));
        const float v2 = *slotp + g;
        if (p < kMrWaves * hop) {                    // no later frame reaches it
          seg[p0 + p] = v2;
          *slotp = 0.0f;
        } else {
          *slotp = v2;
        }
      }
      __syncthreads();                  // buffers and accumulator reused next
    }
  }
  if (want_grad) {
    // the rest of the segment: the last frames' tails (3 hops past the
    // written part), then zeros
    const int done = ((f_end - f_begin + kMrWaves - 1) / kMrWaves) * kMrWaves * hop;
    for (int p = done + tid; p < kSegHops * hop; p += kMrThreads)
      seg[p] = p < done + 3 * hop ? sh.ola[p & (kOlaSlots - 1)] : 0.0f;
  }
  if constexpr (MODE == 1) return;
  // fixed-order reduction of the per-lane loss shares
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
  if (lane == 0) sh.red[wv] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kMrWaves; ++w) s += sh.red[w];
    a.partial[b * a.chunk_base[3] + blk] = s;
  }
}

// One launch per resolution, so that each gets the LDS and registers of its
// own transform size (and the occupancy they allow).
template <int RES, int MODE>
__global__ void __launch_bounds__(kMrThreads) mrstft_frames_kernel(const MrArgs a) {
  __shared__ MrShared<256 << RES> sh;
  mrstft_frames<RES, MODE>(a, sh, blockIdx.y, a.chunk_base[RES] + (int)blockIdx.x);
}

// Log-mel features by FFT, one workgroup of 4 wavefronts per voice: frames
// f < 64 of 2048 samples at hop 2756 (samples past the voice's end read as
// 0), periodic Hann window, power spectrum |X_fk|^2 (k <= 1024) rounded to
// bf16, each mel band's sum over its nonzero bins in float32, log(x + 1e-6)
// into features[b][band][f].  Wavefront w takes frames w, w + 4, ...: a
// 1024-point complex wave FFT of z[m] = w x[2m] + i w x[2m+1], the real
// spectrum from Z_k and Z_{1024-k}, the power row and the band sums in its
// own LDS buffer; the only workgroup barriers are around the staged feature
// stores (every 16 frames).
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// |X|^2 rounded to bf16 (hardware round-to-nearest-even conversion)
__device__ __forceinline__ float pow_bf16(float2 X) {
  return (float)(__bf16)(X.x * X.x + X.y * X.y);
}

// A band's weights are summed in chunks of at most kMelChunk bins, one chunk
// per lane, then each band adds its chunks' sums in order: the work per lane
// stays even although band widths range from 1 to ~60 bins.
constexpr int kMelChunk = 12;
constexpr int kMelChunksMax = kMelWeightsMax / kMelChunk + kMelBands;
constexpr int kMelWaves = 4;
constexpr int kMelThreads = 64 * kMelWaves;

struct MelShared {
  float wt[kMelChunk][kMelChunksMax];   // chunk c's weights, zero-padded to kMelChunk
  int lo[kMelBands];
  int off[kMelBands + 1];
  int cbase[kMelBands + 1];    // band b's chunks: cbase[b] .. cbase[b + 1] - 1
  int chunk[kMelChunksMax];    // first bin of chunk c
  float st[kMelBands][17];     // features of 16 frames, written out together
  alignas(8) float win[2048];  // periodic Hann window
  float2 rs[513];              // exp(-2 pi i k / 2048), k <= 512 (real split)
  float2 pt[wfft::pt_size<1024>()];   // FFT pass twiddles
};

// float -> bf16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t mel_f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Optional standardised output: bf16 (x - mean[c]) * inv_std[c] of feature c
// of voice b to row row_map[b] (b without a map; rows outside [0, batch) are
// not written) instead of the float32 features.
struct MelStd {
  const float* mean;
  const float* inv_std;
  const int64_t* row_map;
  uint16_t* out;
};

template <bool STD>
__global__ void __launch_bounds__(kMelThreads) __attribute__((amdgpu_waves_per_eu(2)))
logmel_fft_kernel(const float* __restrict__ audio, const int64_t* __restrict__ offsets,
                  int64_t n_uniform, const uint16_t* __restrict__ mel, int64_t ldm,
                  float* __restrict__ features, MelStd sd) {
  constexpr int Nc = 1024, P = 16, hop = 2756, frames = 64;
  __shared__ float2 wbuf[kMelWaves][Nc];
  __shared__ MelShared ms;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int64_t b = blockIdx.x;
  int64_t start, len;
  if (offsets) {
    packed_range(offsets, (int64_t)gridDim.x, b, start, len);
  } else {
    start = b * n_uniform;
    len = n_uniform;
  }
  const float* x = audio + start;
  float* feat = STD ? nullptr : features + b * (int64_t)(kMelBands * frames);
  uint16_t* yrow = nullptr;
  if constexpr (STD) {
    const int64_t row = sd.row_map ? sd.row_map[b] : b;
    if (row >= 0 && row < (int64_t)gridDim.x) yrow = sd.out + row * (int64_t)(kMelBands * frames);
  }
  // feature c of this voice takes value v
  auto put = [&](int c, float v) {
    if constexpr (STD) {
      if (yrow) yrow[c] = mel_f2bf((v - sd.mean[c]) * sd.inv_std[c]);
    } else {
      feat[c] = v;
    }
  };

  // ---- set-up: band table (wavefront 0), twiddle table T[k] = exp(-2 pi i k / 2048) ----
  if (tid < 64) {
    int lo[2], wd[2], nc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint16_t* row = mel + (int64_t)(2 * tid + h) * ldm;
      lo[h] = row[Nc + 1] <= Nc ? row[Nc + 1] : Nc;
      const int hi = row[Nc + 2] <= Nc ? row[Nc + 2] : Nc;
      wd[h] = hi >= lo[h] ? hi - lo[h] + 1 : 0;
      nc[h] = (wd[h] + kMelChunk - 1) / kMelChunk;
    }
    const int pw = wd[0] + wd[1], pc = nc[0] + nc[1];
    int iw = pw, ic = pc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int yw = __shfl_up(iw, d), yc = __shfl_up(ic, d);
      if (tid >= d) iw += yw, ic += yc;
    }
    ms.lo[2 * tid] = lo[0];
    ms.lo[2 * tid + 1] = lo[1];
    ms.off[2 * tid] = iw - pw;
    ms.off[2 * tid + 1] = iw - pw + wd[0];
    ms.cbase[2 * tid] = min(ic - pc, kMelChunksMax);
    ms.cbase[2 * tid + 1] = min(ic - pc + nc[0], kMelChunksMax);
    if (tid == 63) {
      ms.off[kMelBands] = iw;
      ms.cbase[kMelBands] = min(ic, kMelChunksMax);
    }
  }
  for (int k = tid; k <= Nc / 2; k += kMelThreads) {
    float sn, cs;
    sincospif((float)k / (float)Nc, &sn, &cs);
    ms.rs[k] = make_float2(cs, -sn);
  }
  for (int k = tid; k < 2 * Nc; k += kMelThreads)
    ms.win[k] = 0.5f - 0.5f * cospif(2.0f * (float)k / (float)(2 * Nc));
  wfft::build_pass_twiddles<Nc>(ms.pt, tid, kMelThreads);
  __syncthreads();                      // band table and LDS tables written
  for (int e = tid; e < kMelBands * 4; e += kMelThreads) {
    const int bd = e >> 2;
    const int wd = ms.off[bd + 1] - ms.off[bd];
    const uint16_t* row = mel + (int64_t)bd * ldm + ms.lo[bd];
    for (int c = ms.cbase[bd] + (e & 3), q = e & 3; c < ms.cbase[bd + 1]; c += 4, q += 4) {
      ms.chunk[c] = ms.lo[bd] + q * kMelChunk;
#pragma unroll
      for (int i = 0; i < kMelChunk; ++i)
        ms.wt[i][c] = q * kMelChunk + i < wd ? bf2f(row[q * kMelChunk + i]) : 0.0f;
    }
  }
  __syncthreads();
  const int nchunks = ms.cbase[kMelBands];

  float2* buf = wbuf[wv];
  // power row P[0..1024] (a chunk may read up to 11 slots past it, where its
  // weights are 0), chunk sums from 1040
  float* Pw = reinterpret_cast<float*>(buf);
  float* part = Pw + 1040;
  // Frames that start at or past the voice's end hold only zero padding:
  // their features are log(1e-6) and they skip the FFT.
  const int64_t nlive = len <= 0 ? 0 : (len + hop - 1) / hop;
  const int live = (int)(nlive < frames ? nlive : frames);
  // this wavefront's next frame's samples, fetched during the current one
  float s[2 * P];
#define LM_FETCH(f_)                                                    \
  {                                                                     \
    const int64_t pos = (int64_t)(f_) * hop;                            \
    _Pragma("unroll") for (int r = 0; r < P; ++r) {                     \
      const int64_t i0 = pos + 2 * (lane + 64 * r);                     \
      s[2 * r] = i0 < len ? x[i0] : 0.0f;                               \
      s[2 * r + 1] = i0 + 1 < len ? x[i0 + 1] : 0.0f;                   \
    }                                                                   \
  }
  if (wv < live) LM_FETCH(wv)
  for (int g = 0; 16 * g < live; ++g) {
#pragma unroll 1
    for (int i = 0; i < 4; ++i) {
      const int f = 16 * g + wv + 4 * i;
      if (f >= live) break;
      float2 v[P];
#pragma unroll
      for (int r = 0; r < P; ++r) {
        const float2 w2 = *reinterpret_cast<const float2*>(&ms.win[2 * (lane + 64 * r)]);
        v[r] = make_float2(w2.x * s[2 * r], w2.y * s[2 * r + 1]);
      }
      if (f + 4 < live) LM_FETCH(f + 4)
      wfft::wave_fft<Nc, true>(v, buf, ms.pt, lane);
      // ---- real spectrum: X_k = E + W^k O, X_{Nc-k} = conj(E - W^k O) ----
      float pk[9], pm[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int k = q < 8 ? lane + 64 * q : 512;
        const float2 zk = buf[wfft::swz<Nc>(k)];
        const float2 zc = buf[wfft::swz<Nc>((Nc - k) & (Nc - 1))];
        const float2 E = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y - zc.y));
        const float2 O = make_float2(0.5f * (zk.y + zc.y), -0.5f * (zk.x - zc.x));
        const float2 w = ms.rs[k];
        const float2 WO = wfft::cmul(w, O);
        pk[q] = pow_bf16(wfft::add(E, WO));
        pm[q] = pow_bf16(wfft::sub(E, WO));
      }
      wfft::wave_fence();
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = lane + 64 * q;
        Pw[k] = pk[q];
        Pw[Nc - k] = pm[q];
      }
      if (lane == 0) Pw[512] = pk[8];
      wfft::wave_fence();
      // ---- band sums: chunk c = lane + 64 i, then band b = lane, lane + 64 ----
      for (int c = lane; c < nchunks; c += 64) {
        const float* pc = Pw + ms.chunk[c];
        float acc = 0.0f;
#pragma unroll
        for (int i2 = 0; i2 < kMelChunk; ++i2) acc = fmaf(ms.wt[i2][c], pc[i2], acc);
        part[c] = acc;
      }
      wfft::wave_fence();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int bd = lane + 64 * h;
        const int c0 = ms.cbase[bd], c1 = ms.cbase[bd + 1];
        float acc = 0.0f;
#pragma unroll
        for (int i2 = 0; i2 < 6; ++i2) {
          const float pv = part[min(c0 + i2, kMelChunksMax - 1)];
          acc += c0 + i2 < c1 ? pv : 0.0f;
        }
        for (int c = c0 + 6; c < c1; ++c) acc += part[c];
        ms.st[bd][f & 15] = logf(acc + 1e-6f);
      }
    }
    // write out frames 16 g .. of the group: 16 consecutive frames of a band
    // are 64 contiguous bytes
    __syncthreads();
    const int cnt = min(16, live - 16 * g);
    for (int e = tid; e < kMelBands * 16; e += kMelThreads) {
      const int bd = e >> 4, fr = e & 15;
      if (fr < cnt) put(bd * frames + 16 * g + fr, ms.st[bd][fr]);
    }
    __syncthreads();
  }
#undef LM_FETCH
  const int nz = frames - live;
  if (nz > 0) {
    float zero = 0.0f;
    asm volatile("" : "+v"(zero));      // log(0 + 1e-6) evaluated as for a computed frame
    const float floor_v = logf(zero + 1e-6f);
    for (int e = tid; e < kMelBands * nz; e += kMelThreads) {
      const int bd = e / nz;
      put(bd * frames + live + (e - bd * nz), floor_v);
    }
  }
}

// grad[b][i] = sum over resolutions, then over the (at most two) workgroup
// segments covering i, in workgroup order; block x == 0 also sums voice b's
// loss partials.
__global__ void __launch_bounds__(256) mrstft_combine_kernel(const MrArgs a) {
  const int64_t b = blockIdx.y;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int c = 0; c < a.chunk_base[3]; ++c) s += a.partial[b * a.chunk_base[3] + c];
    a.loss[b] = s;
  }
  if (!a.grad) return;
  // four consecutive samples per thread: hops are multiples of 4, so they
  // share their segments, and segment rows are 16-byte aligned
  const int64_t i0 = 4 * (blockIdx.x * (int64_t)blockDim.x + threadIdx.x);
  if (i0 >= a.n) return;
  float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int r = 0; r < 3; ++r) {
    const int n = 512 << r, hop = n / 4;
    const int nch = a.chunk_base[r + 1] - a.chunk_base[r];
    if (nch == 0) continue;
    const int64_t h = i0 / hop;                      // hop of samples i0 .. i0 + 3
    int64_t khi = h / kFramesPerBlock;
    if (khi > nch - 1) khi = nch - 1;
    const int64_t klo = h >= kSegHops ? (h - kSegHops) / kFramesPerBlock + 1 : 0;
    const int64_t seglen = (int64_t)kSegHops * hop;
    const float* segs = a.wgrad + a.wbase[r] + b * nch * seglen;
    for (int64_t k = klo; k <= khi; ++k) {
      const float4 v = *reinterpret_cast<const float4*>(segs + k * seglen +
                                                        (i0 - k * kFramesPerBlock * hop));
      g.x += v.x;
      g.y += v.y;
      g.z += v.z;
      g.w += v.w;
    }
  }
  float* out = a.grad + b * a.n + i0;
  if (i0 + 4 <= a.n && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
    *reinterpret_cast<float4*>(out) = g;
  } else {
    const float gv[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (i0 + e < a.n) out[e] = gv[e];
  }
}

void plan(int64_t batch, int64_t n_samples, MrArgs& a, size_t& partial_bytes, size_t& wgrad_floats,
          size_t* tlog_floats = nullptr) {
  int cb = 0;
  int64_t wb = 0, tb = 0;
  for (int r = 0; r < 3; ++r) {
    const int n = 512 << r;
    const int64_t F = n_samples < n ? 0 : (n_samples - n) / (n / 4) + 1;
    a.F[r] = (int)F;
    a.chunk_base[r] = cb;
    cb += (int)((F + kFramesPerBlock - 1) / kFramesPerBlock);
    a.wbase[r] = wb;
    wb += batch * ((F + kFramesPerBlock - 1) / kFramesPerBlock) * kSegHops * (n / 4);
    a.tbase[r] = tb;
    tb += batch * F * (n / 2 + 1);
    a.scale[r] = F > 0 ? 1.0 / ((double)F * (double)(n / 2 + 1)) : 0.0;
  }
  if (tlog_floats) *tlog_floats = (size_t)tb;
  a.chunk_base[3] = cb;
  partial_bytes = (size_t)batch * (size_t)(cb > 0 ? cb : 1) * sizeof(double);
  wgrad_floats = (size_t)wb;
}

}  // namespace

hipError_t launch_logmel_fft(const float* audio, const int64_t* offsets, int64_t n_uniform,
                            int64_t batch, const void* mel_basis, int64_t ldm, float* features,
                            hipStream_t s) {
  if (batch == 0) return hipSuccess;
  if (batch > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(logmel_fft_kernel<false>, dim3((unsigned)batch), dim3(kMelThreads), 0, s,
                     audio, offsets, n_uniform, (const uint16_t*)mel_basis, ldm, features,
                     MelStd{});
  return hipGetLastError();
}

hipError_t launch_logmel_fft_std(const float* audio, const int64_t* offsets, int64_t n_uniform,
                                 int64_t batch, const void* mel_basis, int64_t ldm,
                                 const float* mean, const float* inv_std, const int64_t* row_map,
                                 void* out_bf16, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  if (batch > 0x7FFFFFFF) return hipErrorInvalidValue;
  const MelStd sd{mean, inv_std, row_map, static_cast<uint16_t*>(out_bf16)};
  hipLaunchKernelGGL(logmel_fft_kernel<true>, dim3((unsigned)batch), dim3(kMelThreads), 0, s,
                     audio, offsets, n_uniform, (const uint16_t*)mel_basis, ldm, nullptr, sd);
  return hipGetLastError();
}

size_t mrstft_workspace_bytes(int64_t batch, int64_t n_samples, bool with_grad) {
  MrArgs a = {};
  size_t pb, wf;
  plan(batch, n_samples, a, pb, wf);
  pb = (pb + 255) & ~(size_t)255;
  return pb + (with_grad ? wf * sizeof(float) : 0);
}

namespace {
template <int MODE>
void launch_frames(const MrArgs& a, hipStream_t s) {
  const int nch[3] = {a.chunk_base[1] - a.chunk_base[0], a.chunk_base[2] - a.chunk_base[1],
                      a.chunk_base[3] - a.chunk_base[2]};
  const unsigned B = (unsigned)a.batch;
  if (nch[0] > 0)
    hipLaunchKernelGGL((mrstft_frames_kernel<0, MODE>), dim3((unsigned)nch[0], B), dim3(kMrThreads),
                       0, s, a);
  if (nch[1] > 0)
    hipLaunchKernelGGL((mrstft_frames_kernel<1, MODE>), dim3((unsigned)nch[1], B), dim3(kMrThreads),
                       0, s, a);
  if (nch[2] > 0)
    hipLaunchKernelGGL((mrstft_frames_kernel<2, MODE>), dim3((unsigned)nch[2], B), dim3(kMrThreads),
                       0, s, a);
}
}  // namespace

size_t mrstft_target_bytes(int64_t batch, int64_t n_samples) {
  MrArgs a = {};
  size_t pb, wf, tf;
  plan(batch, n_samples, a, pb, wf, &tf);
  return tf * sizeof(float);
}

hipError_t launch_mrstft_target(const float* target, int64_t batch, int64_t n_samples, float* tlog,
                                hipStream_t s) {
  if (batch == 0) return hipSuccess;
  if (batch > 65535) return hipErrorInvalidValue;
  MrArgs a = {};
  size_t pb, wf;
  plan(batch, n_samples, a, pb, wf);
  a.t = target;
  a.x = target;
  a.n = n_samples;
  a.batch = batch;
  a.tlog = tlog;
  launch_frames<1>(a, s);
  return hipGetLastError();
}

hipError_t launch_mrstft(const float* x, const float* target, const float* tlog, int64_t batch,
                         int64_t n_samples, double* loss, float* grad, void* workspace,
                         hipStream_t s) {
  if (batch == 0) return hipSuccess;
  MrArgs a = {};
  size_t pb, wf;
  plan(batch, n_samples, a, pb, wf);
  pb = (pb + 255) & ~(size_t)255;
  a.x = x;
  a.t = target ? target : x;
  a.tlog = const_cast<float*>(tlog);
  a.n = n_samples;
  a.batch = batch;
  a.partial = reinterpret_cast<double*>(workspace);
  a.wgrad = grad ? reinterpret_cast<float*>(reinterpret_cast<char*>(workspace) + pb) : nullptr;
  a.grad = grad;
  a.loss = loss;
  if (batch > 65535) return hipErrorInvalidValue;
  if (tlog)
    launch_frames<2>(a, s);
  else
    launch_frames<0>(a, s);
  if (a.chunk_base[3] > 0) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // (with no complete frame at any resolution the combine kernel writes
  // loss 0 and a zero gradient)
  const int64_t gx = grad ? (n_samples + 1023) / 1024 : 1;
  hipLaunchKernelGGL(mrstft_combine_kernel, dim3((unsigned)gx, (unsigned)batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace synth
