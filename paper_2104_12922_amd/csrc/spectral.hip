// Multi-resolution log-magnitude STFT L1 loss and its gradient (float32 FFT).
//
// The paper scores sounds with a multi-scale spectrogram distance over several
// FFT sizes and prefers L1 (Section 4, distance evaluation).  Per voice:
//   loss = sum over n in (512, 1024, 2048), hop n/4, of
//          mean_{frame t, bin k <= n/2} |log(|X_tk| + 1e-5) - log(|T_tk| + 1e-5)|
// with X, T the periodic-Hann STFTs (no padding) of the render x and target.
//
// Frames are independent jobs.  Kernel 1 (512 threads per workgroup, grid =
// voices x (frame chunks of every resolution)) takes 16 frames of one
// resolution per workgroup.  A real frame of n samples is transformed as a
// complex sequence of n/2 points (even samples real, odd imaginary) by a
// Stockham autosort FFT - radix-4 passes and one radix-2 pass when log2(n/2)
// is odd - with one radix-4 butterfly per thread and pass, twiddles from an
// LDS table, then split into the n/2 + 1 bins of the real spectrum.  Render
// and target frames get separate FFTs (a shared complex FFT would leak the
// louder signal's rounding noise into the quieter one's spectrum).  For the
// gradient, G_k = sign(d_k) X_k / (|X_k| (|X_k| + eps)) / (F (n/2 + 1)) is
// extended to a Hermitian spectrum H (H_0 = 2 Re G_0, H_{n/2} = 2 Re G_{n/2}),
// inverted by the same half-size complex FFT, and the frame's gradient
// 0.5 w(m) h(m) is written to a workspace row of its own.  Kernel 2 adds,
// for every sample, the rows of the frames that cover it in a fixed order
// (resolution, then frame), and sums the per-workgroup loss partials in a
// fixed order: bitwise deterministic, no atomics.
#include <math.h>

#include "synth_internal.h"
#include "wave_fft.h"

namespace synth {
namespace {

constexpr int kThreads = 512;
constexpr int kMaxN = 2048;
constexpr int kFramesPerBlock = 16;
// A workgroup's frames f0 .. f0 + 15 cover hops f0 .. f0 + 18 of the voice:
// their gradient rows are overlap-added in LDS into one segment of 19 hops.
constexpr int kSegHops = kFramesPerBlock + 3;
constexpr int kOlaSlots = 2048;
constexpr float kEps = 1e-5f;
// LDS slot swizzle (a bijection within each block of 128 float2): XORs index
// bits 4-6 into bits 0-4 so that the strided writes of the first Stockham
// passes (strides of 4 and 16 slots) and the contiguous reads all fall on
// distinct banks, for 32 or 64 four-byte banks.
__device__ __forceinline__ int swz(int i) { return i ^ (5 * ((i >> 4) & 3)) ^ ((i >> 2) & 16); }
constexpr int kPadded = kMaxN;

constexpr int kPassTw = 1280;  // per-pass twiddles (Nc = 512 needs 1276)

struct SpecShared {
  float2 tw[kMaxN / 2];        // tw[k] = exp(-2 pi i k / n), k < n / 2
  float2 ptw[kPassTw];         // per-pass twiddles, contiguous in the butterfly index
  float win[kMaxN];            // periodic Hann window
  float2 buf[2][kPadded];      // FFT ping-pong: (512 / (n/8)) transforms of n/2 points (swizzled)
  double red[kThreads / 64];
};

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
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// One Stockham pass of radix R on the transform of NC points whose butterfly
// j (0 <= j < NC / R) this thread owns: inputs v[r] = src[j + r NC / R], the
// twiddles exp(dir 2 pi i (j mod NS) r / (NS R)), the R-point DFT, outputs to
// dst[(j / NS) NS R + (j mod NS) + r NS].  tw holds exp(-2 pi i k / (2 NC)).
// NS and NC are powers of two known at compile time.
// Per-pass twiddle tables: the radix-4 pass with stride NS (NS >= 4) keeps
// exp(-2 pi i k r / (4 NS)) for k < NS, r = 1..3 at ptw[off4(NS) + 3 k + r - 1];
// the radix-2 pass (stride NS) keeps exp(-2 pi i k / (2 NS)) at ptw[off4(NS) + k].
// Lanes read consecutive entries.
constexpr int off4(int ns) { return ns <= 4 ? 0 : off4(ns / 4) + 3 * (ns / 4); }

template <int R, int NS, int NC>
__device__ __forceinline__ void butterfly(float2 (&v)[4], int j, float dir, const float2* ptw) {
  const int k = j & (NS - 1);
  if constexpr (NS > 1) {
#pragma unroll
    for (int r = 1; r < R; ++r) {
      float2 w = ptw[off4(NS) + (R - 1) * k + (r - 1)];
      if (dir > 0.0f) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
  }
  if constexpr (R == 4) {
    const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]);
    float2 t3 = csub(v[1], v[3]);
    t3 = dir < 0.0f ? make_float2(t3.y, -t3.x) : make_float2(-t3.y, t3.x);   // -i or +i
    v[0] = cadd(t0, t2);
    v[1] = cadd(t1, t3);
    v[2] = csub(t0, t2);
    v[3] = csub(t1, t3);
  } else {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
}

// The passes of a complex FFT of NC points held by NC / 4 threads (thread j
// of the transform), starting from v (the first pass's inputs v[r] =
// z[j + r NC / 4]), ping-ponging between base0 and base1 (each NC points).
// Every thread of the workgroup calls it (it contains barriers); `active`
// marks the threads that own a butterfly.  CUR is the buffer the pass writes;
// the natural-order result ends in the buffer whose index is returned.
template <int NC, int NS, int CUR>
__device__ __forceinline__ int fft_passes(float2 (&v)[4], int j, float dir, const float2* ptw,
                                          float2* base0, float2* base1, bool active) {
  constexpr int REM = NC / NS;
  if constexpr (REM <= 1) {
    return CUR ^ 1;
  } else {
    constexpr int R = (REM % 4 == 0) ? 4 : 2;
    float2* dst = CUR == 0 ? base0 : base1;
    const float2* src = CUR == 0 ? base1 : base0;
    constexpr bool first = NS == 1;
    if (active) {
      if constexpr (R == 4) {
        if constexpr (!first) {
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = src[swz(j + r * (NC / 4))];
        }
        butterfly<4, NS, NC>(v, j, dir, ptw);
        const int d = ((j & ~(NS - 1)) << 2) + (j & (NS - 1));
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[swz(d + r * NS)] = v[r];
      } else {
        // radix 2 (last pass): NC / 2 butterflies, two per thread (j, j + NC / 4)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int jj = j + h * (NC / 4);
          float2 u[4];
          u[0] = src[swz(jj)];
          u[1] = src[swz(jj + NC / 2)];
          butterfly<2, NS, NC>(u, jj, dir, ptw);
          const int d = ((jj & ~(NS - 1)) << 1) + (jj & (NS - 1));
          dst[swz(d)] = u[0];
          dst[swz(d + NS)] = u[1];
        }
      }
    }
    __syncthreads();
    return fft_passes<NC, NS * R, CUR ^ 1>(v, j, dir, ptw, base0, base1, active);
  }
}

// Twiddle, window and per-pass tables for frames of n = 512 << RES samples
// (every thread of the workgroup takes part; ends with a barrier).
template <int RES>
__device__ __forceinline__ void fft_tables(SpecShared& sh) {
  constexpr int n = 512 << RES;
  constexpr int Nc = n / 2;
  const int tid = threadIdx.x;
  for (int k = tid; k < n; k += kThreads) {
    if (k < Nc) {
      float s, c;
      sincospif(2.0f * (float)k / (float)n, &s, &c);
      sh.tw[k] = make_float2(c, -s);
    }
    sh.win[k] = 0.5f - 0.5f * cospif(2.0f * (float)k / (float)n);
  }
  for (int ns = 4, rem = Nc / 4; rem > 1; ns *= 4, rem /= 4) {
    const int R = rem % 4 == 0 ? 4 : 2;       // radix of the pass with stride ns
    for (int e = tid; e < (R - 1) * ns; e += kThreads) {
      const int k = e / (R - 1), r = e % (R - 1) + 1;
      float sn, cs;
      sincospif(-2.0f * (float)(k * r) / (float)(R * ns), &sn, &cs);
      sh.ptw[off4(ns) + e] = make_float2(cs, sn);
    }
    if (R == 2) break;
  }
  __syncthreads();
}

// Bin k (0 <= k <= Nc) of the real spectrum of a frame of 2 Nc samples from
// the half-size complex FFT Z (even samples real, odd imaginary; swizzled).
template <int Nc>
__device__ __forceinline__ float2 real_bin(const float2* Z, const float2* tw, int k) {
  const float2 w = k < Nc ? tw[k] : make_float2(-1.0f, 0.0f);
  const int kc = k == Nc ? 0 : k, km = k == 0 ? 0 : Nc - k;   // Z_Nc = Z_0
  const float2 zk = Z[swz(kc)], zc = cconj(Z[swz(km)]);
  const float2 E = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
  const float2 D = csub(zk, zc);
  const float2 O = make_float2(0.5f * D.y, -0.5f * D.x);       // -i D / 2
  return cadd(E, cmul(w, O));
}

template <int RES>
__device__ __forceinline__ void mrstft_frames(const MrArgs& a, SpecShared& sh, float* ola,
                                              int64_t b, int blk) {
  constexpr int r = RES;
  const int tid = threadIdx.x;
  const int chunk = blk - a.chunk_base[r];
  constexpr int n = 512 << r;
  constexpr int Nc = n / 2;             // complex points per transform
  constexpr int tpt = Nc / 4;           // threads per transform
  constexpr int ntr = kThreads / tpt;   // transforms in flight: 8, 4, 2
  constexpr int fpi = ntr / 2;          // frames per iteration: 4, 2, 1
  constexpr int hop = n / 4;
  const int F = a.F[r];
  const bool want_grad = a.wgrad != nullptr;

  fft_tables<RES>(sh);

  const int tr = tid / tpt;             // transform of this thread
  const int j = tid - tr * tpt;         // butterfly index within the transform
  const int slot = tr >> 1;             // frame slot of the iteration
  const int sig = tr & 1;               // 0: render, 1: target
  const float* src = (sig ? a.t : a.x) + b * a.n;
  const double scale = a.scale[r];
  double acc = 0.0;

  const int f_begin = chunk * kFramesPerBlock;
  const int f_end = min(F, f_begin + kFramesPerBlock);
  // Overlap-add accumulator: block-relative position p lives at ola[p % 2048]
  // (the unfinished positions never span more than (fpi - 1) hop + n <= 2048);
  // a position is written out to the segment, and its slot cleared, as soon
  // as no later frame of the block covers it.
  const int nch = a.chunk_base[r + 1] - a.chunk_base[r];
  float* seg = want_grad ? a.wgrad + a.wbase[r] + ((int64_t)b * nch + chunk) * (kSegHops * hop)
                         : nullptr;
  if (want_grad)
    for (int i = tid; i < kOlaSlots; i += kThreads) ola[i] = 0.0f;
  for (int f0 = f_begin; f0 < f_end; f0 += fpi) {
    const int f = f0 + slot;
    const bool live = f < f_end;
    // ---- forward transforms: z[m] = w x[2m] + i w x[2m+1] ----
    float2 v[4];
    const float* fr = src + (int64_t)f * hop;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = j + q * tpt;
      v[q] = live ? make_float2(sh.win[2 * m] * fr[2 * m], sh.win[2 * m + 1] * fr[2 * m + 1])
                  : make_float2(0.f, 0.f);
    }
    float2* b0 = sh.buf[0] + tr * Nc;
    float2* b1 = sh.buf[1] + tr * Nc;
    const int zb = fft_passes<Nc, 1, 0>(v, j, -1.0f, sh.ptw, b0, b1, true);
    // ---- bins: frame slot's 2 * tpt threads take bins k = u, u + 2 tpt, ... ----
    const float2* Zx = sh.buf[zb] + (2 * slot) * Nc;
    const float2* Zt = sh.buf[zb] + (2 * slot + 1) * Nc;
    float2* Hs = sh.buf[zb ^ 1] + slot * (Nc + 4);   // Hermitian half H_0 .. H_Nc (plain)
    const int u = tid - slot * 2 * tpt;
    for (int k = u; k <= Nc; k += 2 * tpt) {
      const float2 X = real_bin<Nc>(Zx, sh.tw, k);
      const float2 T = real_bin<Nc>(Zt, sh.tw, k);
      // hardware sqrt, log2 and reciprocal (about 1 ulp each)
      const float ax = __builtin_amdgcn_sqrtf(X.x * X.x + X.y * X.y);
      const float at = __builtin_amdgcn_sqrtf(T.x * T.x + T.y * T.y);
      const float d = 0.69314718055994531f *
                      (__builtin_amdgcn_logf(ax + kEps) - __builtin_amdgcn_logf(at + kEps));
      if (live) acc += scale * (double)fabsf(d);
      if (want_grad) {
        float2 G = make_float2(0.f, 0.f);
        if (live && ax > 0.0f && d != 0.0f) {
          const float gm = copysignf((float)scale, d) * __builtin_amdgcn_rcpf((ax + kEps) * ax);
          G = make_float2(gm * X.x, gm * X.y);
        }
        if (k == 0 || k == Nc) G = make_float2(2.0f * G.x, 0.0f);
        Hs[k] = G;
      }
    }
    __syncthreads();
    if (want_grad) {
      // ---- inverse: Y_k = (H_k + conj H_{Nc-k}) + i conj(tw_k) (H_k - conj H_{Nc-k}) ----
      const bool inv_active = sig == 0;             // one inverse per frame
      float2 y[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = j + q * tpt;
        const float2 hk = Hs[k], hc = cconj(Hs[Nc - k]);
        const float2 A = cadd(hk, hc), D = csub(hk, hc);
        const float2 c = cconj(sh.tw[k]);
        const float2 cd = cmul(c, D);
        y[q] = make_float2(A.x - cd.y, A.y + cd.x);   // A + i (c D)
      }
      __syncthreads();                              // H read before buffers are reused
      float2* c0 = sh.buf[0] + slot * 2 * Nc;  // the frame slot's two transform areas
      float2* c1 = sh.buf[1] + slot * 2 * Nc;
      const int yb = fft_passes<Nc, 1, 0>(y, j, 1.0f, sh.ptw, c0, c1, inv_active);
      // ---- overlap-add: frame f0 + s contributes 0.5 w(o) y(o) at o = p - s hop ----
      const int p0 = (f0 - f_begin) * hop;           // block-relative start of frame f0
      for (int p = tid; p < (fpi - 1) * hop + n; p += kThreads) {
        float g = 0.0f;
#pragma unroll
        for (int s2 = 0; s2 < fpi; ++s2) {
          const int o = p - s2 * hop;
          if (o >= 0 && o < n && f0 + s2 < f_end) {
            const float2 yy = (sh.buf[yb] + s2 * 2 * Nc)[swz(o >> 1)];
            g += 0.5f * sh.win[o] * ((o & 1) ? yy.y : yy.x);
          }
        }
        float* slotp = ola + ((p0 + p) & (kOlaSlots - 1));
        const float v = *slotp + g;
        if (p < fpi * hop) {                         // no later frame reaches it
          seg[p0 + p] = v;
          *slotp = 0.0f;
        } else {
          *slotp = v;
        }
      }
      __syncthreads();
    }
  }
  if (want_grad) {
    // the rest of the segment: the last frames' tails (3 hops past the
    // written part), then zeros
    const int done = ((f_end - f_begin + fpi - 1) / fpi) * fpi * hop;
    for (int p = done + tid; p < kSegHops * hop; p += kThreads)
      seg[p] = p < done + 3 * hop ? ola[p & (kOlaSlots - 1)] : 0.0f;
  }
  // fixed-order reduction of the per-thread loss shares
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
  if ((tid & 63) == 0) sh.red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += sh.red[w];
    a.partial[b * a.chunk_base[3] + blk] = s;
  }
}

__global__ void __launch_bounds__(kThreads) mrstft_frames_kernel(const MrArgs a) {
  __shared__ SpecShared sh;
  __shared__ float ola[kOlaSlots];
  const int64_t b = blockIdx.y;
  const int blk = blockIdx.x;
  if (blk < a.chunk_base[1])
    mrstft_frames<0>(a, sh, ola, b, blk);
  else if (blk < a.chunk_base[2])
    mrstft_frames<1>(a, sh, ola, b, blk);
  else
    mrstft_frames<2>(a, sh, ola, b, blk);
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

__global__ void __launch_bounds__(kMelThreads) __attribute__((amdgpu_waves_per_eu(2)))
logmel_fft_kernel(const float* __restrict__ audio, const int64_t* __restrict__ offsets,
                  int64_t n_uniform, const uint16_t* __restrict__ mel, int64_t ldm,
                  float* __restrict__ features) {
  constexpr int Nc = 1024, P = 16, hop = 2756, frames = 64;
  __shared__ float2 wbuf[kMelWaves][Nc];
  __shared__ MelShared ms;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int64_t b = blockIdx.x;
  int64_t start, len;
  if (offsets) {
    start = offsets[b];
    len = offsets[b + 1] - start;
  } else {
    start = b * n_uniform;
    len = n_uniform;
  }
  const float* x = audio + start;
  float* feat = features + b * (int64_t)(kMelBands * frames);

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
      if (fr < cnt) feat[bd * frames + 16 * g + fr] = ms.st[bd][fr];
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
      feat[bd * frames + live + (e - bd * nz)] = floor_v;
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
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  float g = 0.0f;
  for (int r = 0; r < 3; ++r) {
    const int n = 512 << r, hop = n / 4;
    const int nch = a.chunk_base[r + 1] - a.chunk_base[r];
    if (nch == 0) continue;
    const int64_t h = i / hop;                       // hop of sample i
    int64_t khi = h / kFramesPerBlock;
    if (khi > nch - 1) khi = nch - 1;
    const int64_t klo = h >= kSegHops ? (h - kSegHops) / kFramesPerBlock + 1 : 0;
    const int64_t seglen = (int64_t)kSegHops * hop;
    const float* segs = a.wgrad + a.wbase[r] + b * nch * seglen;
    for (int64_t k = klo; k <= khi; ++k)
      g += segs[k * seglen + (i - k * kFramesPerBlock * hop)];
  }
  a.grad[b * a.n + i] = g;
}

void plan(int64_t batch, int64_t n_samples, MrArgs& a, size_t& partial_bytes, size_t& wgrad_floats) {
  int cb = 0;
  int64_t wb = 0;
  for (int r = 0; r < 3; ++r) {
    const int n = 512 << r;
    const int64_t F = n_samples < n ? 0 : (n_samples - n) / (n / 4) + 1;
    a.F[r] = (int)F;
    a.chunk_base[r] = cb;
    cb += (int)((F + kFramesPerBlock - 1) / kFramesPerBlock);
    a.wbase[r] = wb;
    wb += batch * ((F + kFramesPerBlock - 1) / kFramesPerBlock) * kSegHops * (n / 4);
    a.scale[r] = F > 0 ? 1.0 / ((double)F * (double)(n / 2 + 1)) : 0.0;
  }
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
  hipLaunchKernelGGL(logmel_fft_kernel, dim3((unsigned)batch), dim3(kMelThreads), 0, s, audio,
                     offsets, n_uniform, (const uint16_t*)mel_basis, ldm, features);
  return hipGetLastError();
}

size_t mrstft_workspace_bytes(int64_t batch, int64_t n_samples, bool with_grad) {
  MrArgs a = {};
  size_t pb, wf;
  plan(batch, n_samples, a, pb, wf);
  pb = (pb + 255) & ~(size_t)255;
  return pb + (with_grad ? wf * sizeof(float) : 0);
}

hipError_t launch_mrstft(const float* x, const float* target, int64_t batch, int64_t n_samples,
                         double* loss, float* grad, void* workspace, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  MrArgs a = {};
  size_t pb, wf;
  plan(batch, n_samples, a, pb, wf);
  pb = (pb + 255) & ~(size_t)255;
  a.x = x;
  a.t = target;
  a.n = n_samples;
  a.batch = batch;
  a.partial = reinterpret_cast<double*>(workspace);
  a.wgrad = grad ? reinterpret_cast<float*>(reinterpret_cast<char*>(workspace) + pb) : nullptr;
  a.grad = grad;
  a.loss = loss;
  if (batch > 65535) return hipErrorInvalidValue;
  if (a.chunk_base[3] > 0) {
    hipLaunchKernelGGL(mrstft_frames_kernel, dim3((unsigned)a.chunk_base[3], (unsigned)batch),
                       dim3(kThreads), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // (with no complete frame at any resolution the combine kernel writes
  // loss 0 and a zero gradient)
  const int64_t gx = grad ? (n_samples + 255) / 256 : 1;
  hipLaunchKernelGGL(mrstft_combine_kernel, dim3((unsigned)gx, (unsigned)batch), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace synth
