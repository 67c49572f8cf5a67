// Multi-resolution log-magnitude STFT L1 loss and its gradient (float32 FFT).
//
// The paper scores sounds with a multi-scale spectrogram distance over several
// FFT sizes and prefers L1 (Section 4.3).  Per voice:
//   loss = sum over n in (512, 1024, 2048), hop n/4, of
//          mean_{frame t, bin k <= n/2} |log(|X_tk| + 1e-5) - log(|T_tk| + 1e-5)|
// with X, T the periodic-Hann STFTs (no padding) of the render x and target.
//
// One 1024-thread workgroup per voice walks the voice in blocks of 512
// samples.  For every resolution a block is one group of S = 2048/n frames
// (S * hop = 512), so each thread owns exactly one radix-2 butterfly per FFT
// stage.  Render and target frames get separate FFTs.  The gradient
// w.r.t. x of a frame is w(m) Re(sum_k G_k e^{2 pi i k m / n}) with
// G_k = sign(d_k) X_k / (|X_k| (|X_k| + eps)) / (F (n/2 + 1)); it is formed by
// an inverse FFT of the Hermitian extension of G and overlap-added into an LDS
// ring covering [block, block + 2560).  After a block no later frame reaches
// its first 512 samples, which are then written once: no atomics, no
// read-modify-write of global memory, bitwise deterministic.
#include <math.h>

#include "synth_internal.h"

namespace synth {
namespace {

constexpr int kThreads = 1024;
constexpr int kMaxN = 2048;
constexpr int kBlock = 512;                 // output samples finalised per step
constexpr int kRing = kBlock + kMaxN;       // 2560
constexpr float kEps = 1e-5f;

struct SpecShared {
  float2 buf[2][kMaxN];                     // FFT ping-pong
  float ring[kRing];                        // gradient overlap-add window
  double red[kThreads / 64];                // per-wave loss partial sums
};

// Stockham radix-2 autosort FFT of S independent length-n sequences stored
// back to back in buf[src] (S * n == 2048).  dir = -1 forward, +1 inverse
// (unnormalised).  Thread t owns butterfly t of the stage.  Returns the index
// of the buffer holding the result.
__device__ int fft_group(SpecShared& sh, int src, int n, int logn, float dir) {
  const int t = threadIdx.x;
  const int half = n >> 1;
  const int slot = t / half;
  const int b = t - slot * half;
  int len = n;       // current sub-transform length
  int stride = 1;    // number of interleaved sub-transforms
  for (int st = 0; st < logn; ++st) {
    const int m = len >> 1;
    const int p = b / stride;
    const int qq = b - p * stride;
    const float2* x = sh.buf[src] + slot * n;
    float2* y = sh.buf[src ^ 1] + slot * n;
    const float2 a = x[qq + stride * p];
    const float2 c = x[qq + stride * (p + m)];
    float sn, cs;
    sincospif(dir * 2.0f * (float)p / (float)len, &sn, &cs);
    const float2 d = make_float2(a.x - c.x, a.y - c.y);
    y[qq + stride * (2 * p)] = make_float2(a.x + c.x, a.y + c.y);
    y[qq + stride * (2 * p + 1)] = make_float2(d.x * cs - d.y * sn, d.x * sn + d.y * cs);
    src ^= 1;
    len = m;
    stride <<= 1;
    __syncthreads();
  }
  return src;
}

__device__ __forceinline__ float hann_f(int m, int n) {
  return 0.5f - 0.5f * cospif(2.0f * (float)m / (float)n);
}

__global__ void __launch_bounds__(kThreads) mrstft_kernel(const float* __restrict__ x,
                                                          const float* __restrict__ target,
                                                          int64_t N, double* __restrict__ loss,
                                                          float* __restrict__ grad) {
  __shared__ SpecShared sh;
  const int t = threadIdx.x;
  const int64_t b = blockIdx.x;
  const float* xv = x + b * N;
  const float* tv = target + b * N;
  float* gv = grad ? grad + b * N : nullptr;
  double acc = 0.0;                          // this thread's share of the loss

  int F[3], logn[3];
  double scale[3];
  for (int r = 0; r < 3; ++r) {
    const int n = 512 << r;
    logn[r] = 9 + r;
    F[r] = N < n ? 0 : (int)((N - n) / (n / 4)) + 1;
    scale[r] = F[r] > 0 ? 1.0 / ((double)F[r] * (double)(n / 2 + 1)) : 0.0;
  }
  if (gv)
    for (int i = t; i < kRing; i += kThreads) sh.ring[i] = 0.0f;
  __syncthreads();

  const int64_t nblocks = (N + kBlock - 1) / kBlock;
  for (int64_t blk = 0; blk < nblocks; ++blk) {
    const int64_t base = blk * kBlock;
    for (int r = 0; r < 3; ++r) {
      const int n = 512 << r;
      const int hop = n / 4;
      const int S = kMaxN / n;
      const int64_t f0 = blk * S;            // first frame of this group
      if (f0 >= F[r]) continue;              // uniform across the workgroup
      // bins owned by this thread: k = t mod (n/2) of its frame slot, plus
      // k = n/2 for the thread with k == 0
      const int half = n >> 1;
      const int slot = t / half;
      const int k = t - slot * half;
      const int64_t fr = f0 + slot;
      const bool live = fr < F[r];
      // Two real-input FFTs, render then target, each with its own float32
      // noise floor (sharing one complex FFT would leak the louder signal's
      // rounding noise into the quieter one's spectrum).
      float2 Xa, Xb, Ta, Tb;
      int res = 0;
      for (int which = 0; which < 2; ++which) {
        const float* sig = which == 0 ? xv : tv;
        for (int e = t; e < kMaxN; e += kThreads) {
          const int sl = e / n;
          const int m = e - sl * n;
          const int64_t frm = f0 + sl;
          float v = 0.0f;
          if (frm < F[r]) v = hann_f(m, n) * sig[frm * hop + m];
          sh.buf[0][e] = make_float2(v, 0.0f);
        }
        __syncthreads();
        res = fft_group(sh, 0, n, logn[r], -1.0f);
        const float2* Z = sh.buf[res] + slot * n;
        const float2 za = Z[k];
        const float2 zb = k == 0 ? Z[half] : make_float2(0.f, 0.f);
        if (which == 0) { Xa = za; Xb = zb; } else { Ta = za; Tb = zb; }
        __syncthreads();                     // buffers are reused
      }
      float2 G0 = make_float2(0.f, 0.f), G1 = make_float2(0.f, 0.f);
      for (int pass = 0; pass < (k == 0 ? 2 : 1); ++pass) {
        const float2 X = pass == 0 ? Xa : Xb;
        const float2 T = pass == 0 ? Ta : Tb;
        const float ax = sqrtf(X.x * X.x + X.y * X.y);
        const float at = sqrtf(T.x * T.x + T.y * T.y);
        const float d = logf(ax + kEps) - logf(at + kEps);
        if (live) acc += scale[r] * (double)fabsf(d);
        float2 G = make_float2(0.f, 0.f);
        if (live && ax > 0.0f && d != 0.0f) {
          const float gm = copysignf((float)scale[r], d) / ((ax + kEps) * ax);
          G = make_float2(gm * X.x, gm * X.y);
        }
        if (pass == 0) G0 = G; else G1 = G;
      }
      if (gv) {
        // Hermitian extension H of G (H_0 = 2 Re G_0, H_{n/2} = 2 Re G_{n/2},
        // H_{n-k} = conj G_k)
        float2* H = sh.buf[0] + slot * n;
        if (k == 0) {
          H[0] = make_float2(2.0f * G0.x, 0.0f);
          H[half] = make_float2(2.0f * G1.x, 0.0f);
        } else {
          H[k] = G0;
          H[n - k] = make_float2(G0.x, -G0.y);
        }
        __syncthreads();
        const int ri = fft_group(sh, 0, n, logn[r], 1.0f);
        // frame gradient 0.5 w(m) Re(h(m)), overlap-added in frame order
        for (int s = 0; s < S; ++s) {
          if (f0 + s < F[r]) {
            const int off = s * hop;          // ring position of frame s's first sample
            for (int m = t; m < n; m += kThreads)
              sh.ring[off + m] += 0.5f * hann_f(m, n) * sh.buf[ri][s * n + m].x;
          }
          __syncthreads();
        }
      }
    }
    if (gv) {
      // samples [base, base + 512) are final: write, then slide the ring
      for (int i = t; i < kBlock; i += kThreads)
        if (base + i < N) gv[base + i] = sh.ring[i];
      __syncthreads();
      float carry[3];
      int nc = 0;
      for (int i = t; i < kRing - kBlock; i += kThreads) carry[nc++] = sh.ring[i + kBlock];
      __syncthreads();
      nc = 0;
      for (int i = t; i < kRing - kBlock; i += kThreads) sh.ring[i] = carry[nc++];
      for (int i = kRing - kBlock + t; i < kRing; i += kThreads) sh.ring[i] = 0.0f;
      __syncthreads();
    }
  }
  // fixed-order reduction of the per-thread loss shares
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o);
  if ((t & 63) == 0) sh.red[t >> 6] = acc;
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += sh.red[w];
    loss[b] = s;
  }
}

}  // namespace

hipError_t launch_mrstft(const float* x, const float* target, int64_t batch, int64_t n_samples,
                         double* loss, float* grad, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(mrstft_kernel, dim3((unsigned)batch), dim3(kThreads), 0, s, x, target,
                     n_samples, loss, grad);
  return hipGetLastError();
}

}  // namespace synth
