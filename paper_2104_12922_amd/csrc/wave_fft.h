// Wave-level complex FFT for gfx950: one 64-lane wavefront transforms NC =
// 64 P points (NC = 256, 512, 1024) with no workgroup barrier.
//
// Stockham autosort passes of radix R (1024: 16, 16, 4; 512: 8, 8, 8;
// 256: 4, 4, 4, 4).  In a pass of stride NS, butterfly j (lane + 64 q)
// takes inputs j + r NC / R, multiplies input r by W_{NS R}^{(j mod NS) r},
// does an R-point DFT in registers and writes output r to
// (j / NS) NS R + (j mod NS) + r NS.  The first pass has one butterfly per
// lane whose inputs are the lane's own points z[lane + 64 r], so a caller
// loads them straight from memory; the result ends in natural order in a
// wave-private LDS buffer of NC float2, read through swz().  Twiddles are
// read from a shared per-pass LDS table (build_pass_twiddles).
//
// LDS traffic stays inside the wavefront: its LDS instructions execute in
// program order, so only the compiler has to be kept from moving a write
// across a read of another lane's value (wave_fence).
#pragma once

#include <hip/hip_runtime.h>

namespace synth {
namespace wfft {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool FWD>
__device__ __forceinline__ float2 rot(float2 a) {
  return FWD ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

__device__ __forceinline__ void wave_fence() { asm volatile("" ::: "memory"); }

// Slot swizzle of the exchange buffer (a bijection inside every 32 slots): the
// strided writes of the first passes land on distinct LDS banks.
template <int NC>
__device__ __forceinline__ int swz(int i) {
  constexpr int sh = NC == 1024 ? 4 : 3;
  return i ^ ((i >> sh) & 31);
}

template <int NC> struct Plan;
template <> struct Plan<1024> {
  static constexpr int passes = 3;
  static constexpr int radix(int p) { return p < 2 ? 16 : 4; }
};
template <> struct Plan<512> {
  static constexpr int passes = 3;
  static constexpr int radix(int p) { return 8; }
};
template <> struct Plan<256> {
  static constexpr int passes = 4;
  static constexpr int radix(int p) { return 4; }
};

template <int NC>
constexpr int stride_of(int p) {   // NS of pass p
  return p == 0 ? 1 : stride_of<NC>(p - 1) * Plan<NC>::radix(p - 1);
}
// Per-pass twiddle table: pass p (>= 1) keeps W_{NS R}^{k r} at
// pt_offset(p) + (r - 1) NS + k, so the lanes of a butterfly row read
// consecutive entries.
template <int NC>
constexpr int pt_offset(int p) {
  return p <= 1 ? 0 : pt_offset<NC>(p - 1) + (Plan<NC>::radix(p - 1) - 1) * stride_of<NC>(p - 1);
}
template <int NC>
constexpr int pt_size() { return pt_offset<NC>(Plan<NC>::passes); }

// Fills the per-pass table (forward twiddles) with threads t < nthreads.
template <int NC, int p = 1>
__device__ __forceinline__ void build_pass_twiddles(float2* PT, int t, int nthreads) {
  if constexpr (p < Plan<NC>::passes) {
    constexpr int NS = stride_of<NC>(p), R = Plan<NC>::radix(p), OFF = pt_offset<NC>(p);
    for (int i = t; i < (R - 1) * NS; i += nthreads) {
      const int r = i / NS + 1, k = i % NS;
      float sn, cs;
      sincospif(-2.0f * (float)(k * r) / (float)(NS * R), &sn, &cs);
      PT[OFF + i] = make_float2(cs, sn);
    }
    build_pass_twiddles<NC, p + 1>(PT, t, nthreads);
  }
}

// ---- R-point DFTs in registers ----
template <bool FWD>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = add(a0, a2), t1 = sub(a0, a2), t2 = add(a1, a3);
  const float2 t3 = rot<FWD>(sub(a1, a3));
  a0 = add(t0, t2);
  a1 = add(t1, t3);
  a2 = sub(t0, t2);
  a3 = sub(t1, t3);
}

// W_R^e for the forward direction; the inverse uses the conjugate
__device__ __forceinline__ float2 wconst(int R, int e) {
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
  const int k = (e * (16 / R)) & 15;   // in sixteenths of a turn
  switch (k) {
    case 0: return make_float2(1.0f, 0.0f);
    case 1: return make_float2(c1, -s1);
    case 2: return make_float2(h, -h);
    case 3: return make_float2(s1, -c1);
    case 4: return make_float2(0.0f, -1.0f);
    case 5: return make_float2(-s1, -c1);
    case 6: return make_float2(-h, -h);
    case 7: return make_float2(-c1, -s1);
    case 8: return make_float2(-1.0f, 0.0f);
    case 9: return make_float2(-c1, s1);
    case 10: return make_float2(-h, h);
    case 11: return make_float2(-s1, c1);
    case 12: return make_float2(0.0f, 1.0f);
    case 13: return make_float2(s1, c1);
    case 14: return make_float2(h, h);
    default: return make_float2(c1, s1);
  }
}
template <bool FWD>
__device__ __forceinline__ float2 mulw(float2 a, int R, int e) {
  const float2 w = wconst(R, e);
  return FWD ? cmul(a, w) : cmulc(a, w);
}

template <int R, bool FWD>
__device__ __forceinline__ void dft(float2 (&x)[R]) {
  if constexpr (R == 4) {
    dft4<FWD>(x[0], x[1], x[2], x[3]);
  } else if constexpr (R == 8) {
    // n = 2 m + e: two 4-point DFTs, twiddle W_8^{e k}, then radix 2
    float2 E[4] = {x[0], x[2], x[4], x[6]}, O[4] = {x[1], x[3], x[5], x[7]};
    dft4<FWD>(E[0], E[1], E[2], E[3]);
    dft4<FWD>(O[0], O[1], O[2], O[3]);
#pragma unroll
    for (int k = 1; k < 4; ++k) O[k] = mulw<FWD>(O[k], 8, k);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[k] = add(E[k], O[k]);
      x[k + 4] = sub(E[k], O[k]);
    }
  } else {
    // n = 4 m + e, k = k1 + 4 k2: DFT over m, twiddle W_16^{e k1}, DFT over e
    float2 A[4][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      A[e][0] = x[e];
      A[e][1] = x[4 + e];
      A[e][2] = x[8 + e];
      A[e][3] = x[12 + e];
      dft4<FWD>(A[e][0], A[e][1], A[e][2], A[e][3]);
#pragma unroll
      for (int k1 = 1; k1 < 4; ++k1)
        if (e > 0) A[e][k1] = mulw<FWD>(A[e][k1], 16, e * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 b0 = A[0][k1], b1 = A[1][k1], b2 = A[2][k1], b3 = A[3][k1];
      dft4<FWD>(b0, b1, b2, b3);
      x[k1] = b0;
      x[k1 + 4] = b1;
      x[k1 + 8] = b2;
      x[k1 + 12] = b3;
    }
  }
}

// Pass p: butterflies on v (this pass's inputs), outputs to buf, then the
// next pass's inputs back into v.  Twiddles come from the per-pass table PT.
template <int NC, int p, bool FWD>
__device__ __forceinline__ void run_passes(float2 (&v)[NC / 64], float2* buf, const float2* T,
                                           int lane) {
  if constexpr (p < Plan<NC>::passes) {
    constexpr int P = NC / 64, R = Plan<NC>::radix(p), NS = stride_of<NC>(p), NB = P / R;
    constexpr int OFF = pt_offset<NC>(p);
    wave_fence();                       // earlier reads of buf stay before these writes
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int j = lane + 64 * q;
      const int k = j & (NS - 1);
      float2 x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = v[q * R + r];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 w = T[OFF + (r - 1) * NS + k];
          x[r] = FWD ? cmul(x[r], w) : cmulc(x[r], w);
        }
      }
      dft<R, FWD>(x);
      const int d = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[swz<NC>(d + r * NS)] = x[r];
    }
    wave_fence();
    if constexpr (p + 1 < Plan<NC>::passes) {
      constexpr int R2 = Plan<NC>::radix(p + 1), NB2 = P / R2;
#pragma unroll
      for (int q = 0; q < NB2; ++q)
#pragma unroll
        for (int r = 0; r < R2; ++r) v[q * R2 + r] = buf[swz<NC>(lane + 64 * q + r * (NC / R2))];
    }
    run_passes<NC, p + 1, FWD>(v, buf, T, lane);
  }
}

// v[r] = z[lane + 64 r] on entry; on return Z[k] = buf[swz<NC>(k)] for the
// whole wavefront (natural order).
template <int NC, bool FWD>
__device__ __forceinline__ void wave_fft(float2 (&v)[NC / 64], float2* buf, const float2* T,
                                         int lane) {
  run_passes<NC, 0, FWD>(v, buf, T, lane);
  wave_fence();
}

}  // namespace wfft
}  // namespace synth
