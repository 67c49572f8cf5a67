// Power spectrum of the log-mel frames as one bf16 MFMA GEMM (gfx950):
//   P[m][f] = |sum_k x_m(k) w(k) e^{-2 pi i f k / 2048}|^2,  f = 0..1024,
// m = voice * 64 + frame, x_m the frame's samples (hop 2756, zero past the
// voice's end), w the periodic Hann window.
//
// The window is folded into the basis B[n][k] (n = 0..2047, K-major):
//   n = 0: w(k) (bin 0, real), n = 1: w(k) (-1)^k (bin 1024, real),
//   n = 2f, 2f + 1 (f = 1..1023): w(k) cos(2 pi f k / 2048), -w(k) sin(...),
// so bins 0 and 1024, whose imaginary parts vanish, share one column pair and
// N is exactly 2048.  The frames operand is read straight from the float32
// audio and rounded to bf16 while it is staged (v_cvt_pk_bf16_f32).
//
// Workgroup tile 256 (M) x 256 (N) x 32 (K), 512 threads = 8 wavefronts in
// 2 (M) x 4 (N), each owning 128 x 64 = 4 x 2 blocks of
// v_mfma_f32_32x32x16_bf16 (two wavefronts per SIMD).
// Global loads for k-step s + 1 are issued before the MFMAs of step s and
// land in the other LDS buffer afterwards (one barrier per k-step).  Tiles
// are assigned so that consecutive tiles of one M row share an XCD (and its
// L2), which reads every frame from HBM about once.
//
// MFMA 32x32x16 lane layout: A fragment = row (lane % 32), k = 8 (lane / 32)
// .. +7; B fragment = column (lane % 32), same k; the 16 accumulators of a
// lane are column (lane % 32), rows 8 (v / 4) + 4 (lane / 32) + (v % 4).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "synth_internal.h"

namespace synth {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kN = 2048;            // DFT size == K == N of the GEMM
constexpr int kBM = 256, kBN = 256, kBK = 32, kLDK = kBK + 8, kThreads = 512;
constexpr int kKSteps = kN / kBK;   // 64
constexpr int kXcds = 8;

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__global__ void __launch_bounds__(kThreads) dft_power_kernel(const float* __restrict__ audio,
                                                        const int64_t* __restrict__ offsets,
                                                        int64_t n_uniform, int64_t rows,
                                                        const uint16_t* __restrict__ basis,
                                                        uint16_t* __restrict__ power,
                                                        int64_t ldp) {
  __shared__ __align__(16) uint16_t As[2][kBM][kLDK];
  __shared__ __align__(16) uint16_t Bs[2][kBN][kLDK];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;

  // XCD-aware tile order: workgroup b runs on XCD b % 8; give each XCD a
  // contiguous range of tiles (N-tiles of one M row are consecutive).
  constexpr int64_t tiles_n = kN / kBN;   // 8
  const int64_t nblk = gridDim.x;
  const int64_t b = blockIdx.x;
  const int64_t per = nblk / kXcds, extra = nblk % kXcds;
  const int64_t x = b % kXcds, i = b / kXcds;
  const int64_t tile = x * per + (x < extra ? x : extra) + i;
  const int64_t m0 = (tile / tiles_n) * kBM, n0 = (tile % tiles_n) * kBN;

  // A staging: 8 threads per row (one float4 each), 64 rows per pass, 4
  // passes.  The 256 rows of the tile are 4 whole voices (64 frames each):
  // pass p reads frame a_r of voice m0 / 64 + p.
  const int a_c = (t & 7) * 4;
  const int a_r = t >> 3;
  const int64_t batch = rows >> 6;
  int64_t vstart[4], vlen[4];
  bool vvec[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t v = (m0 >> 6) + q;
    vstart[q] = 0;
    vlen[q] = 0;
    if (v < batch) {
      if (offsets) {
        vstart[q] = offsets[v];
        vlen[q] = offsets[v + 1] - vstart[q];
      } else {
        vstart[q] = v * n_uniform;
        vlen[q] = n_uniform;
      }
    }
    vvec[q] = ((reinterpret_cast<uintptr_t>(audio + vstart[q]) & 15u) == 0);
  }
  const int pos = a_r * 2756;          // frame start (hop 2756)
  // B staging: 4 threads per row (16 bytes each), 128 rows per pass, 2 passes.
  const int b_c = (t & 3) * 8;
  const int b_r = t >> 2;

  float4 ra[4];
  uint4 rb[2];

  auto load = [&](int ks) {
    const int k0 = ks * kBK + a_c;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t av = vlen[q] - pos - k0;          // samples left in the voice
      const float* src = audio + vstart[q] + pos + k0;
      if (vvec[q] && av >= 4) {
        ra[q] = *reinterpret_cast<const float4*>(src);
      } else {
        ra[q].x = av > 0 ? src[0] : 0.0f;
        ra[q].y = av > 1 ? src[1] : 0.0f;
        ra[q].z = av > 2 ? src[2] : 0.0f;
        ra[q].w = av > 3 ? src[3] : 0.0f;
      }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
      rb[p] = *reinterpret_cast<const uint4*>(basis + (n0 + p * 128 + b_r) * (int64_t)kN +
                                              ks * kBK + b_c);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint2 w;
      w.x = pack_bf16(ra[q].x, ra[q].y);
      w.y = pack_bf16(ra[q].z, ra[q].w);
      *reinterpret_cast<uint2*>(&As[buf][q * 64 + a_r][a_c]) = w;
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) *reinterpret_cast<uint4*>(&Bs[buf][p * 128 + b_r][b_c]) = rb[p];
  };

  f32x16 acc[4][2];
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[ii][j][v] = 0.0f;

  load(0);
  store(0);
  __syncthreads();
  for (int ks = 0; ks < kKSteps; ++ks) {
    const int buf = ks & 1;
    if (ks + 1 < kKSteps) load(ks + 1);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
      const int kq = kk + 8 * (lane >> 5);
      bf16x8 af[4], bf[2];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
        af[ii] = *reinterpret_cast<const bf16x8*>(&As[buf][wm * 128 + ii * 32 + (lane & 31)][kq]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bf[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn * 64 + j * 32 + (lane & 31)][kq]);
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[ii][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[ii], bf[j], acc[ii][j], 0, 0, 0);
    }
    if (ks + 1 < kKSteps) store(buf ^ 1);
    __syncthreads();
  }

  // Epilogue: (Re, Im) of a bin sit in adjacent columns = adjacent lanes.
  // Column pair (0, 1) holds the real bins 0 and 1024.
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = (int)n0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float xv = acc[ii][j][v];
        const float other = __shfl_xor(xv, 1);            // every lane takes part
        const int64_t row = m0 + wm * 128 + ii * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (row >= rows) continue;
        uint16_t* prow = power + row * ldp;
        if (col == 0) {
          prow[0] = f2bf(xv * xv);
        } else if (col == 1) {
          prow[kN / 2] = f2bf(xv * xv);
        } else if ((col & 1) == 0) {
          prow[col >> 1] = f2bf(xv * xv + other * other);
        }
      }
    }
}

// Basis rows as described above, float64 angle and window, rounded to bf16.
__global__ void dft_basis_kernel(uint16_t* __restrict__ basis) {
  const int64_t total = (int64_t)kN * kN;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(idx / kN), k = (int)(idx % kN);
    const double w = 0.5 - 0.5 * cospi(2.0 * (double)k / (double)kN);
    double val;
    if (n == 0) {
      val = w;
    } else if (n == 1) {
      val = (k & 1) ? -w : w;
    } else {
      const int64_t f = n >> 1;
      const int64_t ph = (f * k) % kN;                  // exact angle reduction
      const double a = 2.0 * (double)ph / (double)kN;
      val = (n & 1) ? -w * sinpi(a) : w * cospi(a);
    }
    basis[idx] = f2bf((float)val);
  }
}

}  // namespace

hipError_t launch_dft_power(const float* audio, const int64_t* offsets, int64_t n_uniform,
                            int64_t batch, const void* basis, void* power, int64_t ldp,
                            hipStream_t s) {
  const int64_t rows = batch * 64;
  if (rows == 0) return hipSuccess;
  const int64_t tiles = ((rows + kBM - 1) / kBM) * (kN / kBN);
  if (tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dft_power_kernel, dim3((unsigned)tiles), dim3(kThreads), 0, s, audio, offsets,
                     n_uniform, rows, (const uint16_t*)basis, (uint16_t*)power, ldp);
  return hipGetLastError();
}

hipError_t launch_dft_basis(void* basis_bf16, hipStream_t s) {
  hipLaunchKernelGGL(dft_basis_kernel, dim3(4096), dim3(256), 0, s, (uint16_t*)basis_bf16);
  return hipGetLastError();
}

}  // namespace synth
