// bf16 MFMA GEMM for gfx950 with fused epilogues: C[M x N] = A[M x K] B[K x N],
// float32 accumulation (v_mfma_f32_32x32x16_bf16).
//
// Operand layouts: kOpKMajor (row r of the operand has K contiguous:
// X[r * ld + k]) and kOpRowMajorMN (X[k * ld + r]).
//
// Tiles of 128 x 128 x 32 per 256-thread workgroup (four wavefronts in 2 x 2,
// each 64 x 64 as 2 x 2 MFMA 32 x 32 blocks).  Tiles are staged in LDS as
// [row][k] with K contiguous (rows padded by 16 bytes), so every lane's
// 8-element MFMA fragment is one 16-byte LDS read.
//
// MFMA 32x32x16 lane layout (verified on gfx950): A fragment = row (lane % 32),
// k = 8 (lane / 32) .. +7; B fragment = column (lane % 32), same k; the 16
// accumulators of a lane are column (lane % 32), rows 8 (v / 4) + 4 (lane / 32)
// + (v % 4), v = 0..15.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "synth_internal.h"

namespace synth {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int BM = 128, BN = 128, BK = 32, PADK = BK + 8;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bf16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float gelu_erf(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752440f));
}
// d/dx x Phi(x) = Phi(x) + x phi(x)
__device__ __forceinline__ float gelu_erf_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752440f)) +
         x * 0.39894228040143267794f * expf(-0.5f * x * x);
}

__device__ __forceinline__ bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// Stage a 128 x 32 tile (rows row0.., k k0..) of an operand into dst[row][k].
template <int OP>
__device__ __forceinline__ void stage(uint16_t (*dst)[PADK], const GemmArgs& g, const void* srcv,
                                      int64_t ld, int64_t row0, int64_t nrows, int64_t k0) {
  const int t = threadIdx.x;
  const int64_t K = g.K;
  if constexpr (OP == kOpKMajor) {
    const uint16_t* src = reinterpret_cast<const uint16_t*>(srcv);
    const int r = t >> 1;                 // 128 rows, 2 threads per row
    const int kk = (t & 1) * 16;
    const int64_t gr = row0 + r;
    const bool full = gr < nrows && k0 + kk + 16 <= K && ((ld & 7) == 0) && aligned16(src);
    if (full) {
      const uint4* p = reinterpret_cast<const uint4*>(src + gr * ld + k0 + kk);
      *reinterpret_cast<uint4*>(&dst[r][kk]) = p[0];
      *reinterpret_cast<uint4*>(&dst[r][kk + 8]) = p[1];
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t gk = k0 + kk + e;
        dst[r][kk + e] = (gr < nrows && gk < K) ? src[gr * ld + gk] : (uint16_t)0;
      }
    }
  } else if constexpr (OP == kOpRowMajorMN) {
    const uint16_t* src = reinterpret_cast<const uint16_t*>(srcv);
    const int kk = t >> 3;                // 32 k rows, 8 threads per k
    const int r0 = (t & 7) * 16;
    const int64_t gk = k0 + kk;
    uint16_t v[16];
    const bool full = gk < K && row0 + r0 + 16 <= nrows && ((ld & 7) == 0) && aligned16(src);
    if (full) {
      const uint4* p = reinterpret_cast<const uint4*>(src + gk * ld + row0 + r0);
      const uint4 a = p[0], b = p[1];
      const uint16_t* pa = reinterpret_cast<const uint16_t*>(&a);
      const uint16_t* pb = reinterpret_cast<const uint16_t*>(&b);
#pragma unroll
      for (int e = 0; e < 8; ++e) { v[e] = pa[e]; v[8 + e] = pb[e]; }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t gr = row0 + r0 + e;
        v[e] = (gk < K && gr < nrows) ? src[gk * ld + gr] : (uint16_t)0;
      }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) dst[r0 + e][kk] = v[e];
  }
}

template <int AOP, int BOP>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[BM][PADK];
  __shared__ __align__(16) uint16_t Bs[BN][PADK];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  const int64_t tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int64_t m0 = tm * BM, n0 = tn * BN;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  for (int64_t k0 = 0; k0 < g.K; k0 += BK) {
    stage<AOP>(As, g, g.A, g.lda, m0, g.M, k0);
    stage<BOP>(Bs, g, g.B, g.ldb, n0, g.N, k0);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const int kq = ks + 8 * (lane >> 5);
      bf16x8 af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        af[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 64 + i * 32 + (lane & 31)][kq]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 64 + j * 32 + (lane & 31)][kq]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  // ---- epilogue ----
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = n0 + wn * 64 + j * 32 + (lane & 31);
      const bool col_ok = col < g.N;
      const float bias = (g.bias && col_ok) ? g.bias[col] : 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        float x = acc[i][j][v] * g.alpha + bias;
        if (g.epilogue == kEpiPowerPairs) {
          // (Re, Im) sit in adjacent columns = adjacent lanes; every lane shuffles
          const float other = __shfl_xor(x, 1);
          if ((col & 1) == 0 && col_ok && row < g.M) {
            const float p = x * x + other * other;
            const int64_t o = row * g.ldc + (col >> 1);
            if (g.c_bf16) reinterpret_cast<uint16_t*>(g.C)[o] = f2bf(p);
            else reinterpret_cast<float*>(g.C)[o] = p;
          }
          continue;
        }
        if (!col_ok || row >= g.M) continue;
        if (g.epilogue == kEpiLogMelT) {
          const int64_t o = (row / 64) * 8192 + col * 64 + (row % 64);
          reinterpret_cast<float*>(g.C)[o] = logf(x + 1e-6f);
          continue;
        }
        const int64_t o = row * g.ldc + col;
        if (g.pre) g.pre[o] = x;
        if (g.epilogue == kEpiGelu) x = gelu_erf(x);
        else if (g.epilogue == kEpiSigmoid) x = 1.0f / (1.0f + expf(-x));
        else if (g.epilogue == kEpiGeluGrad) x = x * gelu_erf_grad(g.aux[o]);
        if (g.beta != 0.0f)
          x += g.beta * (g.c_bf16 ? bf2f(reinterpret_cast<const uint16_t*>(g.C)[o])
                                  : reinterpret_cast<const float*>(g.C)[o]);
        if (g.c_bf16) reinterpret_cast<uint16_t*>(g.C)[o] = f2bf(x);
        else reinterpret_cast<float*>(g.C)[o] = x;
      }
    }
}

template <int AOP>
hipError_t launch_b(const GemmArgs& g, int b_op, dim3 grid, hipStream_t s) {
  if (b_op == kOpKMajor)
    hipLaunchKernelGGL((gemm_bf16_kernel<AOP, kOpKMajor>), grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<AOP, kOpRowMajorMN>), grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_bf16(const GemmArgs& g, int a_op, int b_op, hipStream_t s) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  if (tiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 grid((unsigned)tiles);
  switch (a_op) {
    case kOpKMajor: return launch_b<kOpKMajor>(g, b_op, grid, s);
    case kOpRowMajorMN: return launch_b<kOpRowMajorMN>(g, b_op, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace synth
