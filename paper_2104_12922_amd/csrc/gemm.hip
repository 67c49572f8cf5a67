// bf16 MFMA GEMM for gfx950 with fused epilogues: C[M x N] = A[M x K] B[K x N],
// float32 accumulation (v_mfma_f32_32x32x16_bf16).
//
// Operand layouts: kOpKMajor (row r of the operand has K contiguous:
// X[r * ld + k]) and kOpRowMajorMN (X[k * ld + r]).
//
// Tiles of 128 x 128 x 32 per 256-thread workgroup (four wavefronts in 2 x 2,
// each 64 x 64 as 2 x 2 MFMA 32 x 32 blocks).  Tiles are staged in LDS as
// [row][k] with K contiguous (rows padded by 16 bytes, 16-byte k-chunks
// permuted per row, swz_k), so every lane's 8-element MFMA fragment is one
// 16-byte LDS read; the LDS tiles are double
// buffered and the next k-step is prefetched into registers.
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

// 16 elements as eight 4-byte loads (rows of an even leading dimension that
// is not a multiple of 8, e.g. the MLP's 78-wide output rows)
__device__ __forceinline__ void load16_by4(const uint16_t* p, uint4& r0, uint4& r1) {
  const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
  r0 = make_uint4(q[0], q[1], q[2], q[3]);
  r1 = make_uint4(q[4], q[5], q[6], q[7]);
}

// Staging of a 128 x 32 tile (rows row0.., k k0..) of an operand into
// dst[row][k], in two phases so that the loads of the next k-step can be in
// flight during the MFMAs: load() fills two 16-byte registers per thread,
// store() writes them to LDS.
//   K-major: thread t takes row t / 2, k (t & 1) * 16 .. +15 (32 bytes).
//   row-major (X[k * ld + r]): with G = NT / 32 groups of 16 rows, thread t
//   takes k t / G, rows (t % G) * 16 .. +15, written to LDS transposed (16
//   two-byte writes).  NT threads cover NT / 2 rows (a 128- or 256-row tile).
// Rows of an even leading dimension that is not a multiple of 8 are read as
// 4-byte words.  Tiles at the matrix edge or at the end K of the k-range (or
// unaligned operands) are read element by element with bounds checks and zero
// fill.
template <int OP, int NT = 256>
__device__ __forceinline__ void load_tile(uint4& r0, uint4& r1, int64_t K, const void* srcv,
                                          int64_t ld, int64_t row0, int64_t nrows, int64_t k0) {
  constexpr int G = NT / 32;          // row-major: groups of 16 rows per k
  const int t = threadIdx.x;
  const uint16_t* src = reinterpret_cast<const uint16_t*>(srcv);
  uint16_t v[16];
  if constexpr (OP == kOpKMajor) {
    const int64_t gr = row0 + (t >> 1);
    const int64_t kb = k0 + (t & 1) * 16;
    if (gr < nrows && kb + 16 <= K && ((ld & 7) == 0) && aligned16(src)) {
      const uint4* p = reinterpret_cast<const uint4*>(src + gr * ld + kb);
      r0 = p[0];
      r1 = p[1];
      return;
    }
    if (gr < nrows && kb + 16 <= K && ((ld & 1) == 0) &&
        (reinterpret_cast<uintptr_t>(src) & 3u) == 0) {
      load16_by4(src + gr * ld + kb, r0, r1);
      return;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e)
      v[e] = (gr < nrows && kb + e < K) ? src[gr * ld + kb + e] : (uint16_t)0;
  } else {
    const int64_t gk = k0 + t / G;
    const int64_t gr = row0 + (t % G) * 16;
    if (gk < K && gr + 16 <= nrows && ((ld & 7) == 0) && aligned16(src)) {
      const uint4* p = reinterpret_cast<const uint4*>(src + gk * ld + gr);
      r0 = p[0];
      r1 = p[1];
      return;
    }
    if (gk < K && gr + 16 <= nrows && ((ld & 1) == 0) &&
        (reinterpret_cast<uintptr_t>(src) & 3u) == 0) {
      load16_by4(src + gk * ld + gr, r0, r1);
      return;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e)
      v[e] = (gk < K && gr + e < nrows) ? src[gk * ld + gr + e] : (uint16_t)0;
  }
  r0 = make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16),
                  v[4] | ((uint32_t)v[5] << 16), v[6] | ((uint32_t)v[7] << 16));
  r1 = make_uint4(v[8] | ((uint32_t)v[9] << 16), v[10] | ((uint32_t)v[11] << 16),
                  v[12] | ((uint32_t)v[13] << 16), v[14] | ((uint32_t)v[15] << 16));
}

// load_tile for tiles known to lie inside the operand with 16-byte aligned
// rows (the large-tile kernel's shapes): two unconditional 16-byte loads, so
// that the loads of two k-steps can be in flight with exact wait counts.
template <int OP, int NT>
__device__ __forceinline__ void load_tile_full(uint4& r0, uint4& r1, const void* srcv, int64_t ld,
                                               int64_t row0, int64_t k0) {
  constexpr int G = NT / 32;
  const int t = threadIdx.x;
  const uint16_t* src = reinterpret_cast<const uint16_t*>(srcv);
  const uint4* p;
  if constexpr (OP == kOpKMajor)
    p = reinterpret_cast<const uint4*>(src + (row0 + (t >> 1)) * ld + k0 + (t & 1) * 16);
  else
    p = reinterpret_cast<const uint4*>(src + (k0 + t / G) * ld + row0 + (t % G) * 16);
  r0 = p[0];
  r1 = p[1];
}

// LDS column of element k of tile row `row`: the four 8-element (16-byte)
// k-chunks of a row are permuted by (row / 16) mod 4.  The transposed stores
// of row-major operands (the lanes of a wavefront at 8 k values, 16 rows
// apart, rows 20 dwords apart) then spread over 16 banks instead of 4 (a
// 2-way instead of an 8-way conflict), and an MFMA fragment (8 consecutive
// k from a multiple of 8) is still one 16-byte read.
__device__ __forceinline__ int swz_k(int row, int k) { return k ^ (((row >> 4) & 3) << 3); }

template <int OP, int NT = 256>
__device__ __forceinline__ void store_tile(const uint4& r0, const uint4& r1,
                                           uint16_t (*dst)[PADK]) {
  constexpr int G = NT / 32;
  const int t = threadIdx.x;
  if constexpr (OP == kOpKMajor) {
    const int r = t >> 1, kk = (t & 1) * 16;
    *reinterpret_cast<uint4*>(&dst[r][swz_k(r, kk)]) = r0;
    *reinterpret_cast<uint4*>(&dst[r][swz_k(r, kk + 8)]) = r1;
  } else {
    const int kk = t / G, rr = (t % G) * 16;
    const uint32_t w[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
    const int kc = swz_k(rr, kk);       // rows rr .. rr + 15 share the permutation
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      dst[rr + 2 * e][kc] = (uint16_t)(w[e] & 0xFFFFu);
      dst[rr + 2 * e + 1][kc] = (uint16_t)(w[e] >> 16);
    }
  }
}

// Element (row, col) of the standard epilogues: x is alpha A B (+ bias added here).
__device__ __forceinline__ void epi_store(const GemmArgs& g, int64_t row, int64_t col, float x) {
  const int64_t o = row * g.ldc + col;
  if (g.bias) x += g.bias[col];
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

// The standard epilogue for the 16 accumulators of one lane (column col,
// rows row0 + 8 (v / 4) + (v % 4)): the GELU' pre-activations it reads are
// loaded for all 16 first, so the loads are in flight together instead of
// one round trip per element.
__device__ __forceinline__ void epi_store16(const GemmArgs& g, int64_t row0, int64_t col,
                                            f32x16 acc) {
  if (col >= g.N) return;
  float aux[16];
  if (g.epilogue == kEpiGeluGrad) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = row0 + 8 * (v >> 2) + (v & 3);
      aux[v] = row < g.M ? g.aux[row * g.ldc + col] : 0.0f;
    }
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t row = row0 + 8 * (v >> 2) + (v & 3);
    if (row >= g.M) continue;
    float x = acc[v] * g.alpha;
    if (g.epilogue == kEpiGeluGrad) {
      const int64_t o = row * g.ldc + col;
      if (g.bias) x += g.bias[col];
      if (g.pre) g.pre[o] = x;
      x *= gelu_erf_grad(aux[v]);
      if (g.beta != 0.0f)
        x += g.beta * (g.c_bf16 ? bf2f(reinterpret_cast<const uint16_t*>(g.C)[o])
                                : reinterpret_cast<const float*>(g.C)[o]);
      if (g.c_bf16) reinterpret_cast<uint16_t*>(g.C)[o] = f2bf(x);
      else reinterpret_cast<float*>(g.C)[o] = x;
    } else {
      epi_store(g, row, col, x);
    }
  }
}

template <int AOP, int BOP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
    gemm_bf16_kernel(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[2][BM][PADK];
  __shared__ __align__(16) uint16_t Bs[2][BN][PADK];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t tiles_n = (g.N + BN - 1) / BN;
  const int64_t tiles = ((g.M + BM - 1) / BM) * tiles_n;
  const int64_t tile = blockIdx.x % tiles;
  const int64_t tm = tile / tiles_n, tn = tile % tiles_n;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  // split K: workgroup part p takes [kbeg, kend), a whole number of k-steps
  const int split = g.split > 1 ? g.split : 1;
  const int64_t part = blockIdx.x / tiles;
  const int64_t kper = ((g.K + split - 1) / split + BK - 1) / BK * BK;
  const int64_t kbeg = part * kper;
  const int64_t kend = kbeg + kper < g.K ? kbeg + kper : g.K;

  // four named accumulators (an array of them is not kept in registers)
  f32x16 s00 = {}, s01 = {}, s10 = {}, s11 = {};
#define SYNTH_SACC(i, j) ((i) == 0 ? ((j) == 0 ? s00 : s01) : ((j) == 0 ? s10 : s11))

  // LDS double buffer; the next k-step's tiles are loaded into registers
  // before this step's MFMAs and written to the other buffer after them.
  uint4 a0, a1, b0, b1;
  load_tile<AOP>(a0, a1, kend, g.A, g.lda, m0, g.M, kbeg);
  load_tile<BOP>(b0, b1, kend, g.B, g.ldb, n0, g.N, kbeg);
  store_tile<AOP>(a0, a1, As[0]);
  store_tile<BOP>(b0, b1, Bs[0]);
  __syncthreads();
  const int64_t nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  for (int64_t ks = 0; ks < nk; ++ks) {
    const int buf = (int)(ks & 1);
    const bool more = ks + 1 < nk;
    if (more) {
      load_tile<AOP>(a0, a1, kend, g.A, g.lda, m0, g.M, kbeg + (ks + 1) * BK);
      load_tile<BOP>(b0, b1, kend, g.B, g.ldb, n0, g.N, kbeg + (ks + 1) * BK);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int kq = kk + 8 * (lane >> 5);
      bf16x8 af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = wm * 64 + i * 32 + (lane & 31);
        af[i] = *reinterpret_cast<const bf16x8*>(&As[buf][r][swz_k(r, kq)]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = wn * 64 + j * 32 + (lane & 31);
        bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][r][swz_k(r, kq)]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          SYNTH_SACC(i, j) = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], SYNTH_SACC(i, j), 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (more) {
      store_tile<AOP>(a0, a1, As[buf ^ 1]);
      store_tile<BOP>(b0, b1, Bs[buf ^ 1]);
    }
    __syncthreads();
  }

  // ---- epilogue ----
  if (split > 1) {
    // raw partial sums; the reduction applies the epilogue
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t col = n0 + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          if (col < g.N && row < g.M) g.partial[(part * g.M + row) * g.N + col] = SYNTH_SACC(i, j)[v];
        }
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = n0 + wn * 64 + j * 32 + (lane & 31);
      const bool col_ok = col < g.N;
      if (g.epilogue <= kEpiGeluGrad) {
        epi_store16(g, m0 + wm * 64 + i * 32 + 4 * (lane >> 5), col, SYNTH_SACC(i, j));
        continue;
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = m0 + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        float x = SYNTH_SACC(i, j)[v] * g.alpha;
        if (g.epilogue == kEpiPowerPairs) {
          x += (g.bias && col_ok) ? g.bias[col] : 0.0f;
          // (Re, Im) sit in adjacent columns = adjacent lanes; every lane shuffles
          const float other = __shfl_xor(x, 1);
          if ((col & 1) == 0 && col_ok && row < g.M) {
            const float p = x * x + other * other;
            const int64_t o = row * g.ldc + (col >> 1);
            if (g.c_bf16) reinterpret_cast<uint16_t*>(g.C)[o] = f2bf(p);
            else reinterpret_cast<float*>(g.C)[o] = p;
          }
        } else if (col_ok && row < g.M) {    // kEpiLogMelT
          if (g.bias) x += g.bias[col];
          const int64_t o = (row / 64) * 8192 + col * 64 + (row % 64);
          reinterpret_cast<float*>(g.C)[o] = logf(x + 1e-6f);
        }
      }
    }
}

#undef SYNTH_SACC

// Large tiles for the MLP's big products (output dims multiples of 256):
// 256 x 256 x 32 per 512-thread workgroup, eight wavefronts in 2 x 4, each
// 128 x 64 as 4 x 2 MFMA 32 x 32 blocks.  Per k-step a workgroup moves 32 KB
// of operands for 4.2 MFLOP, half the bytes per flop of the 128 x 128 tile,
// so the operand traffic from L2 and the last-level cache stays below what
// the matrix cores consume.  Same staging, LDS layout, double buffering, split
// K and epilogues (the standard ones; split K writes partials).
constexpr int BM2 = 256, BN2 = 256;

template <int AOP, int BOP>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(1, 2)))
    gemm_bf16_big_kernel(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[2][BM2][PADK];
  __shared__ __align__(16) uint16_t Bs[2][BN2][PADK];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int64_t tiles_n = g.N / BN2;
  const int64_t tiles = (g.M / BM2) * tiles_n;
  // Workgroups are dispatched to the 8 XCDs round-robin by index; renumber
  // them so that each XCD takes a contiguous run of (part, tile) with the
  // tiles row-major: the workgroups sharing an L2 then share A's rows and
  // the same B, instead of every XCD streaming all of both.
  const int64_t nblk = gridDim.x;
  const int64_t vid = (nblk % 8 == 0) ? (int64_t)(blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8
                                      : (int64_t)blockIdx.x;
  const int64_t tile = vid % tiles;
  const int64_t tm = tile / tiles_n, tn = tile % tiles_n;
  const int64_t m0 = tm * BM2, n0 = tn * BN2;
  const int split = g.split > 1 ? g.split : 1;
  const int64_t part = vid / tiles;
  const int64_t kper = ((g.K + split - 1) / split + BK - 1) / BK * BK;
  const int64_t kbeg = part * kper;
  const int64_t kend = kbeg + kper < g.K ? kbeg + kper : g.K;

  // eight named accumulators (an array of them is not kept in registers)
  f32x16 c00 = {}, c01 = {}, c10 = {}, c11 = {}, c20 = {}, c21 = {}, c30 = {}, c31 = {};
#define SYNTH_ACC(i, j) ((i) == 0 ? ((j) == 0 ? c00 : c01) : (i) == 1 ? ((j) == 0 ? c10 : c11) \
                         : (i) == 2 ? ((j) == 0 ? c20 : c21) : ((j) == 0 ? c30 : c31))

  // Two k-steps of loads in flight: while the MFMAs run on the LDS tile of
  // step ks, the registers hold step ks + 1 (stored to the other LDS buffer
  // after the MFMAs) and the loads of step ks + 2 are issued, so each global
  // load has two steps of matrix work to arrive.  The loop is unrolled by two
  // so that the register sets alternate without copies.
  uint4 a0, a1, b0, b1, p0, p1, q0, q1;
  load_tile_full<AOP, 512>(a0, a1, g.A, g.lda, m0, kbeg);
  load_tile_full<BOP, 512>(b0, b1, g.B, g.ldb, n0, kbeg);
  store_tile<AOP, 512>(a0, a1, As[0]);
  store_tile<BOP, 512>(b0, b1, Bs[0]);
  const int64_t nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 1) {
    load_tile_full<AOP, 512>(a0, a1, g.A, g.lda, m0, kbeg + BK);
    load_tile_full<BOP, 512>(b0, b1, g.B, g.ldb, n0, kbeg + BK);
  }
  __syncthreads();
  auto mfma_step = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const int kq = kk + 8 * (lane >> 5);
      bf16x8 af[4], bfr[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wm * 128 + i * 32 + (lane & 31);
        af[i] = *reinterpret_cast<const bf16x8*>(&As[buf][r][swz_k(r, kq)]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = wn * 64 + j * 32 + (lane & 31);
        bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][r][swz_k(r, kq)]);
      }
      c00 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[0], bfr[0], c00, 0, 0, 0);
      c01 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[0], bfr[1], c01, 0, 0, 0);
      c10 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[1], bfr[0], c10, 0, 0, 0);
      c11 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[1], bfr[1], c11, 0, 0, 0);
      c20 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[2], bfr[0], c20, 0, 0, 0);
      c21 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[2], bfr[1], c21, 0, 0, 0);
      c30 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[3], bfr[0], c30, 0, 0, 0);
      c31 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[3], bfr[1], c31, 0, 0, 0);
    }
  };
  for (int64_t ks = 0; ks < nk; ks += 2) {
    // step ks (LDS buffer 0); registers a/b hold step ks + 1
    if (ks + 2 < nk) {
      load_tile_full<AOP, 512>(p0, p1, g.A, g.lda, m0, kbeg + (ks + 2) * BK);
      load_tile_full<BOP, 512>(q0, q1, g.B, g.ldb, n0, kbeg + (ks + 2) * BK);
    }
    __builtin_amdgcn_sched_barrier(0);
    mfma_step(0);
    __builtin_amdgcn_sched_barrier(0);
    if (ks + 1 < nk) {
      store_tile<AOP, 512>(a0, a1, As[1]);
      store_tile<BOP, 512>(b0, b1, Bs[1]);
    }
    __syncthreads();
    if (ks + 1 >= nk) break;
    // step ks + 1 (LDS buffer 1); registers p/q hold step ks + 2
    if (ks + 3 < nk) {
      load_tile_full<AOP, 512>(a0, a1, g.A, g.lda, m0, kbeg + (ks + 3) * BK);
      load_tile_full<BOP, 512>(b0, b1, g.B, g.ldb, n0, kbeg + (ks + 3) * BK);
    }
    __builtin_amdgcn_sched_barrier(0);
    mfma_step(1);
    __builtin_amdgcn_sched_barrier(0);
    if (ks + 2 < nk) {
      store_tile<AOP, 512>(p0, p1, As[0]);
      store_tile<BOP, 512>(q0, q1, Bs[0]);
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = n0 + wn * 64 + j * 32 + (lane & 31);
      const int64_t row0 = m0 + wm * 128 + i * 32 + 4 * (lane >> 5);
      if (split > 1) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
          g.partial[(part * g.M + row0 + 8 * (v >> 2) + (v & 3)) * g.N + col] = SYNTH_ACC(i, j)[v];
      } else {
        epi_store16(g, row0, col, SYNTH_ACC(i, j));
      }
    }
#undef SYNTH_ACC
}

// The large-tile kernel applies when both output dims are multiples of 256
// (no edge tiles), K is a multiple of 32, the epilogue is a standard one, and
// the operands take the 16-byte load path (leading dims multiples of 8,
// 16-byte aligned pointers).
bool big_tiles(const GemmArgs& g) {
  return g.M % BM2 == 0 && g.N % BN2 == 0 && g.K % BK == 0 && g.K > 0 &&
         g.epilogue <= kEpiGeluGrad && g.lda % 8 == 0 && g.ldb % 8 == 0 &&
         (reinterpret_cast<uintptr_t>(g.A) & 15u) == 0 && (reinterpret_cast<uintptr_t>(g.B) & 15u) == 0;
}

// Sum of the split-K partials in part order, then the epilogue.
__global__ void __launch_bounds__(256) gemm_split_reduce_kernel(GemmArgs g) {
  // One workgroup per output row (rows strided over the grid): the row's
  // columns are read from each part as 16-byte vectors when N is a multiple
  // of 4 and the workspace 16-byte aligned, else one by one; no index
  // division.
  const int64_t n = g.M * g.N;
  const int t = threadIdx.x;
  const bool vec = (g.N & 3) == 0 && (reinterpret_cast<uintptr_t>(g.partial) & 15u) == 0;
  for (int64_t row = blockIdx.x; row < g.M; row += gridDim.x) {
    const float* src = g.partial + row * g.N;
    if (vec) {
      for (int64_t c4 = t; 4 * c4 < g.N; c4 += 256) {
        float4 x = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        int p = 0;
        for (; p + 4 <= g.split; p += 4) {     // four parts' loads in flight, added in order
          float4 v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const float4*>(src + (p + u) * n + 4 * c4);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            x.x += v[u].x;
            x.y += v[u].y;
            x.z += v[u].z;
            x.w += v[u].w;
          }
        }
        for (; p < g.split; ++p) {
          const float4 v = *reinterpret_cast<const float4*>(src + p * n + 4 * c4);
          x.x += v.x;
          x.y += v.y;
          x.z += v.z;
          x.w += v.w;
        }
        epi_store(g, row, 4 * c4, x.x * g.alpha);
        epi_store(g, row, 4 * c4 + 1, x.y * g.alpha);
        epi_store(g, row, 4 * c4 + 2, x.z * g.alpha);
        epi_store(g, row, 4 * c4 + 3, x.w * g.alpha);
      }
    } else {
      for (int64_t col = t; col < g.N; col += 256) {
        float x = 0.0f;
        int p = 0;
        for (; p + 4 <= g.split; p += 4) {
          float v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = src[(p + u) * n + col];
#pragma unroll
          for (int u = 0; u < 4; ++u) x += v[u];
        }
        for (; p < g.split; ++p) x += src[p * n + col];
        epi_store(g, row, col, x * g.alpha);
      }
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

int gemm_split_for(int64_t M, int64_t N, int64_t K) {
  if (M % BM2 == 0 && N % BN2 == 0 && K % BK == 0 && K > 0) {
    // large tiles: one 512-thread workgroup per CU, each part >= 8 k-steps
    const int64_t tiles2 = (M / BM2) * (N / BN2);
    int64_t split = 1;
    while (tiles2 * split < 256 && K >= split * 2 * 8 * BK) split *= 2;
    return (int)split;
  }
  const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int64_t split = 1;
  // double the split while the grid is under two workgroups per CU (one
  // leaves each SIMD a single wavefront to hide load latency with; two
  // measured 14% faster on the MLP's GEMMs, four slower again) and each part
  // keeps at least 4 k-steps
  while (tiles * split < 512 && K >= split * 2 * 4 * BK) split *= 2;
  return (int)split;
}

size_t gemm_split_bytes(int64_t M, int64_t N, int split) {
  return split > 1 ? (size_t)split * (size_t)M * (size_t)N * sizeof(float) : 0;
}

hipError_t launch_gemm_bf16(const GemmArgs& g, int a_op, int b_op, hipStream_t s) {
  if (g.M == 0 || g.N == 0) return hipSuccess;
  const int split = g.split > 1 ? g.split : 1;
  if (split > 1 && (!g.partial || g.epilogue > kEpiGeluGrad)) return hipErrorInvalidValue;
  if ((a_op != kOpKMajor && a_op != kOpRowMajorMN) || (b_op != kOpKMajor && b_op != kOpRowMajorMN))
    return hipErrorInvalidValue;
  hipError_t e;
  if (big_tiles(g)) {
    const int64_t tiles2 = (g.M / BM2) * (g.N / BN2);
    if (tiles2 * split > 0x7FFFFFFF) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(tiles2 * split));
    if (a_op == kOpKMajor) {
      if (b_op == kOpKMajor)
        hipLaunchKernelGGL((gemm_bf16_big_kernel<kOpKMajor, kOpKMajor>), grid, dim3(512), 0, s, g);
      else
        hipLaunchKernelGGL((gemm_bf16_big_kernel<kOpKMajor, kOpRowMajorMN>), grid, dim3(512), 0, s, g);
    } else {
      if (b_op == kOpKMajor)
        hipLaunchKernelGGL((gemm_bf16_big_kernel<kOpRowMajorMN, kOpKMajor>), grid, dim3(512), 0, s, g);
      else
        hipLaunchKernelGGL((gemm_bf16_big_kernel<kOpRowMajorMN, kOpRowMajorMN>), grid, dim3(512), 0,
                           s, g);
    }
    e = hipGetLastError();
  } else {
    const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
    if (tiles * split > 0x7FFFFFFF) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(tiles * split));
    e = a_op == kOpKMajor ? launch_b<kOpKMajor>(g, b_op, grid, s)
                          : launch_b<kOpRowMajorMN>(g, b_op, grid, s);
  }
  if (e != hipSuccess || split == 1) return e;
  const int64_t blocks = g.M < 65535 ? g.M : 65535;
  hipLaunchKernelGGL(gemm_split_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace synth
