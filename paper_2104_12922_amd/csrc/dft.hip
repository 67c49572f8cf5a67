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
// Global loads for k-step s + 2 are issued before the MFMAs of step s (two
// register sets) and written to LDS two steps later; the LDS tile is double
// buffered (one barrier per k-step).  Tiles
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

// Source of the zeros read for frame samples past a voice's end.
__device__ __align__(16) const float kZeros[4] = {0.0f, 0.0f, 0.0f, 0.0f};

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// The k-loop and epilogue of one tile.  The four frame rows this thread
// stages start at abase[q] with lim[q] samples left in their voice; past that
// the frame reads as 0: those loads are redirected to a zero constant, so the
// loads are unconditional and nothing waits on a load before the MFMAs.
// VEC: every voice is 16-byte aligned with a length divisible by 4, so one
// float4 is wholly inside or wholly outside; otherwise four scalar loads.
template <bool VEC>
__device__ __forceinline__ void dft_tile(const float* __restrict__ audio, const float* const (&abase)[4],
                                         const int (&lim)[4], const uint16_t* bsrc0,
                                         const uint16_t* bsrc1, uint16_t (*As)[kBM][kLDK],
                                         uint16_t (*Bs)[kBN][kLDK], int64_t m0, int64_t n0,
                                         int64_t rows, uint16_t* __restrict__ power, int64_t ldp) {
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int a_c = (t & 7) * 4;
  const int a_r = t >> 3;
  const int b_c = (t & 3) * 8;
  const int b_r = t >> 2;

  // Two sets of prefetch registers (named scalars, so that they stay in
  // VGPRs): the loads for k-step s + 2 are issued at the start of step s, so
  // each has two steps of MFMA work to arrive before it is written to LDS.
  float4 ra0, ra1, ra2, ra3, sa0, sa1, sa2, sa3;
  uint4 rb0, rb1, sb0, sb1;

#define DFT_LD1(RA, Q, K0)                                                      \
  if constexpr (VEC) {                                                          \
    const float* p_ = (K0) < lim[Q] ? abase[Q] + (K0) : kZeros;                 \
    RA = *reinterpret_cast<const float4*>(p_);                                  \
  } else {                                                                      \
    RA.x = *((K0) + 0 < lim[Q] ? abase[Q] + (K0) + 0 : kZeros);                 \
    RA.y = *((K0) + 1 < lim[Q] ? abase[Q] + (K0) + 1 : kZeros);                 \
    RA.z = *((K0) + 2 < lim[Q] ? abase[Q] + (K0) + 2 : kZeros);                 \
    RA.w = *((K0) + 3 < lim[Q] ? abase[Q] + (K0) + 3 : kZeros);                 \
  }
#define DFT_LOAD(A0, A1, A2, A3, B0, B1, KS)                                    \
  {                                                                             \
    const int k0 = (KS) * kBK + a_c;                                            \
    DFT_LD1(A0, 0, k0) DFT_LD1(A1, 1, k0) DFT_LD1(A2, 2, k0) DFT_LD1(A3, 3, k0) \
    B0 = *reinterpret_cast<const uint4*>(bsrc0 + (KS) * kBK);                   \
    B1 = *reinterpret_cast<const uint4*>(bsrc1 + (KS) * kBK);                   \
  }
#define DFT_ST1(RA, Q, K0, BUF)                                                 \
  {                                                                             \
    uint2 w_;                                                                   \
    w_.x = pack_bf16(RA.x, RA.y);                                               \
    w_.y = pack_bf16(RA.z, RA.w);                                               \
    *reinterpret_cast<uint2*>(&As[BUF][(Q) * 64 + a_r][a_c]) = w_;              \
  }
#define DFT_STORE(A0, A1, A2, A3, B0, B1, KS, BUF)                              \
  {                                                                             \
    const int k0 = (KS) * kBK + a_c;                                            \
    DFT_ST1(A0, 0, k0, BUF) DFT_ST1(A1, 1, k0, BUF) DFT_ST1(A2, 2, k0, BUF)     \
    DFT_ST1(A3, 3, k0, BUF)                                                     \
    *reinterpret_cast<uint4*>(&Bs[BUF][b_r][b_c]) = B0;                         \
    *reinterpret_cast<uint4*>(&Bs[BUF][128 + b_r][b_c]) = B1;                   \
  }
#define DFT_MFMA(BUF)                                                           \
  _Pragma("unroll") for (int kk = 0; kk < kBK; kk += 16) {                      \
    const int kq = kk + 8 * (lane >> 5);                                        \
    bf16x8 af[4], bf[2];                                                        \
    _Pragma("unroll") for (int ii = 0; ii < 4; ++ii) af[ii] =                   \
        *reinterpret_cast<const bf16x8*>(&As[BUF][wm * 128 + ii * 32 + (lane & 31)][kq]); \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) bf[j] =                       \
        *reinterpret_cast<const bf16x8*>(&Bs[BUF][wn * 64 + j * 32 + (lane & 31)][kq]); \
    _Pragma("unroll") for (int ii = 0; ii < 4; ++ii)                            \
      _Pragma("unroll") for (int j = 0; j < 2; ++j)                             \
        acc[ii][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[ii], bf[j], acc[ii][j], 0, 0, 0); \
  }

  f32x16 acc[4][2];
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[ii][j][v] = 0.0f;

  static_assert(kKSteps % 2 == 0, "the k-loop is unrolled by two");
  DFT_LOAD(ra0, ra1, ra2, ra3, rb0, rb1, 0)
  DFT_LOAD(sa0, sa1, sa2, sa3, sb0, sb1, 1)
  DFT_STORE(ra0, ra1, ra2, ra3, rb0, rb1, 0, 0)
  __syncthreads();
  for (int ks = 0; ks < kKSteps; ks += 2) {
    // step ks: LDS buffer 0 holds ks, set s (ks + 1) is in flight, set r is free
    if (ks + 2 < kKSteps) DFT_LOAD(ra0, ra1, ra2, ra3, rb0, rb1, ks + 2)
    __builtin_amdgcn_sched_barrier(0);
    DFT_MFMA(0)
    __builtin_amdgcn_sched_barrier(0);
    DFT_STORE(sa0, sa1, sa2, sa3, sb0, sb1, ks + 1, 1)
    __syncthreads();
    // step ks + 1: LDS buffer 1 holds ks + 1, set r (ks + 2) is in flight
    if (ks + 3 < kKSteps) DFT_LOAD(sa0, sa1, sa2, sa3, sb0, sb1, ks + 3)
    __builtin_amdgcn_sched_barrier(0);
    DFT_MFMA(1)
    __builtin_amdgcn_sched_barrier(0);
    if (ks + 2 < kKSteps) DFT_STORE(ra0, ra1, ra2, ra3, rb0, rb1, ks + 2, 0)
    __syncthreads();
  }
#undef DFT_LD1
#undef DFT_LOAD
#undef DFT_ST1
#undef DFT_STORE
#undef DFT_MFMA

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

template <bool VEC>
__global__ void __launch_bounds__(kThreads) dft_power_kernel(const float* __restrict__ audio,
                                                        const int64_t* __restrict__ offsets,
                                                        int64_t n_uniform, int64_t rows,
                                                        const uint16_t* __restrict__ basis,
                                                        uint16_t* __restrict__ power,
                                                        int64_t ldp) {
  __shared__ __align__(16) uint16_t As[2][kBM][kLDK];
  __shared__ __align__(16) uint16_t Bs[2][kBN][kLDK];
  const int t = threadIdx.x;

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
  // pass q reads frame a_r of voice m0 / 64 + q, which starts at a_r * 2756.
  const int a_r = t >> 3;
  const int64_t batch = rows >> 6;
  const int64_t pos = a_r * 2756;
  const float* abase[4];
  int lim[4];
  bool vec = true;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t v = (m0 >> 6) + q;
    int64_t start = 0, len = 0;
    if (v < batch) {
      if (offsets) {
        packed_range(offsets, batch, v, start, len);
      } else {
        start = v * n_uniform;
        len = n_uniform;
      }
    }
    vec = vec && (len & 3) == 0 && (reinterpret_cast<uintptr_t>(audio + start) & 15u) == 0;
    abase[q] = audio + start + pos;
    const int64_t l = len - pos;                 // samples of the frame in the voice
    lim[q] = (int)(l < 4096 ? (l > -1 ? l : -1) : 4096);
  }
  // B staging: 4 threads per row (16 bytes each), 128 rows per pass, 2 passes.
  const int b_c = (t & 3) * 8;
  const int b_r = t >> 2;
  const uint16_t* bsrc0 = basis + (n0 + b_r) * (int64_t)kN + b_c;
  const uint16_t* bsrc1 = basis + (n0 + 128 + b_r) * (int64_t)kN + b_c;
  // Both instantiations run over the same grid; each takes the tiles whose
  // voices suit it (the flag is uniform across the workgroup), so every tile
  // is computed once and each instantiation gets its own register budget.
  if (vec != VEC) return;
  dft_tile<VEC>(audio, abase, lim, bsrc0, bsrc1, As, Bs, m0, n0, rows, power, ldp);
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
  hipLaunchKernelGGL(dft_power_kernel<true>, dim3((unsigned)tiles), dim3(kThreads), 0, s, audio,
                     offsets, n_uniform, rows, (const uint16_t*)basis, (uint16_t*)power, ldp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Tiles with a voice that is not 16-byte aligned or whose length is not a
  // multiple of 4 (none for uniform batches of aligned audio).
  const bool all_vec = !offsets && (n_uniform & 3) == 0 &&
                       (reinterpret_cast<uintptr_t>(audio) & 15u) == 0;
  if (!all_vec)
    hipLaunchKernelGGL(dft_power_kernel<false>, dim3((unsigned)tiles), dim3(kThreads), 0, s, audio,
                       offsets, n_uniform, rows, (const uint16_t*)basis, (uint16_t*)power, ldp);
  return hipGetLastError();
}

hipError_t launch_dft_basis(void* basis_bf16, hipStream_t s) {
  hipLaunchKernelGGL(dft_basis_kernel, dim3(4096), dim3(256), 0, s, (uint16_t*)basis_bf16);
  return hipGetLastError();
}

}  // namespace synth
