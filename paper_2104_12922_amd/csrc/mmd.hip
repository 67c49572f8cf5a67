// Sums of pairwise L1 distances between two sets of embeddings, and the
// maximum mean discrepancy built from them (Section 5, equation "mmd": sets
// of sounds compared through an auditory distance d; here d is the L1
// distance between embedding vectors):
//   S(A, B) = sum_{i < n, j < m} sum_k |A[i][k] - B[j][k]|
//   MMD(X, Y) = 2 S(X, Y) / (n m) - S(X, X) / n^2 - S(Y, Y) / m^2.
//
// Workgroups of 256 threads take tiles of 64 x 64 pairs and one share of
// the embedding dimension (whole runs of 256 dimensions, so tiles x shares
// fills the chip even for sets of a few hundred sounds).  The dimension is
// walked in chunks of 32 staged in LDS (rows padded to 36 floats).  Thread
// (ty, tx) holds the 4 x 4 pairs rows ty + 16 a, columns tx + 16 b: per four
// staged dimensions, 8 16-byte LDS reads (conflict-free: the A reads are
// broadcasts, B rows 36 floats apart cover distinct banks) feed 64 |x - y|
// accumulations.  A pair's distance is accumulated in float32 over each run
// of 256 dimensions, then added to a float64 accumulator; a workgroup sums
// its pairs in a fixed order, and a second kernel sums the workgroups in
// order, so S is bitwise reproducible and S(X, X) equals S(A = X, B = X).
// Bound by VALU issue: two instructions (subtract, add of the absolute
// value) per pair and dimension.
#include "synth_internal.h"

namespace synth {
namespace {

constexpr int kPT = 64;          // pairs per tile side
constexpr int kPK = 32;          // dimensions per LDS chunk
constexpr int kPLd = 36;         // padded LDS row (floats)
constexpr int kF32Run = 256;     // dimensions accumulated in float32 before promotion
constexpr int64_t kFillBlocks = 1024;

struct PairPlan {
  int64_t tiles_n, tiles_m, shares, runs_per_share;
};

PairPlan pair_plan(int64_t n, int64_t m, int64_t dim) {
  PairPlan p;
  p.tiles_n = (n + kPT - 1) / kPT;
  p.tiles_m = (m + kPT - 1) / kPT;
  const int64_t tiles = p.tiles_n * p.tiles_m;
  const int64_t runs = dim > 0 ? (dim + kF32Run - 1) / kF32Run : 1;
  int64_t want = tiles >= kFillBlocks ? 1 : (kFillBlocks + tiles - 1) / (tiles > 0 ? tiles : 1);
  if (want > runs) want = runs;
  p.runs_per_share = (runs + want - 1) / want;
  p.shares = (runs + p.runs_per_share - 1) / p.runs_per_share;
  return p;
}

// Stage rows r0 .. r0 + 63, dimensions k0 .. k0 + 31 of X (rows < rows, dims
// < dim; anything outside reads as 0, and |0 - 0| adds nothing).
__device__ __forceinline__ void stage_rows(float (*S)[kPLd], const float* __restrict__ X,
                                           int64_t ld, int64_t rows, int64_t r0, int64_t k0,
                                           int64_t dim, bool vec) {
  const int t = threadIdx.x;
  const int lr = t >> 2, lk = (t & 3) * 8;
  const int64_t r = r0 + lr, k = k0 + lk;
  float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
  if (r < rows) {
    const float* p = X + r * ld + k;
    if (vec && k + 8 <= dim) {
      v0 = *reinterpret_cast<const float4*>(p);
      v1 = *reinterpret_cast<const float4*>(p + 4);
    } else {
      float e[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) e[i] = (k + i < dim) ? p[i] : 0.0f;
      v0 = make_float4(e[0], e[1], e[2], e[3]);
      v1 = make_float4(e[4], e[5], e[6], e[7]);
    }
  }
  *reinterpret_cast<float4*>(&S[lr][lk]) = v0;
  *reinterpret_cast<float4*>(&S[lr][lk + 4]) = v1;
}

__global__ void __launch_bounds__(256) l1_pair_sum_kernel(const float* __restrict__ A, int64_t lda,
                                                          int64_t n, const float* __restrict__ B,
                                                          int64_t ldb, int64_t m, int64_t dim,
                                                          PairPlan plan, int vec,
                                                          double* __restrict__ partial) {
  __shared__ __align__(16) float As[kPT][kPLd];
  __shared__ __align__(16) float Bs[kPT][kPLd];
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  const int64_t share = blockIdx.x % plan.shares;
  const int64_t tile = blockIdx.x / plan.shares;
  const int64_t i0 = (tile / plan.tiles_m) * kPT, j0 = (tile % plan.tiles_m) * kPT;
  const int64_t kbeg = share * plan.runs_per_share * kF32Run;
  int64_t kend = kbeg + plan.runs_per_share * kF32Run;
  if (kend > dim) kend = dim;
  float acc[4][4];
  double dacc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc[a][b] = 0.0f;
      dacc[a][b] = 0.0;
    }
  for (int64_t k0 = kbeg; k0 < kend; k0 += kPK) {
    stage_rows(As, A, lda, n, i0, k0, kend, vec != 0);
    stage_rows(Bs, B, ldb, m, j0, k0, kend, vec != 0);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kPK; kk += 4) {
      float4 xa[4], yb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xa[a] = *reinterpret_cast<const float4*>(&As[ty + 16 * a][kk]);
#pragma unroll
      for (int b = 0; b < 4; ++b) yb[b] = *reinterpret_cast<const float4*>(&Bs[tx + 16 * b][kk]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b] += fabsf(xa[a].x - yb[b].x);
          acc[a][b] += fabsf(xa[a].y - yb[b].y);
          acc[a][b] += fabsf(xa[a].z - yb[b].z);
          acc[a][b] += fabsf(xa[a].w - yb[b].w);
        }
    }
    __syncthreads();
    if ((k0 + kPK - kbeg) % kF32Run == 0 || k0 + kPK >= kend) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          dacc[a][b] += (double)acc[a][b];
          acc[a][b] = 0.0f;
        }
    }
  }
  // this thread's pairs inside the sets, in a fixed order
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (i0 + ty + 16 * a < n && j0 + tx + 16 * b < m) s += dacc[a][b];
  red[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) partial[blockIdx.x] = red[0];
}

// out[0] = sum of partial[0 .. count) in order (one workgroup: per-thread
// strided sums, then a fixed tree).
__global__ void __launch_bounds__(256) ordered_sum_kernel(const double* __restrict__ partial,
                                                          int64_t count, double* __restrict__ out) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t i = t; i < count; i += 256) s += partial[i];
  red[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[0] = red[0];
}

// out[0] = 2 s_xy / (n m) - s_xx / n^2 - s_yy / m^2 from out[1..3].
__global__ void mmd_combine_kernel(double* out, int64_t n, int64_t m) {
  if (threadIdx.x == 0) {
    const double dn = (double)n, dm = (double)m;
    out[0] = 2.0 * out[1] / (dn * dm) - out[2] / (dn * dn) - out[3] / (dm * dm);
  }
}

}  // namespace

size_t l1_pair_sum_workspace(int64_t n, int64_t m, int64_t dim) {
  const PairPlan p = pair_plan(n, m, dim);
  return (size_t)(p.tiles_n * p.tiles_m * p.shares) * sizeof(double);
}

hipError_t launch_l1_pair_sum(const float* A, int64_t lda, int64_t n, const float* B, int64_t ldb,
                              int64_t m, int64_t dim, double* partial, double* out, hipStream_t s) {
  const PairPlan p = pair_plan(n, m, dim);
  const int64_t blocks = p.tiles_n * p.tiles_m * p.shares;
  if (blocks > 0 && dim > 0) {
    const int vec = ((lda | ldb) % 4 == 0) && (reinterpret_cast<uintptr_t>(A) % 16 == 0) &&
                    (reinterpret_cast<uintptr_t>(B) % 16 == 0);
    hipLaunchKernelGGL(l1_pair_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, s, A, lda, n, B,
                       ldb, m, dim, p, vec, partial);
  }
  hipLaunchKernelGGL(ordered_sum_kernel, dim3(1), dim3(256), 0, s, partial,
                     dim > 0 ? blocks : (int64_t)0, out);
  return hipGetLastError();
}

hipError_t launch_mmd_combine(double* out, int64_t n, int64_t m, hipStream_t s) {
  hipLaunchKernelGGL(mmd_combine_kernel, dim3(1), dim3(64), 0, s, out, n, m);
  return hipGetLastError();
}

}  // namespace synth
