// Small fixed-order reductions over device matrices (float64 accumulation):
// per-row or per-column sums of |a - b| or (a - b)^2, the sum of a float64
// vector, and a per-row rescale.  They close the learned and sound-matching
// paths on the device: the proposal's training loss, the chain rule of the
// spectral loss, and the evaluation metrics (log-mel L1 between renders,
// parameter squared error).  Every sum runs in a fixed order, so results are
// bitwise reproducible.
#include "synth_internal.h"

namespace synth {
namespace {

constexpr int kRedThreads = 256;

__device__ __forceinline__ double diff_term(int kind, float a, float b) {
  const double d = (double)a - (double)b;
  return kind == 0 ? fabs(d) : d * d;
}

// Tree over the workgroup's 256 partial sums in a fixed order; thread 0 returns it.
__device__ __forceinline__ double block_sum(double x, double* red) {
  const int t = threadIdx.x;
  red[t] = x;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  return red[0];
}

// One workgroup per row: thread t adds columns t, t + 256, ... in order.
__global__ void __launch_bounds__(kRedThreads)
    diff_rows_kernel(int kind, const float* __restrict__ a, const float* __restrict__ b,
                     int64_t cols, int64_t lda, int64_t ldb, double scale, int accumulate,
                     double* __restrict__ out) {
  __shared__ double red[kRedThreads];
  const int64_t r = blockIdx.x;
  const float* ar = a + r * lda;
  const float* br = b ? b + r * ldb : nullptr;
  double acc = 0.0;
  for (int64_t c = threadIdx.x; c < cols; c += kRedThreads)
    acc += diff_term(kind, ar[c], br ? br[c] : 0.0f);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[r] = (accumulate ? out[r] : 0.0) + scale * s;
}

// One thread per column, rows in order.
__global__ void __launch_bounds__(kRedThreads)
    diff_cols_kernel(int kind, const float* __restrict__ a, const float* __restrict__ b,
                     int64_t rows, int64_t cols, int64_t lda, int64_t ldb, double scale,
                     int accumulate, double* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
  if (c >= cols) return;
  double acc = 0.0;
  for (int64_t r = 0; r < rows; ++r) acc += diff_term(kind, a[r * lda + c], b ? b[r * ldb + c] : 0.0f);
  out[c] = (accumulate ? out[c] : 0.0) + scale * acc;
}

__global__ void __launch_bounds__(kRedThreads)
    sum_f64_kernel(const double* __restrict__ x, int64_t n, double scale, double* __restrict__ out) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRedThreads) acc += x[i];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = scale * s;
}

__global__ void scale_rows_kernel(const float* __restrict__ g, const double* __restrict__ s,
                                  int64_t rows, int64_t cols, float* __restrict__ out) {
  const int64_t n = rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = g[i] * (float)s[i / cols];
}

}  // namespace

hipError_t launch_diff_reduce(int kind, int axis, const float* a, const float* b, int64_t rows,
                              int64_t cols, int64_t lda, int64_t ldb, double scale, int accumulate,
                              double* out, hipStream_t s) {
  if (axis == 1) {
    if (rows == 0) return hipSuccess;
    hipLaunchKernelGGL(diff_rows_kernel, dim3((unsigned)rows), dim3(kRedThreads), 0, s, kind, a, b,
                       cols, lda, ldb, scale, accumulate, out);
  } else {
    if (cols == 0) return hipSuccess;
    const unsigned grid = (unsigned)((cols + kRedThreads - 1) / kRedThreads);
    hipLaunchKernelGGL(diff_cols_kernel, dim3(grid), dim3(kRedThreads), 0, s, kind, a, b, rows,
                       cols, lda, ldb, scale, accumulate, out);
  }
  return hipGetLastError();
}

hipError_t launch_sum_f64(const double* x, int64_t n, double scale, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(kRedThreads), 0, s, x, n, scale, out);
  return hipGetLastError();
}

hipError_t launch_scale_rows(const float* g, const double* sc, int64_t rows, int64_t cols,
                             float* out, hipStream_t s) {
  const int64_t n = rows * cols;
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(scale_rows_kernel, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256),
                     0, s, g, sc, rows, cols, out);
  return hipGetLastError();
}

}  // namespace synth
