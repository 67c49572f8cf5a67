// Elementwise and reduction kernels of the learned proposal: bf16 casts,
// per-column sums (bias gradients, feature statistics), feature
// standardisation, the sigmoid-output MSE gradient, Adam, and the
// logit-space updates and best-so-far tracking of sound matching.  All deterministic (fixed-order reductions).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "synth_internal.h"

namespace synth {
namespace {

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}

// Column reductions use 1024-thread workgroups of 16 columns x 64 row groups:
// thread (g, c) accumulates rows g, g + 64, ... of column c in float64, then
// the 64 partial sums are added in a fixed tree order - deterministic.
constexpr int kRedCols = 16, kRedGroups = 64;

__device__ __forceinline__ double tree_sum(double* red, int c, int g, double v) {
  red[g * kRedCols + c] = v;
  __syncthreads();
  for (int s = kRedGroups / 2; s > 0; s >>= 1) {
    if (g < s) red[g * kRedCols + c] += red[(g + s) * kRedCols + c];
    __syncthreads();
  }
  const double r = red[c];
  __syncthreads();
  return r;
}

// sum (and sum of squares) of each column over rows.
__global__ void __launch_bounds__(1024) colsum_kernel(const void* __restrict__ x, int x_bf16,
                                                      int64_t rows, int64_t cols, int64_t ld,
                                                      float* __restrict__ sum,
                                                      float* __restrict__ sumsq) {
  __shared__ double red[kRedGroups * kRedCols];
  const int c = threadIdx.x % kRedCols, g = threadIdx.x / kRedCols;
  const int64_t col = blockIdx.x * (int64_t)kRedCols + c;
  double s = 0.0, s2 = 0.0;
  if (col < cols) {
    for (int64_t r = g; r < rows; r += kRedGroups) {
      const float v = x_bf16 ? bf2f(reinterpret_cast<const uint16_t*>(x)[r * ld + col])
                             : reinterpret_cast<const float*>(x)[r * ld + col];
      s += v;
      s2 += (double)v * v;
    }
  }
  s = tree_sum(red, c, g, s);
  if (sumsq) s2 = tree_sum(red, c, g, s2);
  if (g == 0 && col < cols) {
    sum[col] = (float)s;
    if (sumsq) sumsq[col] = (float)s2;
  }
}

// Column sums of a bf16 matrix in two passes, for the bias gradients:
// workgroup (column tile t, row slice r) of 4 wavefronts sums rows
// [r R0, (r + 1) R0) of 128 columns (each lane two adjacent columns, read as
// one 4-byte word, so a wavefront reads 256 contiguous bytes of a row;
// wavefront w takes rows w, w + 4, ... of the slice), adds the four
// wavefronts' sums in a fixed order and writes ws[r][col] (float64); the
// second pass adds the slices in order.  Deterministic.
constexpr int kColTile = 128, kColWaves = 4;

__global__ void __launch_bounds__(64 * kColWaves) colsum_part_kernel(const uint16_t* __restrict__ x,
                                                                     int64_t rows, int64_t cols,
                                                                     int64_t ld, int64_t r0n,
                                                                     double* __restrict__ ws) {
  __shared__ double red[kColWaves][kColTile];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t c0 = blockIdx.x * (int64_t)kColTile + 2 * lane;
  const int64_t rb = blockIdx.y * r0n, re = min(rows, rb + r0n);
  double s0 = 0.0, s1 = 0.0;
  if (c0 + 1 < cols) {
    // eight rows' loads in flight before their adds (in row order)
    int64_t r = rb + w;
    for (; r + 7 * kColWaves < re; r += 8 * kColWaves) {
      uint32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = *reinterpret_cast<const uint32_t*>(x + (r + u * kColWaves) * ld + c0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s0 += (double)bf2f((uint16_t)(v[u] & 0xFFFFu));
        s1 += (double)bf2f((uint16_t)(v[u] >> 16));
      }
    }
    for (; r < re; r += kColWaves) {
      const uint32_t v = *reinterpret_cast<const uint32_t*>(x + r * ld + c0);
      s0 += (double)bf2f((uint16_t)(v & 0xFFFFu));
      s1 += (double)bf2f((uint16_t)(v >> 16));
    }
  } else if (c0 < cols) {
    for (int64_t r = rb + w; r < re; r += kColWaves) s0 += (double)bf2f(x[r * ld + c0]);
  }
  red[w][2 * lane] = s0;
  red[w][2 * lane + 1] = s1;
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int cc = 2 * lane + e;
      const double t = ((red[0][cc] + red[1][cc]) + red[2][cc]) + red[3][cc];
      if (c0 + e < cols) ws[blockIdx.y * cols + c0 + e] = t;
    }
  }
}

__global__ void __launch_bounds__(256) colsum_final_kernel(const double* __restrict__ ws,
                                                           int64_t slices, int64_t cols,
                                                           float* __restrict__ sum) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  int64_t r = 0;
  for (; r + 8 <= slices; r += 8) {      // eight slices' loads in flight, added in order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ws[(r + u) * cols + c];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; r < slices; ++r) s += ws[r * cols + c];
  sum[c] = (float)s;
}

// Per-column mean and 1 / sqrt(max(var, min_var)) (population variance), two
// float64 passes over the rows.
__global__ void __launch_bounds__(1024) feature_stats_kernel(const float* __restrict__ x,
                                                             int64_t rows, int64_t cols,
                                                             float min_var,
                                                             float* __restrict__ mean,
                                                             float* __restrict__ inv_std) {
  __shared__ double red[kRedGroups * kRedCols];
  const int c = threadIdx.x % kRedCols, g = threadIdx.x / kRedCols;
  const int64_t col = blockIdx.x * (int64_t)kRedCols + c;
  double s = 0.0;
  if (col < cols)
    for (int64_t r = g; r < rows; r += kRedGroups) s += x[r * cols + col];
  const double mu = tree_sum(red, c, g, s) / (double)rows;
  double s2 = 0.0;
  if (col < cols)
    for (int64_t r = g; r < rows; r += kRedGroups) {
      const double d = x[r * cols + col] - mu;
      s2 += d * d;
    }
  s2 = tree_sum(red, c, g, s2);
  if (g == 0 && col < cols) {
    const double var = fmax(s2 / (double)rows, (double)min_var);
    mean[col] = (float)mu;
    inv_std[col] = (float)(1.0 / sqrt(var));
  }
}

// y = bf16((x - mean[col]) * inv_std[col])
__global__ void standardize_kernel(const float* __restrict__ x, const float* __restrict__ mean,
                                   const float* __restrict__ inv_std, int64_t rows, int64_t cols,
                                   uint16_t* __restrict__ y) {
  const int64_t n = rows * cols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i % cols;
    y[i] = f2bf((x[i] - mean[c]) * inv_std[c]);
  }
}

// MSE on sigmoid outputs: loss_rows[r] = sum_c (o - u)^2; dz = 2 (o - u) o (1 - o) / (rows cols)
// One wavefront per row: lane c takes columns c, c + 64, ...; the row's
// squared error is summed over lanes in a fixed tree (deterministic).
__global__ void __launch_bounds__(256) mse_sigmoid_grad_kernel(const float* __restrict__ out,
                                                               const float* __restrict__ target,
                                                               int64_t rows, int64_t cols,
                                                               uint16_t* __restrict__ dz,
                                                               double* __restrict__ loss_rows) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const float scale = 2.0f / ((float)rows * (float)cols);
  double l = 0.0;
  for (int64_t c = lane; c < cols; c += 64) {
    const float o = out[r * cols + c];
    const float d = o - target[r * cols + c];
    l += (double)d * d;
    dz[r * cols + c] = f2bf(scale * d * o * (1.0f - o));
  }
  for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off);
  if (lane == 0) loss_rows[r] = l;
}

// Adam (bias-corrected) on float32 master weights, refreshing the bf16 copy.
__global__ void adam_kernel(int64_t n, float* __restrict__ w, uint16_t* __restrict__ wb,
                            const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
  }
}

// Sound matching in logit space (u = sigmoid(z)).
__global__ void logit_init_kernel(const float* __restrict__ u, float* __restrict__ z,
                                  float* __restrict__ u_out, int64_t n, float eps) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float uc = fminf(fmaxf(u[i], eps), 1.0f - eps);
    const float zi = logf(uc) - log1pf(-uc);
    z[i] = zi;
    u_out[i] = 1.0f / (1.0f + expf(-zi));
  }
}

// dL/dz = dL/du * u (1 - u) at the current u; Adam on z; u <- sigmoid(z).
__global__ void logit_adam_kernel(int64_t n, float* __restrict__ z, float* __restrict__ u,
                                  const float* __restrict__ gu, float* __restrict__ m,
                                  float* __restrict__ v, float lr, float b1, float b2, float eps,
                                  float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float ui = u[i];
    const float gi = gu[i] * ui * (1.0f - ui);
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float zi = z[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    z[i] = zi;
    u[i] = 1.0f / (1.0f + expf(-zi));
  }
}

// Per row r: the smallest loss over columns c (element r * rs + c * cs; the
// first one on ties); if it beats best[r], record it, its column index
// (col_base + c) and, if params is given, that element's param_dim floats.
__global__ void best_update_kernel(const double* __restrict__ loss, int64_t rows, int64_t cols,
                                   int64_t rs, int64_t cs, int64_t col_base,
                                   const float* __restrict__ params, int64_t param_dim,
                                   double* __restrict__ best, int64_t* __restrict__ best_idx,
                                   float* __restrict__ best_params) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double lm = 0.0;
  int64_t cm = -1;
  for (int64_t c = 0; c < cols; ++c) {
    const double l = loss[r * rs + c * cs];
    if (cm < 0 || l < lm) { lm = l; cm = c; }
  }
  if (cm < 0 || !(lm < best[r])) return;
  best[r] = lm;
  if (best_idx) best_idx[r] = col_base + cm;
  if (params && best_params) {
    const float* src = params + (r * rs + cm * cs) * param_dim;
    for (int64_t p = 0; p < param_dim; ++p) best_params[r * param_dim + p] = src[p];
  }
}

dim3 grid_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b > 65535 * 4) b = 65535 * 4;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

}  // namespace

hipError_t launch_f32_to_bf16(const float* x, void* y, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(f32_to_bf16_kernel, grid_for(n, 256), dim3(256), 0, s, x, (uint16_t*)y, n);
  return hipGetLastError();
}

hipError_t launch_colsum(const void* x, int x_bf16, int64_t rows, int64_t cols, int64_t ld,
                         float* sum, float* sumsq, hipStream_t s) {
  if (cols == 0) return hipSuccess;
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)((cols + kRedCols - 1) / kRedCols)), dim3(1024),
                     0, s, x, x_bf16, rows, cols, ld, sum, sumsq);
  return hipGetLastError();
}

size_t colsum_ws_bytes(int64_t rows, int64_t cols) {
  const int64_t slices = rows < 32 ? rows : 32;
  return (size_t)(slices > 0 ? slices : 1) * (size_t)cols * sizeof(double);
}

hipError_t launch_colsum_bf16_ws(const void* x, int64_t rows, int64_t cols, int64_t ld, float* sum,
                                 void* ws, size_t ws_bytes, hipStream_t s) {
  if (cols == 0) return hipSuccess;
  // two-byte elements read in pairs: rows must start 4-byte aligned
  const bool pairs = (ld % 2 == 0) && (reinterpret_cast<uintptr_t>(x) & 3u) == 0;
  if (!ws || ws_bytes < colsum_ws_bytes(rows, cols) || rows < 1 || !pairs ||
      (reinterpret_cast<uintptr_t>(ws) & 7u) != 0)
    return launch_colsum(x, 1, rows, cols, ld, sum, nullptr, s);
  const int64_t slices = rows < 32 ? rows : 32;
  const int64_t r0n = (rows + slices - 1) / slices;
  const dim3 grid((unsigned)((cols + kColTile - 1) / kColTile), (unsigned)slices);
  hipLaunchKernelGGL(colsum_part_kernel, grid, dim3(64 * kColWaves), 0, s,
                     static_cast<const uint16_t*>(x), rows, cols, ld, r0n, static_cast<double*>(ws));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_final_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s,
                     static_cast<const double*>(ws), slices, cols, sum);
  return hipGetLastError();
}

hipError_t launch_feature_stats(const float* x, int64_t rows, int64_t cols, float min_var,
                                float* mean, float* inv_std, hipStream_t s) {
  if (cols == 0) return hipSuccess;
  hipLaunchKernelGGL(feature_stats_kernel, dim3((unsigned)((cols + kRedCols - 1) / kRedCols)),
                     dim3(1024), 0, s, x, rows, cols, min_var, mean, inv_std);
  return hipGetLastError();
}

hipError_t launch_standardize(const float* x, const float* mean, const float* inv_std,
                              int64_t rows, int64_t cols, void* y_bf16, hipStream_t s) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(standardize_kernel, grid_for(rows * cols, 256), dim3(256), 0, s, x, mean,
                     inv_std, rows, cols, (uint16_t*)y_bf16);
  return hipGetLastError();
}

hipError_t launch_mse_sigmoid_grad(const float* out, const float* target, int64_t rows,
                                   int64_t cols, void* dz_bf16, double* loss_rows,
                                   hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(mse_sigmoid_grad_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0,
                     s, out, target, rows, cols, (uint16_t*)dz_bf16, loss_rows);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float* w, void* w_bf16, const float* g, float* m, float* v,
                       float lr, float b1, float b2, float eps, int step, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, grid_for(n, 256), dim3(256), 0, s, n, w, (uint16_t*)w_bf16, g,
                     m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_logit_init(const float* u, float* z, float* u_out, int64_t n, float eps,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(logit_init_kernel, grid_for(n, 256), dim3(256), 0, s, u, z, u_out, n, eps);
  return hipGetLastError();
}

hipError_t launch_logit_adam(int64_t n, float* z, float* u, const float* grad_u, float* m,
                             float* v, float lr, float b1, float b2, float eps, int step,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(logit_adam_kernel, grid_for(n, 256), dim3(256), 0, s, n, z, u, grad_u, m, v,
                     lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_best_update(const double* loss, int64_t rows, int64_t cols, int64_t row_stride,
                              int64_t col_stride, int64_t col_base, const float* params,
                              int64_t param_dim, double* best, int64_t* best_idx,
                              float* best_params, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(best_update_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s,
                     loss, rows, cols, row_stride, col_stride, col_base, params, param_dim, best,
                     best_idx, best_params);
  return hipGetLastError();
}

}  // namespace synth
