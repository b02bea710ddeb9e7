// FP64 vector kernels of the FGMRES outer iteration (Sec. 7.1): blocked
// multi-vector dot products and updates for classical Gram-Schmidt applied
// twice, scaling, axpy and a finite-value check.  Reductions are two-pass
// (fixed block partials, then one block) so results are run-to-run
// deterministic.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sipg {

namespace {

constexpr int kT = 256;
constexpr int kMaxVec = 65;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // wave64 reduction, then across the 4 waves of the block
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kT / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// partial[i * gridDim.x + block] = sum over the block's range of V_i . w
__global__ __launch_bounds__(kT) void mdot_kernel(const double* __restrict__ V, int64_t ld,
                                                  int nv, const double* __restrict__ w,
                                                  int64_t n, double* __restrict__ partial) {
  __shared__ double sh[kT / 64];
  double acc[8];
  for (int i0 = 0; i0 < nv; i0 += 8) {
    const int cnt = min(8, nv - i0);
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
      const double we = w[e];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < cnt) acc[i] = fma(V[(int64_t)(i0 + i) * ld + e], we, acc[i]);
    }
    for (int i = 0; i < cnt; ++i) {
      const double s = block_sum(acc[i], sh);
      if (threadIdx.x == 0) partial[(int64_t)(i0 + i) * gridDim.x + blockIdx.x] = s;
    }
  }
}

__global__ __launch_bounds__(kT) void reduce_rows_kernel(const double* __restrict__ partial,
                                                         int nb, double* __restrict__ out) {
  __shared__ double sh[kT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += kT) s += partial[(int64_t)blockIdx.x * nb + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// w -= sign * sum_i coef[i] V_i; acc[i] += coef[i] (one thread does it)
__global__ __launch_bounds__(kT) void maxpy_kernel(const double* __restrict__ V, int64_t ld,
                                                   int nv, const double* __restrict__ coef,
                                                   double* __restrict__ w, int64_t n,
                                                   double* __restrict__ acc, double sign) {
  __shared__ double c[kMaxVec];
  for (int i = threadIdx.x; i < nv; i += kT) c[i] = coef[i];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    double s = 0.0;
    for (int i = 0; i < nv; ++i) s = fma(c[i], V[(int64_t)i * ld + e], s);
    w[e] -= sign * s;
  }
  if (acc && blockIdx.x == 0)
    for (int i = threadIdx.x; i < nv; i += kT) acc[i] += c[i];
}

__global__ __launch_bounds__(kT) void scale_copy_kernel(const double* __restrict__ src,
                                                        double alpha, double* __restrict__ dst,
                                                        int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    dst[e] = alpha * src[e];
}

__global__ __launch_bounds__(kT) void axpy_kernel(double alpha, const double* __restrict__ x,
                                                  double* __restrict__ y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    y[e] = fma(alpha, x[e], y[e]);
}

__global__ __launch_bounds__(kT) void fill_kernel(double* __restrict__ x, double value, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    x[e] = value;
}

__global__ __launch_bounds__(kT) void finite_kernel(const double* __restrict__ x, int64_t n,
                                                    int* __restrict__ flag) {
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    bad |= !isfinite(x[e]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ __launch_bounds__(kT) void to_f32_kernel(const double* __restrict__ src,
                                                    float* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    dst[e] = (float)src[e];
}

__global__ __launch_bounds__(kT) void to_f64_kernel(const float* __restrict__ src,
                                                    double* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    dst[e] = (double)src[e];
}

__global__ __launch_bounds__(kT) void fill_f32_kernel(float* __restrict__ x, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    x[e] = 0.0f;
}

int grid_for(int64_t n) {
  int64_t g = (n + kT - 1) / kT;
  return (int)(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

}  // namespace

hipError_t launch_mdot(const double* V, int64_t ld, int nv, const double* w, int64_t n,
                       double* partial, double* out, hipStream_t s) {
  if (nv < 1 || nv > kMaxVec || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mdot_kernel, dim3(kDotBlocks), dim3(kT), 0, s, V, ld, nv, w, n, partial);
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(nv), dim3(kT), 0, s, partial, kDotBlocks, out);
  return hipGetLastError();
}

hipError_t launch_maxpy(const double* V, int64_t ld, int nv, const double* coef, double* w,
                        int64_t n, double* acc, double sign, hipStream_t s) {
  if (nv < 1 || nv > kMaxVec || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(maxpy_kernel, dim3(grid_for(n)), dim3(kT), 0, s, V, ld, nv, coef, w, n, acc,
                     sign);
  return hipGetLastError();
}

hipError_t launch_scale_copy(const double* src, double alpha, double* dst, int64_t n,
                             hipStream_t s) {
  hipLaunchKernelGGL(scale_copy_kernel, dim3(grid_for(n)), dim3(kT), 0, s, src, alpha, dst, n);
  return hipGetLastError();
}

hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(n)), dim3(kT), 0, s, alpha, x, y, n);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, double value, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(kT), 0, s, x, value, n);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n)), dim3(kT), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_to_f64(const float* src, double* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to_f64_kernel, dim3(grid_for(n)), dim3(kT), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_zero_f32(float* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n)), dim3(kT), 0, s, x, n);
  return hipGetLastError();
}

hipError_t launch_finite_check(const double* x, int64_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(finite_kernel, dim3(grid_for(n)), dim3(kT), 0, s, x, n, flag);
  return hipGetLastError();
}

}  // namespace sipg
