// Manufactured right-hand side and L2 error (Sec. 7.2: Poisson problem with
// the analytical solution sin(pi x) sin(pi y) sin(pi z); sums of such modes).
// For a separable mode the tensor Gauss rule factors into 1D integrals per
// direction, which the host tabulates per cell coordinate; the kernels
// combine them.  The L2 error interpolates u_h to the (k+3)^3 Gauss points
// of each cell by sum factorization (Sec. 2.1, interpolation formula).
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace sipg {

// Workspace of the allocation-free L2 error (sipg_l2_error_sines_noalloc):
// its host-prepared tables, the per-workgroup partial sums and the result.
// Each device holds its own copy until the process ends; host code reaches
// it only through the address hipGetSymbolAddress returns for that device.
static __device__ __align__(256) double scratch[kL2ScratchDoubles];

namespace {

constexpr int kT = 256;

// b[c, i + N j + N^2 l] = sum_m coef_m bx[m][cx][i] by[m][cy][j] bz[m][cz][l]
__global__ __launch_bounds__(kT) void rhs_kernel(int N, int n, int nm, const double* __restrict__ coef,
                                                 const double* __restrict__ bx,
                                                 const double* __restrict__ by,
                                                 const double* __restrict__ bz,
                                                 double* __restrict__ b, int64_t total) {
  const int N3 = N * N * N;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kT) {
    const int64_t c = e / N3;
    const int loc = (int)(e - c * N3);
    const int i = loc % N, j = (loc / N) % N, l = loc / (N * N);
    const int cx = (int)(c % n), cy = (int)((c / n) % n), cz = (int)(c / ((int64_t)n * n));
    double s = 0.0;
    for (int m = 0; m < nm; ++m)
      s += coef[m] * bx[((int64_t)m * n + cx) * N + i] * by[((int64_t)m * n + cy) * N + j] *
           bz[((int64_t)m * n + cz) * N + l];
    b[e] = s;
  }
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
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

constexpr int kMaxQ = 10;  // (k+3) points for k = 7


__global__ __launch_bounds__(kT) void l2_kernel(int N, int nq, int n, int nm,
                                                const double* __restrict__ amps,
                                                const double* __restrict__ sx,
                                                const double* __restrict__ sy,
                                                const double* __restrict__ sz,
                                                const double* __restrict__ interp,
                                                const double* __restrict__ wq, double h,
                                                const double* __restrict__ x,
                                                double* __restrict__ partial) {
  __shared__ double s_phi[kMaxQ * kMaxN];
  __shared__ double s_w[kMaxQ];
  __shared__ double s_X[kMaxN * kMaxN * kMaxN];
  __shared__ double s_T1[kMaxQ * kMaxN * kMaxN];
  __shared__ double s_T2[kMaxQ * kMaxQ * kMaxN];
  __shared__ double sh[kT / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < nq * N; i += kT) s_phi[i] = interp[i];
  if (tid < nq) s_w[tid] = wq[tid];
  const int N2 = N * N, N3 = N2 * N;
  const int64_t ncells = (int64_t)n * n * n;
  const double h3 = h * h * h;
  double acc = 0.0;
  for (int64_t c = blockIdx.x; c < ncells; c += gridDim.x) {
    __syncthreads();
    for (int i = tid; i < N3; i += kT) s_X[i] = x[c * N3 + i];
    __syncthreads();
    for (int t = tid; t < nq * N2; t += kT) {  // T1[qa][j][l]
      const int qa = t % nq, jl = t / nq;
      double s = 0.0;
      for (int i = 0; i < N; ++i) s = fma(s_phi[qa * N + i], s_X[jl * N + i], s);
      s_T1[jl * nq + qa] = s;
    }
    __syncthreads();
    for (int t = tid; t < nq * nq * N; t += kT) {  // T2[qa][qb][l]
      const int qa = t % nq, qb = (t / nq) % nq, l = t / (nq * nq);
      double s = 0.0;
      for (int j = 0; j < N; ++j) s = fma(s_phi[qb * N + j], s_T1[(l * N + j) * nq + qa], s);
      s_T2[(l * nq + qb) * nq + qa] = s;
    }
    __syncthreads();
    const int cx = (int)(c % n), cy = (int)((c / n) % n), cz = (int)(c / ((int64_t)n * n));
    for (int t = tid; t < nq * nq * nq; t += kT) {
      const int qa = t % nq, qb = (t / nq) % nq, qc = t / (nq * nq);
      double uh = 0.0;
      for (int l = 0; l < N; ++l) uh = fma(s_phi[qc * N + l], s_T2[(l * nq + qb) * nq + qa], uh);
      double ue = 0.0;
      for (int m = 0; m < nm; ++m)
        ue += amps[m] * sx[((int64_t)m * n + cx) * nq + qa] * sy[((int64_t)m * n + cy) * nq + qb] *
              sz[((int64_t)m * n + cz) * nq + qc];
      const double d = ue - uh;
      acc += s_w[qa] * s_w[qb] * s_w[qc] * h3 * d * d;
    }
  }
  const double s = block_sum(acc, sh);
  if (tid == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kT) void sum_kernel(const double* __restrict__ partial, int nb,
                                                 double* __restrict__ out) {
  __shared__ double sh[kT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += kT) s += partial[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = s;
}

}  // namespace

hipError_t launch_rhs_sines(int N, int n, int n_modes, const double* coef, const double* bx,
                            const double* by, const double* bz, double* b, hipStream_t s) {
  const int64_t total = (int64_t)n * n * n * N * N * N;
  int64_t g = (total + kT - 1) / kT;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(rhs_kernel, dim3((int)g), dim3(kT), 0, s, N, n, n_modes, coef, bx, by, bz, b,
                     total);
  return hipGetLastError();
}

hipError_t launch_l2_sines(int N, int nq, int n, int n_modes, const double* amps, const double* sx,
                           const double* sy, const double* sz, const double* interp,
                           const double* wq, double h, const double* x, double* partial,
                           double* out, hipStream_t s) {
  if (N > kMaxN || nq > kMaxQ) return hipErrorInvalidValue;
  const int64_t ncells = (int64_t)n * n * n;
  const int grid = (int)(ncells < kDotBlocks ? ncells : kDotBlocks);
  hipLaunchKernelGGL(l2_kernel, dim3(grid), dim3(kT), 0, s, N, nq, n, n_modes, amps, sx, sy, sz,
                     interp, wq, h, x, partial);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kT), 0, s, partial, grid, out);
  return hipGetLastError();
}

hipError_t l2_scratch(double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  static std::mutex mu;
  static double* ptr[kMaxDevices] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));  // the current device's copy
    if (e != hipSuccess) return e;
    ptr[dev] = (double*)a;
  }
  *out = ptr[dev];
  return hipSuccess;
}

}  // namespace sipg
