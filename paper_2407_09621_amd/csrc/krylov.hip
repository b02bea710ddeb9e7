// Flexible GMRES (Sec. 7.1) of many independent problems with its scalars on
// the device: classical Gram-Schmidt applied twice as batched multi-dot /
// multi-axpy launches over all problems (one launch per stage, the problem
// in blockIdx.y), and the Arnoldi normalization, Givens rotations, residual
// estimate, stopping test and the final triangular solve in small kernels
// with one thread per problem.  No value has to reach the host between two
// Krylov steps, so a whole step (V-cycle, apply, Gram-Schmidt, update) can
// be captured once as a graph and replayed; the host reads the problems'
// flags only to decide when to stop issuing steps.  Problems that have
// stopped carry zero vectors through the remaining steps (their step
// scale is 0), and their scalars stay frozen.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sipg {

namespace {

constexpr int kT = 256;
constexpr int kBlocks = 256;  // dot-product blocks per problem

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

// partial[i * kBlocks + block] = sum over the block's range of V_{first+i} . V_w
// (problem blockIdx.y); i < nv <= 8 per launch pass
__global__ __launch_bounds__(kT) void bmdot_kernel(const KrylovDesc* __restrict__ D, int first,
                                                   int nv, int widx) {
  __shared__ double sh[kT / 64];
  const KrylovDesc d = D[blockIdx.y];
  const int64_t n = d.n;
  const double* __restrict__ w = d.V + (int64_t)widx * n;
  for (int i0 = 0; i0 < nv; i0 += 8) {
    const int cnt = min(8, nv - i0);
    double acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)kBlocks * kT) {
      const double we = w[e];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < cnt) acc[i] = fma(d.V[(int64_t)(first + i0 + i) * n + e], we, acc[i]);
    }
    for (int i = 0; i < cnt; ++i) {
      const double s = block_sum(acc[i], sh);
      if (threadIdx.x == 0) d.partial[(int64_t)(i0 + i) * kBlocks + blockIdx.x] = s;
    }
  }
}

// small[off + i] = sum of the kBlocks partials of row i (row blockIdx.x,
// problem blockIdx.y)
__global__ __launch_bounds__(kT) void breduce_kernel(const KrylovDesc* __restrict__ D, int off) {
  __shared__ double sh[kT / 64];
  const KrylovDesc d = D[blockIdx.y];
  double s = 0.0;
  for (int i = threadIdx.x; i < kBlocks; i += kT) s += d.partial[(int64_t)blockIdx.x * kBlocks + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) d.small[off + blockIdx.x] = s;
}

// V_w -= sum_{i < nv} small[coef + i] V_i; if acc >= 0, small[acc + i] += the
// coefficients (block 0 of the problem, after every block has read them:
// the coefficients are staged in LDS first and acc never overlaps coef)
__global__ __launch_bounds__(kT) void bmaxpy_kernel(const KrylovDesc* __restrict__ D, int nv,
                                                    int widx, int coef, int acc) {
  __shared__ double c[kMaxKrylov + 1];
  const KrylovDesc d = D[blockIdx.y];
  for (int i = threadIdx.x; i < nv; i += kT) c[i] = d.small[coef + i];
  __syncthreads();
  const int64_t n = d.n;
  double* __restrict__ w = d.V + (int64_t)widx * n;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    double s = 0.0;
    for (int i = 0; i < nv; ++i) s = fma(c[i], d.V[(int64_t)i * n + e], s);
    w[e] -= s;
  }
  if (acc >= 0 && blockIdx.x == 0)
    for (int i = threadIdx.x; i < nv; i += kT) d.small[acc + i] += c[i];
}

// V_w *= st[kSInv] of the problem
__global__ __launch_bounds__(kT) void bscale_kernel(const KrylovDesc* __restrict__ D, int widx) {
  const KrylovDesc d = D[blockIdx.y];
  const double a = d.st[kSInv];
  const int64_t n = d.n;
  double* __restrict__ w = d.V + (int64_t)widx * n;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    w[e] *= a;
}

// x += sum_{i < m} y_i Z_i with y = st[kSY ..] (zero beyond the steps done)
__global__ __launch_bounds__(kT) void bupdate_kernel(const KrylovDesc* __restrict__ D, int m) {
  __shared__ double c[kMaxKrylov];
  const KrylovDesc d = D[blockIdx.y];
  for (int i = threadIdx.x; i < m; i += kT) c[i] = d.st[kSY + i];
  __syncthreads();
  const int64_t n = d.n;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s = fma(c[i], d.Z[(int64_t)i * n + e], s);
    d.x[e] += s;
  }
}

__device__ __forceinline__ void push_history(double* st, double v) {
  const int h = (int)st[kSHist];
  if (h < kHistory) st[kSHistory + h] = v;
  st[kSHist] = h + 1;
}

// Start of a restart cycle: V_0 = b - A x is in place and ||V_0||^2 in
// small[kNormSlot].  Sets g = (beta, 0, ..), the step scale 1 / beta, or
// stops the problem (converged, budget spent, or not finite).
__global__ __launch_bounds__(64) void fg_start_kernel(const KrylovDesc* __restrict__ D, int P,
                                                      int m) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p >= P) return;
  double* st = D[p].st;
  st[kSJd] = 0.0;
  st[kSInv] = 0.0;
  st[kSActive] = 0.0;
  if (st[kSConv] != 0.0 || st[kSIts] >= st[kSMaxIts] || st[kSBad] != 0.0) return;
  const double beta = sqrt(D[p].small[kNormSlot]);
  if (!isfinite(beta)) {
    st[kSBad] = 1.0;
    return;
  }
  st[kSEst] = beta / st[kSNb];
  push_history(st, st[kSEst]);
  if (beta <= st[kSTol]) {
    st[kSConv] = 1.0;
    return;
  }
  for (int i = 0; i <= m; ++i) st[kSG + i] = 0.0;
  st[kSG] = beta;
  st[kSInv] = 1.0 / beta;
  st[kSActive] = 1.0;
}

// Arnoldi step j of every active problem: the CGS2 column h_{0..j} is in
// small[0 ..], ||w||^2 in small[kNormSlot].  Stores the rotated column of R,
// the new Givens rotation and g, the estimate |g_{j+1}| / ||b||; sets the
// scale of w (1 / h_{j+1,j}, or 0 when the problem stops here).
__global__ __launch_bounds__(64) void fg_step_kernel(const KrylovDesc* __restrict__ D, int P,
                                                     int j, int m) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p >= P) return;
  double* st = D[p].st;
  const double* h = D[p].small;
  st[kSInv] = 0.0;
  if (st[kSActive] == 0.0) return;
  const double hn = sqrt(h[kNormSlot]);
  bool finite = isfinite(hn);
  for (int i = 0; i <= j; ++i) finite = finite && isfinite(h[i]);
  if (!finite) {
    st[kSBad] = 1.0;
    st[kSActive] = 0.0;
    return;
  }
  double col[kMaxKrylov + 1];
  for (int i = 0; i <= j; ++i) col[i] = h[i];
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double c = st[kSCs + i], s = st[kSSn + i];
    const double t = c * col[i] + s * col[i + 1];
    col[i + 1] = -s * col[i] + c * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[j], col[j + 1]);
  const double c = den > 0.0 ? col[j] / den : 1.0, s = den > 0.0 ? col[j + 1] / den : 0.0;
  st[kSCs + j] = c;
  st[kSSn + j] = s;
  col[j] = den;
  for (int i = 0; i <= j; ++i) st[kSR + i + m * j] = col[i];
  const double gj = st[kSG + j];
  st[kSG + j + 1] = -s * gj;
  st[kSG + j] = c * gj;
  st[kSIts] += 1.0;
  st[kSJd] = j + 1;
  st[kSEst] = fabs(st[kSG + j + 1]) / st[kSNb];
  push_history(st, st[kSEst]);
  const bool stop = fabs(st[kSG + j + 1]) <= st[kSTol] || st[kSIts] >= st[kSMaxIts] ||
                    den == 0.0 || !(hn > 0.0) || j + 1 >= m;
  if (stop) {
    st[kSActive] = 0.0;
  } else {
    st[kSInv] = 1.0 / hn;
  }
}

// End of a cycle: y = R^{-1} g over the steps done (zero beyond), and the
// convergence flag from |g_jd|.
__global__ __launch_bounds__(64) void fg_finish_kernel(const KrylovDesc* __restrict__ D, int P,
                                                       int m) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p >= P) return;
  double* st = D[p].st;
  const int J = (int)st[kSJd];
  for (int i = m - 1; i >= 0; --i) {
    double a = 0.0;
    if (i < J) {
      a = st[kSG + i];
      for (int c = i + 1; c < J; ++c) a -= st[kSR + i + m * c] * st[kSY + c];
      a /= st[kSR + i + m * i];
    }
    st[kSY + i] = a;
  }
  if (J > 0 && fabs(st[kSG + J]) <= st[kSTol]) st[kSConv] = 1.0;
  st[kSActive] = 0.0;
}

// flags[p * kFlagCount + i] = st[kSActive + i] (the host's view of every problem)
__global__ __launch_bounds__(64) void fg_flags_kernel(const KrylovDesc* __restrict__ D, int P,
                                                      double* __restrict__ flags) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p >= P) return;
  for (int i = 0; i < kFlagCount; ++i) flags[p * kFlagCount + i] = D[p].st[kSActive + i];
}

int vec_grid(int64_t nmax) {
  const int64_t g = (nmax + kT - 1) / kT;
  return (int)(g < 1024 ? (g < 1 ? 1 : g) : 1024);
}

}  // namespace

hipError_t launch_krylov_dots(const KrylovDesc* D, int P, int first, int nv, int widx, int off,
                              hipStream_t s) {
  if (P < 1 || P > 65535 || nv < 1 || nv > kMaxKrylov + 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bmdot_kernel, dim3(kBlocks, P), dim3(kT), 0, s, D, first, nv, widx);
  hipLaunchKernelGGL(breduce_kernel, dim3(nv, P), dim3(kT), 0, s, D, off);
  return hipGetLastError();
}

hipError_t launch_krylov_axpy(const KrylovDesc* D, int P, int64_t nmax, int nv, int widx,
                              int coef, int acc, hipStream_t s) {
  if (P < 1 || P > 65535 || nv < 1 || nv > kMaxKrylov + 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bmaxpy_kernel, dim3(vec_grid(nmax), P), dim3(kT), 0, s, D, nv, widx, coef,
                     acc);
  return hipGetLastError();
}

hipError_t launch_krylov_scale(const KrylovDesc* D, int P, int64_t nmax, int widx, hipStream_t s) {
  if (P < 1 || P > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bscale_kernel, dim3(vec_grid(nmax), P), dim3(kT), 0, s, D, widx);
  return hipGetLastError();
}

hipError_t launch_krylov_update(const KrylovDesc* D, int P, int64_t nmax, int m, hipStream_t s) {
  if (P < 1 || P > 65535 || m < 1 || m > kMaxKrylov) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bupdate_kernel, dim3(vec_grid(nmax), P), dim3(kT), 0, s, D, m);
  return hipGetLastError();
}

hipError_t launch_krylov_scalars(int stage, const KrylovDesc* D, int P, int j, int m,
                                 double* flags, hipStream_t s) {
  if (P < 1 || m < 1 || m > kMaxKrylov || j < 0 || j >= m) return hipErrorInvalidValue;
  const dim3 grid((P + 63) / 64);
  switch (stage) {
    case 0: hipLaunchKernelGGL(fg_start_kernel, grid, dim3(64), 0, s, D, P, m); break;
    case 1: hipLaunchKernelGGL(fg_step_kernel, grid, dim3(64), 0, s, D, P, j, m); break;
    case 2: hipLaunchKernelGGL(fg_finish_kernel, grid, dim3(64), 0, s, D, P, m); break;
    case 3:
      if (!flags) return hipErrorInvalidValue;
      hipLaunchKernelGGL(fg_flags_kernel, grid, dim3(64), 0, s, D, P, flags);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace sipg
