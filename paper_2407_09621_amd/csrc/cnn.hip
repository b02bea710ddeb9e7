// Kernels of the learned correction stage (see cnn.h for the network and
// the data layouts).  The two 32 -> 32 layers, which carry almost all of
// the arithmetic, run on the matrix cores as implicit GEMMs
// (v_mfma_f32_16x16x32_f16: 16 grid points x 16 output channels x 32 input
// channels per instruction); the 1-channel first and last layers, the
// training reductions and Adam are plain vector code.
#include <hip/hip_runtime.h>

#include "cnn.h"

namespace sipg {
namespace cnn {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr int kR = 4;  // receptive radius of four 3x3x3 layers

// neighbour of grid point (gx, gy, gz) at offset index d (d = 9 (dz+1) +
// 3 (dy+1) + dx + 1), or -1 outside the grid; `sign` = -1 mirrors the offset
__device__ __forceinline__ int neighbour(int gx, int gy, int gz, int d, int G, int sign) {
  const int dz = (d / 9 - 1) * sign, dy = ((d / 3) % 3 - 1) * sign, dx = (d % 3 - 1) * sign;
  const int x = gx + dx, y = gy + dy, z = gz + dz;
  if (x < 0 || x >= G || y < 0 || y >= G || z < 0 || z >= G) return -1;
  return (z * G + y) * G + x;
}

// cell-blocked index of grid point (gx, gy, gz): n^3 cells of N^3 nodes
__device__ __forceinline__ int64_t cell_index(int gx, int gy, int gz, int n, int N) {
  const int cx = gx / N, cy = gy / N, cz = gz / N;
  const int i = gx - cx * N, j = gy - cy * N, l = gz - cz * N;
  return ((int64_t)(cx + n * (cy + n * cz)) * N + l) * N * N + j * N + i;
}

// ---- layer 1: 1 -> 32, ReLU -------------------------------------------------
__global__ __launch_bounds__(kT) void in_fwd_kernel(const _Float16* __restrict__ x, int G,
                                                    int64_t total, const float* __restrict__ prm,
                                                    _Float16* __restrict__ a1) {
  __shared__ float w[27 * kC];
  __shared__ float bb[kC];
  for (int i = threadIdx.x; i < 27 * kC; i += kT) w[(i % 27) * kC + i / 27] = prm[kW1 + i];
  if (threadIdx.x < kC) bb[threadIdx.x] = prm[kB1 + threadIdx.x];
  __syncthreads();
  const int64_t gp = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (gp >= total) return;
  const int64_t G3 = (int64_t)G * G * G;
  const int64_t base = gp - gp % G3;
  const int p = (int)(gp - base);
  const int gx = p % G, gy = (p / G) % G, gz = p / (G * G);
  float nb[27];
#pragma unroll
  for (int d = 0; d < 27; ++d) {
    const int q = neighbour(gx, gy, gz, d, G, 1);
    nb[d] = q >= 0 ? (float)x[base + q] : 0.0f;
  }
  h8 o[4];
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    float acc = bb[c];
#pragma unroll
    for (int d = 0; d < 27; ++d) acc = fmaf(w[d * kC + c], nb[d], acc);
    o[c / 8][c % 8] = (_Float16)fmaxf(acc, 0.0f);
  }
  h8* dst = reinterpret_cast<h8*>(a1 + gp * kC);
#pragma unroll
  for (int c = 0; c < 4; ++c) dst[c] = o[c];
}

// ---- layers 2 and 3: 32 -> 32 on the matrix cores ------------------------------
// One wave computes 16 consecutive x-points of TY x TZ grid lines for all 32
// output channels: 2 x 16-channel blocks x TY x TZ accumulator tiles.  For
// each x-shift the wave holds the 18 weight fragments of the 9 (dy, dz)
// offsets and 2 channel blocks in registers and streams the (TY+2)(TZ+2)
// shifted input lines past them; each line feeds every output line it
// touches.  Operand layouts of the instruction (A 16x32, B 32x16, D 16x16):
// lane L holds A[L%16][8(L/16)..+7], B[8(L/16)..+7][L%16] and
// D[4(L/16)+r][L%16], r = 0..3.
constexpr int TY = 4, TZ = 2;

template <int MODE>
__global__ __launch_bounds__(kT) void mid_kernel(const _Float16* __restrict__ in,
                                                 const h8* __restrict__ wp,
                                                 const float* __restrict__ bias,
                                                 const _Float16* __restrict__ act_prev,
                                                 _Float16* __restrict__ out, int G, int ns) {
  const int lane = threadIdx.x & 63;
  const int nbx = G / 16, nby = G / TY, nbz = G / TZ;
  const int64_t nwb = (int64_t)ns * nbx * nby * nbz;
  int64_t t = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
  if (t >= nwb) return;
  const int bx = (int)(t % nbx);
  t /= nbx;
  const int by = (int)(t % nby);
  t /= nby;
  const int bz = (int)(t % nbz);
  const int smp = (int)(t / nbz);
  const int x0 = bx * 16, y0 = by * TY, z0 = bz * TZ;
  const int64_t G3 = (int64_t)G * G * G;
  const _Float16* src = in + (int64_t)smp * G3 * kC;
  const int li = lane & 15, lg = lane >> 4;

  f4 acc[TZ][TY][2];
#pragma unroll
  for (int a = 0; a < TZ; ++a)
#pragma unroll
    for (int b = 0; b < TY; ++b) {
      acc[a][b][0] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      acc[a][b][1] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }

#pragma unroll
  for (int dxi = 0; dxi < 3; ++dxi) {
    h8 B[3][3][2];
#pragma unroll
    for (int dyi = 0; dyi < 3; ++dyi)
#pragma unroll
      for (int dzi = 0; dzi < 3; ++dzi)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
          B[dzi][dyi][nb] = wp[(((dxi * 3 + dyi) * 3 + dzi) * 2 + nb) * 64 + lane];
    const int xs = x0 + li + dxi - 1;
    const bool xok = xs >= 0 && xs < G;
#pragma unroll
    for (int iz = 0; iz < TZ + 2; ++iz) {
      const int zs = z0 + iz - 1;
#pragma unroll
      for (int iy = 0; iy < TY + 2; ++iy) {
        const int ys = y0 + iy - 1;
        h8 A = h8{0, 0, 0, 0, 0, 0, 0, 0};
        if (xok && ys >= 0 && ys < G && zs >= 0 && zs < G)
          A = *reinterpret_cast<const h8*>(src + (((int64_t)zs * G + ys) * G + xs) * kC + lg * 8);
#pragma unroll
        for (int dzi = 0; dzi < 3; ++dzi) {
          const int oz = iz - dzi;
          if (oz < 0 || oz >= TZ) continue;
#pragma unroll
          for (int dyi = 0; dyi < 3; ++dyi) {
            const int oy = iy - dyi;
            if (oy < 0 || oy >= TY) continue;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
              acc[oz][oy][nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, B[dzi][dyi][nb],
                                                                       acc[oz][oy][nb], 0, 0, 0);
          }
        }
      }
    }
  }

  _Float16* dst = out + (int64_t)smp * G3 * kC;
  const _Float16* prev = act_prev ? act_prev + (int64_t)smp * G3 * kC : nullptr;
#pragma unroll
  for (int oz = 0; oz < TZ; ++oz)
#pragma unroll
    for (int oy = 0; oy < TY; ++oy)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int co = nb * 16 + li;
        const float bv = MODE == 0 ? bias[co] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t o =
              (((int64_t)(z0 + oz) * G + (y0 + oy)) * G + x0 + lg * 4 + r) * kC + co;
          float v = acc[oz][oy][nb][r];
          if (MODE == 0) v = fmaxf(v + bv, 0.0f);
          else v = (float)prev[o] > 0.0f ? v : 0.0f;
          dst[o] = (_Float16)v;
        }
      }
}

// ---- layer 4: 32 -> 1 ------------------------------------------------------------
__device__ __forceinline__ float out_point(const _Float16* __restrict__ a3, int gx, int gy,
                                           int gz, int G, const float* w, float b4) {
  float acc = b4;
  for (int d = 0; d < 27; ++d) {
    const int q = neighbour(gx, gy, gz, d, G, 1);
    if (q < 0) continue;
    const h8* v = reinterpret_cast<const h8*>(a3 + (int64_t)q * kC);
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      const h8 u = v[c4];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc = fmaf(w[d * kC + c4 * 8 + e], (float)u[e], acc);
    }
  }
  return acc;
}

__global__ __launch_bounds__(kT) void out_fwd_kernel(const _Float16* __restrict__ a3, int G,
                                                     int64_t total, const float* __restrict__ prm,
                                                     float scale, float* __restrict__ y) {
  __shared__ float w[27 * kC];
  for (int i = threadIdx.x; i < 27 * kC; i += kT) w[(i % 27) * kC + i / 27] = prm[kW4 + i];
  __syncthreads();
  const int64_t gp = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (gp >= total) return;
  const int64_t G3 = (int64_t)G * G * G;
  const int64_t base = gp - gp % G3;
  const int p = (int)(gp - base);
  y[gp] = scale * out_point(a3 + base * kC, p % G, (p / G) % G, p / (G * G), G, w, prm[kB4]);
}

__global__ __launch_bounds__(kT) void out_scatter_kernel(const _Float16* __restrict__ a3, int n,
                                                         int N, const float* __restrict__ prm,
                                                         float sigma,
                                                         const double* __restrict__ scale,
                                                         double* __restrict__ z) {
  __shared__ float w[27 * kC];
  for (int i = threadIdx.x; i < 27 * kC; i += kT) w[(i % 27) * kC + i / 27] = prm[kW4 + i];
  __syncthreads();
  const int G = n * N;
  const int64_t total = (int64_t)G * G * G;
  const int64_t gp = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (gp >= total) return;
  const int p = (int)gp;
  const int gx = p % G, gy = (p / G) % G, gz = p / (G * G);
  const double s = scale[0];
  if (s == 0.0) return;
  const float v = out_point(a3, gx, gy, gz, G, w, prm[kB4]);
  z[cell_index(gx, gy, gz, n, N)] += s * (double)sigma * (double)v;
}

// ---- FP16 weight fragments ---------------------------------------------------------
__global__ __launch_bounds__(kT) void pack_kernel(const float* __restrict__ prm,
                                                  _Float16* __restrict__ packed) {
  const int e = blockIdx.x * kT + threadIdx.x;
  if (e >= 4 * kPacked) return;
  const int which = e / kPacked, q = e % kPacked;
  const int el = q % 8, lane = (q / 8) % 64, nb = (q / 512) % 2, f = q / 1024;
  const int dzi = f % 3, dyi = (f / 3) % 3, dxi = f / 9;
  const int base = (which & 1) ? kW3 : kW2;
  const int j = nb * 16 + lane % 16, k = (lane / 16) * 8 + el;
  float v;
  if (which < 2)  // forward: B[k = ci][j = co]
    v = prm[base + (j * kC + k) * 27 + dzi * 9 + dyi * 3 + dxi];
  else  // data gradient: B[k = co][j = ci] at the mirrored offset
    v = prm[base + (k * kC + j) * 27 + (2 - dzi) * 9 + (2 - dyi) * 3 + (2 - dxi)];
  packed[e] = (_Float16)v;
}

// ---- grid mapping --------------------------------------------------------------------
constexpr int kRedBlocks = 1024;

__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kT / 64; ++i) r = fmax(r, sh[i]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kT) void absmax_kernel(const double* __restrict__ v, int64_t n,
                                                    double* __restrict__ partial) {
  __shared__ double sh[kT / 64];
  double m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    m = fmax(m, fabs(v[e]));
  m = block_max(m, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(kT) void pow2_kernel(const double* __restrict__ partial, int nb,
                                                  double* __restrict__ scale) {
  __shared__ double sh[kT / 64];
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += kT) m = fmax(m, partial[i]);
  m = block_max(m, sh);
  if (threadIdx.x == 0) {
    double s = 0.0;
    if (m > 0.0) {
      int e;
      const double f = frexp(m, &e);  // m = f 2^e, f in [0.5, 1)
      s = ldexp(1.0, f == 0.5 ? e - 1 : e);
    }
    scale[0] = s;
  }
}

__global__ __launch_bounds__(kT) void gather16_kernel(const double* __restrict__ v, int n, int N,
                                                      const double* __restrict__ scale,
                                                      _Float16* __restrict__ x) {
  const int G = n * N;
  const int64_t gp = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (gp >= (int64_t)G * G * G) return;
  const int p = (int)gp;
  const double s = scale[0];
  const double u = v[cell_index(p % G, (p / G) % G, p / (G * G), n, N)];
  x[gp] = (_Float16)(s > 0.0 ? (float)(u / s) : 0.0f);
}

__global__ __launch_bounds__(kT) void gather32_kernel(const double* __restrict__ v, int n, int N,
                                                      const double* __restrict__ scale,
                                                      float* __restrict__ g) {
  const int G = n * N;
  const int64_t gp = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (gp >= (int64_t)G * G * G) return;
  const int p = (int)gp;
  const double s = scale[0];
  const double u = v[cell_index(p % G, (p / G) % G, p / (G * G), n, N)];
  g[gp] = s > 0.0 ? (float)(u / s) : 0.0f;
}

__global__ __launch_bounds__(kT) void axpy_ratio_kernel(const double* __restrict__ num,
                                                        const double* __restrict__ den,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ y, int64_t n) {
  const double d = den[0];
  const double a = d > 0.0 ? num[0] / d : 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    y[e] = fma(a, x[e], y[e]);
}

// out = v / scale[0] (0 where scale[0] = 0)
__global__ __launch_bounds__(kT) void div_scale_kernel(const double* __restrict__ v,
                                                       const double* __restrict__ scale,
                                                       double* __restrict__ out, int64_t n) {
  const double d = scale[0];
  const double a = d > 0.0 ? 1.0 / d : 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    out[e] = a * v[e];
}

// sums[0] = rr / pp (the relative residual loss), sums[1] = sigma pp / (2 S)
// (the normalisation that turns the scaled output gradient -grid(A r) / S
// into dL/dy, see launch_reduce_rows)
__global__ void residual_sums_kernel(const double* __restrict__ rr, const double* __restrict__ pp,
                                     const double* __restrict__ S, const double* __restrict__ ab,
                                     float sigma, float* __restrict__ sums) {
  if (threadIdx.x == 0) {
    const double p = pp[0], sc = S[0], a = ab[0], b = ab[1];
    sums[0] = p > 0.0 ? (float)(rr[0] / p) : 0.0f;
    // gradient factor 2 sigma alpha S / p with alpha = a / b; 0: no gradient
    sums[1] = (p > 0.0 && sc > 0.0 && a != 0.0 && b > 0.0)
                  ? (float)(sigma * p * b / (2.0 * a * sc)) : 0.0f;
  }
}

__global__ __launch_bounds__(kT) void f32_to_f16_kernel(const float* __restrict__ a,
                                                        _Float16* __restrict__ b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT)
    b[e] = (_Float16)a[e];
}

// ---- training ------------------------------------------------------------------------
__device__ __forceinline__ float block_sumf(float v, float* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = 0.0f;
  if (threadIdx.x == 0)
    for (int i = 0; i < kT / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kT) void loss_kernel(const float* __restrict__ y,
                                                  const float* __restrict__ t,
                                                  const float* __restrict__ m, int64_t n,
                                                  float sigma, float* __restrict__ g4,
                                                  float* __restrict__ partial) {
  __shared__ float sh[kT / 64];
  float se = 0.0f, sm = 0.0f;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    // residual in units of the network output; the sigma^2 of the loss
    // gradient is applied in the final reduction (keeps g4 O(1) for FP16)
    const float d = y[e] - t[e] / sigma;
    g4[e] = 2.0f * m[e] * d;
    se = fmaf(m[e] * d, d, se);
    sm += m[e];
  }
  se = block_sumf(se, sh);
  sm = block_sumf(sm, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = se;
    partial[2 * blockIdx.x + 1] = sm;
  }
}

__global__ __launch_bounds__(kT) void loss_final_kernel(const float* __restrict__ partial, int nb,
                                                        float sigma2, float* __restrict__ sums) {
  __shared__ float sh[kT / 64];
  float se = 0.0f, sm = 0.0f;
  for (int i = threadIdx.x; i < nb; i += kT) {
    se += partial[2 * i];
    sm += partial[2 * i + 1];
  }
  se = block_sumf(se, sh);
  sm = block_sumf(sm, sh);
  if (threadIdx.x == 0) {
    sums[0] = sm > 0.0f ? sigma2 * se / sm : 0.0f;  // the masked mean of (sigma y - t)^2
    sums[1] = sm;
  }
}

__global__ __launch_bounds__(kT) void out_bwd_kernel(const float* __restrict__ g4,
                                                     const _Float16* __restrict__ a3, int G,
                                                     int64_t total, const float* __restrict__ prm,
                                                     _Float16* __restrict__ g3) {
  __shared__ float w[27 * kC];
  for (int i = threadIdx.x; i < 27 * kC; i += kT) w[(i % 27) * kC + i / 27] = prm[kW4 + i];
  __syncthreads();
  const int64_t gq = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (gq >= total) return;
  const int64_t G3 = (int64_t)G * G * G;
  const int64_t base = gq - gq % G3;
  const int q = (int)(gq - base);
  const int gx = q % G, gy = (q / G) % G, gz = q / (G * G);
  float gn[27];
#pragma unroll
  for (int d = 0; d < 27; ++d) {
    const int p = neighbour(gx, gy, gz, d, G, -1);  // p = q - offset(d)
    gn[d] = p >= 0 ? g4[base + p] : 0.0f;
  }
  const h8* av = reinterpret_cast<const h8*>(a3 + gq * kC);
  h8* dst = reinterpret_cast<h8*>(g3 + gq * kC);
#pragma unroll
  for (int c4 = 0; c4 < 4; ++c4) {
    const h8 a = av[c4];
    h8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int c = c4 * 8 + e;
      float acc = 0.0f;
#pragma unroll
      for (int d = 0; d < 27; ++d) acc = fmaf(w[d * kC + c], gn[d], acc);
      o[e] = (_Float16)((float)a[e] > 0.0f ? acc : 0.0f);
    }
    dst[c4] = o;
  }
}

// ---- weight gradients on the matrix cores ---------------------------------------
// Every weight gradient is a sum over grid points of a product of two
// point-indexed operands, dW[m][n] = sum_p A[p][m] B[p][n]: a GEMM whose
// contraction runs over the points.  The matrix-core operand of one lane is
// 8 consecutive contraction indices, so both operands are read as "octets",
// 8 consecutive x-points of one channel (16 bytes), from copies laid out
// [p / 8][channel][p % 8] (octets_kernel, or scalar_octets_kernel for the
// one-channel fields).  A tap's x-shift is built into the copy (one copy per
// shift s, holding src[p + s] and zero where x + s leaves the grid); its y
// and z shifts move whole octets, because G is a multiple of 16.
//   layers 2, 3: A = g^T (output channel), B = a shifted by the tap (input
//                channel); 27 taps, each a 32 x 32 block; bias: B = ones.
//   layer 1:     A = g1^T, B = x shifted by tap (tap d = column), column 27 =
//                ones for the bias.
//   layer 4:     A = a3^T, B = g4 shifted back by the tap (sum_p g4[p]
//                a3[p + d] = sum_q a3[q] g4[q - d]); bias: A = ones, tap 13.
// Operands as in the forward kernel (16x16x32: lane L holds A[L%16][8(L/16)
// ..+7], B[8(L/16)..+7][L%16], D[4(L/16)+r][L%16]).

__device__ __align__(16) _Float16 g_zero_octet[8];

// dst[(o 32 + c) 8 + e] = src[(8 o + e + sh) 32 + c], zero where x + sh
// leaves the grid line; one thread per (octet, 8 channels)
__global__ __launch_bounds__(kT) void octets_kernel(const _Float16* __restrict__ src, int G,
                                                    int64_t noct, int sh,
                                                    _Float16* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= noct * 4) return;
  const int64_t o = t >> 2;
  const int cg = (int)(t & 3);
  const int x0 = (int)((8 * o) % G);
  h8 v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int xs = x0 + e + sh;
    v[e] = (xs >= 0 && xs < G)
               ? *reinterpret_cast<const h8*>(src + (8 * o + e + sh) * kC + cg * 8)
               : h8{0, 0, 0, 0, 0, 0, 0, 0};
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    h8 w;
#pragma unroll
    for (int e = 0; e < 8; ++e) w[e] = v[e][c];
    *reinterpret_cast<h8*>(dst + (o * kC + cg * 8 + c) * 8) = w;
  }
}

// dst[p] = src[p + sh] as FP16, zero where x + sh leaves the grid line
template <typename T>
__global__ __launch_bounds__(kT) void scalar_octets_kernel(const T* __restrict__ src, int G,
                                                           int64_t np, int sh,
                                                           _Float16* __restrict__ dst) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= np) return;
  const int xs = (int)(p % G) + sh;
  dst[p] = (xs >= 0 && xs < G) ? (_Float16)src[p + sh] : (_Float16)0.0f;
}

__device__ __forceinline__ h8 load_octet(const _Float16* p) {
  return *reinterpret_cast<const h8*>(p);
}

// KIND 0: layers 2, 3 (At = g^T, Bs = shifted a^T copies, bstride = np * 32)
// KIND 1: layer 1 (At = g1^T, Bs = shifted x copies, bstride = np)
// KIND 2: layer 4 (At = a3^T, Bs = shifted g4 copies, bstride = np)
// A step is 32 points (4 octets, one per lane group); block b takes steps
// [b spb, (b + 1) spb).  KIND 0 (512 threads): the eight waves share the
// steps and split the 27 taps and the bias (at most 4 each, 64 accumulators
// per lane); KINDs 1 and 2 (256 threads): the waves split the steps and sum
// through LDS.  One partial row per block.
constexpr int kWgradMidThreads = 512;
template <int KIND>
__global__ __launch_bounds__(KIND == 0 ? kWgradMidThreads : kT) void wgrad_mfma_kernel(const _Float16* __restrict__ At,
                                                        const _Float16* __restrict__ Bs,
                                                        int64_t bstride, int G, int64_t nsteps,
                                                        int64_t spb, float* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = lane & 15, h = lane >> 4;
  const int64_t G3 = (int64_t)G * G * G;
  const int64_t s0 = (int64_t)blockIdx.x * spb;
  const int64_t s1 = s0 + spb < nsteps ? s0 + spb : nsteps;
  const h8 ones = h8{1, 1, 1, 1, 1, 1, 1, 1};
  const int64_t oy = G / 8, oz = (int64_t)G * G / 8;  // octets per y and z step

  if constexpr (KIND == 0) {
    constexpr int kSeg = kC * kC * 27 + kC;
    constexpr int W = kWgradMidThreads / 64, TPW = (28 + W - 1) / W;  // taps (+ bias) per wave
    f4 acc[TPW][2][2], accb[2];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int a = 0; a < 2; ++a) acc[t][a][0] = acc[t][a][1] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    accb[0] = accb[1] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t st = s0; st < s1; ++st) {
      const int64_t o = 4 * st + h;
      const int64_t pp = (8 * o) % G3;
      const int y = (int)((pp / G) % G), z = (int)(pp / ((int64_t)G * G));
      const h8 A0 = load_octet(At + (o * kC + i) * 8);
      const h8 A1 = load_octet(At + (o * kC + 16 + i) * 8);
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int d = wave + W * t;
        if (d < 27) {
          const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
          const bool ok = (unsigned)(y + dy) < (unsigned)G && (unsigned)(z + dz) < (unsigned)G;
          const _Float16* b = Bs + (dx + 1) * bstride + ((o + dy * oy + dz * oz) * kC + i) * 8;
          const h8 B0 = load_octet(ok ? b : g_zero_octet);
          const h8 B1 = load_octet(ok ? b + 16 * 8 : g_zero_octet);
          acc[t][0][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, B0, acc[t][0][0], 0, 0, 0);
          acc[t][0][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, B1, acc[t][0][1], 0, 0, 0);
          acc[t][1][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, B0, acc[t][1][0], 0, 0, 0);
          acc[t][1][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, B1, acc[t][1][1], 0, 0, 0);
        } else if (d == 27) {
          accb[0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, ones, accb[0], 0, 0, 0);
          accb[1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, ones, accb[1], 0, 0, 0);
        }
      }
    }
    float* row = part + (int64_t)blockIdx.x * kSeg;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int d = wave + W * t;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = a * 16 + 4 * h + r;
          if (d < 27) {
            row[(co * kC + i) * 27 + d] = acc[t][a][0][r];
            row[(co * kC + 16 + i) * 27 + d] = acc[t][a][1][r];
          } else if (d == 27 && i == 0) {
            row[kC * kC * 27 + co] = accb[a][r];
          }
        }
    }
  } else {
    constexpr int kSeg = KIND == 1 ? kC * 27 + kC : kC * 27 + 1;
    __shared__ float s_red[3][20][64];
    f4 acc[2][2], accb;
    acc[0][0] = acc[0][1] = acc[1][0] = acc[1][1] = accb = f4{0.0f, 0.0f, 0.0f, 0.0f};
    // this lane's tap in each of the two column blocks
    int dxs[2], dys[2], dzs[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      const int d = nb * 16 + i;
      dxs[nb] = d % 3 - 1;
      dys[nb] = (d / 3) % 3 - 1;
      dzs[nb] = d / 9 - 1;
    }
    for (int64_t st = s0 + wave; st < s1; st += kT / 64) {
      const int64_t o = 4 * st + h;
      const int64_t pp = (8 * o) % G3;
      const int y = (int)((pp / G) % G), z = (int)(pp / ((int64_t)G * G));
      const h8 A0 = load_octet(At + (o * kC + i) * 8);
      const h8 A1 = load_octet(At + (o * kC + 16 + i) * 8);
      h8 B[2];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int d = nb * 16 + i;
        // layer 1 reads x at p + tap, layer 4 reads g4 at q - tap
        const int sg = KIND == 1 ? 1 : -1;
        const int dx = sg * dxs[nb], dy = sg * dys[nb], dz = sg * dzs[nb];
        const bool ok = d < 27 && (unsigned)(y + dy) < (unsigned)G &&
                        (unsigned)(z + dz) < (unsigned)G;
        const _Float16* b = Bs + (dx + 1) * bstride + (o + dy * oy + dz * oz) * 8;
        B[nb] = load_octet(ok ? b : g_zero_octet);
        if (KIND == 1 && d == 27) B[nb] = ones;
      }
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, B[0], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A0, B[1], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, B[0], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, B[1], acc[1][1], 0, 0, 0);
      if constexpr (KIND == 2)
        accb = __builtin_amdgcn_mfma_f32_16x16x32_f16(ones, B[0], accb, 0, 0, 0);
    }
    // sum the four waves' accumulators through LDS, wave 0 writes the row
    if (wave > 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        s_red[wave - 1][0 + r][lane] = acc[0][0][r];
        s_red[wave - 1][4 + r][lane] = acc[0][1][r];
        s_red[wave - 1][8 + r][lane] = acc[1][0][r];
        s_red[wave - 1][12 + r][lane] = acc[1][1][r];
        s_red[wave - 1][16 + r][lane] = accb[r];
      }
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc[0][0][r] += s_red[w][0 + r][lane];
        acc[0][1][r] += s_red[w][4 + r][lane];
        acc[1][0][r] += s_red[w][8 + r][lane];
        acc[1][1][r] += s_red[w][12 + r][lane];
        accb[r] += s_red[w][16 + r][lane];
      }
    float* row = part + (int64_t)blockIdx.x * kSeg;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = a * 16 + 4 * h + r;  // output channel (layer 1) / input channel (4)
          const int d = nb * 16 + i;
          if (d < 27) row[m * 27 + d] = acc[a][nb][r];
          else if (KIND == 1 && d == 27) row[kC * 27 + m] = acc[a][nb][r];
        }
    if (KIND == 2 && lane == 13) row[kC * 27] = accb[0];
  }
}

__global__ __launch_bounds__(kT) void reduce_rows_kernel(const float* __restrict__ part, int seg,
                                                         const float* __restrict__ sums,
                                                         float sigma2, float* __restrict__ grad) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= seg) return;
  float s = 0.0f;
  for (int b = 0; b < kWgradRows; ++b) s += part[(int64_t)b * seg + i];
  const float tot = sums[1];
  grad[i] = tot != 0.0f ? sigma2 * s / tot : 0.0f;
}

__global__ __launch_bounds__(kT) void adam_kernel(float* __restrict__ prm, float* __restrict__ m,
                                                  float* __restrict__ v,
                                                  const float* __restrict__ grad, int n, float lr,
                                                  float b1, float b2, float eps, float c1,
                                                  float c2) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  prm[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ __launch_bounds__(kT) void crops_kernel(const float* __restrict__ in,
                                                   const float* __restrict__ target, int G, int c,
                                                   CropJob j, _Float16* __restrict__ x16,
                                                   float* __restrict__ t,
                                                   float* __restrict__ m) {
  const int64_t c3 = (int64_t)c * c * c;
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= c3 * j.count) return;
  const int k = (int)(e / c3);
  const int loc = (int)(e - (int64_t)k * c3);
  const int lx = loc % c, ly = (loc / c) % c, lz = loc / (c * c);
  const int oz = j.off[k][0], oy = j.off[k][1], ox = j.off[k][2];
  const int64_t src = ((int64_t)(oz + lz) * G + (oy + ly)) * G + (ox + lx);
  auto keep = [&](int o, int l) {
    if (o > 0 && l < kR) return false;
    if (o + c < G && l >= c - kR) return false;
    return true;
  };
  x16[e] = (_Float16)in[src];
  t[e] = target[src];
  m[e] = (keep(oz, lz) && keep(oy, ly) && keep(ox, lx)) ? 1.0f : 0.0f;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

hipError_t launch_in_fwd(const _Float16* x, int G, int ns, const float* prm, _Float16* a1,
                         hipStream_t s) {
  if (G < 1 || ns < 1) return hipErrorInvalidValue;
  const int64_t total = (int64_t)ns * G * G * G;
  hipLaunchKernelGGL(in_fwd_kernel, dim3(blocks_for(total)), dim3(kT), 0, s, x, G, total, prm, a1);
  return hipGetLastError();
}

hipError_t launch_mid(int mode, const _Float16* in, const _Float16* packed, const float* bias,
                      const _Float16* act_prev, _Float16* out, int G, int ns, hipStream_t s) {
  if (G < kTile || G % kTile || ns < 1) return hipErrorInvalidValue;
  if (mode == 1 && !act_prev) return hipErrorInvalidValue;
  const int64_t nwb = (int64_t)ns * (G / 16) * (G / TY) * (G / TZ);
  const dim3 grid((unsigned)((nwb + 3) / 4));
  const h8* wp = reinterpret_cast<const h8*>(packed);
  if (mode == 0)
    hipLaunchKernelGGL(mid_kernel<0>, grid, dim3(kT), 0, s, in, wp, bias, act_prev, out, G, ns);
  else
    hipLaunchKernelGGL(mid_kernel<1>, grid, dim3(kT), 0, s, in, wp, bias, act_prev, out, G, ns);
  return hipGetLastError();
}

hipError_t launch_out_fwd(const _Float16* a3, int G, int ns, const float* prm, float scale,
                          float* y, hipStream_t s) {
  if (G < 1 || ns < 1) return hipErrorInvalidValue;
  const int64_t total = (int64_t)ns * G * G * G;
  hipLaunchKernelGGL(out_fwd_kernel, dim3(blocks_for(total)), dim3(kT), 0, s, a3, G, total, prm,
                     scale, y);
  return hipGetLastError();
}

hipError_t launch_out_scatter(const _Float16* a3, int n, int N, const float* prm, float sigma,
                              const double* scale, double* z, hipStream_t s) {
  const int64_t G = (int64_t)n * N;
  hipLaunchKernelGGL(out_scatter_kernel, dim3(blocks_for(G * G * G)), dim3(kT), 0, s, a3, n, N,
                     prm, sigma, scale, z);
  return hipGetLastError();
}

hipError_t launch_pack(const float* prm, _Float16* packed4, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(4 * kPacked)), dim3(kT), 0, s, prm, packed4);
  return hipGetLastError();
}

hipError_t launch_pow2_absmax(const double* v, int64_t n, double* partial, double* scale,
                              hipStream_t s) {
  if (n < 1) return hipErrorInvalidValue;
  int64_t g = (n + kT - 1) / kT;
  const int nb = (int)(g < kRedBlocks ? g : kRedBlocks);
  hipLaunchKernelGGL(absmax_kernel, dim3(nb), dim3(kT), 0, s, v, n, partial);
  hipLaunchKernelGGL(pow2_kernel, dim3(1), dim3(kT), 0, s, partial, nb, scale);
  return hipGetLastError();
}

hipError_t launch_gather_f16(const double* v, int n, int N, const double* scale, _Float16* x,
                             hipStream_t s) {
  const int64_t G = (int64_t)n * N;
  hipLaunchKernelGGL(gather16_kernel, dim3(blocks_for(G * G * G)), dim3(kT), 0, s, v, n, N, scale, x);
  return hipGetLastError();
}

hipError_t launch_gather_f32(const double* v, int n, int N, const double* scale, float* g,
                             hipStream_t s) {
  const int64_t G = (int64_t)n * N;
  hipLaunchKernelGGL(gather32_kernel, dim3(blocks_for(G * G * G)), dim3(kT), 0, s, v, n, N, scale, g);
  return hipGetLastError();
}

hipError_t launch_axpy_ratio(const double* num, const double* den, const double* x, double* y,
                             int64_t n, hipStream_t s) {
  int64_t g = (n + kT - 1) / kT;
  hipLaunchKernelGGL(axpy_ratio_kernel, dim3((unsigned)(g < 8192 ? (g < 1 ? 1 : g) : 8192)),
                     dim3(kT), 0, s, num, den, x, y, n);
  return hipGetLastError();
}

hipError_t launch_div_scale(const double* v, const double* scale, double* out, int64_t n,
                            hipStream_t s) {
  int64_t g = (n + kT - 1) / kT;
  hipLaunchKernelGGL(div_scale_kernel, dim3((unsigned)(g < 8192 ? (g < 1 ? 1 : g) : 8192)),
                     dim3(kT), 0, s, v, scale, out, n);
  return hipGetLastError();
}

hipError_t launch_residual_sums(const double* rr, const double* pp, const double* S,
                                const double* ab, float sigma, float* sums, hipStream_t s) {
  hipLaunchKernelGGL(residual_sums_kernel, dim3(1), dim3(64), 0, s, rr, pp, S, ab, sigma, sums);
  return hipGetLastError();
}

hipError_t launch_f32_to_f16(const float* a, _Float16* b, int64_t n, hipStream_t s) {
  int64_t g = (n + kT - 1) / kT;
  hipLaunchKernelGGL(f32_to_f16_kernel, dim3((unsigned)(g < 8192 ? (g < 1 ? 1 : g) : 8192)),
                     dim3(kT), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t launch_loss(const float* y, const float* t, const float* m, int64_t n, float sigma,
                       float* g4, float* partial, float* sums, hipStream_t s) {
  if (n < 1) return hipErrorInvalidValue;
  int64_t g = (n + kT - 1) / kT;
  const int nb = (int)(g < kRedBlocks ? g : kRedBlocks);
  hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(kT), 0, s, y, t, m, n, sigma, g4, partial);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(kT), 0, s, partial, nb, sigma * sigma, sums);
  return hipGetLastError();
}

hipError_t launch_out_bwd(const float* g4, const _Float16* a3, int G, int ns, const float* prm,
                          _Float16* g3, hipStream_t s) {
  const int64_t total = (int64_t)ns * G * G * G;
  hipLaunchKernelGGL(out_bwd_kernel, dim3(blocks_for(total)), dim3(kT), 0, s, g4, a3, G, total,
                     prm, g3);
  return hipGetLastError();
}

// octet copies for one layer's weight gradient and the MFMA kernel
template <int KIND>
static hipError_t wgrad(const _Float16* At, const _Float16* Bs, int64_t bstride, int G,
                        int64_t np, float* part, hipStream_t s) {
  const int64_t nsteps = np / 32;
  const int64_t spb = (nsteps + kWgradRows - 1) / kWgradRows;
  hipLaunchKernelGGL(wgrad_mfma_kernel<KIND>, dim3(kWgradRows),
                     dim3(KIND == 0 ? kWgradMidThreads : kT), 0, s, At, Bs, bstride,
                     G, nsteps, spb, part);
  return hipGetLastError();
}

hipError_t launch_out_wgrad(const _Float16* a3, const float* g4, int G, int ns,
                            const WgradBufs& w, float* part, hipStream_t s) {
  const int64_t np = (int64_t)ns * G * G * G, noct = np / 8;
  hipLaunchKernelGGL(octets_kernel, dim3(blocks_for(noct * 4)), dim3(kT), 0, s, a3, G, noct, 0,
                     w.ot);
  for (int sh = -1; sh <= 1; ++sh)
    hipLaunchKernelGGL(scalar_octets_kernel<float>, dim3(blocks_for(np)), dim3(kT), 0, s, g4, G,
                       np, sh, w.os + (sh + 1) * np);
  return wgrad<2>(w.ot, w.os, np, G, np, part, s);
}

hipError_t launch_mid_wgrad(const _Float16* a, const _Float16* g, int G, int ns,
                            const WgradBufs& w, float* part, hipStream_t s) {
  const int64_t np = (int64_t)ns * G * G * G, noct = np / 8;
  hipLaunchKernelGGL(octets_kernel, dim3(blocks_for(noct * 4)), dim3(kT), 0, s, g, G, noct, 0,
                     w.ot);
  for (int sh = -1; sh <= 1; ++sh)
    hipLaunchKernelGGL(octets_kernel, dim3(blocks_for(noct * 4)), dim3(kT), 0, s, a, G, noct, sh,
                       w.os + (sh + 1) * np * kC);
  return wgrad<0>(w.ot, w.os, np * kC, G, np, part, s);
}

hipError_t launch_in_wgrad(const _Float16* x, const _Float16* g1, int G, int ns,
                           const WgradBufs& w, float* part, hipStream_t s) {
  const int64_t np = (int64_t)ns * G * G * G, noct = np / 8;
  hipLaunchKernelGGL(octets_kernel, dim3(blocks_for(noct * 4)), dim3(kT), 0, s, g1, G, noct, 0,
                     w.ot);
  for (int sh = -1; sh <= 1; ++sh)
    hipLaunchKernelGGL(scalar_octets_kernel<_Float16>, dim3(blocks_for(np)), dim3(kT), 0, s, x,
                       G, np, sh, w.os + (sh + 1) * np);
  return wgrad<1>(w.ot, w.os, np, G, np, part, s);
}

hipError_t launch_reduce_rows(const float* part, int seg, const float* sums, float sigma,
                              float* grad, hipStream_t s) {
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(blocks_for(seg)), dim3(kT), 0, s, part, seg, sums,
                     sigma * sigma, grad);
  return hipGetLastError();
}

hipError_t launch_adam(float* prm, float* m, float* v, const float* grad, int n, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(kT), 0, s, prm, m, v, grad, n, lr,
                     beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_crops(const float* in, const float* target, int G, int c, const CropJob& j,
                        _Float16* x16, float* t, float* m, hipStream_t s) {
  if (j.count < 1 || j.count > 16 || c < 1 || c > G) return hipErrorInvalidValue;
  for (int k = 0; k < j.count; ++k)
    for (int a = 0; a < 3; ++a)
      if (j.off[k][a] < 0 || j.off[k][a] + c > G) return hipErrorInvalidValue;
  const int64_t total = (int64_t)c * c * c * j.count;
  hipLaunchKernelGGL(crops_kernel, dim3(blocks_for(total)), dim3(kT), 0, s, in, target, G, c, j,
                     x16, t, m);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace sipg
