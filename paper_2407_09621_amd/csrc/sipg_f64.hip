// FP64 kernels of the SIPG operator, the vertex-patch fast-diagonalization
// smoother, the exact coarse solve and the level transfers on gfx950.
//
// Operator (Sec. 2.1, eq. tensorproduct_3d): on a uniform Cartesian level
// A = h (Mh (x) Mh (x) Lh + Mh (x) Lh (x) Mh + Lh (x) Mh (x) Mh), where the
// global Lh is block-tridiagonal: its diagonal blocks hold the cell
// stiffness plus the face terms seen from inside the cell, and the
// off-diagonal blocks couple a cell to its face neighbour only through the
// neighbour's face value and normal derivative (the 1 x N evaluators S_f and
// D_f of Sec. 2.1).  The cell part is applied by sum factorization, one
// direction at a time (the N x N by N x N^2 products of Sec. 4.1):
//   t1 = Lx u + (x-face terms),  t2 = Mx u
//   c  = My t1 + Ly t2 + (y-face terms, after Mx),  e = My t2
//   v  = h (Mz c + Lz e + (z-face terms, after Mx My)).
// The DG "pull" form writes each cell's block from exactly one work item:
// no atomics.  Work items map to workgroups through an XCD-aware permutation
// so that consecutive cells (and their face neighbours) share an L2.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sipg {

namespace {

constexpr int kThreads = 256;

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of work items instead.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

template <int N>
__device__ __forceinline__ void matvec(const double* __restrict__ A, const double (&x)[N],
                                       double (&y)[N]) {
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) s = fma(A[a * N + b], x[b], s);
    y[a] = s;
  }
}

template <int N>
__device__ __forceinline__ void matvec_acc(const double* __restrict__ A, const double (&x)[N],
                                           double (&y)[N]) {
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double s = y[a];
#pragma unroll
    for (int b = 0; b < N; ++b) s = fma(A[a * N + b], x[b], s);
    y[a] = s;
  }
}

// y = A^T x
template <int N>
__device__ __forceinline__ void matvec_t(const double* __restrict__ A, const double (&x)[N],
                                         double (&y)[N]) {
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) s = fma(A[b * N + a], x[b], s);
    y[a] = s;
  }
}

// Face coupling to the lower neighbour (its high-end value f and derivative
// g = d1 . u) and to the upper neighbour (low-end value f, g = d0 . u).
template <int N>
__device__ __forceinline__ void add_lower_face(double (&t)[N], double f, double g, double gam,
                                               const double* __restrict__ d0) {
  t[0] += -gam * f + 0.5 * g;
#pragma unroll
  for (int a = 0; a < N; ++a) t[a] = fma(-0.5 * d0[a], f, t[a]);
}
template <int N>
__device__ __forceinline__ void add_upper_face(double (&t)[N], double f, double g, double gam,
                                               const double* __restrict__ d1) {
  t[N - 1] += -gam * f - 0.5 * g;
#pragma unroll
  for (int a = 0; a < N; ++a) t[a] = fma(0.5 * d1[a], f, t[a]);
}

__device__ __forceinline__ int bdry_variant(int coord, int n) {
  return (coord == 0 ? 1 : 0) | (coord == n - 1 ? 2 : 0);
}

// ---------------------------------------------------------------------------
// Operator apply: CPB cells per workgroup, one thread per 1D line per stage.
// ---------------------------------------------------------------------------
template <int N, bool RES>
__global__ __launch_bounds__(kThreads) void apply_f64_kernel(
    const double* __restrict__ u, double* __restrict__ v, const double* __restrict__ bvec,
    const double* __restrict__ tab, TableLayout lay, int n, double h, int ncells) {
  constexpr int N2 = N * N, N3 = N2 * N, CPB = kThreads / N2;
  __shared__ double s_M[N2];
  __shared__ double s_L[4 * N2];
  __shared__ double s_d0[N], s_d1[N];
  __shared__ double s_u[CPB * N3];
  __shared__ double s_t1[CPB * N3];
  __shared__ double s_t2[CPB * N3];
  __shared__ double s_tr[CPB * 12 * N2];  // [cell][face 0..5][value, derivative][N2]

  const int tid = threadIdx.x;
  const int c0 = xcd_remap(blockIdx.x, gridDim.x) * CPB;
  const int nc = min(CPB, ncells - c0);
  if (nc <= 0) return;
  for (int i = tid; i < N2; i += kThreads) s_M[i] = tab[lay.mass + i];
  for (int i = tid; i < 4 * N2; i += kThreads) s_L[i] = tab[lay.lcell + i];
  if (tid < N) {
    s_d0[tid] = tab[lay.d0 + tid];
    s_d1[tid] = tab[lay.d1 + tid];
  }
  const double gam = tab[lay.gam];
  const double* ug = u + (size_t)c0 * N3;
  for (int i = tid; i < nc * N3; i += kThreads) s_u[i] = ug[i];
  __syncthreads();

  // Face traces of the six neighbours: value on the shared face and the
  // normal derivative there (reference coordinates).
  const int nn = n * n;
  for (int w = tid; w < nc * 6 * N2; w += kThreads) {
    const int cl = w / (6 * N2), r = w - cl * 6 * N2;
    const int face = r / N2, pq = r - face * N2;
    const int p = pq % N, q = pq / N;
    const int c = c0 + cl;
    const int d = face >> 1, upper = face & 1;
    const int coord = d == 0 ? c % n : (d == 1 ? (c / n) % n : c / nn);
    const bool has = upper ? (coord < n - 1) : (coord > 0);
    double f = 0.0, g = 0.0;
    if (has) {
      const int sc = d == 0 ? 1 : (d == 1 ? n : nn);
      const int cn = upper ? c + sc : c - sc;
      const double* src = (cn >= c0 && cn < c0 + nc) ? s_u + (cn - c0) * N3 : u + (size_t)cn * N3;
      const int sn = d == 0 ? 1 : (d == 1 ? N : N2);
      const int base = d == 0 ? (p * N + q * N2) : (d == 1 ? (p + q * N2) : (p + q * N));
      const double* dv = upper ? s_d0 : s_d1;
      f = src[base + (upper ? 0 : (N - 1) * sn)];
#pragma unroll
      for (int a = 0; a < N; ++a) g = fma(dv[a], src[base + a * sn], g);
    }
    s_tr[(cl * 12 + face * 2 + 0) * N2 + pq] = f;
    s_tr[(cl * 12 + face * 2 + 1) * N2 + pq] = g;
  }
  __syncthreads();
  // Mass along x on the y- and z-face traces (index p).
  for (int w = tid; w < nc * 8 * N; w += kThreads) {
    const int cl = w / (8 * N), r = w - cl * 8 * N, fa = r / N, q = r - fa * N;
    double* t = s_tr + (cl * 12 + 4 + fa) * N2 + q * N;
    double x[N], y[N];
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = t[a];
    matvec<N>(s_M, x, y);
#pragma unroll
    for (int a = 0; a < N; ++a) t[a] = y[a];
  }
  __syncthreads();
  // Mass along y on the z-face traces (index q).
  for (int w = tid; w < nc * 4 * N; w += kThreads) {
    const int cl = w / (4 * N), r = w - cl * 4 * N, fa = r / N, p = r - fa * N;
    double* t = s_tr + (cl * 12 + 8 + fa) * N2 + p;
    double x[N], y[N];
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = t[a * N];
    matvec<N>(s_M, x, y);
#pragma unroll
    for (int a = 0; a < N; ++a) t[a * N] = y[a];
  }
  __syncthreads();

  // x stage: lines (j, l)
  if (tid < nc * N2) {
    const int cl = tid / N2, jl = tid - cl * N2;
    const int cx = (c0 + cl) % n;
    double x[N], t1[N], t2[N];
    const double* src = s_u + cl * N3 + jl * N;
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = src[a];
    matvec<N>(s_L + bdry_variant(cx, n) * N2, x, t1);
    matvec<N>(s_M, x, t2);
    const double* tr = s_tr + cl * 12 * N2;
    if (cx > 0) add_lower_face<N>(t1, tr[0 * N2 + jl], tr[1 * N2 + jl], gam, s_d0);
    if (cx < n - 1) add_upper_face<N>(t1, tr[2 * N2 + jl], tr[3 * N2 + jl], gam, s_d1);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      s_t1[cl * N3 + jl * N + a] = t1[a];
      s_t2[cl * N3 + jl * N + a] = t2[a];
    }
  }
  __syncthreads();

  // y stage: lines (i, l)
  if (tid < nc * N2) {
    const int cl = tid / N2, il = tid - cl * N2;
    const int i = il % N, l = il / N;
    const int cy = ((c0 + cl) / n) % n;
    double a1[N], a2[N], cc[N], e[N];
    const int base = cl * N3 + i + l * N2;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      a1[b] = s_t1[base + b * N];
      a2[b] = s_t2[base + b * N];
    }
    matvec<N>(s_M, a1, cc);
    matvec_acc<N>(s_L + bdry_variant(cy, n) * N2, a2, cc);
    matvec<N>(s_M, a2, e);
    const double* tr = s_tr + cl * 12 * N2;
    if (cy > 0) add_lower_face<N>(cc, tr[4 * N2 + il], tr[5 * N2 + il], gam, s_d0);
    if (cy < n - 1) add_upper_face<N>(cc, tr[6 * N2 + il], tr[7 * N2 + il], gam, s_d1);
#pragma unroll
    for (int b = 0; b < N; ++b) {
      s_t1[base + b * N] = cc[b];
      s_t2[base + b * N] = e[b];
    }
  }
  __syncthreads();

  // z stage: lines (i, j), written straight to global memory
  if (tid < nc * N2) {
    const int cl = tid / N2, ij = tid - cl * N2;
    const int c = c0 + cl;
    const int cz = c / nn;
    double a1[N], a2[N], o[N];
    const int base = cl * N3 + ij;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      a1[b] = s_t1[base + b * N2];
      a2[b] = s_t2[base + b * N2];
    }
    matvec<N>(s_M, a1, o);
    matvec_acc<N>(s_L + bdry_variant(cz, n) * N2, a2, o);
    const double* tr = s_tr + cl * 12 * N2;
    if (cz > 0) add_lower_face<N>(o, tr[8 * N2 + ij], tr[9 * N2 + ij], gam, s_d0);
    if (cz < n - 1) add_upper_face<N>(o, tr[10 * N2 + ij], tr[11 * N2 + ij], gam, s_d1);
    double* dst = v + (size_t)c * N3 + ij;
    if (RES) {
      const double* bs = bvec + (size_t)c * N3 + ij;
#pragma unroll
      for (int a = 0; a < N; ++a) dst[a * N2] = bs[a * N2] - h * o[a];
    } else {
#pragma unroll
      for (int a = 0; a < N; ++a) dst[a * N2] = h * o[a];
    }
  }
}

// ---------------------------------------------------------------------------
// Fast-diagonalization solve on vertex patches of one colour:
//   x_P += (1/h) (Sz (x) Sy (x) Sx) diag(1/(lx_i + ly_j + lz_l)) (..)^T r_P
// with (S, l) the generalized eigenpairs of the 2N x 2N patch matrices
// (Lh_P S = Mh_P S diag(l), S^T Mh_P S = I).  Patch layout in LDS:
// i' + G j' + G^2 l' with i' = dx N + i over the two cells of each direction.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kThreads) void patch_fd_f64_kernel(
    const double* __restrict__ r, double* __restrict__ x, const double* __restrict__ tab,
    TableLayout lay, int n, double h, int bx, int by, int bz, int npx, int npy, int npatch) {
  constexpr int G = 2 * N, G2 = G * G, G3 = G2 * G, N2 = N * N, N3 = N2 * N;
  constexpr int PPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  __shared__ double s_S[4 * G2];
  __shared__ double s_l[4 * G];
  __shared__ double s_X[PPB * G3];
  const int tid = threadIdx.x;
  const int p0 = xcd_remap(blockIdx.x, gridDim.x) * PPB;
  const int np = min(PPB, npatch - p0);
  if (np <= 0) return;
  for (int i = tid; i < 4 * G2; i += kThreads) s_S[i] = tab[lay.fd_s + i];
  for (int i = tid; i < 4 * G; i += kThreads) s_l[i] = tab[lay.fd_l + i];

  // vertex of a patch and its first cell
  auto vertex = [&](int pl, int& vx, int& vy, int& vz) {
    const int p = p0 + pl;
    const int px = p % npx, py = (p / npx) % npy, pz = p / (npx * npy);
    vx = 2 * px + (bx ? 1 : 2);
    vy = 2 * py + (by ? 1 : 2);
    vz = 2 * pz + (bz ? 1 : 2);
  };
  const int nn = n * n;
  // gather r_P
  for (int w = tid; w < np * G3; w += kThreads) {
    const int pl = w / G3, rr = w - pl * G3;
    int vx, vy, vz;
    vertex(pl, vx, vy, vz);
    const int cell8 = rr / N3, loc = rr - cell8 * N3;
    const int dx = cell8 & 1, dy = (cell8 >> 1) & 1, dz = cell8 >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int c = (vx - 1 + dx) + n * (vy - 1 + dy) + nn * (vz - 1 + dz);
    s_X[pl * G3 + (dx * N + i) + G * (dy * N + j) + G2 * (dz * N + l)] = r[(size_t)c * N3 + loc];
  }
  __syncthreads();

  const bool act = tid < np * G2;
  const int pl = act ? tid / G2 : 0, ln = tid - pl * G2;
  int vx = 1, vy = 1, vz = 1;
  if (act) vertex(pl, vx, vy, vz);
  const int tx = (vx == 1 ? 1 : 0) | (vx == n - 1 ? 2 : 0);
  const int ty = (vy == 1 ? 1 : 0) | (vy == n - 1 ? 2 : 0);
  const int tz = (vz == 1 ? 1 : 0) | (vz == n - 1 ? 2 : 0);
  double* X = s_X + pl * G3;
  const int la = ln % G, lb = ln / G;
  // offsets of line ln in direction d: start and stride
  const int o0 = la * G + lb * G2, o1 = la + lb * G2, o2 = la + lb * G;
  double in[G], out[G];
  // forward: S^T along x, y, z
  if (act) {
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[o0 + a];
    matvec_t<G>(s_S + tx * G2, in, out);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o0 + a] = out[a];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[o1 + a * G];
    matvec_t<G>(s_S + ty * G2, in, out);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o1 + a * G] = out[a];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[o2 + a * G2];
    matvec_t<G>(s_S + tz * G2, in, out);
    // eigenvalue scaling: line (la, lb) = (i', j'), running over l'
    const double lij = s_l[tx * G + la] + s_l[ty * G + lb];
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = out[a] / (h * (lij + s_l[tz * G + a]));
    matvec<G>(s_S + tz * G2, in, out);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o2 + a * G2] = out[a];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[o1 + a * G];
    matvec<G>(s_S + ty * G2, in, out);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o1 + a * G] = out[a];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[o0 + a];
    matvec<G>(s_S + tx * G2, in, out);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o0 + a] = out[a];
  }
  __syncthreads();
  // scatter-add into x
  for (int w = tid; w < np * G3; w += kThreads) {
    const int q = w / G3, rr = w - q * G3;
    int ux, uy, uz;
    vertex(q, ux, uy, uz);
    const int cell8 = rr / N3, loc = rr - cell8 * N3;
    const int dx = cell8 & 1, dy = (cell8 >> 1) & 1, dz = cell8 >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int c = (ux - 1 + dx) + n * (uy - 1 + dy) + nn * (uz - 1 + dz);
    x[(size_t)c * N3 + loc] += s_X[q * G3 + (dx * N + i) + G * (dy * N + j) + G2 * (dz * N + l)];
  }
}

// ---------------------------------------------------------------------------
// Exact coarse solve by fast diagonalization of the whole n0^3-cell level
// (one workgroup; G = n0 N <= 3N).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kThreads) void coarse_fd_f64_kernel(
    const double* __restrict__ b, double* __restrict__ x, const double* __restrict__ tab,
    TableLayout lay, int n0, double h) {
  constexpr int GM = 3 * N, N2 = N * N, N3 = N2 * N;
  extern __shared__ double s_dyn[];
  const int G = n0 * N, G2 = G * G, G3 = G2 * G;
  double* s_S = s_dyn;
  double* s_l = s_S + G2;
  double* X = s_l + G;
  const int tid = threadIdx.x;
  for (int i = tid; i < G2; i += kThreads) s_S[i] = tab[lay.fdc_s + i];
  for (int i = tid; i < G; i += kThreads) s_l[i] = tab[lay.fdc_l + i];
  const int nn = n0 * n0;
  for (int w = tid; w < G3; w += kThreads) {
    const int c = w / N3, loc = w - c * N3;
    const int cx = c % n0, cy = (c / n0) % n0, cz = c / nn;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    X[(cx * N + i) + G * (cy * N + j) + G2 * (cz * N + l)] = b[w];
  }
  __syncthreads();
  double in[GM], out[GM];
  for (int pass = 0; pass < 6; ++pass) {
    const int d = pass < 3 ? pass : 5 - pass;
    const int sd = d == 0 ? 1 : (d == 1 ? G : G2);
    for (int ln = tid; ln < G2; ln += kThreads) {
      const int la = ln % G, lb = ln / G;
      const int o = d == 0 ? la * G + lb * G2 : (d == 1 ? la + lb * G2 : la + lb * G);
      for (int a = 0; a < G; ++a) in[a] = X[o + a * sd];
      for (int a = 0; a < G; ++a) {
        double s = 0.0;
        if (pass < 3)
          for (int c = 0; c < G; ++c) s = fma(s_S[c * G + a], in[c], s);
        else
          for (int c = 0; c < G; ++c) s = fma(s_S[a * G + c], in[c], s);
        out[a] = s;
      }
      if (pass == 2)
        for (int a = 0; a < G; ++a) out[a] /= h * (s_l[la] + s_l[lb] + s_l[a]);
      for (int a = 0; a < G; ++a) X[o + a * sd] = out[a];
    }
    __syncthreads();
  }
  for (int w = tid; w < G3; w += kThreads) {
    const int c = w / N3, loc = w - c * N3;
    const int cx = c % n0, cy = (c / n0) % n0, cz = c / nn;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    x[w] = X[(cx * N + i) + G * (cy * N + j) + G2 * (cz * N + l)];
  }
}

// ---------------------------------------------------------------------------
// Transfers, one coarse cell per work item.  P1 (2N x N): fine node
// (child c, node a) from coarse node b.  Restriction applies P1^T along x,
// y, z to the 8 children (2N)^3 -> N^3; prolongation applies P1.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kThreads) void restrict_f64_kernel(
    const double* __restrict__ rf, double* __restrict__ rc, const double* __restrict__ tab,
    TableLayout lay, int nc) {
  constexpr int G = 2 * N, G2 = G * G, G3 = G2 * G, N2 = N * N, N3 = N2 * N;
  constexpr int CPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  __shared__ double s_P[G * N];
  __shared__ double s_X[CPB * G3];
  const int tid = threadIdx.x;
  const int ncells = nc * nc * nc;
  const int c0 = xcd_remap(blockIdx.x, gridDim.x) * CPB;
  const int cnt = min(CPB, ncells - c0);
  if (cnt <= 0) return;
  for (int i = tid; i < G * N; i += kThreads) s_P[i] = tab[lay.p1 + i];
  const int nf = 2 * nc;
  for (int w = tid; w < cnt * G3; w += kThreads) {
    const int cl = w / G3, rr = w - cl * G3;
    const int cc = c0 + cl;
    const int cx = cc % nc, cy = (cc / nc) % nc, cz = cc / (nc * nc);
    const int child = rr / N3, loc = rr - child * N3;
    const int ox = child & 1, oy = (child >> 1) & 1, oz = child >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int f = (2 * cx + ox) + nf * (2 * cy + oy) + nf * nf * (2 * cz + oz);
    s_X[cl * G3 + (ox * N + i) + G * (oy * N + j) + G2 * (oz * N + l)] = rf[(size_t)f * N3 + loc];
  }
  __syncthreads();
  // x: lines (j', l') of length G -> N values, stored in place at stride 1
  for (int w = tid; w < cnt * G2; w += kThreads) {
    const int cl = w / G2, ln = w - cl * G2;
    double* X = s_X + cl * G3 + ln * G;
    double in[G];
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[a];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < G; ++a) s = fma(s_P[a * N + b], in[a], s);
      X[b] = s;
    }
  }
  __syncthreads();
  // y: lines (b, l') over j'
  for (int w = tid; w < cnt * N * G; w += kThreads) {
    const int cl = w / (N * G), ln = w - cl * N * G;
    const int bx = ln % N, lz = ln / N;
    double* X = s_X + cl * G3 + bx + lz * G2;
    double in[G];
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[a * G];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < G; ++a) s = fma(s_P[a * N + b], in[a], s);
      X[b * G] = s;
    }
  }
  __syncthreads();
  // z: lines (b, b') over l', written to the coarse vector
  for (int w = tid; w < cnt * N2; w += kThreads) {
    const int cl = w / N2, ln = w - cl * N2;
    const int bx = ln % N, by = ln / N;
    const double* X = s_X + cl * G3 + bx + by * G;
    double in[G];
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[a * G2];
    double* dst = rc + (size_t)(c0 + cl) * N3 + bx + by * N;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < G; ++a) s = fma(s_P[a * N + b], in[a], s);
      dst[b * N2] = s;
    }
  }
}

template <int N>
__global__ __launch_bounds__(kThreads) void prolongate_add_f64_kernel(
    const double* __restrict__ ec, double* __restrict__ xf, const double* __restrict__ tab,
    TableLayout lay, int nc) {
  constexpr int G = 2 * N, G2 = G * G, G3 = G2 * G, N2 = N * N, N3 = N2 * N;
  constexpr int CPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  __shared__ double s_P[G * N];
  __shared__ double s_X[CPB * G3];
  const int tid = threadIdx.x;
  const int ncells = nc * nc * nc;
  const int c0 = xcd_remap(blockIdx.x, gridDim.x) * CPB;
  const int cnt = min(CPB, ncells - c0);
  if (cnt <= 0) return;
  for (int i = tid; i < G * N; i += kThreads) s_P[i] = tab[lay.p1 + i];
  // coarse values at X[b + G b' + G^2 b''] (the low corner of the box)
  for (int w = tid; w < cnt * N3; w += kThreads) {
    const int cl = w / N3, loc = w - cl * N3;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    s_X[cl * G3 + i + G * j + G2 * l] = ec[(size_t)(c0 + cl) * N3 + loc];
  }
  __syncthreads();
  // z first: lines (b, b') over l: N -> G
  for (int w = tid; w < cnt * N2; w += kThreads) {
    const int cl = w / N2, ln = w - cl * N2;
    double* X = s_X + cl * G3 + (ln % N) + (ln / N) * G;
    double in[N];
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = X[b * G2];
#pragma unroll
    for (int a = 0; a < G; ++a) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) s = fma(s_P[a * N + b], in[b], s);
      X[a * G2] = s;
    }
  }
  __syncthreads();
  // y: lines (b, l') over j: N -> G
  for (int w = tid; w < cnt * N * G; w += kThreads) {
    const int cl = w / (N * G), ln = w - cl * N * G;
    double* X = s_X + cl * G3 + (ln % N) + (ln / N) * G2;
    double in[N];
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = X[b * G];
#pragma unroll
    for (int a = 0; a < G; ++a) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) s = fma(s_P[a * N + b], in[b], s);
      X[a * G] = s;
    }
  }
  __syncthreads();
  // x: lines (j', l') over i: N -> G
  for (int w = tid; w < cnt * G2; w += kThreads) {
    const int cl = w / G2, ln = w - cl * G2;
    double* X = s_X + cl * G3 + ln * G;
    double in[N];
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = X[b];
#pragma unroll
    for (int a = 0; a < G; ++a) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) s = fma(s_P[a * N + b], in[b], s);
      X[a] = s;
    }
  }
  __syncthreads();
  const int nf = 2 * nc;
  for (int w = tid; w < cnt * G3; w += kThreads) {
    const int cl = w / G3, rr = w - cl * G3;
    const int cc = c0 + cl;
    const int cx = cc % nc, cy = (cc / nc) % nc, cz = cc / (nc * nc);
    const int child = rr / N3, loc = rr - child * N3;
    const int ox = child & 1, oy = (child >> 1) & 1, oz = child >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int f = (2 * cx + ox) + nf * (2 * cy + oy) + nf * nf * (2 * cz + oz);
    xf[(size_t)f * N3 + loc] += s_X[cl * G3 + (ox * N + i) + G * (oy * N + j) + G2 * (oz * N + l)];
  }
}

template <int N>
hipError_t apply_impl(const double* u, double* v, const double* b, const DevTab& t, int n,
                      double h, hipStream_t s) {
  constexpr int CPB = kThreads / (N * N);
  const int64_t ncells = (int64_t)n * n * n;
  if (ncells <= 0 || ncells > (int64_t)1 << 30) return hipErrorInvalidValue;
  const int grid = (int)((ncells + CPB - 1) / CPB);
  if (b)
    hipLaunchKernelGGL((apply_f64_kernel<N, true>), dim3(grid), dim3(kThreads), 0, s, u, v, b,
                       t.tab, t.lay, n, h, (int)ncells);
  else
    hipLaunchKernelGGL((apply_f64_kernel<N, false>), dim3(grid), dim3(kThreads), 0, s, u, v,
                       nullptr, t.tab, t.lay, n, h, (int)ncells);
  return hipGetLastError();
}

template <int N>
hipError_t patch_impl(int colour, const double* r, double* x, const DevTab& t, int n, double h,
                      hipStream_t s) {
  constexpr int G2 = 4 * N * N;
  constexpr int PPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  const int bx = colour & 1, by = (colour >> 1) & 1, bz = (colour >> 2) & 1;
  // vertices v in [1, n-1]: odd ones 1,3,..; even ones 2,4,..
  auto count = [&](int bit) { return bit ? n / 2 : (n - 1) / 2; };
  const int npx = count(bx), npy = count(by), npz = count(bz);
  const int64_t np = (int64_t)npx * npy * npz;
  if (np == 0) return hipSuccess;
  const int grid = (int)((np + PPB - 1) / PPB);
  hipLaunchKernelGGL((patch_fd_f64_kernel<N>), dim3(grid), dim3(kThreads), 0, s, r, x, t.tab,
                     t.lay, n, h, bx, by, bz, npx, npy, (int)np);
  return hipGetLastError();
}

template <int N>
hipError_t coarse_impl(int n0, const double* b, double* x, const DevTab& t, double h,
                       hipStream_t s) {
  if (n0 < 1 || n0 > 3 || t.lay.Gc != n0 * N) return hipErrorInvalidValue;
  const int G = n0 * N;
  const size_t shm = sizeof(double) * ((size_t)G * G + G + (size_t)G * G * G);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)coarse_fd_f64_kernel<N>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((coarse_fd_f64_kernel<N>), dim3(1), dim3(kThreads), shm, s, b, x, t.tab,
                     t.lay, n0, h);
  return hipGetLastError();
}

template <int N>
hipError_t transfer_impl(bool restr, const double* in, double* out, const DevTab& t, int nc,
                         hipStream_t s) {
  constexpr int G2 = 4 * N * N;
  constexpr int CPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  const int64_t ncells = (int64_t)nc * nc * nc;
  const int grid = (int)((ncells + CPB - 1) / CPB);
  if (restr)
    hipLaunchKernelGGL((restrict_f64_kernel<N>), dim3(grid), dim3(kThreads), 0, s, in, out,
                       t.tab, t.lay, nc);
  else
    hipLaunchKernelGGL((prolongate_add_f64_kernel<N>), dim3(grid), dim3(kThreads), 0, s, in,
                       out, t.tab, t.lay, nc);
  return hipGetLastError();
}

}  // namespace

#define SIPG_DISPATCH_N(N, CALL)                \
  switch (N) {                                  \
    case 2: return CALL(2);                     \
    case 3: return CALL(3);                     \
    case 4: return CALL(4);                     \
    case 5: return CALL(5);                     \
    case 6: return CALL(6);                     \
    case 7: return CALL(7);                     \
    case 8: return CALL(8);                     \
    default: return hipErrorInvalidValue;       \
  }

hipError_t launch_apply_f64(int N, const double* u, double* v, const double* b, const DevTab& t,
                            int n, double h, hipStream_t s) {
  if (t.lay.N != N) return hipErrorInvalidValue;
#define CALL(NN) apply_impl<NN>(u, v, b, t, n, h, s)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_patch_fd_f64(int N, int colour, const double* r, double* x, const DevTab& t,
                               int n, double h, hipStream_t s) {
  if (t.lay.N != N || colour < 0 || colour > 7 || n < 2) return hipErrorInvalidValue;
#define CALL(NN) patch_impl<NN>(colour, r, x, t, n, h, s)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_coarse_fd_f64(int N, int n0, const double* b, double* x, const DevTab& t,
                                double h, hipStream_t s) {
  if (t.lay.N != N) return hipErrorInvalidValue;
#define CALL(NN) coarse_impl<NN>(n0, b, x, t, h, s)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_restrict_f64(int N, const double* rf, double* rc, const DevTab& t, int nc,
                               hipStream_t s) {
  if (t.lay.N != N || nc < 1) return hipErrorInvalidValue;
#define CALL(NN) transfer_impl<NN>(true, rf, rc, t, nc, s)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_prolongate_add_f64(int N, const double* ec, double* xf, const DevTab& t, int nc,
                                     hipStream_t s) {
  if (t.lay.N != N || nc < 1) return hipErrorInvalidValue;
#define CALL(NN) transfer_impl<NN>(false, ec, xf, t, nc, s)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

}  // namespace sipg
