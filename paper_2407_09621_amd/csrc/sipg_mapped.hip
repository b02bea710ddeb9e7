// Operator apply on trilinear hexahedra (general geometry, Sec. 2.1): every
// cell is the image of the reference cube under the trilinear map of its 8
// vertices, and the cell integral becomes
//   A^K = G^T W G,   W = w_q det J J^{-1} J^{-T}  at each quadrature point,
// with G the values / reference gradients of the basis at the points (sum
// factorization along x, y, z).  The face terms of eq. bilinear_form use the
// physical normal and surface measure: on the reference face
//   n dsigma = det J J^{-T} n_hat dA = C n_hat dA,  C = cof(J),
// so that grad u . n dsigma = grad_xi u . (C^T nu / det J) with nu = C n_hat w.
//
// Quadrature is N-point Gauss per direction on cells and N x N on faces (the
// rule of the Cartesian operator, exact on affine cells).  The penalty of a
// face is k(k+1)(1/h- + 1/h+) with h = |K| / |e| on each side (2k(k+1)/h-
// on the boundary), computed once per face on the host.
//
// One workgroup per cell: the cell's block and the stage arrays live in LDS,
// the 16 one-dimensional contractions of the cell term and the two-
// dimensional contractions of the six face terms run over the workgroup's
// threads.  The Jacobians are computed on the fly from the 8 vertices at
// every quadrature point (a few dozen flops per point instead of 48 B per
// point of stored metric terms), so the kernel reads the vector once (plus
// its neighbours' blocks, mostly from L2) and 72 B of geometry per cell.
// Workgroups are mapped to cells in contiguous chunks per XCD so that a
// cell's neighbours are likely in the same L2.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sipg {

namespace {

// column `col` of the Jacobian dx_i / dxi_col of the trilinear map through X
// (vertex a + 2b + 4c at X[3 (a + 2b + 4c) + i]); it depends only on the two
// other reference coordinates, xa < xb in direction order
__device__ __forceinline__ void jac_column(const double* X, int col, double xa, double xb,
                                           double out[3]) {
  // vertex pairs (hi, lo) along col, ordered by the other two corner bits
  const int step = col == 0 ? 1 : (col == 1 ? 2 : 4);
  const int sa = col == 0 ? 2 : 1;          // bit of the first other direction
  const int sb = col == 2 ? 2 : 4;          // bit of the second
  const double wa[2] = {1.0 - xa, xa}, wb[2] = {1.0 - xb, xb};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
#pragma unroll
    for (int bb = 0; bb < 2; ++bb)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int lo = a * sa + bb * sb;
        s += (X[3 * (lo + step) + i] - X[3 * lo + i]) * wa[a] * wb[bb];
      }
    out[i] = s;
  }
}

// cofactor matrix C (J^{-T} = C / det J) and the determinant
__device__ __forceinline__ double cofactor(const double J[3][3], double C[3][3]) {
  C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  return J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
}

template <int N>
constexpr int mapped_threads() {
  return N <= 3 ? 64 : (N == 4 ? 128 : 256);
}

// The points a thread of a T-thread workgroup takes in the stage loops over
// a cell block (p = tid + j T < N^3) with their three coordinates, and over
// the six faces' N x N arrays (it = tid + j T < 6 N^2) with their two
// tangential coordinates, computed once instead of in every stage.
template <int N, int T>
struct CellPts {
  static constexpr int PP = (N * N * N + T - 1) / T;
  int p[PP], o[3][PP];
  __device__ __forceinline__ explicit CellPts(int tid) {
#pragma unroll
    for (int j = 0; j < PP; ++j) {
      const int q = tid + j * T;
      p[j] = q;
      o[0][j] = q % N;
      o[1][j] = (q / N) % N;
      o[2][j] = q / (N * N);
    }
  }
  __device__ __forceinline__ bool ok(int j) const { return PP * T == N * N * N || p[j] < N * N * N; }
};

template <int N, int T>
struct FacePts {
  static constexpr int PF = (6 * N * N + T - 1) / T;
  int p[PF], o[2][PF];
  __device__ __forceinline__ explicit FacePts(int tid) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int q = tid + j * T;
      p[j] = q;
      o[0][j] = (q % (N * N)) % N;
      o[1][j] = (q % (N * N)) / N;
    }
  }
  __device__ __forceinline__ bool ok(int j) const { return PF * T == 6 * N * N || p[j] < 6 * N * N; }
};

// dst[p] (+)= sum_a M'[o][a] src[p with its index o along DIR replaced by a]
// over the N^3 points of a cell block (x fastest); M' = M (row-major
// M[o * N + a]) or, for TR, its transpose
template <int N, int T, int DIR, bool TR, bool ACC>
__device__ __forceinline__ void line3(const double* M, const double* src, double* dst,
                                      const CellPts<N, T>& P) {
  constexpr int st = DIR == 0 ? 1 : (DIR == 1 ? N : N * N);
#pragma unroll
  for (int j = 0; j < CellPts<N, T>::PP; ++j) {
    if (!P.ok(j)) continue;
    const int p = P.p[j], o = P.o[DIR][j];
    const int base = p - o * st;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) s += (TR ? M[a * N + o] : M[o * N + a]) * src[base + a * st];
    dst[p] = ACC ? dst[p] + s : s;
  }
}

// the same on the six N x N face arrays (index t1 + N t2, face-major);
// DIR 0 contracts along t1, 1 along t2
template <int N, int T, int DIR, bool TR, bool ACC>
__device__ __forceinline__ void line2(const double* M, const double* src, double* dst,
                                      const FacePts<N, T>& P) {
  constexpr int st = DIR == 0 ? 1 : N;
#pragma unroll
  for (int j = 0; j < FacePts<N, T>::PF; ++j) {
    if (!P.ok(j)) continue;
    const int it = P.p[j], o = P.o[DIR][j];
    const int base = it - o * st;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) s += (TR ? M[a * N + o] : M[o * N + a]) * src[base + a * st];
    dst[it] = ACC ? dst[it] + s : s;
  }
}

// v = A u, or v = b - A u when b != nullptr.  mtab: S [N x N] (basis at the
// Gauss points, S[q * N + a] = phi_a(g_q)), D [N x N] (derivatives), Gauss
// weights [N], Gauss points [N], phi'(0) [N], phi'(1) [N].  Cell c of the
// launch is (blockIdx % 8) * chunk + blockIdx / 8 (contiguous chunks of
// cells per XCD); blocks beyond n^3 cells return at once.  VT is the vector
// type: FP32 vectors (the FP32 V-cycle's residuals) are widened on load and
// the result is rounded to FP32 on store; the arithmetic is FP64.
template <typename VT, int N>
__global__ __launch_bounds__(mapped_threads<N>()) void apply_mapped_kernel(
    const VT* __restrict__ u, VT* __restrict__ v, const VT* __restrict__ b,
    const double* __restrict__ vert, const double* __restrict__ gam,
    const double* __restrict__ mtab, int n, int chunk) {
  constexpr int T = mapped_threads<N>();
  constexpr int N2 = N * N, N3 = N * N * N, F = 6 * N2;
  constexpr int RA = (5 * N3 > 6 * F) ? 5 * N3 : 6 * F;
  __shared__ double s_tab[2 * N2 + 4 * N];
  __shared__ double s_X[24];
  __shared__ double s_Xn[6 * 24];
  __shared__ double s_gam[6];
  __shared__ double s_u[N3];
  __shared__ double s_v[N3];
  __shared__ double s_a[RA];     // cell stage arrays, then face region 2 (6 arrays)
  __shared__ double s_r1[8 * F]; // face region 1 (8 arrays)
  // Jacobian columns at the Gauss points and the ends 0, 1 (extended index
  // N + side): column c at the extended indices (ea, eb) of the two other
  // directions, s_J[((3 c + i) * E + eb) * E + ea]
  constexpr int E = N + 2;
  __shared__ double s_J[9 * E * E];
  const int tid = threadIdx.x;
  const CellPts<N, T> P3(tid);
  const FacePts<N, T> P2(tid);
  const int nc = n * n * n;
  const int c = (int)(blockIdx.x % 8) * chunk + (int)(blockIdx.x / 8);
  if (c >= nc) return;  // the whole workgroup, before any barrier
  const int pos[3] = {c % n, (c / n) % n, c / (n * n)};
  const int cstride[3] = {1, n, n * n};
  const size_t n1 = (size_t)n + 1;
  auto vtx = [&](int x, int y, int z, int i) { return vert[((z * n1 + y) * n1 + x) * 3 + i]; };

  for (int i = tid; i < 2 * N2 + 4 * N; i += T) s_tab[i] = mtab[i];
  if (tid < 24) {
    const int w = tid / 3, i = tid % 3;
    s_X[tid] = vtx(pos[0] + (w & 1), pos[1] + ((w >> 1) & 1), pos[2] + (w >> 2), i);
  }
  for (int it = tid; it < 6 * 24; it += T) {
    const int f = it / 24, r = it % 24, d = f >> 1, side = f & 1;
    int q[3] = {pos[0], pos[1], pos[2]};
    q[d] += side ? 1 : -1;
    double val = 0.0;
    if (q[d] >= 0 && q[d] < n) {
      const int w = r / 3, i = r % 3;
      val = vtx(q[0] + (w & 1), q[1] + ((w >> 1) & 1), q[2] + (w >> 2), i);
    }
    s_Xn[it] = val;
  }
  if (tid < 6) s_gam[tid] = gam[(size_t)c * 6 + tid];
  const VT* __restrict__ uc = u + (size_t)c * N3;
  for (int p = tid; p < N3; p += T) s_u[p] = (double)uc[p];
  __syncthreads();

  const double* S = s_tab;
  const double* D = s_tab + N2;
  const double* W = s_tab + 2 * N2;
  const double* G = W + N;
  const double* D0 = G + N;
  const double* D1 = D0 + N;

  for (int e = tid; e < 9 * E * E; e += T) {
    const int ea = e % E, eb = (e / E) % E, ci = e / (E * E);
    const double xa = ea < N ? G[ea] : (double)(ea - N);
    const double xb = eb < N ? G[eb] : (double)(eb - N);
    double col[3];
    jac_column(s_X, ci / 3, xa, xb, col);
    s_J[e] = col[ci % 3];
  }
  // J at the point with extended indices (e0, e1, e2)
  auto jac_at = [&](int e0, int e1, int e2, double J[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      J[i][0] = s_J[((0 * 3 + i) * E + e2) * E + e1];
      J[i][1] = s_J[((1 * 3 + i) * E + e2) * E + e0];
      J[i][2] = s_J[((2 * 3 + i) * E + e1) * E + e0];
    }
  };

  // ---- cell term: reference gradient at the Gauss points, metric, transpose
  double* t0 = s_a;
  double* t1 = s_a + N3;
  double* p1 = s_a + 2 * N3;
  double* p2 = s_a + 3 * N3;
  double* p3 = s_a + 4 * N3;
  line3<N, T, 0, false, false>(S, s_u, t0, P3);
  line3<N, T, 0, false, false>(D, s_u, t1, P3);
  __syncthreads();
  line3<N, T, 1, false, false>(S, t1, p1, P3);  // d/dxi0 branch
  line3<N, T, 1, false, false>(D, t0, p2, P3);  // d/dxi1 branch
  line3<N, T, 1, false, false>(S, t0, p3, P3);  // d/dxi2 branch
  __syncthreads();
  line3<N, T, 2, false, false>(S, p1, t0, P3);
  line3<N, T, 2, false, false>(S, p2, t1, P3);
  line3<N, T, 2, false, false>(D, p3, s_v, P3);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < CellPts<N, T>::PP; ++j) {
    if (!P3.ok(j)) continue;
    const int p = P3.p[j], qx = P3.o[0][j], qy = P3.o[1][j], qz = P3.o[2][j];
    double J[3][3], C[3][3];
    jac_at(qx, qy, qz, J);
    const double det = cofactor(J, C);
    const double g0 = t0[p], g1 = t1[p], g2 = s_v[p];
    double h[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) h[i] = C[i][0] * g0 + C[i][1] * g1 + C[i][2] * g2;
    const double w = W[qx] * W[qy] * W[qz] / det;
    t0[p] = w * (C[0][0] * h[0] + C[1][0] * h[1] + C[2][0] * h[2]);
    t1[p] = w * (C[0][1] * h[0] + C[1][1] * h[1] + C[2][1] * h[2]);
    s_v[p] = w * (C[0][2] * h[0] + C[1][2] * h[1] + C[2][2] * h[2]);
  }
  __syncthreads();
  line3<N, T, 2, true, false>(S, t0, p1, P3);
  line3<N, T, 2, true, false>(S, t1, p2, P3);
  line3<N, T, 2, true, false>(D, s_v, p3, P3);
  __syncthreads();
  line3<N, T, 1, true, false>(S, p1, t0, P3);
  line3<N, T, 1, true, false>(D, p2, t1, P3);
  line3<N, T, 1, true, true>(S, p3, t1, P3);
  __syncthreads();
  line3<N, T, 0, true, false>(D, t0, s_v, P3);
  line3<N, T, 0, true, true>(S, t1, s_v, P3);
  __syncthreads();

  // ---- face terms of the six faces (face f = 2 d + side, side 1 at xi_d = 1)
  double* R1 = s_r1;
  double* R2 = s_a;
  auto tdirs = [](int d, int& a, int& bb) {
    a = d == 0 ? 1 : 0;
    bb = d == 2 ? 1 : 2;
  };
  const int st3[3] = {1, N, N2};
#pragma unroll
  for (int j = 0; j < FacePts<N, T>::PF; ++j) {  // traces at the face nodes
    if (!P2.ok(j)) continue;
    const int it = P2.p[j], f = it / N2, d = f >> 1, side = f & 1;
    const int t1i = P2.o[0][j], t2i = P2.o[1][j];
    int d1, d2;
    tdirs(d, d1, d2);
    const int base = t1i * st3[d1] + t2i * st3[d2];
    const double* Ds = side ? D1 : D0;
    double lm = s_u[base + (side ? N - 1 : 0) * st3[d]], dm = 0.0;
#pragma unroll
    for (int e = 0; e < N; ++e) dm += Ds[e] * s_u[base + e * st3[d]];
    double lp = 0.0, dp = 0.0;
    const int qd = pos[d] + (side ? 1 : -1);
    if (qd >= 0 && qd < n) {
      const VT* __restrict__ un = u + (size_t)(c + (side ? 1 : -1) * cstride[d]) * N3 + base;
      const double* Do = side ? D0 : D1;
      lp = (double)un[(side ? 0 : N - 1) * st3[d]];
#pragma unroll
      for (int e = 0; e < N; ++e) dp += Do[e] * (double)un[e * st3[d]];
    }
    R1[it] = lm;
    R1[F + it] = dm;
    R1[2 * F + it] = lp;
    R1[3 * F + it] = dp;
  }
  __syncthreads();
  line2<N, T, 0, false, false>(S, R1, R2, P2);                  // minus value, along t1
  line2<N, T, 0, false, false>(D, R1, R2 + F, P2);              // minus d/dt1
  line2<N, T, 0, false, false>(S, R1 + F, R2 + 2 * F, P2);      // minus d/dn
  line2<N, T, 0, false, false>(S, R1 + 2 * F, R2 + 3 * F, P2);  // plus value
  line2<N, T, 0, false, false>(D, R1 + 2 * F, R2 + 4 * F, P2);  // plus d/dt1
  line2<N, T, 0, false, false>(S, R1 + 3 * F, R2 + 5 * F, P2);  // plus d/dn
  __syncthreads();
  line2<N, T, 1, false, false>(S, R2, R1, P2);                  // u-
  line2<N, T, 1, false, false>(S, R2 + F, R1 + F, P2);          // du-/dt1
  line2<N, T, 1, false, false>(D, R2, R1 + 2 * F, P2);          // du-/dt2
  line2<N, T, 1, false, false>(S, R2 + 2 * F, R1 + 3 * F, P2);  // du-/dn
  line2<N, T, 1, false, false>(S, R2 + 3 * F, R1 + 4 * F, P2);  // u+
  line2<N, T, 1, false, false>(S, R2 + 4 * F, R1 + 5 * F, P2);  // du+/dt1
  line2<N, T, 1, false, false>(D, R2 + 3 * F, R1 + 6 * F, P2);  // du+/dt2
  line2<N, T, 1, false, false>(S, R2 + 5 * F, R1 + 7 * F, P2);  // du+/dn
  __syncthreads();
#pragma unroll
  for (int j = 0; j < FacePts<N, T>::PF; ++j) {  // integrand at the face quadrature points
    if (!P2.ok(j)) continue;
    const int it = P2.p[j], f = it / N2, d = f >> 1, side = f & 1;
    const int q1 = P2.o[0][j], q2 = P2.o[1][j];
    int d1, d2;
    tdirs(d, d1, d2);
    int ex[3];
    ex[d] = N + side;
    ex[d1] = q1;
    ex[d2] = q2;
    const double wf = W[q1] * W[q2];
    double J[3][3], C[3][3];
    jac_at(ex[0], ex[1], ex[2], J);
    const double det = cofactor(J, C);
    const double sg = side ? wf : -wf;
    const double nu[3] = {sg * C[0][d], sg * C[1][d], sg * C[2][d]};
    const double ds = sqrt(nu[0] * nu[0] + nu[1] * nu[1] + nu[2] * nu[2]);
    double mm[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) mm[e] = (C[0][e] * nu[0] + C[1][e] * nu[1] + C[2][e] * nu[2]) / det;
    double gm[3];
    gm[d] = R1[3 * F + it];
    gm[d1] = R1[F + it];
    gm[d2] = R1[2 * F + it];
    const double um = R1[it];
    const double gmm = gm[0] * mm[0] + gm[1] * mm[1] + gm[2] * mm[2];
    const double gmf = s_gam[f];
    double cv, cs;  // value coefficient, scale of m- in the gradient coefficient
    const int qd = pos[d] + (side ? 1 : -1);
    if (qd >= 0 && qd < n) {
      // the neighbour's Jacobian on the shared face: the same tangential
      // columns (the same bilinear face), its own normal column
      double cn[3];
      jac_column(s_Xn + 24 * f, d, G[q1], G[q2], cn);
      J[0][d] = cn[0];
      J[1][d] = cn[1];
      J[2][d] = cn[2];
      const double detp = cofactor(J, C);
      double gp[3];
      gp[d] = R1[7 * F + it];
      gp[d1] = R1[5 * F + it];
      gp[d2] = R1[6 * F + it];
      double gpm = 0.0;
#pragma unroll
      for (int e = 0; e < 3; ++e)
        gpm += gp[e] * (C[0][e] * nu[0] + C[1][e] * nu[1] + C[2][e] * nu[2]);
      gpm /= detp;
      const double jump = um - R1[4 * F + it];
      cv = gmf * ds * jump - 0.5 * (gmm + gpm);
      cs = -0.5 * jump;
    } else {
      cv = gmf * ds * um - gmm;
      cs = -um;
    }
    R2[it] = cv;
    R2[F + it] = cs * mm[d1];
    R2[2 * F + it] = cs * mm[d2];
    R2[3 * F + it] = cs * mm[d];
  }
  __syncthreads();
  line2<N, T, 1, true, false>(S, R2, R1, P2);
  line2<N, T, 1, true, true>(D, R2 + 2 * F, R1, P2);
  line2<N, T, 1, true, false>(S, R2 + F, R1 + F, P2);
  line2<N, T, 1, true, false>(S, R2 + 3 * F, R1 + 2 * F, P2);
  __syncthreads();
  line2<N, T, 0, true, false>(S, R1, R2, P2);
  line2<N, T, 0, true, true>(D, R1 + F, R2, P2);
  line2<N, T, 0, true, false>(S, R1 + 2 * F, R2 + F, P2);
  __syncthreads();
  const VT* __restrict__ bc = b ? b + (size_t)c * N3 : nullptr;
  VT* __restrict__ vc = v + (size_t)c * N3;
#pragma unroll
  for (int j = 0; j < CellPts<N, T>::PP; ++j) {
    if (!P3.ok(j)) continue;
    const int p = P3.p[j];
    const int id[3] = {P3.o[0][j], P3.o[1][j], P3.o[2][j]};
    double val = s_v[p];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, side = f & 1;
      int d1, d2;
      tdirs(d, d1, d2);
      const int t = f * N2 + id[d1] + N * id[d2];
      if (id[d] == (side ? N - 1 : 0)) val += R2[t];
      val += (side ? D1 : D0)[id[d]] * R2[F + t];
    }
    vc[p] = (VT)(bc ? (double)bc[p] - val : val);
  }
}

// Contraction along DIR of a (d0, d1, d2) array (x fastest) with the table
// M = [NQ][NB] (row-major, basis at the quadrature points): INTERP maps NB
// nodes to NQ points, out[o] = sum_a M[o NB + a] in[a]; otherwise NQ points
// to NB nodes, out[o] = sum_a M[a NB + o] in[a] (the transpose).
template <int T, int DIR, bool INTERP, int NB, int NQ>
__device__ __forceinline__ void contract_q(const double* M, const double* src, double* dst,
                                           int d0, int d1, int d2, int tid) {
  constexpr int IN = INTERP ? NB : NQ, OUT = INTERP ? NQ : NB;
  const int e0 = DIR == 0 ? OUT : d0, e1 = DIR == 1 ? OUT : d1, e2 = DIR == 2 ? OUT : d2;
  const int total = e0 * e1 * e2;
  for (int p = tid; p < total; p += T) {
    const int o0 = p % e0, o1 = (p / e0) % e1, o2 = p / (e0 * e1);
    const int o = DIR == 0 ? o0 : (DIR == 1 ? o1 : o2);
    const int sst = DIR == 0 ? 1 : (DIR == 1 ? d0 : d0 * d1);
    const int base = (DIR == 0 ? 0 : o0) + (DIR == 1 ? 0 : o1) * d0 + (DIR == 2 ? 0 : o2) * d0 * d1;
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < IN; ++a)
      acc += (INTERP ? M[o * NB + a] : M[a * NB + o]) * src[base + a * sst];
    dst[p] = acc;
  }
}

// position and det J of the trilinear map through X at (x0, x1, x2)
__device__ __forceinline__ double map_point(const double* X, double x0, double x1, double x2,
                                            double pos[3]) {
  const double w0[2] = {1.0 - x0, x0}, w1[2] = {1.0 - x1, x1}, w2[2] = {1.0 - x2, x2};
  pos[0] = pos[1] = pos[2] = 0.0;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const double w = w0[v & 1] * w1[(v >> 1) & 1] * w2[v >> 2];
    pos[0] += w * X[3 * v];
    pos[1] += w * X[3 * v + 1];
    pos[2] += w * X[3 * v + 2];
  }
  double J[3][3], C[3][3], col[3];
  jac_column(X, 0, x1, x2, col);
  J[0][0] = col[0]; J[1][0] = col[1]; J[2][0] = col[2];
  jac_column(X, 1, x0, x2, col);
  J[0][1] = col[0]; J[1][1] = col[1]; J[2][1] = col[2];
  jac_column(X, 2, x0, x1, col);
  J[0][2] = col[0]; J[1][2] = col[1]; J[2][2] = col[2];
  return cofactor(J, C);
}

// sum_m s_m[4m] sin(s_m[4m+1] pi x) sin(s_m[4m+2] pi y) sin(s_m[4m+3] pi z)
__device__ __forceinline__ double sine_modes(const double* m, int nm, const double pos[3]) {
  double s = 0.0;
  for (int i = 0; i < nm; ++i)
    s += m[4 * i] * sin(m[4 * i + 1] * M_PI * pos[0]) * sin(m[4 * i + 2] * M_PI * pos[1]) *
         sin(m[4 * i + 3] * M_PI * pos[2]);
  return s;
}

constexpr int kMappedRhsT = 256;

// b_I = int_K f phi_I dx on every trilinear cell (one workgroup per cell),
// (N+1)-point Gauss rule per direction with det J at every point.  modes:
// [nm][coefficient of -Laplace u, p, q, r]; qtab: basis at the points
// [Q][N], weights [Q], points [Q].
template <int N>
__global__ __launch_bounds__(kMappedRhsT) void rhs_mapped_kernel(
    const double* __restrict__ vert, int n, int nm, const double* __restrict__ modes,
    const double* __restrict__ qtab, double* __restrict__ b) {
  constexpr int Q = N + 1, T = kMappedRhsT;
  __shared__ double s_X[24];
  __shared__ double s_tab[Q * N + 2 * Q];
  __shared__ double s_m[4 * 64];
  __shared__ double s_F[Q * Q * Q];
  __shared__ double s_T1[N * Q * Q];
  __shared__ double s_T2[N * N * Q];
  const int tid = threadIdx.x;
  const int c = blockIdx.x;
  const int pos0[3] = {c % n, (c / n) % n, c / (n * n)};
  const size_t n1 = (size_t)n + 1;
  if (tid < 24) {
    const int w = tid / 3, i = tid % 3;
    s_X[tid] = vert[(((pos0[2] + (w >> 2)) * n1 + pos0[1] + ((w >> 1) & 1)) * n1 + pos0[0] +
                     (w & 1)) * 3 + i];
  }
  for (int i = tid; i < Q * N + 2 * Q; i += T) s_tab[i] = qtab[i];
  for (int i = tid; i < 4 * nm; i += T) s_m[i] = modes[i];
  __syncthreads();
  const double* Vq = s_tab;
  const double* wq = s_tab + Q * N;
  const double* xq = wq + Q;
  for (int q = tid; q < Q * Q * Q; q += T) {
    const int qa = q % Q, qb = (q / Q) % Q, qc = q / (Q * Q);
    double pos[3];
    const double det = map_point(s_X, xq[qa], xq[qb], xq[qc], pos);
    s_F[q] = wq[qa] * wq[qb] * wq[qc] * det * sine_modes(s_m, nm, pos);
  }
  __syncthreads();
  contract_q<T, 0, false, N, Q>(Vq, s_F, s_T1, Q, Q, Q, tid);
  __syncthreads();
  contract_q<T, 1, false, N, Q>(Vq, s_T1, s_T2, N, Q, Q, tid);
  __syncthreads();
  contract_q<T, 2, false, N, Q>(Vq, s_T2, b + (size_t)c * N * N * N, N, N, Q, tid);
}

// Partial sums of int (u - u_h)^2 dx over the trilinear cells, (N+2)-point
// Gauss rule per direction: workgroup g takes cells g, g + grid, ...;
// modes: [nm][amplitude, p, q, r].
template <int N>
__global__ __launch_bounds__(kMappedRhsT) void l2_mapped_kernel(
    const double* __restrict__ vert, int n, int nm, const double* __restrict__ modes,
    const double* __restrict__ qtab, const double* __restrict__ x, double* __restrict__ partial) {
  constexpr int Q = N + 2, T = kMappedRhsT, N3 = N * N * N;
  __shared__ double s_X[24];
  __shared__ double s_tab[Q * N + 2 * Q];
  __shared__ double s_m[4 * 64];
  __shared__ double s_U[N3];
  __shared__ double s_T1[Q * N * N];
  __shared__ double s_T2[Q * Q * N];
  __shared__ double s_T3[Q * Q * Q];
  __shared__ double s_red[T / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < Q * N + 2 * Q; i += T) s_tab[i] = qtab[i];
  for (int i = tid; i < 4 * nm; i += T) s_m[i] = modes[i];
  const double* Vq = s_tab;
  const double* wq = s_tab + Q * N;
  const double* xq = wq + Q;
  const int nc = n * n * n;
  const size_t n1 = (size_t)n + 1;
  double acc = 0.0;
  for (int c = blockIdx.x; c < nc; c += gridDim.x) {
    __syncthreads();
    const int pos0[3] = {c % n, (c / n) % n, c / (n * n)};
    if (tid < 24) {
      const int w = tid / 3, i = tid % 3;
      s_X[tid] = vert[(((pos0[2] + (w >> 2)) * n1 + pos0[1] + ((w >> 1) & 1)) * n1 + pos0[0] +
                       (w & 1)) * 3 + i];
    }
    for (int i = tid; i < N3; i += T) s_U[i] = x[(size_t)c * N3 + i];
    __syncthreads();
    contract_q<T, 0, true, N, Q>(Vq, s_U, s_T1, N, N, N, tid);
    __syncthreads();
    contract_q<T, 1, true, N, Q>(Vq, s_T1, s_T2, Q, N, N, tid);
    __syncthreads();
    contract_q<T, 2, true, N, Q>(Vq, s_T2, s_T3, Q, Q, N, tid);
    __syncthreads();
    for (int q = tid; q < Q * Q * Q; q += T) {
      const int qa = q % Q, qb = (q / Q) % Q, qc = q / (Q * Q);
      double pos[3];
      const double det = map_point(s_X, xq[qa], xq[qb], xq[qc], pos);
      const double e = sine_modes(s_m, nm, pos) - s_T3[q];
      acc += wq[qa] * wq[qb] * wq[qc] * det * e * e;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((tid & 63) == 0) s_red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int i = 0; i < T / 64; ++i) s += s_red[i];
    partial[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partial,
                                                           int nb, double* __restrict__ out) {
  __shared__ double s_red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) acc += partial[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

}  // namespace

namespace {

template <typename VT>
hipError_t apply_mapped(int N, const VT* u, VT* v, const VT* b, const MappedLevel& g,
                        const double* mtab, hipStream_t s) {
  if (N < 2 || N > kMaxN || g.n < 1 || g.n > 1024 || !u || !v || !g.vert || !g.gam || !mtab)
    return hipErrorInvalidValue;
  const int nc = g.n * g.n * g.n;
  const int chunk = (nc + 7) / 8;
  const dim3 grid(8 * chunk);
#define LAUNCH(NN)                                                                      \
  hipLaunchKernelGGL((apply_mapped_kernel<VT, NN>), grid, dim3(mapped_threads<NN>()), 0, s, \
                     u, v, b, g.vert, g.gam, mtab, g.n, chunk)
  switch (N) {
    case 2: LAUNCH(2); break;
    case 3: LAUNCH(3); break;
    case 4: LAUNCH(4); break;
    case 5: LAUNCH(5); break;
    case 6: LAUNCH(6); break;
    case 7: LAUNCH(7); break;
    case 8: LAUNCH(8); break;
    default: return hipErrorInvalidValue;
  }
#undef LAUNCH
  return hipGetLastError();
}

}  // namespace

hipError_t launch_apply_mapped(int N, const double* u, double* v, const double* b,
                               const MappedLevel& g, const double* mtab, hipStream_t s) {
  return apply_mapped<double>(N, u, v, b, g, mtab, s);
}

hipError_t launch_apply_mapped_f32(int N, const float* u, float* v, const float* b,
                                   const MappedLevel& g, const double* mtab, hipStream_t s) {
  return apply_mapped<float>(N, u, v, b, g, mtab, s);
}

hipError_t launch_rhs_mapped(int N, const MappedLevel& g, int nm, const double* modes,
                             const double* qtab, double* b, hipStream_t s) {
  if (N < 2 || N > kMaxN || g.n < 1 || g.n > 1024 || nm < 1 || nm > 64 || !g.vert || !modes ||
      !qtab || !b)
    return hipErrorInvalidValue;
  const dim3 grid(g.n * g.n * g.n);
#define LAUNCH(NN)                                                                     \
  hipLaunchKernelGGL(rhs_mapped_kernel<NN>, grid, dim3(kMappedRhsT), 0, s, g.vert, g.n, nm, \
                     modes, qtab, b)
  switch (N) {
    case 2: LAUNCH(2); break;
    case 3: LAUNCH(3); break;
    case 4: LAUNCH(4); break;
    case 5: LAUNCH(5); break;
    case 6: LAUNCH(6); break;
    case 7: LAUNCH(7); break;
    case 8: LAUNCH(8); break;
    default: return hipErrorInvalidValue;
  }
#undef LAUNCH
  return hipGetLastError();
}

hipError_t launch_l2_mapped(int N, const MappedLevel& g, int nm, const double* modes,
                            const double* qtab, const double* x, double* partial, int max_blocks,
                            double* out, hipStream_t s) {
  if (N < 2 || N > kMaxN || g.n < 1 || g.n > 1024 || nm < 1 || nm > 64 || !g.vert || !modes ||
      !qtab || !x || !partial || !out || max_blocks < 1)
    return hipErrorInvalidValue;
  const int nc = g.n * g.n * g.n;
  const int nb = nc < max_blocks ? nc : max_blocks;
#define LAUNCH(NN)                                                                          \
  hipLaunchKernelGGL(l2_mapped_kernel<NN>, dim3(nb), dim3(kMappedRhsT), 0, s, g.vert, g.n, nm, \
                     modes, qtab, x, partial)
  switch (N) {
    case 2: LAUNCH(2); break;
    case 3: LAUNCH(3); break;
    case 4: LAUNCH(4); break;
    case 5: LAUNCH(5); break;
    case 6: LAUNCH(6); break;
    case 7: LAUNCH(7); break;
    case 8: LAUNCH(8); break;
    default: return hipErrorInvalidValue;
  }
#undef LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, partial, nb, out);
  return hipGetLastError();
}

}  // namespace sipg
