// VALU kernels (FP64 and FP32 instantiations) of the SIPG operator, the vertex-patch fast-diagonalization
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

#include "batch.h"
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

// A cell of zeros (up to N = 8): loads of a missing face neighbour point
// here, so the loaded values need no select.  Never written.
__device__ __align__(16) double g_zero_cell_f64[512];
__device__ __align__(16) float g_zero_cell_f32[512];
template <typename T>
__device__ __forceinline__ const T* zero_cell();
template <>
__device__ __forceinline__ const double* zero_cell<double>() { return g_zero_cell_f64; }
template <>
__device__ __forceinline__ const float* zero_cell<float>() { return g_zero_cell_f32; }

// 16 contiguous bytes of a vector (two doubles or four floats): one load or
// LDS store instruction; both addresses must be 16-byte aligned.
template <typename T>
struct Piece16 {
  static constexpr int kPer = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(16 / sizeof(T))));
  V v;
  static __device__ __forceinline__ Piece16 load(const T* p) {
    Piece16 q;
    q.v = *reinterpret_cast<const V*>(p);
    return q;
  }
  static __device__ __forceinline__ void store(T* p, const Piece16& q) {
    *reinterpret_cast<V*>(p) = q.v;
  }
};

template <int N, typename T>
__device__ __forceinline__ void matvec(const T* __restrict__ A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int a = 0; a < N; ++a) {
    T s = 0;
#pragma unroll
    for (int b = 0; b < N; ++b) s = fma(A[a * N + b], x[b], s);
    y[a] = s;
  }
}

template <int N, typename T>
__device__ __forceinline__ void matvec_acc(const T* __restrict__ A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int a = 0; a < N; ++a) {
    T s = y[a];
#pragma unroll
    for (int b = 0; b < N; ++b) s = fma(A[a * N + b], x[b], s);
    y[a] = s;
  }
}

// Even-odd form of a J-symmetric N x N matrix (Q[N-1-a][N-1-b] = Q[a][b],
// as the mass matrix and the interior cell block on the symmetric GLL
// nodes): with e_b = x_b + x_{N-1-b}, o_b = x_b - x_{N-1-b} (b < N/2; for
// odd N the middle e = 2 x_mid) and the half-blocks QE[a][b] = (Q[a][b] +
// Q[a][N-1-b]) / 2 (Q[a][mid] / 2 in the middle column) and QO[a][b] =
// (Q[a][b] - Q[a][N-1-b]) / 2, y_a = (QE e)_a + (QO o)_a and y_{N-1-a} =
// (QE e)_a - (QO o)_a: 2 (N/2)^2 products instead of N^2.
template <int N, typename T>
struct Split {
  static constexpr int P = N / 2, PE = (N + 1) / 2;
  T e[PE], o[P > 0 ? P : 1];
  __device__ __forceinline__ explicit Split(const T (&x)[N]) {
#pragma unroll
    for (int b = 0; b < P; ++b) {
      e[b] = x[b] + x[N - 1 - b];
      o[b] = x[b] - x[N - 1 - b];
    }
    if constexpr (N % 2) e[P] = x[P] + x[P];
  }
};

// y (+)= Q x for J-symmetric Q given by its half-blocks QE [PE x PE] and
// QO [P x P] (row-major), on split input
template <int N, bool ACC, typename T>
__device__ __forceinline__ void matvec_sym(const T* __restrict__ QE, const T* __restrict__ QO,
                                           const Split<N, T>& x, T (&y)[N]) {
  constexpr int P = N / 2, PE = (N + 1) / 2;
#pragma unroll
  for (int a = 0; a < PE; ++a) {
    T se = 0;
#pragma unroll
    for (int b = 0; b < PE; ++b) se = fma(QE[a * PE + b], x.e[b], se);
    if (a < P) {
      T so = 0;
#pragma unroll
      for (int b = 0; b < P; ++b) so = fma(QO[a * P + b], x.o[b], so);
      y[a] = ACC ? y[a] + (se + so) : se + so;
      y[N - 1 - a] = ACC ? y[N - 1 - a] + (se - so) : se - so;
    } else {
      y[a] = ACC ? y[a] + se : se;
    }
  }
}

// y = A^T x
template <int N, typename T>
__device__ __forceinline__ void matvec_t(const T* __restrict__ A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int a = 0; a < N; ++a) {
    T s = 0;
#pragma unroll
    for (int b = 0; b < N; ++b) s = fma(A[b * N + a], x[b], s);
    y[a] = s;
  }
}

// For large N: keep loop-invariant LDS matrix reads inside the loop (a
// compiler-only memory clobber; without it the whole matrix is hoisted into
// registers, 256 VGPRs and one wave per SIMD at N = 8).
template <int N>
__device__ __forceinline__ void keep_lds_reads_local() {
  if constexpr (N >= 6) asm volatile("" ::: "memory");
}

// Patch-size products with the matrix in LDS: one output row at a time,
// with a scheduling barrier between rows, so the compiler does not hoist all
// G^2 matrix reads ahead of the arithmetic (that filled the register file:
// 256 VGPRs and one wave per SIMD for N >= 6).
template <int G, typename T>
__device__ __forceinline__ void matvec_rows(const T* __restrict__ A, const T (&x)[G], T (&y)[G]) {
#pragma unroll
  for (int a = 0; a < G; ++a) {
    T s = 0;
#pragma unroll
    for (int b = 0; b < G; ++b) s = fma(A[a * G + b], x[b], s);
    y[a] = s;
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int G, typename T>
__device__ __forceinline__ void matvec_rows_t(const T* __restrict__ A, const T (&x)[G], T (&y)[G]) {
#pragma unroll
  for (int a = 0; a < G; ++a) {
    T s = 0;
#pragma unroll
    for (int b = 0; b < G; ++b) s = fma(A[b * G + a], x[b], s);
    y[a] = s;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Patch transforms of the interior patch type in even-odd form: YE, YO are
// H x H (H = G/2; row = node a < H, column = eigenvector, 1/sqrt 2 folded
// in).  Forward c = S^T x with c = [even eigen-indices, odd ones], from
// e = x_a + x_{G-1-a} and o = x_a - x_{G-1-a}; backward x = S c, with
// x_a = (YE c_E)_a + (YO c_O)_a and x_{G-1-a} = (YE c_E)_a - (YO c_O)_a.
// 2 H^2 products instead of G^2; one row per scheduling region as in
// matvec_rows (the matrices are in LDS).
template <int G, typename T>
__device__ __forceinline__ void fd_fwd_eo(const T* __restrict__ YE, const T* __restrict__ YO,
                                          const T (&x)[G], T (&y)[G]) {
  constexpr int H = G / 2;
  T e[H], o[H];
#pragma unroll
  for (int a = 0; a < H; ++a) {
    e[a] = x[a] + x[G - 1 - a];
    o[a] = x[a] - x[G - 1 - a];
  }
#pragma unroll
  for (int k = 0; k < H; ++k) {
    T se = 0, so = 0;
#pragma unroll
    for (int a = 0; a < H; ++a) {
      se = fma(YE[a * H + k], e[a], se);
      so = fma(YO[a * H + k], o[a], so);
    }
    y[k] = se;
    y[H + k] = so;
    __builtin_amdgcn_sched_barrier(0);
  }
}
template <int G, typename T>
__device__ __forceinline__ void fd_bwd_eo(const T* __restrict__ YE, const T* __restrict__ YO,
                                          const T (&c)[G], T (&x)[G]) {
  constexpr int H = G / 2;
#pragma unroll
  for (int a = 0; a < H; ++a) {
    T ye = 0, yo = 0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
      ye = fma(YE[a * H + k], c[k], ye);
      yo = fma(YO[a * H + k], c[H + k], yo);
    }
    x[a] = ye + yo;
    x[G - 1 - a] = ye - yo;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Face coupling to the lower neighbour (its high-end value f and derivative
// g = d1 . u) and to the upper neighbour (low-end value f, g = d0 . u).
template <int N, typename T>
__device__ __forceinline__ void add_lower_face(T (&t)[N], T f, T g, T gam,
                                               const T* __restrict__ d0) {
  t[0] += -gam * f + T(0.5) * g;
#pragma unroll
  for (int a = 0; a < N; ++a) t[a] = fma(T(-0.5) * d0[a], f, t[a]);
}
template <int N, typename T>
__device__ __forceinline__ void add_upper_face(T (&t)[N], T f, T g, T gam,
                                               const T* __restrict__ d1) {
  t[N - 1] += -gam * f - T(0.5) * g;
#pragma unroll
  for (int a = 0; a < N; ++a) t[a] = fma(T(0.5) * d1[a], f, t[a]);
}

__device__ __forceinline__ int bdry_variant(int coord, int n) {
  return (coord == 0 ? 1 : 0) | (coord == n - 1 ? 2 : 0);
}

// The diagonal block of a cell at a boundary differs from the interior one
// by a rank-2 term: at x = 0 the boundary face adds (s0 d0^T + d0 s0^T)/2
// more than an interior face, at x = 1 it adds -(s1 d1^T + d1 s1^T)/2.
// Applied to the line x (before any face term is added to t).
template <int N, typename T>
__device__ __forceinline__ void add_boundary_correction(T (&t)[N], const T (&x)[N], bool lo,
                                                        bool hi, const T* __restrict__ d0,
                                                        const T* __restrict__ d1) {
  if (lo) {
    T g = 0;
#pragma unroll
    for (int a = 0; a < N; ++a) g = fma(d0[a], x[a], g);
    t[0] += T(0.5) * g;
#pragma unroll
    for (int a = 0; a < N; ++a) t[a] = fma(T(0.5) * d0[a], x[0], t[a]);
  }
  if (hi) {
    T g = 0;
#pragma unroll
    for (int a = 0; a < N; ++a) g = fma(d1[a], x[a], g);
    t[N - 1] -= T(0.5) * g;
#pragma unroll
    for (int a = 0; a < N; ++a) t[a] = fma(T(-0.5) * d1[a], x[N - 1], t[a]);
  }
}

// ---------------------------------------------------------------------------
// Operator apply.  A wave owns a tile of TX consecutive cells along x (TX
// divides n, TX * N^2 <= 64 lanes), one lane per 1D line per stage; waves
// run independently (cells never straddle a wave).  Tiles are ordered so
// that a cell's six face neighbours are processed close in time on the same
// XCD: x-tiles fastest, then z and y in 8 x 8 blocks.
// ---------------------------------------------------------------------------
struct TileMap {
  int n, tx, ntx, blk;  // blk = 8 when n % 8 == 0 (blocked order), else 1
  int ngroups;          // number of tiles (wave-level variant)
};

__device__ __forceinline__ int tile_first_cell(const TileMap& m, int t) {
  const int txi = t % m.ntx;
  int r = t / m.ntx;
  int cy, cz;
  if (m.blk > 1) {
    const int zi = r % m.blk;
    r /= m.blk;
    const int yi = r % m.blk;
    r /= m.blk;
    const int nb = m.n / m.blk;
    const int zb = r % nb, yb = r / nb;
    cz = zb * m.blk + zi;
    cy = yb * m.blk + yi;
  } else {
    cy = r % m.n;
    cz = r / m.n;
  }
  return (cz * m.n + cy) * m.n + txi * m.tx;
}

// Order LDS traffic between the lanes of one wave: LDS instructions of a
// wave execute in order; the wait and the memory clobber keep the compiler
// from moving accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Global loads: for N >= 5 every cell the tile touches (its own and the six
// face neighbours) is read in the coalesced z-line pattern -- lane (p, q)
// reads nodes (p, q, a), a = 0..N-1, so consecutive lanes read consecutive
// doubles -- and transposed into x- or y-lines through the wave's LDS
// slice.  The staging slice is reused for the face traces once consumed
// (8 N^2 <= 2 N^3 for N >= 4).  For N <= 4 the lanes read their lines
// directly (measured faster at N = 4, where a line is 32 bytes).  Both
// paths feed identical values to identical arithmetic.  (Also measured:
// persistent waves that prefetch the next tile during the y and z stages
// lose more to the lower occupancy than they gain.)
//
// WG: the workgroup's waves share one tile of CPT = kThreads / N^2 cells
// (consecutive in memory order) and synchronise with workgroup barriers;
// used where whole cells per wave would leave many lanes idle (N = 6: 7
// cells on 252 of 256 lanes instead of one cell on 36 of 64).
template <typename T, int N, bool RES, bool WG = false>
__global__ __launch_bounds__(kThreads) void apply_wave_kernel(
    Batch<T> B, const T* __restrict__ tab, TableLayout lay) {
  constexpr int N2 = N * N, N3 = N2 * N, CPB = (64 / N2) > 0 ? 64 / N2 : 1;
  constexpr int WAVES = kThreads / 64;
  constexpr int CPT = kThreads / N2;            // cells of a workgroup tile (WG)
  constexpr int CS = WG ? CPT : CPB;            // cells of one LDS slice
  constexpr int SLOTS = WG ? CPT : WAVES * CPB;  // cells of all slices
  constexpr bool COAL = N >= 5;
  // cells split evenly into 16-byte pieces, NP per lane
  constexpr bool V16 = (N * sizeof(T)) % 16 == 0;
  constexpr int NP = V16 ? (int)(N * sizeof(T) / 16) : 1;
  static_assert(!WG || COAL, "the workgroup tile is implemented for the staged loads");
  // per cell: t1, t2 and a region holding first (COAL) one staged neighbour
  // cell, then the y-face traces [face 0,1][value, derivative][i + N l] and
  // z-face traces [face 0,1][value, derivative][i + N j]; the z-traces after
  // Mx overwrite the y-traces once those are read
  constexpr int NR = (COAL && N3 > 8 * N2) ? N3 : 8 * N2;
  __shared__ __align__(16) T s_t1_all[SLOTS * N3];
  __shared__ __align__(16) T s_t2_all[SLOTS * N3];
  __shared__ __align__(16) T s_r_all[SLOTS * NR];
  // LDS ordering between the lanes sharing a tile
  auto lds_sync = [&]() {
    if constexpr (WG) __syncthreads();
    else wave_lds_sync();
  };

  const int tid = WG ? threadIdx.x : (threadIdx.x & 63), wave = WG ? 0 : (threadIdx.x >> 6);
  const int gi = __builtin_amdgcn_readfirstlane(WG ? xcd_remap(blockIdx.x, gridDim.x)
                                                   : xcd_remap(blockIdx.x, gridDim.x) * WAVES + wave);
  // wave-uniform (workgroup-uniform with WG): every barrier below is reached
  // by all threads that pass this point
  if (gi >= B.start[B.count]) return;
  const int pb = batch_find(B, gi);
  const int grp = gi - B.start[pb];
  const T* __restrict__ u = B.d[pb].in;
  T* __restrict__ v = B.d[pb].out;
  const T* __restrict__ bvec = B.d[pb].aux;
  const T h = B.d[pb].h;
  TileMap tm;
  tm.n = B.d[pb].n;
  tm.tx = B.d[pb].a0;
  tm.ntx = B.d[pb].a1;
  tm.blk = B.d[pb].a2;
  tm.ngroups = B.start[pb + 1] - B.start[pb];
  T* s_t1 = s_t1_all + wave * (CS * N3);
  T* s_t2 = s_t2_all + wave * (CS * N3);
  T* s_ty = s_r_all + wave * (CS * NR);
  T* s_tz = s_ty + CS * 4 * N2;
  T* s_tzm = s_ty;
  // staging (COAL): t1 and t2 are free until the x stage writes them
  T* s_n0 = s_t2;
  T* s_n1 = s_ty;
  const int n = tm.n, nn = n * n, nc = tm.tx;
  // WG: CPT consecutive cells of the blocked order (x fastest, then (z, y)
  // in blk x blk blocks, so the tiles that share y/z neighbours run close
  // in time) from index grp * CPT; the last tile may be short.  Else TX
  // cells of an x-row.
  TileMap t1 = tm;
  t1.tx = 1;
  t1.ntx = n;
  const int c0 = WG ? grp * CPT : tile_first_cell(tm, grp);
  const bool act = WG ? (tid < CPT * N2 && c0 + tid / N2 < nn * n) : (tid < nc * N2);
  const int cl = act ? tid / N2 : 0, ln = tid - cl * N2;
  const int c = WG ? tile_first_cell(t1, c0 + cl) : c0 + cl;
  // cell coordinates: per lane with WG, else the tile's row plus cl
  const int cx = WG ? c % n : c0 % n + cl;
  const int cy = WG ? (c / n) % n : (c0 / n) % n;
  const int cz = WG ? c / nn : c0 / nn;
  // this thread owns x-line (j, l) = (ln % N, ln / N) of cell c and the
  // y-/z-face trace lines at (i, l) = (ln % N, ln / N) and (i, j) = ln.
  const int lp = ln % N, lq = ln / N;

  // ---- all global loads of the tile are issued first
  T own[N], xlo[N], xhi[N], ylo[N], yhi[N], zlo[N], zhi[N];
  const bool hx0 = act && cx > 0, hx1 = act && cx < n - 1;
  const bool hy0 = act && cy > 0, hy1 = act && cy < n - 1;
  const bool hz0 = act && cz > 0, hz1 = act && cz < n - 1;
  if constexpr (COAL) {
    // unconditional loads, one basic block: a missing neighbour is read from
    // a cell of zeros, so no value needs a select after its load; idle lanes
    // read the first line of the tile's first cell (lnl = 0) and use
    // nothing, so every address stays inside one cell.  The cells staged
    // through LDS (own, x and y neighbours) are copied in 16-byte pieces
    // where a cell splits evenly into them (lane ln moves pieces ln + N^2 r,
    // in memory order); the z neighbours are read as z-lines, which is the
    // layout their face traces need.
    const int lnl = act ? ln : 0;
    const T* zc = zero_cell<T>();
    const T* cp = u + (size_t)c * N3;
    const ptrdiff_t sx = N3, sy = (ptrdiff_t)n * N3, sz = (ptrdiff_t)nn * N3;
    const T* pxl = hx0 ? cp - sx : zc;
    const T* pxh = hx1 ? cp + sx : zc;
    const T* pyl = hy0 ? cp - sy : zc;
    const T* pyh = hy1 ? cp + sy : zc;
    const T* pzl = (hz0 ? cp - sz : zc) + lnl;
    const T* pzh = (hz1 ? cp + sz : zc) + lnl;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      zlo[a] = pzl[a * N2];
      zhi[a] = pzh[a * N2];
    }
    const int w = cl * N3 + ln;
    if constexpr (V16) {
      using P16 = Piece16<T>;
      P16 qo[NP], ql[NP], qh[NP], yl[NP], yh[NP];
#pragma unroll
      for (int r = 0; r < NP; ++r) {
        const int o = (lnl + N2 * r) * P16::kPer;
        qo[r] = P16::load(cp + o);
        ql[r] = P16::load(pxl + o);
        qh[r] = P16::load(pxh + o);
        yl[r] = P16::load(pyl + o);
        yh[r] = P16::load(pyh + o);
      }
      // own and x-neighbours: cell layout -> x-lines (j, l) = (lp, lq)
      if (act) {
#pragma unroll
        for (int r = 0; r < NP; ++r) {
          const int o = cl * N3 + (ln + N2 * r) * P16::kPer;
          P16::store(s_t1 + o, qo[r]);
          P16::store(s_n0 + o, ql[r]);
          P16::store(s_n1 + o, qh[r]);
        }
      }
      lds_sync();
      const int rx = cl * N3 + ln * N;
      if (act) {
#pragma unroll
        for (int a = 0; a < N; ++a) {
          own[a] = s_t1[rx + a];
          xlo[a] = s_n0[rx + a];
          xhi[a] = s_n1[rx + a];
        }
      }
      lds_sync();
      // y-neighbours: cell layout -> y-lines (i, l) = (lp, lq)
      if (act) {
#pragma unroll
        for (int r = 0; r < NP; ++r) {
          const int o = cl * N3 + (ln + N2 * r) * P16::kPer;
          P16::store(s_n0 + o, yl[r]);
          P16::store(s_n1 + o, yh[r]);
        }
      }
    } else {
#pragma unroll
      for (int a = 0; a < N; ++a) {
        own[a] = cp[lnl + a * N2];
        xlo[a] = pxl[lnl + a * N2];
        xhi[a] = pxh[lnl + a * N2];
        ylo[a] = pyl[lnl + a * N2];
        yhi[a] = pyh[lnl + a * N2];
      }
      // own and x-neighbours: z-lines -> x-lines (j, l) = (lp, lq)
      if (act) {
#pragma unroll
        for (int a = 0; a < N; ++a) {
          s_t1[w + a * N2] = own[a];
          s_n0[w + a * N2] = xlo[a];
          s_n1[w + a * N2] = xhi[a];
        }
      }
      lds_sync();
      const int rx = cl * N3 + ln * N;
      if (act) {
#pragma unroll
        for (int a = 0; a < N; ++a) {
          own[a] = s_t1[rx + a];
          xlo[a] = s_n0[rx + a];
          xhi[a] = s_n1[rx + a];
        }
      }
      lds_sync();
      // y-neighbours: z-lines -> y-lines (i, l) = (lp, lq)
      if (act) {
#pragma unroll
        for (int a = 0; a < N; ++a) {
          s_n0[w + a * N2] = ylo[a];
          s_n1[w + a * N2] = yhi[a];
        }
      }
    }
    lds_sync();
    const int ry = cl * N3 + lp + lq * N2;
    if (act) {
#pragma unroll
      for (int a = 0; a < N; ++a) {
        ylo[a] = s_n0[ry + a * N];
        yhi[a] = s_n1[ry + a * N];
      }
    }
    lds_sync();  // the staging slice becomes the trace buffers below
  } else {
    const T* pc = u + (size_t)c * N3;
    const T* pxl = pc - N3 + ln * N;
    const T* pxh = pc + N3 + ln * N;
    const T* pyl = pc - (size_t)n * N3 + lp + lq * N2;
    const T* pyh = pc + (size_t)n * N3 + lp + lq * N2;
    const T* pzl = pc - (size_t)nn * N3 + ln;
    const T* pzh = pc + (size_t)nn * N3 + ln;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      own[a] = act ? pc[ln * N + a] : 0.0;
      xlo[a] = hx0 ? pxl[a] : 0.0;
      xhi[a] = hx1 ? pxh[a] : 0.0;
      ylo[a] = hy0 ? pyl[a * N] : 0.0;
      yhi[a] = hy1 ? pyh[a * N] : 0.0;
      zlo[a] = hz0 ? pzl[a * N2] : 0.0;
      zhi[a] = hz1 ? pzh[a * N2] : 0.0;
    }
  }
  // 1D tables are uniform over the workgroup: read through the scalar path
  const T* __restrict__ s_M = tab + lay.mass;
  const T* __restrict__ s_L = tab + lay.lcell;  // interior block (variant 0)
  // even-odd half-blocks of the mass and the interior block
  constexpr int PE2 = ((N + 1) / 2) * ((N + 1) / 2);
  const T* __restrict__ s_ME = tab + lay.sym;
  const T* __restrict__ s_MO = s_ME + PE2;
  const T* __restrict__ s_LE = s_MO + (N / 2) * (N / 2);
  const T* __restrict__ s_LO = s_LE + PE2;
  const T* __restrict__ s_d0 = tab + lay.d0;
  const T* __restrict__ s_d1 = tab + lay.d1;
  const T gam = tab[lay.gam];

  // ---- x stage in registers, traces of the y/z neighbours to LDS
  if (act) {
    T t1[N], t2[N];
    const Split<N, T> so(own);
    matvec_sym<N, false>(s_LE, s_LO, so, t1);
    add_boundary_correction<N>(t1, own, cx == 0, cx == n - 1, s_d0, s_d1);
    matvec_sym<N, false>(s_ME, s_MO, so, t2);
    if (hx0) {
      T g = 0.0;
#pragma unroll
      for (int a = 0; a < N; ++a) g = fma(s_d1[a], xlo[a], g);
      add_lower_face<N>(t1, xlo[N - 1], g, gam, s_d0);
    }
    if (hx1) {
      T g = 0.0;
#pragma unroll
      for (int a = 0; a < N; ++a) g = fma(s_d0[a], xhi[a], g);
      add_upper_face<N>(t1, xhi[0], g, gam, s_d1);
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
      s_t1[cl * N3 + ln * N + a] = t1[a];
      s_t2[cl * N3 + ln * N + a] = t2[a];
    }
    T g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      g0 = fma(s_d1[a], ylo[a], g0);
      g1 = fma(s_d0[a], yhi[a], g1);
      g2 = fma(s_d1[a], zlo[a], g2);
      g3 = fma(s_d0[a], zhi[a], g3);
    }
    T* ty = s_ty + cl * 4 * N2;
    T* tz = s_tz + cl * 4 * N2;
    ty[0 * N2 + ln] = ylo[N - 1];
    ty[1 * N2 + ln] = g0;
    ty[2 * N2 + ln] = yhi[0];
    ty[3 * N2 + ln] = g1;
    tz[0 * N2 + ln] = zlo[N - 1];
    tz[1 * N2 + ln] = g2;
    tz[2 * N2 + ln] = zhi[0];
    tz[3 * N2 + ln] = g3;
  }
  lds_sync();

  // ---- y stage: lines (i, l) = (lp, lq); also Mx on the z traces at (i, j)
  T cc[N], e[N];
  const int ybase = cl * N3 + lp + lq * N2;
  const T* Mrow_y = s_M + lp * N;
  if (act) {
    T a1[N], a2[N];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      a1[b] = s_t1[ybase + b * N];
      a2[b] = s_t2[ybase + b * N];
    }
    const Split<N, T> s1(a1), s2(a2);
    matvec_sym<N, false>(s_ME, s_MO, s1, cc);
    matvec_sym<N, true>(s_LE, s_LO, s2, cc);
    add_boundary_correction<N>(cc, a2, cy == 0, cy == n - 1, s_d0, s_d1);
    matvec_sym<N, false>(s_ME, s_MO, s2, e);
    const T* ty = s_ty + cl * 4 * N2 + lq * N;
    T f0 = 0.0, q0 = 0.0, f1 = 0.0, q1 = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) {  // (Mx trace)(i, l) = sum_i' M[i][i'] trace(i', l)
      f0 = fma(Mrow_y[b], ty[0 * N2 + b], f0);
      q0 = fma(Mrow_y[b], ty[1 * N2 + b], q0);
      f1 = fma(Mrow_y[b], ty[2 * N2 + b], f1);
      q1 = fma(Mrow_y[b], ty[3 * N2 + b], q1);
    }
    if (hy0) add_lower_face<N>(cc, f0, q0, gam, s_d0);
    if (hy1) add_upper_face<N>(cc, f1, q1, gam, s_d1);
  }
  lds_sync();  // every lane has read its y-traces before they are overwritten
  if (act) {
    const T* tz = s_tz + cl * 4 * N2 + lq * N;
    T* tzm = s_tzm + cl * 4 * N2 + lq * N + lp;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      T acc = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) acc = fma(Mrow_y[b], tz[r * N2 + b], acc);
      tzm[r * N2] = acc;
    }
#pragma unroll
    for (int b = 0; b < N; ++b) {
      s_t1[ybase + b * N] = cc[b];
      s_t2[ybase + b * N] = e[b];
    }
  }
  lds_sync();

  // ---- z stage: lines (i, j) = ln, written straight to global memory
  if (act) {
    T a1[N], a2[N], o[N];
    const int base = cl * N3 + ln;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      a1[b] = s_t1[base + b * N2];
      a2[b] = s_t2[base + b * N2];
    }
    const Split<N, T> s1(a1), s2(a2);
    matvec_sym<N, false>(s_ME, s_MO, s1, o);
    matvec_sym<N, true>(s_LE, s_LO, s2, o);
    add_boundary_correction<N>(o, a2, cz == 0, cz == n - 1, s_d0, s_d1);
    // (My Mx trace)(i, j) = sum_j' M[j][j'] (Mx trace)(i, j')
    const T* tzm = s_tzm + cl * 4 * N2 + lp;
    const T* Mrow = s_M + lq * N;
    T f0 = 0.0, q0 = 0.0, f1 = 0.0, q1 = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      f0 = fma(Mrow[b], tzm[0 * N2 + b * N], f0);
      q0 = fma(Mrow[b], tzm[1 * N2 + b * N], q0);
      f1 = fma(Mrow[b], tzm[2 * N2 + b * N], f1);
      q1 = fma(Mrow[b], tzm[3 * N2 + b * N], q1);
    }
    if (hz0) add_lower_face<N>(o, f0, q0, gam, s_d0);
    if (hz1) add_upper_face<N>(o, f1, q1, gam, s_d1);
    T* dst = v + (size_t)c * N3 + ln;
    if (RES) {
      const T* bs = bvec + (size_t)c * N3 + ln;
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
//
// FUSED: one colour step of the multiplicative smoother without a separate
// residual.  With r = b - A x, the exact local solve gives
//   x_P + A_PP^{-1} (b - A x)_P = A_PP^{-1} (b_P - A_{P,ext} x_ext),
// where A_{P,ext} couples the patch to the cells across its six faces (the
// principal submatrix A_PP holds everything inside the patch).  So the new
// patch values are the fast-diagonalization solve of f_P = b_P minus the
// face couplings of the outside neighbours, which need only their face
// value and normal derivative (rank 2, as in the operator apply) times the
// tangential masses.  The new values are written to a second vector (x_in is
// read across the faces of neighbouring patches of the same colour, which
// update their own cells in the same launch); cells outside every patch of
// the colour are copied by launch_copy_uncovered.
// ---------------------------------------------------------------------------
template <typename T, int N, bool FUSED = false>
__global__ __launch_bounds__(kThreads) void patch_fd_kernel(
    Batch<T> B, const T* __restrict__ tab, TableLayout lay, int bx, int by, int bz) {
  constexpr int G = 2 * N, G2 = G * G, G3 = G2 * G, N2 = N * N, N3 = N2 * N;
  constexpr int PPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  // One patch per workgroup (N >= 6): only the three matrices of its
  // direction types are staged, which keeps N = 8 in FP64 under 40 KB of LDS
  // (four workgroups per CU).  Several patches: all four types.
  constexpr bool ONE = PPB == 1;
  constexpr int NS = ONE ? 3 : 4;
  __shared__ T s_S[NS * G2];
  // eigenvalues by type, then those of the interior type in even-odd order
  __shared__ T s_l[5 * G];
  // interior type in even-odd form: YE, YO [G/2 x G/2]
  __shared__ T s_eo[G2 / 2];
  __shared__ T s_X[PPB * G3];
  // face traces [patch][face 2 d + side][value, derivative][G2] and the
  // face tables d0, d1, mass
  __shared__ T s_F[FUSED ? PPB * 12 * G2 : 1];
  __shared__ T s_fd[FUSED ? 2 * N + N2 : 1];
  const int tid = threadIdx.x;
  const int bi = xcd_remap(blockIdx.x, gridDim.x);
  if (bi >= B.start[B.count]) return;
  const int pb = batch_find(B, bi);
  const T* __restrict__ r = B.d[pb].in;
  T* __restrict__ x = B.d[pb].out;
  const int n = B.d[pb].n, npx = B.d[pb].a0, npy = B.d[pb].a1, npatch = B.d[pb].a2;
  const T h = B.d[pb].h;
  const int p0 = (bi - B.start[pb]) * PPB;
  const int np = min(PPB, npatch - p0);
  if (np <= 0) return;
  const int nn = n * n;
  // vertex of a patch and its first cell
  auto vertex = [&](int pl, int& vx, int& vy, int& vz) {
    const int p = p0 + pl;
    const int px = p % npx, py = (p / npx) % npy, pz = p / (npx * npy);
    vx = 2 * px + (bx ? 1 : 2);
    vy = 2 * py + (by ? 1 : 2);
    vz = 2 * pz + (bz ? 1 : 2);
  };
  auto vtype = [&](int v) { return (v == 1 ? 1 : 0) | (v == n - 1 ? 2 : 0); };
  int ts[3] = {0, 1, 2};
  if constexpr (ONE) {
    int vx, vy, vz;
    vertex(0, vx, vy, vz);
    ts[0] = vtype(vx);
    ts[1] = vtype(vy);
    ts[2] = vtype(vz);
  }
  for (int i = tid; i < NS * G2; i += kThreads) {
    const int d = i / G2, e = i - d * G2;
    s_S[i] = tab[lay.fd_s + (ONE ? ts[d] : d) * G2 + e];
  }
  for (int i = tid; i < 4 * G; i += kThreads) s_l[i] = tab[lay.fd_l + i];
  const bool eo_ok = lay.fd_eo_ok != 0;
  constexpr int HH = (G / 2) * (G / 2);
  if (eo_ok) {
    for (int i = tid; i < 2 * HH; i += kThreads) s_eo[i] = tab[lay.fd_eo + i];
    for (int i = tid; i < G; i += kThreads) s_l[4 * G + i] = tab[lay.fd_eo + 2 * HH + i];
  }
  if constexpr (FUSED) {
    for (int i = tid; i < N; i += kThreads) {
      s_fd[i] = tab[lay.d0 + i];
      s_fd[N + i] = tab[lay.d1 + i];
    }
    for (int i = tid; i < N2; i += kThreads) s_fd[2 * N + i] = tab[lay.mass + i];
  }
  // A patch of G^2 <= 64 lines that divides 64 lives inside one wave: its
  // waves then synchronise only with themselves after the table load (the
  // fused form shares work items across the workgroup: barriers).
  constexpr bool WL = !FUSED && (G2 <= 64) && (64 % G2 == 0);
  const int lane = tid & 63, wv = tid >> 6;
  auto psync = [&]() {
    if constexpr (WL) wave_lds_sync();
    else __syncthreads();
  };
  const int w_lo = WL ? wv * (G2 <= 64 ? 64 / G2 : 1) * G3 : 0;
  const int w_hi = WL ? min(np * G3, w_lo + (G2 <= 64 ? 64 / G2 : 1) * G3) : np * G3;
  const int w_first = WL ? w_lo + lane : tid, w_step = WL ? 64 : kThreads;

  // first cell of each patch of the block, computed once per patch (the
  // gather and scatter loops below then divide only by compile-time sizes)
  __shared__ int s_cb[PPB];
  for (int q = tid; q < np; q += kThreads) {
    int vx, vy, vz;
    vertex(q, vx, vy, vz);
    s_cb[q] = (vx - 1) + n * (vy - 1) + nn * (vz - 1);
  }
  __syncthreads();
  // gather b_P (fused form; the plain form reads r_P line by line in the
  // first transform below)
  const T* __restrict__ src = FUSED ? B.d[pb].aux : r;
  if constexpr (FUSED)
  for (int w = w_first; w < w_hi; w += w_step) {
    const int pl = w / G3, rr = w - pl * G3;
    const int cell8 = rr / N3, loc = rr - cell8 * N3;
    const int dx = cell8 & 1, dy = (cell8 >> 1) & 1, dz = cell8 >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int c = s_cb[pl] + dx + n * dy + nn * dz;
    s_X[pl * G3 + (dx * N + i) + G * (dy * N + j) + G2 * (dz * N + l)] = src[(size_t)c * N3 + loc];
  }
  psync();
  if constexpr (FUSED) {
    // f_P = b_P - h (tangential masses x face coupling) of the outside
    // neighbours (x_in = r here).  Face f = 2 d + side; its G x G points
    // (ta, tb) run over the tangential directions in increasing order.
    const T gam = tab[lay.gam];
    const T* __restrict__ fd0 = s_fd;
    const T* __restrict__ fd1 = s_fd + N;
    const T* __restrict__ fM = s_fd + 2 * N;
    // cell and node offsets of (d-node a, tangential (ta, tb)) of face d
    auto face_cell = [&](int d, int cd, int pl, int ta, int tb, int& c, int& loc, int& stride) {
      int vx, vy, vz;
      vertex(pl, vx, vy, vz);
      const int ca = ta / N, ia = ta - ca * N, cb = tb / N, ib = tb - cb * N;
      int cx, cy, cz, i, j, l;
      if (d == 0) { cx = cd; cy = vy - 1 + ca; cz = vz - 1 + cb; i = 0; j = ia; l = ib; stride = 1; }
      else if (d == 1) { cx = vx - 1 + ca; cy = cd; cz = vz - 1 + cb; i = ia; j = 0; l = ib; stride = N; }
      else { cx = vx - 1 + ca; cy = vy - 1 + cb; cz = cd; i = ia; j = ib; l = 0; stride = N2; }
      c = (cz * n + cy) * n + cx;
      loc = i + N * j + N2 * l;
    };
    // traces of the outside neighbour lines
    for (int w = tid; w < np * 6 * G2; w += kThreads) {
      const int pl = w / (6 * G2), rem = w - pl * 6 * G2, f = rem / G2, pt = rem - f * G2;
      const int d = f >> 1, side = f & 1;
      int vx, vy, vz;
      vertex(pl, vx, vy, vz);
      const int vd = d == 0 ? vx : (d == 1 ? vy : vz);
      const int cd = side ? vd + 1 : vd - 2;
      T t1 = 0, t2 = 0;
      if (cd >= 0 && cd < n) {
        int c, loc, st;
        face_cell(d, cd, pl, pt % G, pt / G, c, loc, st);
        const T* line = r + (size_t)c * N3 + loc;
        T a[N];
#pragma unroll
        for (int q = 0; q < N; ++q) a[q] = line[q * st];
        t1 = side ? a[0] : a[N - 1];
#pragma unroll
        for (int q = 0; q < N; ++q) t2 = fma(side ? fd0[q] : fd1[q], a[q], t2);
      }
      T* F = s_F + (pl * 6 + f) * 2 * G2;
      F[pt] = t1;
      F[G2 + pt] = t2;
    }
    __syncthreads();
    // tangential masses (each within its cell of the face), through registers
    constexpr int NI = (PPB * 12 * G2 + kThreads - 1) / kThreads;
    T tm[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const int w = tid + q * kThreads;
      tm[q] = 0;
      if (w < np * 12 * G2) {
        const int pt = w % G2, blk = w / G2;
        const int ta = pt % G, tb = pt / G;
        const int ca = ta / N, ia = ta - ca * N, cb = tb / N, ib = tb - cb * N;
        const T* F = s_F + blk * G2 + ca * N + G * (cb * N);
        T acc = 0;
        for (int b2 = 0; b2 < N; ++b2) {
          T row = 0;
#pragma unroll
          for (int a2 = 0; a2 < N; ++a2) row = fma(fM[ia * N + a2], F[a2 + G * b2], row);
          acc = fma(fM[ib * N + b2], row, acc);
        }
        tm[q] = acc;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      const int w = tid + q * kThreads;
      if (w < np * 12 * G2) s_F[w] = tm[q];
    }
    __syncthreads();
    // subtract h times the couplings from f, one direction at a time (the
    // two faces of a direction touch different nodes)
    for (int d = 0; d < 3; ++d) {
      for (int w = tid; w < np * 2 * G2 * N; w += kThreads) {
        const int pl = w / (2 * G2 * N), rem = w - pl * 2 * G2 * N;
        const int side = rem / (G2 * N), rr = rem - side * G2 * N;
        const int pt = rr / N, a = rr - pt * N;
        const int ta = pt % G, tb = pt / G;
        const T* F = s_F + (pl * 6 + 2 * d + side) * 2 * G2;
        const T f1 = F[pt], f2 = F[G2 + pt];
        T val;
        if (side == 0)  // the lower neighbour's coupling into node a of the low cell
          val = (a == 0 ? -gam * f1 + T(0.5) * f2 : T(0)) - T(0.5) * fd0[a] * f1;
        else            // the upper neighbour's coupling into node a of the high cell
          val = (a == N - 1 ? -gam * f1 - T(0.5) * f2 : T(0)) + T(0.5) * fd1[a] * f1;
        const int pos = side ? N + a : a;
        const int idx = d == 0 ? pos + G * ta + G2 * tb
                               : (d == 1 ? ta + G * pos + G2 * tb : ta + G * tb + G2 * pos);
        s_X[pl * G3 + idx] -= h * val;
      }
      __syncthreads();
    }
  }

  const bool act = tid < np * G2;
  const int pl = act ? tid / G2 : 0, ln = tid - pl * G2;
  int vx = 1, vy = 1, vz = 1;
  if (act) vertex(pl, vx, vy, vz);
  const int tx = vtype(vx), ty = vtype(vy), tz = vtype(vz);
  const T* Sx = s_S + (ONE ? 0 : tx) * G2;
  const T* Sy = s_S + (ONE ? 1 : ty) * G2;
  const T* Sz = s_S + (ONE ? 2 : tz) * G2;
  T* X = s_X + pl * G3;
  const int la = ln % G, lb = ln / G;
  // offsets of line ln in direction d: start and stride
  const int o0 = la * G + lb * G2, o1 = la + lb * G2, o2 = la + lb * G;
  // interior directions (type 0) in even-odd form when the table has it;
  // their eigen-indices then run [even, odd] and so do their eigenvalues
  const T* s_YE = s_eo;
  const T* s_YO = s_eo + HH;
  const bool ex = eo_ok && tx == 0, ey = eo_ok && ty == 0, ez = eo_ok && tz == 0;
  const T* lx = s_l + (ex ? 4 : tx) * G;
  const T* ly = s_l + (ey ? 4 : ty) * G;
  const T* lz = s_l + (ez ? 4 : tz) * G;
  T in[G], out[G];
  // x-line (j', l') = (la, lb) of the patch in global memory: the matching
  // x-lines of the cells dx = 0 and dx = 1 (N contiguous values each)
  const int ldy = la / N, lj = la - ldy * N, ldz = lb / N, ll = lb - ldz * N;
  const size_t line0 =
      (size_t)(s_cb[pl] + n * ldy + nn * ldz) * N3 + (size_t)(lj * N + ll * N2);
  // forward: S^T along x, y, z
  if (act) {
    if constexpr (FUSED) {
#pragma unroll
      for (int a = 0; a < G; ++a) in[a] = X[o0 + a];
    } else {  // straight from r: the gather of the plain form
      const T* r0 = r + line0;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        in[a] = r0[a];
        in[N + a] = r0[N3 + a];
      }
    }
    if (ex) fd_fwd_eo<G>(s_YE, s_YO, in, out);
    else matvec_rows_t<G>(Sx, in, out);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o0 + a] = out[a];
  }
  psync();
  if (act) {
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[o1 + a * G];
    if (ey) fd_fwd_eo<G>(s_YE, s_YO, in, out);
    else matvec_rows_t<G>(Sy, in, out);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o1 + a * G] = out[a];
  }
  psync();
  if (act) {
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[o2 + a * G2];
    if (ez) fd_fwd_eo<G>(s_YE, s_YO, in, out);
    else matvec_rows_t<G>(Sz, in, out);
    // eigenvalue scaling: line (la, lb) = (i', j'), running over l'
    const T lij = lx[la] + ly[lb];
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = out[a] / (h * (lij + lz[a]));
    if (ez) fd_bwd_eo<G>(s_YE, s_YO, in, out);
    else matvec_rows<G>(Sz, in, out);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o2 + a * G2] = out[a];
  }
  psync();
  if (act) {
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[o1 + a * G];
    if (ey) fd_bwd_eo<G>(s_YE, s_YO, in, out);
    else matvec_rows<G>(Sy, in, out);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o1 + a * G] = out[a];
  }
  psync();
  if (act) {
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[o0 + a];
    if (ex) fd_bwd_eo<G>(s_YE, s_YO, in, out);
    else matvec_rows<G>(Sx, in, out);
    if constexpr (FUSED) {
#pragma unroll
      for (int a = 0; a < G; ++a) X[o0 + a] = out[a];
    } else {  // add the correction to x line by line (patches of a colour are disjoint)
      T* x0 = x + line0;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        x0[a] += out[a];
        x0[N3 + a] += out[N + a];
      }
    }
  }
  if constexpr (!FUSED) return;
  psync();
  // fused form: store the new values
  for (int w = w_first; w < w_hi; w += w_step) {
    const int q = w / G3, rr = w - q * G3;
    const int cell8 = rr / N3, loc = rr - cell8 * N3;
    const int dx = cell8 & 1, dy = (cell8 >> 1) & 1, dz = cell8 >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int c = s_cb[q] + dx + n * dy + nn * dz;
    const T val = s_X[q * G3 + (dx * N + i) + G * (dy * N + j) + G2 * (dz * N + l)];
    if constexpr (FUSED) x[(size_t)c * N3 + loc] = val;
    else x[(size_t)c * N3 + loc] += val;
  }
}

// ---------------------------------------------------------------------------
// Patch-wise operator evaluation (Sec. 2.1, Fig. patch_int): the vertex
// patches of one colour each add
//   v_P += h (Mz (x) My (x) Lx + Mz (x) Ly (x) Mx + Lz (x) My (x) Mx) u_P
// with the 2N x 2N window matrices of the patch's type per direction: every
// window carries the whole integral of its interior face (and of a boundary
// face of its end cell), the mass and stiffness of a cell are shared by the
// windows that contain it (weight 1/2, or 1 for the first and last cell of
// a line).  Summed over all (n-1)^3 patches this is A u; each DoF lies in up
// to 8 patches, so the work per DoF is about 8 times the cell-wise one (the
// paper's trade of redundant products for tensor-core-sized matrices).
// Patch layout in LDS as in the patch solve: i' + G j' + G^2 l'.
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void patch_apply_kernel(
    Batch<T> B, const T* __restrict__ tab, TableLayout lay, int bx, int by, int bz) {
  constexpr int G = 2 * N, G2 = G * G, G3 = G2 * G, N2 = N * N, N3 = N2 * N;
  constexpr int PPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  __shared__ T s_L[4 * G2];
  __shared__ T s_M[N2];
  __shared__ T s_X[PPB * G3];
  __shared__ T s_Y[PPB * G3];
  const int tid = threadIdx.x;
  const int bi = xcd_remap(blockIdx.x, gridDim.x);
  if (bi >= B.start[B.count]) return;
  const int pb = batch_find(B, bi);
  const T* __restrict__ u = B.d[pb].in;
  T* __restrict__ v = B.d[pb].out;
  const int n = B.d[pb].n, npx = B.d[pb].a0, npy = B.d[pb].a1, npatch = B.d[pb].a2;
  const T h = B.d[pb].h;
  const int p0 = (bi - B.start[pb]) * PPB;
  const int np = min(PPB, npatch - p0);
  if (np <= 0) return;
  for (int i = tid; i < 4 * G2; i += kThreads) s_L[i] = tab[lay.pw_l + i];
  for (int i = tid; i < N2; i += kThreads) s_M[i] = tab[lay.mass + i];
  auto vertex = [&](int pl, int& vx, int& vy, int& vz) {
    const int p = p0 + pl;
    const int px = p % npx, py = (p / npx) % npy, pz = p / (npx * npy);
    vx = 2 * px + (bx ? 1 : 2);
    vy = 2 * py + (by ? 1 : 2);
    vz = 2 * pz + (bz ? 1 : 2);
  };
  const int nn = n * n;
  __shared__ int s_cb[PPB];
  for (int q = tid; q < np; q += kThreads) {
    int vx, vy, vz;
    vertex(q, vx, vy, vz);
    s_cb[q] = (vx - 1) + n * (vy - 1) + nn * (vz - 1);
  }
  __syncthreads();
  for (int w = tid; w < np * G3; w += kThreads) {  // gather u_P
    const int pl = w / G3, rr = w - pl * G3;
    const int cell8 = rr / N3, loc = rr - cell8 * N3;
    const int dx = cell8 & 1, dy = (cell8 >> 1) & 1, dz = cell8 >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int c = s_cb[pl] + dx + n * dy + nn * dz;
    s_X[pl * G3 + (dx * N + i) + G * (dy * N + j) + G2 * (dz * N + l)] = u[(size_t)c * N3 + loc];
  }
  __syncthreads();

  const bool act = tid < np * G2;
  const int pl = act ? tid / G2 : 0, ln = tid - pl * G2;
  int vx = 1, vy = 1, vz = 1;
  if (act) vertex(pl, vx, vy, vz);
  const int tx = (vx == 1 ? 1 : 0) | (vx == n - 1 ? 2 : 0);
  const int ty = (vy == 1 ? 1 : 0) | (vy == n - 1 ? 2 : 0);
  const int tz = (vz == 1 ? 1 : 0) | (vz == n - 1 ? 2 : 0);
  T* X = s_X + pl * G3;
  T* Y = s_Y + pl * G3;
  const int la = ln % G, lb = ln / G;
  const int o0 = la * G + lb * G2, o1 = la + lb * G2, o2 = la + lb * G;
  // the window mass is block-diagonal: the shared cell mass times the
  // weight of each half (1 for an end cell of the line, else 1/2)
  auto mass = [&](int type, const T (&x)[G], T (&y)[G]) {
    const T w0 = (type & 1) ? T(1) : T(0.5), w1 = (type & 2) ? T(1) : T(0.5);
#pragma unroll
    for (int a = 0; a < N; ++a) {
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        s0 = fma(s_M[a * N + b], x[b], s0);
        s1 = fma(s_M[a * N + b], x[N + b], s1);
      }
      y[a] = w0 * s0;
      y[N + a] = w1 * s1;
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  T in1[G], in2[G], out1[G], out2[G];
  if (act) {  // x: t1 = Lx u, t2 = Mx u
#pragma unroll
    for (int a = 0; a < G; ++a) in1[a] = X[o0 + a];
    matvec_rows<G>(s_L + tx * G2, in1, out1);
    mass(tx, in1, out2);
#pragma unroll
    for (int a = 0; a < G; ++a) {
      X[o0 + a] = out1[a];
      Y[o0 + a] = out2[a];
    }
  }
  __syncthreads();
  if (act) {  // y: c = My t1 + Ly t2, e = My t2
#pragma unroll
    for (int a = 0; a < G; ++a) {
      in1[a] = X[o1 + a * G];
      in2[a] = Y[o1 + a * G];
    }
    mass(ty, in1, out1);
    matvec_rows<G>(s_L + ty * G2, in2, out2);
#pragma unroll
    for (int a = 0; a < G; ++a) out1[a] += out2[a];
    mass(ty, in2, out2);
#pragma unroll
    for (int a = 0; a < G; ++a) {
      X[o1 + a * G] = out1[a];
      Y[o1 + a * G] = out2[a];
    }
  }
  __syncthreads();
  if (act) {  // z: v = h (Mz c + Lz e)
#pragma unroll
    for (int a = 0; a < G; ++a) {
      in1[a] = X[o2 + a * G2];
      in2[a] = Y[o2 + a * G2];
    }
    mass(tz, in1, out1);
    matvec_rows<G>(s_L + tz * G2, in2, out2);
#pragma unroll
    for (int a = 0; a < G; ++a) X[o2 + a * G2] = h * (out1[a] + out2[a]);
  }
  __syncthreads();
  for (int w = tid; w < np * G3; w += kThreads) {  // scatter-add into v
    const int q = w / G3, rr = w - q * G3;
    const int cell8 = rr / N3, loc = rr - cell8 * N3;
    const int dx = cell8 & 1, dy = (cell8 >> 1) & 1, dz = cell8 >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int c = s_cb[q] + dx + n * dy + nn * dz;
    v[(size_t)c * N3 + loc] += s_X[q * G3 + (dx * N + i) + G * (dy * N + j) + G2 * (dz * N + l)];
  }
}

// ---------------------------------------------------------------------------
// Exact coarse solve by fast diagonalization of the whole n0^3-cell level
// (one workgroup; G = n0 N <= 3N).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void coarse_fd_kernel(
    Batch<T> B, const T* __restrict__ tab, TableLayout lay) {
  const T* __restrict__ b = B.d[blockIdx.x].in;
  T* __restrict__ x = B.d[blockIdx.x].out;
  const int n0 = B.d[blockIdx.x].n;
  const T h = B.d[blockIdx.x].h;
  constexpr int GM = 3 * N, N2 = N * N, N3 = N2 * N;
  extern __shared__ __align__(16) unsigned char s_raw[];
  T* s_dyn = reinterpret_cast<T*>(s_raw);
  const int G = n0 * N, G2 = G * G, G3 = G2 * G;
  T* s_S = s_dyn;
  T* s_l = s_S + G2;
  T* X = s_l + G;
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
  T in[GM], out[GM];
  for (int pass = 0; pass < 6; ++pass) {
    const int d = pass < 3 ? pass : 5 - pass;
    const int sd = d == 0 ? 1 : (d == 1 ? G : G2);
    for (int ln = tid; ln < G2; ln += kThreads) {
      const int la = ln % G, lb = ln / G;
      const int o = d == 0 ? la * G + lb * G2 : (d == 1 ? la + lb * G2 : la + lb * G);
      for (int a = 0; a < G; ++a) in[a] = X[o + a * sd];
      for (int a = 0; a < G; ++a) {
        T s = 0.0;
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
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void restrict_kernel(
    Batch<T> B, const T* __restrict__ tab, TableLayout lay) {
  constexpr int G = 2 * N, G2 = G * G, G3 = G2 * G, N2 = N * N, N3 = N2 * N;
  constexpr int CPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  __shared__ T s_P[G * N];
  __shared__ T s_X[CPB * G3];
  const int tid = threadIdx.x;
  const int bi = xcd_remap(blockIdx.x, gridDim.x);
  if (bi >= B.start[B.count]) return;
  const int pb = batch_find(B, bi);
  const int nc = B.d[pb].n;
  const int ncells = nc * nc * nc;
  const int c0 = (bi - B.start[pb]) * CPB;
  const int cnt = min(CPB, ncells - c0);
  if (cnt <= 0) return;
  const T* __restrict__ src_in = B.d[pb].in;
  T* __restrict__ dst_out = B.d[pb].out;
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
    s_X[cl * G3 + (ox * N + i) + G * (oy * N + j) + G2 * (oz * N + l)] = src_in[(size_t)f * N3 + loc];
  }
  __syncthreads();
  // x: lines (j', l') of length G -> N values, stored in place at stride 1
  for (int w = tid; w < cnt * G2; w += kThreads) {
    const int cl = w / G2, ln = w - cl * G2;
    T* X = s_X + cl * G3 + ln * G;
    T in[G];
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[a];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      T s = 0.0;
#pragma unroll
      for (int a = 0; a < G; ++a) s = fma(s_P[a * N + b], in[a], s);
      X[b] = s;
      keep_lds_reads_local<N>();
    }
  }
  __syncthreads();
  // y: lines (b, l') over j'
  for (int w = tid; w < cnt * N * G; w += kThreads) {
    const int cl = w / (N * G), ln = w - cl * N * G;
    const int bx = ln % N, lz = ln / N;
    T* X = s_X + cl * G3 + bx + lz * G2;
    T in[G];
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[a * G];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      T s = 0.0;
#pragma unroll
      for (int a = 0; a < G; ++a) s = fma(s_P[a * N + b], in[a], s);
      X[b * G] = s;
      keep_lds_reads_local<N>();
    }
  }
  __syncthreads();
  // z: lines (b, b') over l', written to the coarse vector
  for (int w = tid; w < cnt * N2; w += kThreads) {
    const int cl = w / N2, ln = w - cl * N2;
    const int bx = ln % N, by = ln / N;
    const T* X = s_X + cl * G3 + bx + by * G;
    T in[G];
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = X[a * G2];
    T* dst = dst_out + (size_t)(c0 + cl) * N3 + bx + by * N;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      T s = 0.0;
#pragma unroll
      for (int a = 0; a < G; ++a) s = fma(s_P[a * N + b], in[a], s);
      dst[b * N2] = s;
      keep_lds_reads_local<N>();
    }
  }
}

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void prolongate_add_kernel(
    Batch<T> B, const T* __restrict__ tab, TableLayout lay) {
  constexpr int G = 2 * N, G2 = G * G, G3 = G2 * G, N2 = N * N, N3 = N2 * N;
  constexpr int CPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  __shared__ T s_P[G * N];
  __shared__ T s_X[CPB * G3];
  const int tid = threadIdx.x;
  const int bi = xcd_remap(blockIdx.x, gridDim.x);
  if (bi >= B.start[B.count]) return;
  const int pb = batch_find(B, bi);
  const int nc = B.d[pb].n;
  const int ncells = nc * nc * nc;
  const int c0 = (bi - B.start[pb]) * CPB;
  const int cnt = min(CPB, ncells - c0);
  if (cnt <= 0) return;
  const T* __restrict__ src_in = B.d[pb].in;
  T* __restrict__ dst_out = B.d[pb].out;
  for (int i = tid; i < G * N; i += kThreads) s_P[i] = tab[lay.p1 + i];
  // coarse values at X[b + G b' + G^2 b''] (the low corner of the box)
  for (int w = tid; w < cnt * N3; w += kThreads) {
    const int cl = w / N3, loc = w - cl * N3;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    s_X[cl * G3 + i + G * j + G2 * l] = src_in[(size_t)(c0 + cl) * N3 + loc];
  }
  __syncthreads();
  // z first: lines (b, b') over l: N -> G
  for (int w = tid; w < cnt * N2; w += kThreads) {
    const int cl = w / N2, ln = w - cl * N2;
    T* X = s_X + cl * G3 + (ln % N) + (ln / N) * G;
    T in[N];
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = X[b * G2];
#pragma unroll
    for (int a = 0; a < G; ++a) {
      T s = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) s = fma(s_P[a * N + b], in[b], s);
      X[a * G2] = s;
      keep_lds_reads_local<N>();
    }
  }
  __syncthreads();
  // y: lines (b, l') over j: N -> G
  for (int w = tid; w < cnt * N * G; w += kThreads) {
    const int cl = w / (N * G), ln = w - cl * N * G;
    T* X = s_X + cl * G3 + (ln % N) + (ln / N) * G2;
    T in[N];
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = X[b * G];
#pragma unroll
    for (int a = 0; a < G; ++a) {
      T s = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) s = fma(s_P[a * N + b], in[b], s);
      X[a * G] = s;
      keep_lds_reads_local<N>();
    }
  }
  __syncthreads();
  // x: lines (j', l') over i: N -> G
  for (int w = tid; w < cnt * G2; w += kThreads) {
    const int cl = w / G2, ln = w - cl * G2;
    T* X = s_X + cl * G3 + ln * G;
    T in[N];
#pragma unroll
    for (int b = 0; b < N; ++b) in[b] = X[b];
#pragma unroll
    for (int a = 0; a < G; ++a) {
      T s = 0.0;
#pragma unroll
      for (int b = 0; b < N; ++b) s = fma(s_P[a * N + b], in[b], s);
      X[a] = s;
      keep_lds_reads_local<N>();
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
    dst_out[(size_t)f * N3 + loc] += s_X[cl * G3 + (ox * N + i) + G * (oy * N + j) + G2 * (oz * N + l)];
  }
}

template <typename T>
const T* tab_of(const DevTab& t);
template <>
const double* tab_of<double>(const DevTab& t) { return t.tab; }
template <>
const float* tab_of<float>(const DevTab& t) { return t.tabf; }

// Fill the work ranges of a batch; `items(i)` = work items of job i.
template <typename T, typename F>
hipError_t make_batch(Batch<T>& B, int count, F&& fill) {
  if (count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
  B.count = count;
  B.start[0] = 0;
  for (int i = 0; i < count; ++i) {
    int64_t items = 0;
    hipError_t e = fill(i, B.d[i], items);
    if (e != hipSuccess) return e;
    if ((int64_t)B.start[i] + items > ((int64_t)1 << 30)) return hipErrorInvalidValue;
    B.start[i + 1] = B.start[i] + (int)items;
  }
  for (int i = count; i < kMaxBatch; ++i) B.start[i + 1] = B.start[count];
  return hipSuccess;
}

template <typename T, int N>
hipError_t apply_impl(const ApplyJob* jobs, int count, const DevTab& t, hipStream_t s) {
  constexpr int CPW = (64 / (N * N)) > 0 ? 64 / (N * N) : 1;
  // N = 5, 6, 7: whole cells per wave would leave 14, 28 or 15 of 64 lanes
  // idle; the workgroup shares a tile of kThreads / N^2 = 10, 7 or 5 cells
  // instead (250, 252, 245 of 256 lanes)
  constexpr bool WG = (N >= 5 && N <= 7);
  constexpr int CPT = kThreads / (N * N);
  Batch<T> B;
  bool residual = jobs[0].b != nullptr;
  hipError_t e = make_batch(B, count, [&](int i, Desc<T>& d, int64_t& items) {
    const ApplyJob& j = jobs[i];
    if (j.n < 1 || j.n > 1024 || !j.u || !j.v || (j.b != nullptr) != residual)
      return hipErrorInvalidValue;
    int tx = 1;
    for (int q = 1; q <= CPW && q <= j.n; ++q)
      if (j.n % q == 0) tx = q;  // largest divisor of n that fits a wave
    d.in = (const T*)j.u;
    d.out = (T*)j.v;
    d.aux = (const T*)j.b;
    d.h = (T)j.h;
    d.n = j.n;
    d.a0 = tx;
    d.a1 = j.n / tx;
    d.a2 = (j.order > 0 && j.n % j.order == 0) ? j.order : ((j.n % 8 == 0) ? 8 : 1);
    const int64_t cells = (int64_t)j.n * j.n * j.n;
    items = WG ? (cells + CPT - 1) / CPT : (int64_t)d.a1 * j.n * j.n;
    return hipSuccess;
  });
  if (e != hipSuccess) return e;
  const int per_block = WG ? 1 : kThreads / 64;  // work items (tiles) per workgroup
  const int grid = (B.start[count] + per_block - 1) / per_block;
  if (grid == 0) return hipSuccess;
  if (residual)
    hipLaunchKernelGGL((apply_wave_kernel<T, N, true, WG>), dim3(grid), dim3(kThreads), 0, s, B,
                       tab_of<T>(t), t.lay);
  else
    hipLaunchKernelGGL((apply_wave_kernel<T, N, false, WG>), dim3(grid), dim3(kThreads), 0, s, B,
                       tab_of<T>(t), t.lay);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t patch_impl(int colour, const PatchJob* jobs, int count, const DevTab& t,
                      hipStream_t s, bool apply = false) {
  const bool fused = count > 0 && jobs[0].b != nullptr;
  constexpr int G2 = 4 * N * N;
  constexpr int PPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  const int bx = colour & 1, by = (colour >> 1) & 1, bz = (colour >> 2) & 1;
  Batch<T> B;
  hipError_t e = make_batch(B, count, [&](int i, Desc<T>& d, int64_t& items) {
    const PatchJob& j = jobs[i];
    if (j.n < 2 || j.n > 1024 || !j.r || !j.x) return hipErrorInvalidValue;
    if ((j.b != nullptr) != fused || (fused && (j.b == j.x || j.r == j.x)))
      return hipErrorInvalidValue;
    // vertices v in [1, n-1]: odd ones 1,3,..; even ones 2,4,..
    auto cnt = [&](int bit) { return bit ? j.n / 2 : (j.n - 1) / 2; };
    d.in = (const T*)j.r;
    d.out = (T*)j.x;
    d.aux = (const T*)j.b;
    d.h = (T)j.h;
    d.n = j.n;
    d.a0 = cnt(bx);
    d.a1 = cnt(by);
    d.a2 = d.a0 * d.a1 * cnt(bz);
    items = (d.a2 + PPB - 1) / PPB;
    return hipSuccess;
  });
  if (e != hipSuccess) return e;
  if (B.start[count] == 0) return hipSuccess;
  if (apply)
    hipLaunchKernelGGL((patch_apply_kernel<T, N>), dim3(B.start[count]), dim3(kThreads), 0, s, B,
                       tab_of<T>(t), t.lay, bx, by, bz);
  else if (fused)
    hipLaunchKernelGGL((patch_fd_kernel<T, N, true>), dim3(B.start[count]), dim3(kThreads), 0, s,
                       B, tab_of<T>(t), t.lay, bx, by, bz);
  else
    hipLaunchKernelGGL((patch_fd_kernel<T, N>), dim3(B.start[count]), dim3(kThreads), 0, s, B,
                       tab_of<T>(t), t.lay, bx, by, bz);
  return hipGetLastError();
}

// out = in on the cells of the given layers: slab q is the layer
// c_dir[q] = lay[q] (all n^2 cells of it), N^3 values per cell
template <typename T>
__global__ __launch_bounds__(kThreads) void copy_layers_kernel(const T* __restrict__ in,
                                                               T* __restrict__ out, int n, int N3,
                                                               int nslab, int4 dirs, int4 lays,
                                                               int2 dirs2, int2 lays2) {
  const int64_t per = (int64_t)n * n * N3;
  const int64_t total = per * nslab;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kThreads) {
    const int q = (int)(e / per);
    const int64_t rem = e - q * per;
    const int64_t cl = rem / N3;
    const int loc = (int)(rem - cl * N3);
    const int a = (int)(cl % n), b = (int)(cl / n);
    const int dir = q < 4 ? (&dirs.x)[q] : (&dirs2.x)[q - 4];
    const int layer = q < 4 ? (&lays.x)[q] : (&lays2.x)[q - 4];
    int cx, cy, cz;
    if (dir == 0) { cx = layer; cy = a; cz = b; }
    else if (dir == 1) { cx = a; cy = layer; cz = b; }
    else { cx = a; cy = b; cz = layer; }
    const int64_t idx = (((int64_t)cz * n + cy) * n + cx) * N3 + loc;
    out[idx] = in[idx];
  }
}

template <typename T>
hipError_t copy_uncovered_impl(int N, int colour, const T* in, T* out, int n, hipStream_t s) {
  if (n < 1 || !in || !out || in == out) return hipErrorInvalidValue;
  const int N3 = N * N * N;
  int dirs[6], lays[6], ns = 0;
  for (int d = 0; d < 3; ++d) {
    const int bit = (colour >> d) & 1;
    // vertices 1 <= v <= n - 1 of parity `bit`; a patch covers cells v - 1, v
    const int vmin = bit ? 1 : 2;
    const int vmax = ((n - 1) % 2 == bit) ? n - 1 : n - 2;
    if (vmax < vmin) {  // no patch of this colour: every cell is outside
      const int64_t total = (int64_t)n * n * n * N3;
      return hipMemcpyAsync(out, in, total * sizeof(T), hipMemcpyDeviceToDevice, s);
    }
    for (int c = 0; c < vmin - 1; ++c) { dirs[ns] = d; lays[ns++] = c; }
    for (int c = vmax + 1; c < n; ++c) { dirs[ns] = d; lays[ns++] = c; }
  }
  if (ns == 0) return hipSuccess;
  const int64_t total = (int64_t)ns * n * n * N3;
  int64_t g = (total + kThreads - 1) / kThreads;
  if (g > 16384) g = 16384;
  int4 d4 = {dirs[0], ns > 1 ? dirs[1] : 0, ns > 2 ? dirs[2] : 0, ns > 3 ? dirs[3] : 0};
  int4 l4 = {lays[0], ns > 1 ? lays[1] : 0, ns > 2 ? lays[2] : 0, ns > 3 ? lays[3] : 0};
  int2 d2 = {ns > 4 ? dirs[4] : 0, ns > 5 ? dirs[5] : 0};
  int2 l2 = {ns > 4 ? lays[4] : 0, ns > 5 ? lays[5] : 0};
  hipLaunchKernelGGL(copy_layers_kernel<T>, dim3((unsigned)g), dim3(kThreads), 0, s, in, out, n,
                     N3, ns, d4, l4, d2, l2);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t coarse_impl(const CoarseJob* jobs, int count, const DevTab& t, hipStream_t s) {
  Batch<T> B;
  int gmax = 0;
  hipError_t e = make_batch(B, count, [&](int i, Desc<T>& d, int64_t& items) {
    const CoarseJob& j = jobs[i];
    if (j.n0 < 1 || j.n0 > 3 || t.lay.Gc != j.n0 * N || !j.b || !j.x) return hipErrorInvalidValue;
    d.in = (const T*)j.b;
    d.out = (T*)j.x;
    d.aux = nullptr;
    d.h = (T)j.h;
    d.n = j.n0;
    d.a0 = d.a1 = d.a2 = 0;
    gmax = gmax > j.n0 * N ? gmax : j.n0 * N;
    items = 1;
    return hipSuccess;
  });
  if (e != hipSuccess) return e;
  const int G = gmax;
  const size_t shm = sizeof(T) * ((size_t)G * G + G + (size_t)G * G * G);
  if (shm > 65536) {
    hipError_t e2 = hipFuncSetAttribute((const void*)coarse_fd_kernel<T, N>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e2 != hipSuccess) return e2;
  }
  hipLaunchKernelGGL((coarse_fd_kernel<T, N>), dim3(count), dim3(kThreads), shm, s, B,
                     tab_of<T>(t), t.lay);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t transfer_impl(bool restr, const TransferJob* jobs, int count, const DevTab& t,
                         hipStream_t s) {
  constexpr int G2 = 4 * N * N;
  constexpr int CPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  Batch<T> B;
  hipError_t e = make_batch(B, count, [&](int i, Desc<T>& d, int64_t& items) {
    const TransferJob& j = jobs[i];
    if (j.nc < 1 || j.nc > 512 || !j.in || !j.out) return hipErrorInvalidValue;
    d.in = (const T*)j.in;
    d.out = (T*)j.out;
    d.aux = nullptr;
    d.h = (T)0;
    d.n = j.nc;
    d.a0 = d.a1 = d.a2 = 0;
    items = ((int64_t)j.nc * j.nc * j.nc + CPB - 1) / CPB;
    return hipSuccess;
  });
  if (e != hipSuccess) return e;
  if (restr)
    hipLaunchKernelGGL((restrict_kernel<T, N>), dim3(B.start[count]), dim3(kThreads), 0, s, B,
                       tab_of<T>(t), t.lay);
  else
    hipLaunchKernelGGL((prolongate_add_kernel<T, N>), dim3(B.start[count]), dim3(kThreads), 0,
                       s, B, tab_of<T>(t), t.lay);
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

hipError_t launch_apply_batch(int prec, int N, const ApplyJob* jobs, int count, const DevTab& t,
                              hipStream_t s) {
  if (t.lay.N != N) return hipErrorInvalidValue;
  if ((prec == 0 || prec == 3) && N == 4)
    return launch_apply_mfma4_batch(prec == 0 ? 0 : 1, jobs, count, t, s);
  if (prec == 0 && N == 8) return launch_apply_mfma8_batch(jobs, count, t, s);
  if (prec == 0 || prec == 2) {
#define CALL(NN) apply_impl<double, NN>(jobs, count, t, s)
    SIPG_DISPATCH_N(N, CALL)
#undef CALL
  }
#define CALL(NN) apply_impl<float, NN>(jobs, count, t, s)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_patch_fd_batch(int prec, int N, int colour, const PatchJob* jobs, int count,
                                 const DevTab& t, hipStream_t s) {
  if (t.lay.N != N || colour < 0 || colour > 7) return hipErrorInvalidValue;
  const bool fused = count > 0 && jobs[0].b != nullptr;
  if (N == 4 && !fused) return launch_patch_mfma4_batch(prec, colour, jobs, count, t, s);
  if (prec == 0) {
#define CALL(NN) patch_impl<double, NN>(colour, jobs, count, t, s)
    SIPG_DISPATCH_N(N, CALL)
#undef CALL
  }
#define CALL(NN) patch_impl<float, NN>(colour, jobs, count, t, s)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_copy_uncovered(int prec, int N, int colour, const void* in, void* out, int n,
                                 hipStream_t s) {
  if (N < 2 || N > 8 || colour < 0 || colour > 7) return hipErrorInvalidValue;
  return prec == 0 ? copy_uncovered_impl<double>(N, colour, (const double*)in, (double*)out, n, s)
                   : copy_uncovered_impl<float>(N, colour, (const float*)in, (float*)out, n, s);
}

hipError_t launch_patch_apply_f64(int N, int colour, const double* u, double* v, const DevTab& t,
                                  int n, double h, hipStream_t s) {
  if (t.lay.N != N || colour < 0 || colour > 7) return hipErrorInvalidValue;
  PatchJob j{u, v, n, h};
#define CALL(NN) patch_impl<double, NN>(colour, &j, 1, t, s, true)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_coarse_fd_batch(int prec, int N, const CoarseJob* jobs, int count,
                                  const DevTab& t, hipStream_t s) {
  if (t.lay.N != N) return hipErrorInvalidValue;
  if (prec == 0) {
#define CALL(NN) coarse_impl<double, NN>(jobs, count, t, s)
    SIPG_DISPATCH_N(N, CALL)
#undef CALL
  }
#define CALL(NN) coarse_impl<float, NN>(jobs, count, t, s)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

hipError_t launch_transfer_batch(int prec, int N, bool restr, const TransferJob* jobs, int count,
                                 const DevTab& t, hipStream_t s) {
  if (t.lay.N != N) return hipErrorInvalidValue;
  if (prec == 0) {
#define CALL(NN) transfer_impl<double, NN>(restr, jobs, count, t, s)
    SIPG_DISPATCH_N(N, CALL)
#undef CALL
  }
#define CALL(NN) transfer_impl<float, NN>(restr, jobs, count, t, s)
  SIPG_DISPATCH_N(N, CALL)
#undef CALL
}

// single-problem forms
hipError_t launch_apply_f64(int N, const double* u, double* v, const double* b, const DevTab& t,
                            int n, double h, hipStream_t s) {
  ApplyJob j{u, v, b, n, h};
  return launch_apply_batch(0, N, &j, 1, t, s);
}
hipError_t launch_apply_f32(int N, const float* u, float* v, const float* b, const DevTab& t,
                            int n, double h, hipStream_t s) {
  ApplyJob j{u, v, b, n, h};
  return launch_apply_batch(1, N, &j, 1, t, s);
}
hipError_t launch_residual_f32(int N, const float* u, float* v, const float* b, const DevTab& t,
                               int n, double h, hipStream_t s) {
  ApplyJob j{u, v, b, n, h};
  return launch_apply_batch(3, N, &j, 1, t, s);
}
hipError_t launch_patch_fd_f64(int N, int colour, const double* r, double* x, const DevTab& t,
                               int n, double h, hipStream_t s) {
  PatchJob j{r, x, n, h};
  return launch_patch_fd_batch(0, N, colour, &j, 1, t, s);
}
hipError_t launch_patch_fd_f32(int N, int colour, const float* r, float* x, const DevTab& t,
                               int n, double h, hipStream_t s) {
  PatchJob j{r, x, n, h};
  return launch_patch_fd_batch(1, N, colour, &j, 1, t, s);
}
hipError_t launch_coarse_fd_f64(int N, int n0, const double* b, double* x, const DevTab& t,
                                double h, hipStream_t s) {
  CoarseJob j{b, x, n0, h};
  return launch_coarse_fd_batch(0, N, &j, 1, t, s);
}
hipError_t launch_coarse_fd_f32(int N, int n0, const float* b, float* x, const DevTab& t,
                                double h, hipStream_t s) {
  CoarseJob j{b, x, n0, h};
  return launch_coarse_fd_batch(1, N, &j, 1, t, s);
}
hipError_t launch_restrict_f64(int N, const double* rf, double* rc, const DevTab& t, int nc,
                               hipStream_t s) {
  TransferJob j{rf, rc, nc};
  return launch_transfer_batch(0, N, true, &j, 1, t, s);
}
hipError_t launch_restrict_f32(int N, const float* rf, float* rc, const DevTab& t, int nc,
                               hipStream_t s) {
  TransferJob j{rf, rc, nc};
  return launch_transfer_batch(1, N, true, &j, 1, t, s);
}
hipError_t launch_prolongate_add_f64(int N, const double* ec, double* xf, const DevTab& t, int nc,
                                     hipStream_t s) {
  TransferJob j{ec, xf, nc};
  return launch_transfer_batch(0, N, false, &j, 1, t, s);
}
hipError_t launch_prolongate_add_f32(int N, const float* ec, float* xf, const DevTab& t, int nc,
                                     hipStream_t s) {
  TransferJob j{ec, xf, nc};
  return launch_transfer_batch(1, N, false, &j, 1, t, s);
}

}  // namespace sipg
