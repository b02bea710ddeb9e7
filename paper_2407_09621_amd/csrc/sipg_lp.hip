// Low-precision kernels of the V-cycle (Sec. 7.1 mixed precision): FP32
// storage, 1D contractions on FP16 or BF16 matrix cores with FP32
// accumulation, optional split-operand error correction (Sec. 5.2,
// Alg. matmul).
//
// Building block: v_mfma_f32_4x4x4{f16,bf16_1k} on gfx950 computes 16
// independent 4x4x4 products.  Lane 4b + j supplies column j of block b of
// the B operand (its four K values) and receives column j of block b of the
// result in its four accumulator registers; lane 4b + i supplies row i of
// block b of the A operand.  With the same matrix in every block this is a
// "line per lane" matrix-vector product for 64 lines at once, the layout of
// the VALU kernels.  Lines longer than 4 are split into 4 x 4 sub-blocks
// (lengths padded to a multiple of 4 with zeros).
//
// FP16 range: every line is scaled by a power of two so that its largest
// entry lies in [0.5, 1) before rounding, and the product is scaled back in
// FP32 (exact).  BF16 has the FP32 exponent range and is not scaled.
// Error correction (both operands refined, as the paper's Alg. matmul):
// x = x_hi + 2^-s x_lo with x_lo = round((x - x_hi) 2^s), s = 11 for FP16
// and 8 for BF16; S x ~ S_hi x_hi + 2^-s (S_lo x_hi + S_hi x_lo), the
// correction accumulated in its own FP32 accumulator.  EC = 1 is that
// scheme; EC = 2 refines only the constant matrix operand
// (S x ~ S_hi x_hi + 2^-s S_lo x_hi, two products): the rounded 1D
// operator of BF16 (8 significand bits) moves the lowest eigenvalues of
// the discrete Laplacian by more than their size at degrees >= 4, which
// stalls the smoother, while rounding the vector operand only perturbs
// each entry relatively.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "kernels.h"

namespace sipg {

namespace {

constexpr int kThreads = 256;

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// ---- operand rounding -----------------------------------------------------
template <bool BF>
struct Lp;

template <>
struct Lp<false> {  // FP16
  typedef h4 vec;
  static constexpr float kSplit = 2048.0f;  // 2^11
  static __device__ __forceinline__ float round(float x) { return (float)(_Float16)x; }
  static __device__ __forceinline__ vec pack(float a, float b, float c, float d) {
    vec v = {(_Float16)a, (_Float16)b, (_Float16)c, (_Float16)d};
    return v;
  }
  static __device__ __forceinline__ f4 mfma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x4f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Lp<true> {  // BF16
  typedef s4 vec;
  static constexpr float kSplit = 256.0f;  // 2^8
  static __device__ __forceinline__ short bits(float x) {
    __bf16 b = (__bf16)x;  // round to nearest even
    return __builtin_bit_cast(short, b);
  }
  static __device__ __forceinline__ float round(float x) { return (float)(__bf16)x; }
  static __device__ __forceinline__ vec pack(float a, float b, float c, float d) {
    vec v = {bits(a), bits(b), bits(c), bits(d)};
    return v;
  }
  static __device__ __forceinline__ f4 mfma(vec a, vec b, f4 c) {
    return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0);
  }
};

// y = S x for the line held by every lane (all 64 lanes must call).  NP is
// the padded line length (multiple of 4); S is n x n (n <= NP), row-major,
// possibly different per group of 4 lanes.
template <int NP, bool BF, int EC>
struct LineMV {
  typedef Lp<BF> L;
  static constexpr int C = NP / 4;
  typename L::vec hi[C][C];
  typename L::vec lo[C][C];

  // lane's row of S for block rows: row 4 rc + (lane % 4)
  __device__ __forceinline__ void load(const float* __restrict__ S, int n, bool transpose) {
    const int r = threadIdx.x & 3;
#pragma unroll
    for (int rc = 0; rc < C; ++rc)
#pragma unroll
      for (int kc = 0; kc < C; ++kc) {
        float v[4], w[4];
        const int row = 4 * rc + r;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int col = 4 * kc + q;
          float s = 0.0f;
          if (row < n && col < n) s = transpose ? S[col * n + row] : S[row * n + col];
          v[q] = L::round(s);
          w[q] = (s - v[q]) * L::kSplit;
        }
        hi[rc][kc] = L::pack(v[0], v[1], v[2], v[3]);
        if (EC != 0) lo[rc][kc] = L::pack(w[0], w[1], w[2], w[3]);
      }
  }

  __device__ __forceinline__ void apply(const float (&x)[NP], float (&y)[NP]) const {
    float s = 1.0f, inv = 1.0f;
    if (!BF) {  // per-line power-of-two scale into [0.5, 1)
      float m = 0.0f;
#pragma unroll
      for (int a = 0; a < NP; ++a) m = fmaxf(m, fabsf(x[a]));
      if (m > 0.0f) {
        int e;
        frexpf(m, &e);
        s = ldexpf(1.0f, -e);
        inv = ldexpf(1.0f, e);
      }
    }
    typename L::vec xh[C], xl[C];
#pragma unroll
    for (int kc = 0; kc < C; ++kc) {
      float v[4], w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float t = x[4 * kc + q] * s;
        v[q] = L::round(t);
        w[q] = (t - v[q]) * L::kSplit;
      }
      xh[kc] = L::pack(v[0], v[1], v[2], v[3]);
      if (EC == 1) xl[kc] = L::pack(w[0], w[1], w[2], w[3]);
    }
#pragma unroll
    for (int rc = 0; rc < C; ++rc) {
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kc = 0; kc < C; ++kc) acc = L::mfma(hi[rc][kc], xh[kc], acc);
      if (EC != 0) {
        f4 cor = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kc = 0; kc < C; ++kc) {
          cor = L::mfma(lo[rc][kc], xh[kc], cor);
          if (EC == 1) cor = L::mfma(hi[rc][kc], xl[kc], cor);
        }
        acc += cor * (1.0f / L::kSplit);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) y[4 * rc + i] = acc[i] * inv;
    }
  }
};

template <int N>
struct Pad {
  static constexpr int value = (N + 3) / 4 * 4;
};

template <int N>
__device__ __forceinline__ void add_lower_face(float (&t)[N], float f, float g, float gam,
                                               const float* __restrict__ d0) {
  t[0] += -gam * f + 0.5f * g;
#pragma unroll
  for (int a = 0; a < N; ++a) t[a] = fmaf(-0.5f * d0[a], f, t[a]);
}
template <int N>
__device__ __forceinline__ void add_upper_face(float (&t)[N], float f, float g, float gam,
                                               const float* __restrict__ d1) {
  t[N - 1] += -gam * f - 0.5f * g;
#pragma unroll
  for (int a = 0; a < N; ++a) t[a] = fmaf(0.5f * d1[a], f, t[a]);
}
template <int N>
__device__ __forceinline__ void add_boundary_correction(float (&t)[N], const float (&x)[N],
                                                        bool lo, bool hi,
                                                        const float* __restrict__ d0,
                                                        const float* __restrict__ d1) {
  if (lo) {
    float g = 0.0f;
#pragma unroll
    for (int a = 0; a < N; ++a) g = fmaf(d0[a], x[a], g);
    t[0] += 0.5f * g;
#pragma unroll
    for (int a = 0; a < N; ++a) t[a] = fmaf(0.5f * d0[a], x[0], t[a]);
  }
  if (hi) {
    float g = 0.0f;
#pragma unroll
    for (int a = 0; a < N; ++a) g = fmaf(d1[a], x[a], g);
    t[N - 1] -= 0.5f * g;
#pragma unroll
    for (int a = 0; a < N; ++a) t[a] = fmaf(-0.5f * d1[a], x[N - 1], t[a]);
  }
}

// line of length N inside a padded register array
template <int N, int NP, bool BF, int EC>
__device__ __forceinline__ void line_mv(const LineMV<NP, BF, EC>& m, const float (&x)[N],
                                        float (&y)[N]) {
  float xp[NP], yp[NP];
#pragma unroll
  for (int a = 0; a < NP; ++a) xp[a] = a < N ? x[a] : 0.0f;
  m.apply(xp, yp);
#pragma unroll
  for (int a = 0; a < N; ++a) y[a] = yp[a];
}
template <int N, int NP, bool BF, int EC>
__device__ __forceinline__ void line_mv_acc(const LineMV<NP, BF, EC>& m, const float (&x)[N],
                                            float (&y)[N]) {
  float t[N];
  line_mv<N>(m, x, t);
#pragma unroll
  for (int a = 0; a < N; ++a) y[a] += t[a];
}

struct TileMapLp {
  int n, tx, ntx, blk, ngroups;
};

__device__ __forceinline__ int tile_first_cell(const TileMapLp& m, int t) {
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

// ---------------------------------------------------------------------------
// Operator apply / residual, FP32 storage, contractions on the matrix cores.
// Same decomposition as the VALU kernel (a wave owns TX cells of an x-row,
// one lane per 1D line); the N x N products of the three stages run as
// LineMV calls of all 64 lanes, face traces and rank-2 terms in FP32.
// ---------------------------------------------------------------------------
// WG: the workgroup's waves share one tile of kThreads / N^2 cells of the
// blocked order, with workgroup barriers (as in the FP64 vector kernel).
template <int N, bool BF, int EC, bool RES, bool WG = false>
__global__ __launch_bounds__(kThreads) void apply_lp_kernel(
    Batch<float> B, const float* __restrict__ tab, TableLayout lay) {
  constexpr int N2 = N * N, N3 = N2 * N, CPB = (64 / N2) > 0 ? 64 / N2 : 1;
  constexpr int NP = Pad<N>::value;
  constexpr int WAVES = kThreads / 64;
  constexpr int CPT = kThreads / N2;
  constexpr int CS = WG ? CPT : CPB;
  constexpr int SLOTS = WG ? CPT : WAVES * CPB;
  __shared__ float s_t1_all[SLOTS * N3];
  __shared__ float s_t2_all[SLOTS * N3];
  __shared__ float s_ty_all[SLOTS * 4 * N2];
  __shared__ float s_tz_all[SLOTS * 4 * N2];
  __shared__ float s_tzm_all[SLOTS * 4 * N2];
  auto lds_sync = [&]() {
    if constexpr (WG) __syncthreads();
    else wave_lds_sync();
  };

  const int tid = WG ? threadIdx.x : (threadIdx.x & 63), wave = WG ? 0 : (threadIdx.x >> 6);
  const int gi = __builtin_amdgcn_readfirstlane(WG ? xcd_remap(blockIdx.x, gridDim.x)
                                                   : xcd_remap(blockIdx.x, gridDim.x) * WAVES + wave);
  // wave-uniform (workgroup-uniform with WG)
  if (gi >= B.start[B.count]) return;
  const int pb = batch_find(B, gi);
  const int grp = gi - B.start[pb];
  const float* __restrict__ u = B.d[pb].in;
  float* __restrict__ v = B.d[pb].out;
  const float* __restrict__ bvec = B.d[pb].aux;
  const float h = B.d[pb].h;
  TileMapLp tm;
  tm.n = B.d[pb].n;
  tm.tx = B.d[pb].a0;
  tm.ntx = B.d[pb].a1;
  tm.blk = B.d[pb].a2;
  tm.ngroups = B.start[pb + 1] - B.start[pb];
  float* s_t1 = s_t1_all + wave * (CS * N3);
  float* s_t2 = s_t2_all + wave * (CS * N3);
  float* s_ty = s_ty_all + wave * (CS * 4 * N2);
  float* s_tz = s_tz_all + wave * (CS * 4 * N2);
  float* s_tzm = s_tzm_all + wave * (CS * 4 * N2);
  const int n = tm.n, nn = n * n, nc = tm.tx;
  TileMapLp t1 = tm;
  t1.tx = 1;
  t1.ntx = n;
  const int c0 = WG ? grp * CPT : tile_first_cell(tm, grp);
  const bool act = WG ? (tid < CPT * N2 && c0 + tid / N2 < nn * n) : (tid < nc * N2);
  const int cl = act ? tid / N2 : 0, ln = tid - cl * N2;
  const int c = WG ? tile_first_cell(t1, c0 + cl) : c0 + cl;
  const int cx = WG ? c % n : c0 % n + cl;
  const int cy = WG ? (c / n) % n : (c0 / n) % n;
  const int cz = WG ? c / nn : c0 / nn;
  const int lp = ln % N, lq = ln / N;

  const float* __restrict__ gM = tab + lay.mass;
  const float* __restrict__ gL = tab + lay.lcell;
  const float* __restrict__ d0 = tab + lay.d0;
  const float* __restrict__ d1 = tab + lay.d1;
  const float gam = tab[lay.gam];
  LineMV<NP, BF, EC> mvM, mvL;
  mvM.load(gM, N, false);
  mvL.load(gL, N, false);

  float own[N], xlo[N], xhi[N], ylo[N], yhi[N], zlo[N], zhi[N];
  const bool hx0 = act && cx > 0, hx1 = act && cx < n - 1;
  const bool hy0 = act && cy > 0, hy1 = act && cy < n - 1;
  const bool hz0 = act && cz > 0, hz1 = act && cz < n - 1;
  {
    const float* pc = u + (size_t)c * N3;
    const float* pxl = pc - N3 + ln * N;
    const float* pxh = pc + N3 + ln * N;
    const float* pyl = pc - (size_t)n * N3 + lp + lq * N2;
    const float* pyh = pc + (size_t)n * N3 + lp + lq * N2;
    const float* pzl = pc - (size_t)nn * N3 + ln;
    const float* pzh = pc + (size_t)nn * N3 + ln;
#pragma unroll
    for (int a = 0; a < N; ++a) {
      own[a] = act ? pc[ln * N + a] : 0.0f;
      xlo[a] = hx0 ? pxl[a] : 0.0f;
      xhi[a] = hx1 ? pxh[a] : 0.0f;
      ylo[a] = hy0 ? pyl[a * N] : 0.0f;
      yhi[a] = hy1 ? pyh[a * N] : 0.0f;
      zlo[a] = hz0 ? pzl[a * N2] : 0.0f;
      zhi[a] = hz1 ? pzh[a * N2] : 0.0f;
    }
  }

  // ---- x stage
  {
    float t1[N], t2[N];
    line_mv<N>(mvL, own, t1);
    line_mv<N>(mvM, own, t2);
    if (act) {
      add_boundary_correction<N>(t1, own, cx == 0, cx == n - 1, d0, d1);
      if (hx0) {
        float g = 0.0f;
#pragma unroll
        for (int a = 0; a < N; ++a) g = fmaf(d1[a], xlo[a], g);
        add_lower_face<N>(t1, xlo[N - 1], g, gam, d0);
      }
      if (hx1) {
        float g = 0.0f;
#pragma unroll
        for (int a = 0; a < N; ++a) g = fmaf(d0[a], xhi[a], g);
        add_upper_face<N>(t1, xhi[0], g, gam, d1);
      }
#pragma unroll
      for (int a = 0; a < N; ++a) {
        s_t1[cl * N3 + ln * N + a] = t1[a];
        s_t2[cl * N3 + ln * N + a] = t2[a];
      }
      float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, g3 = 0.0f;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        g0 = fmaf(d1[a], ylo[a], g0);
        g1 = fmaf(d0[a], yhi[a], g1);
        g2 = fmaf(d1[a], zlo[a], g2);
        g3 = fmaf(d0[a], zhi[a], g3);
      }
      float* ty = s_ty + cl * 4 * N2;
      float* tz = s_tz + cl * 4 * N2;
      ty[0 * N2 + ln] = ylo[N - 1];
      ty[1 * N2 + ln] = g0;
      ty[2 * N2 + ln] = yhi[0];
      ty[3 * N2 + ln] = g1;
      tz[0 * N2 + ln] = zlo[N - 1];
      tz[1 * N2 + ln] = g2;
      tz[2 * N2 + ln] = zhi[0];
      tz[3 * N2 + ln] = g3;
    }
  }
  lds_sync();

  // ---- y stage: lines (i, l) = (lp, lq); Mx on the z traces at (i, j)
  {
    float a1[N], a2[N], cc[N], e[N];
    const int base = cl * N3 + lp + lq * N2;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      a1[b] = act ? s_t1[base + b * N] : 0.0f;
      a2[b] = act ? s_t2[base + b * N] : 0.0f;
    }
    line_mv<N>(mvM, a1, cc);
    line_mv_acc<N>(mvL, a2, cc);
    line_mv<N>(mvM, a2, e);
    if (act) {
      add_boundary_correction<N>(cc, a2, cy == 0, cy == n - 1, d0, d1);
      const float* ty = s_ty + cl * 4 * N2 + lq * N;
      const float* Mrow = gM + lp * N;
      float f0 = 0.0f, q0 = 0.0f, f1 = 0.0f, q1 = 0.0f;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        f0 = fmaf(Mrow[b], ty[0 * N2 + b], f0);
        q0 = fmaf(Mrow[b], ty[1 * N2 + b], q0);
        f1 = fmaf(Mrow[b], ty[2 * N2 + b], f1);
        q1 = fmaf(Mrow[b], ty[3 * N2 + b], q1);
      }
      if (hy0) add_lower_face<N>(cc, f0, q0, gam, d0);
      if (hy1) add_upper_face<N>(cc, f1, q1, gam, d1);
      const float* tz = s_tz + cl * 4 * N2 + lq * N;
      float* tzm = s_tzm + cl * 4 * N2 + lq * N + lp;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float acc = 0.0f;
#pragma unroll
        for (int b = 0; b < N; ++b) acc = fmaf(Mrow[b], tz[r * N2 + b], acc);
        tzm[r * N2] = acc;
      }
#pragma unroll
      for (int b = 0; b < N; ++b) {
        s_t1[base + b * N] = cc[b];
        s_t2[base + b * N] = e[b];
      }
    }
  }
  lds_sync();

  // ---- z stage: lines (i, j) = ln
  {
    float a1[N], a2[N], o[N];
    const int base = cl * N3 + ln;
#pragma unroll
    for (int b = 0; b < N; ++b) {
      a1[b] = act ? s_t1[base + b * N2] : 0.0f;
      a2[b] = act ? s_t2[base + b * N2] : 0.0f;
    }
    line_mv<N>(mvM, a1, o);
    line_mv_acc<N>(mvL, a2, o);
    if (act) {
      add_boundary_correction<N>(o, a2, cz == 0, cz == n - 1, d0, d1);
      const float* tzm = s_tzm + cl * 4 * N2 + lp;
      const float* Mrow = gM + lq * N;
      float f0 = 0.0f, q0 = 0.0f, f1 = 0.0f, q1 = 0.0f;
#pragma unroll
      for (int b = 0; b < N; ++b) {
        f0 = fmaf(Mrow[b], tzm[0 * N2 + b * N], f0);
        q0 = fmaf(Mrow[b], tzm[1 * N2 + b * N], q0);
        f1 = fmaf(Mrow[b], tzm[2 * N2 + b * N], f1);
        q1 = fmaf(Mrow[b], tzm[3 * N2 + b * N], q1);
      }
      if (hz0) add_lower_face<N>(o, f0, q0, gam, d0);
      if (hz1) add_upper_face<N>(o, f1, q1, gam, d1);
      float* dst = v + (size_t)c * N3 + ln;
      if (RES) {
        const float* bs = bvec + (size_t)c * N3 + ln;
#pragma unroll
        for (int a = 0; a < N; ++a) dst[a * N2] = bs[a * N2] - h * o[a];
      } else {
#pragma unroll
        for (int a = 0; a < N; ++a) dst[a * N2] = h * o[a];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Fast-diagonalization patch correction, FP32 storage, the six 2N x 2N
// contractions on the matrix cores.  Lines of one patch are consecutive
// lanes, so every group of 4 lanes shares the patch (and its 1D type).
// ---------------------------------------------------------------------------
template <int N, bool BF, int EC>
__global__ __launch_bounds__(kThreads) void patch_fd_lp_kernel(
    Batch<float> B, const float* __restrict__ tab, TableLayout lay, int bx, int by, int bz) {
  constexpr int G = 2 * N, G2 = G * G, G3 = G2 * G, N2 = N * N, N3 = N2 * N;
  constexpr int PPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  constexpr int GP = Pad<G>::value;
  __shared__ float s_l[4 * G];
  __shared__ float s_X[PPB * G3];
  const int tid = threadIdx.x;
  const int bi = xcd_remap(blockIdx.x, gridDim.x);
  if (bi >= B.start[B.count]) return;
  const int pb = batch_find(B, bi);
  const float* __restrict__ r = B.d[pb].in;
  float* __restrict__ x = B.d[pb].out;
  const int n = B.d[pb].n, npx = B.d[pb].a0, npy = B.d[pb].a1, npatch = B.d[pb].a2;
  const float h = B.d[pb].h;
  const int p0 = (bi - B.start[pb]) * PPB;
  const int np = min(PPB, npatch - p0);
  if (np <= 0) return;
  for (int i = tid; i < 4 * G; i += kThreads) s_l[i] = tab[lay.fd_l + i];
  // A patch of G^2 <= 64 lines that divides 64 lives inside one wave: its
  // waves then synchronise only with themselves after the table load.
  constexpr bool WL = (G2 <= 64) && (64 % G2 == 0);
  const int lane = tid & 63, wv = tid >> 6;
  auto psync = [&]() {
    if constexpr (WL) wave_lds_sync();
    else __syncthreads();
  };
  const int w_lo = WL ? wv * (G2 <= 64 ? 64 / G2 : 1) * G3 : 0;
  const int w_hi = WL ? min(np * G3, w_lo + (G2 <= 64 ? 64 / G2 : 1) * G3) : np * G3;
  const int w_first = WL ? w_lo + lane : tid, w_step = WL ? 64 : kThreads;
  auto vertex = [&](int pl, int& vx, int& vy, int& vz) {
    const int p = p0 + pl;
    const int px = p % npx, py = (p / npx) % npy, pz = p / (npx * npy);
    vx = 2 * px + (bx ? 1 : 2);
    vy = 2 * py + (by ? 1 : 2);
    vz = 2 * pz + (bz ? 1 : 2);
  };
  const int nn = n * n;
  // first cell of each patch of the block, computed once per patch (the
  // gather and scatter loops below then divide only by compile-time sizes)
  __shared__ int s_cb[PPB];
  for (int q = tid; q < np; q += kThreads) {
    int vx, vy, vz;
    vertex(q, vx, vy, vz);
    s_cb[q] = (vx - 1) + n * (vy - 1) + nn * (vz - 1);
  }
  __syncthreads();
  for (int w = w_first; w < w_hi; w += w_step) {
    const int pl = w / G3, rr = w - pl * G3;
    const int cell8 = rr / N3, loc = rr - cell8 * N3;
    const int dx = cell8 & 1, dy = (cell8 >> 1) & 1, dz = cell8 >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int c = s_cb[pl] + dx + n * dy + nn * dz;
    s_X[pl * G3 + (dx * N + i) + G * (dy * N + j) + G2 * (dz * N + l)] = r[(size_t)c * N3 + loc];
  }
  psync();

  const bool act = tid < np * G2;
  const int pl = act ? tid / G2 : 0, ln = tid - pl * G2;
  int vx = 1, vy = 1, vz = 1;
  if (act) vertex(pl, vx, vy, vz);
  const int tx = (vx == 1 ? 1 : 0) | (vx == n - 1 ? 2 : 0);
  const int ty = (vy == 1 ? 1 : 0) | (vy == n - 1 ? 2 : 0);
  const int tz = (vz == 1 ? 1 : 0) | (vz == n - 1 ? 2 : 0);
  float* X = s_X + pl * G3;
  const int la = ln % G, lb = ln / G;
  const int o0 = la * G + lb * G2, o1 = la + lb * G2, o2 = la + lb * G;
  const float* S = tab + lay.fd_s;
  float in[G], out[G];
  {
    LineMV<GP, BF, EC> m;
    m.load(S + tx * G2, G, true);
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = act ? X[o0 + a] : 0.0f;
    line_mv<G>(m, in, out);
    if (act)
#pragma unroll
      for (int a = 0; a < G; ++a) X[o0 + a] = out[a];
  }
  psync();
  {
    LineMV<GP, BF, EC> m;
    m.load(S + ty * G2, G, true);
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = act ? X[o1 + a * G] : 0.0f;
    line_mv<G>(m, in, out);
    if (act)
#pragma unroll
      for (int a = 0; a < G; ++a) X[o1 + a * G] = out[a];
  }
  psync();
  {
    // the transposed and the plain matrix one after the other: a scheduling
    // barrier keeps the second one's fragments from being loaded (and held)
    // while the first is in use
    {
      LineMV<GP, BF, EC> mt;
      mt.load(S + tz * G2, G, true);
#pragma unroll
      for (int a = 0; a < G; ++a) in[a] = act ? X[o2 + a * G2] : 0.0f;
      line_mv<G>(mt, in, out);
    }
    const float lij = act ? s_l[tx * G + la] + s_l[ty * G + lb] : 1.0f;
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = act ? out[a] / (h * (lij + s_l[tz * G + a])) : 0.0f;
    __builtin_amdgcn_sched_barrier(0);
    LineMV<GP, BF, EC> mf;
    mf.load(S + tz * G2, G, false);
    line_mv<G>(mf, in, out);
    if (act)
#pragma unroll
      for (int a = 0; a < G; ++a) X[o2 + a * G2] = out[a];
  }
  psync();
  {
    LineMV<GP, BF, EC> m;
    m.load(S + ty * G2, G, false);
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = act ? X[o1 + a * G] : 0.0f;
    line_mv<G>(m, in, out);
    if (act)
#pragma unroll
      for (int a = 0; a < G; ++a) X[o1 + a * G] = out[a];
  }
  psync();
  {
    LineMV<GP, BF, EC> m;
    m.load(S + tx * G2, G, false);
#pragma unroll
    for (int a = 0; a < G; ++a) in[a] = act ? X[o0 + a] : 0.0f;
    line_mv<G>(m, in, out);
    if (act)
#pragma unroll
      for (int a = 0; a < G; ++a) X[o0 + a] = out[a];
  }
  psync();
  for (int w = w_first; w < w_hi; w += w_step) {
    const int q = w / G3, rr = w - q * G3;
    const int cell8 = rr / N3, loc = rr - cell8 * N3;
    const int dx = cell8 & 1, dy = (cell8 >> 1) & 1, dz = cell8 >> 2;
    const int i = loc % N, j = (loc / N) % N, l = loc / N2;
    const int c = s_cb[q] + dx + n * dy + nn * dz;
    x[(size_t)c * N3 + loc] += s_X[q * G3 + (dx * N + i) + G * (dy * N + j) + G2 * (dz * N + l)];
  }
}

template <int N, bool BF, int EC>
hipError_t apply_lp_impl(const ApplyJob* jobs, int count, const DevTab& t, hipStream_t s) {
  constexpr int CPW = (64 / (N * N)) > 0 ? 64 / (N * N) : 1;
  constexpr bool WG = (N >= 5 && N <= 7);  // workgroup tiles of 10, 7, 5 cells
  constexpr int CPT = kThreads / (N * N);
  if (count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
  Batch<float> B;
  const bool residual = jobs[0].b != nullptr;
  B.count = count;
  B.start[0] = 0;
  for (int i = 0; i < count; ++i) {
    const ApplyJob& j = jobs[i];
    if (j.n < 1 || j.n > 1024 || !j.u || !j.v || (j.b != nullptr) != residual)
      return hipErrorInvalidValue;
    int tx = 1;
    for (int q = 1; q <= CPW && q <= j.n; ++q)
      if (j.n % q == 0) tx = q;
    Desc<float>& d = B.d[i];
    d.in = (const float*)j.u;
    d.out = (float*)j.v;
    d.aux = (const float*)j.b;
    d.h = (float)j.h;
    d.n = j.n;
    d.a0 = tx;
    d.a1 = j.n / tx;
    d.a2 = (j.order > 0 && j.n % j.order == 0) ? j.order : ((j.n % 8 == 0) ? 8 : 1);
    const int64_t cells = (int64_t)j.n * j.n * j.n;
    const int64_t items = WG ? (cells + CPT - 1) / CPT : (int64_t)d.a1 * j.n * j.n;
    if (B.start[i] + items > ((int64_t)1 << 30)) return hipErrorInvalidValue;
    B.start[i + 1] = B.start[i] + (int)items;
  }
  for (int i = count; i < kMaxBatch; ++i) B.start[i + 1] = B.start[count];
  const int per_block = WG ? 1 : kThreads / 64;
  const int grid = (B.start[count] + per_block - 1) / per_block;
  if (grid == 0) return hipSuccess;
  if (residual)
    hipLaunchKernelGGL((apply_lp_kernel<N, BF, EC, true, WG>), dim3(grid), dim3(kThreads), 0, s,
                       B, t.tabf, t.lay);
  else
    hipLaunchKernelGGL((apply_lp_kernel<N, BF, EC, false, WG>), dim3(grid), dim3(kThreads), 0, s,
                       B, t.tabf, t.lay);
  return hipGetLastError();
}

template <int N, bool BF, int EC>
hipError_t patch_lp_impl(int colour, const PatchJob* jobs, int count, const DevTab& t,
                         hipStream_t s) {
  constexpr int G2 = 4 * N * N;
  constexpr int PPB = (kThreads / G2) > 0 ? kThreads / G2 : 1;
  if (count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
  const int bx = colour & 1, by = (colour >> 1) & 1, bz = (colour >> 2) & 1;
  Batch<float> B;
  B.count = count;
  B.start[0] = 0;
  for (int i = 0; i < count; ++i) {
    const PatchJob& j = jobs[i];
    if (j.n < 2 || j.n > 1024 || !j.r || !j.x) return hipErrorInvalidValue;
    auto cnt = [&](int bit) { return bit ? j.n / 2 : (j.n - 1) / 2; };
    Desc<float>& d = B.d[i];
    d.in = (const float*)j.r;
    d.out = (float*)j.x;
    d.aux = nullptr;
    d.h = (float)j.h;
    d.n = j.n;
    d.a0 = cnt(bx);
    d.a1 = cnt(by);
    d.a2 = d.a0 * d.a1 * cnt(bz);
    B.start[i + 1] = B.start[i] + (d.a2 + PPB - 1) / PPB;
  }
  for (int i = count; i < kMaxBatch; ++i) B.start[i + 1] = B.start[count];
  if (B.start[count] == 0) return hipSuccess;
  hipLaunchKernelGGL((patch_fd_lp_kernel<N, BF, EC>), dim3(B.start[count]), dim3(kThreads), 0, s,
                     B, t.tabf, t.lay, bx, by, bz);
  return hipGetLastError();
}

}  // namespace

#define SIPG_LP_EC(NN, BF, EC, CALL)                                      \
  switch (EC) {                                                           \
    case 0: return BF ? CALL(NN, true, 0) : CALL(NN, false, 0);           \
    case 1: return BF ? CALL(NN, true, 1) : CALL(NN, false, 1);           \
    case 2: return BF ? CALL(NN, true, 2) : CALL(NN, false, 2);           \
    default: return hipErrorInvalidValue;                                 \
  }
#define SIPG_LP_DISPATCH(N, BF, EC, CALL) \
  switch (N) {                            \
    case 2: SIPG_LP_EC(2, BF, EC, CALL)   \
    case 3: SIPG_LP_EC(3, BF, EC, CALL)   \
    case 4: SIPG_LP_EC(4, BF, EC, CALL)   \
    case 5: SIPG_LP_EC(5, BF, EC, CALL)   \
    case 6: SIPG_LP_EC(6, BF, EC, CALL)   \
    case 7: SIPG_LP_EC(7, BF, EC, CALL)   \
    case 8: SIPG_LP_EC(8, BF, EC, CALL)   \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_apply_lp_batch(int N, bool bf16, int ec, const ApplyJob* jobs, int count,
                                 const DevTab& t, hipStream_t s) {
  if (t.lay.N != N) return hipErrorInvalidValue;
#define CALL(NN, BB, EE) apply_lp_impl<NN, BB, EE>(jobs, count, t, s)
  SIPG_LP_DISPATCH(N, bf16, ec, CALL)
#undef CALL
}

hipError_t launch_patch_fd_lp_batch(int N, bool bf16, int ec, int colour, const PatchJob* jobs,
                                    int count, const DevTab& t, hipStream_t s) {
  if (t.lay.N != N || colour < 0 || colour > 7) return hipErrorInvalidValue;
#define CALL(NN, BB, EE) patch_lp_impl<NN, BB, EE>(colour, jobs, count, t, s)
  SIPG_LP_DISPATCH(N, bf16, ec, CALL)
#undef CALL
}

hipError_t launch_apply_lp(int N, bool bf16, int ec, const float* u, float* v, const float* b,
                           const DevTab& t, int n, double h, hipStream_t s) {
  ApplyJob j{u, v, b, n, h};
  return launch_apply_lp_batch(N, bf16, ec, &j, 1, t, s);
}

hipError_t launch_patch_fd_lp(int N, bool bf16, int ec, int colour, const float* r, float* x,
                              const DevTab& t, int n, double h, hipStream_t s) {
  PatchJob j{r, x, n, h};
  return launch_patch_fd_lp_batch(N, bf16, ec, colour, &j, 1, t, s);
}

}  // namespace sipg
