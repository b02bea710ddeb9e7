// FP64 SIPG operator apply on the matrix cores for degrees 3 (N = 4) and
// 7 (N = 8).
//
// v_mfma_f64_4x4x4f64 computes four 4x4x4 products at once; its operands put
// the contraction index k at lane bits 4-5 (A[b][i][k] at lane 16k + 4b + i,
// B[b][k][j] at lane 16k + 4b + j) and its result D[b][i][j] at lane
// 16i + 4b + j.  A cell's coefficients of one 4-index block per direction
// fill the 64 lanes with one direction per lane-bit pair, so a 1D matrix Q
// applied along the direction at bits 4-5 is one instruction:
//   normal  (A = Q, B = data): the layout is unchanged;
//   swapped (A = data, B = Q): the new index lands at bits 0-1 and the
//            direction that was at bits 0-1 moves to bits 4-5.
// The swapped form changes layouts for free; the remaining layout changes
// are one ds_bpermute per 32-bit half.
//
// The operator (Sec. 2.1, eq. tensorproduct_3d) with the block-tridiagonal
// 1D matrices written out per cell:
//   v = h [ Mz My Lx~ u + Mz Mx Ly~ u + My Mx Lz~ u ],
//   Ld~ u = Lcc u_c + Lrl u_{c-e_d} + Llr u_{c+e_d}
// where Lcc is the cell block (by boundary type) and Lrl, Llr are the
// rank-2 couplings to the lower and upper face neighbour (Sec. 2.1's face
// evaluators folded into blocks).  Every term is a contraction with a small
// matrix: 9 for the three Ld~ (own cell and two neighbours each) and 5 for
// the mass factors.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "kernels.h"

namespace sipg {

namespace {

// 512 zeros (one degree-7 cell, or the 8 cells of a degree-3 row): the
// loads of a missing face neighbour read here, so the loaded values need
// no per-value select.  The choice of pointer is wave-uniform (scalar).
// Never written.
__device__ __align__(16) double g_zero_cells[512];
__device__ __align__(16) float g_zero_cells_f[512];

template <typename T>
__device__ __forceinline__ const T* zero_cells();
template <>
__device__ __forceinline__ const double* zero_cells<double>() {
  return g_zero_cells;
}
template <>
__device__ __forceinline__ const float* zero_cells<float>() {
  return g_zero_cells_f;
}

constexpr int kT = 256;  // 4 waves per workgroup

__device__ __forceinline__ double mma(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// value of `v` held by lane `src`
__device__ __forceinline__ double gather(double v, int src) {
  const int addr = src << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// A operand of a 4x4 matrix Q (row-major at q): lane 16k + 4b + i holds Q[i][k]
__device__ __forceinline__ double a_operand(const double* __restrict__ q, int lane) {
  return q[(lane & 3) * 4 + (lane >> 4)];
}

// workgroup b of nb -> its position in an order that gives each of the 8 XCDs
// (which receive workgroups round-robin) one contiguous range
__device__ __forceinline__ int xcd_remap4(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// cell index of work item t: x fastest, then (z, y) in blk x blk blocks
__device__ __forceinline__ int cell_of(int t, int n, int blk) {
  const int cx = t % n;
  int r = t / n, cy, cz;
  if (blk > 1) {
    const int zi = r % blk;
    r /= blk;
    const int yi = r % blk;
    r /= blk;
    const int nb = n / blk;
    cz = (r % nb) * blk + zi;
    cy = (r / nb) * blk + yi;
  } else {
    cy = r % n;
    cz = r / n;
  }
  return (cz * n + cy) * n + cx;
}

// One wave owns CPW consecutive cells of an x-row: their dependency chains
// (load, permute, product, permute, ...) are independent and interleave,
// and the x-neighbours inside the row come from registers.
//
// With the data as the A operand (B = the matrix, same lane pattern), a
// product contracts the direction at bits 4-5 and exchanges bit pairs 0-1
// and 4-5 of the layout at no cost.  Writing (a, b, c) for the directions at
// bit pairs 0-1, 2-3, 4-5 (loads and stores use (x, y, z)):
//   t3 = My Mx Lz~ u:  (x,y,z) -Lz~ swapped-> (z,y,x) -Mx-> (z,y,x)
//                       -permute-> (z,x,y) -My swapped-> (y,x,z)
//   s1 = My Lx~ u:      row in (y,z,x) -Lx~ swapped-> (x,z,y) -My swapped-> (y,z,x)
//   s2 = Mx Ly~ u:      (x,z,y) -Ly~ swapped-> (y,z,x) -Mx-> (y,z,x)
//   v  = h [Mz (s1 + s2) + t3]: (y,z,x) -permute-> (y,x,z) -Mz, plus t3->
//        (y,x,z) -permute-> (x,y,z)
// The y neighbours are read directly in (x,z,y).  Per cell: 14 products and
// about five permutations.
// T is the vector type: FP32 vectors (the FP32 V-cycle's residuals) are
// widened on load and the result is rounded to FP32 on store; the products
// are FP64.
template <typename T, bool RES, int CPW>
__global__ __launch_bounds__(kT) void apply_mfma4_kernel(Batch<T> B,
                                                         const double* __restrict__ tab,
                                                         TableLayout lay) {
  const int lane = threadIdx.x & 63;
  const int gi = __builtin_amdgcn_readfirstlane(xcd_remap4(blockIdx.x, gridDim.x) * (kT / 64) +
                                                (threadIdx.x >> 6));
  if (gi >= B.start[B.count]) return;  // wave-uniform; no barriers in this kernel
  const int pb = batch_find(B, gi);
  const T* __restrict__ u = B.d[pb].in;
  T* __restrict__ v = B.d[pb].out;
  const T* __restrict__ bv = B.d[pb].aux;
  const double h = B.d[pb].h;
  const int n = B.d[pb].n, nn = n * n;
  // tile t covers cells c0 .. c0 + CPW - 1 along x
  const int t = gi - B.start[pb];
  const int ntx = n / CPW;
  const int c0 = cell_of(t / ntx * n + (t % ntx) * CPW, n, B.d[pb].a2);
  const int cx0 = c0 % n, cy = (c0 / n) % n, cz = c0 / nn;

  // lane sources of the layout changes (permutations of bit pairs)
  const int p0 = lane & 3, p1 = (lane >> 2) & 3, p2 = lane >> 4;
  const int sToX = p2 | (p0 << 2) | (p1 << 4);  // (x,y,z) -> (y,z,x)
  const int s12 = p0 | (p2 << 2) | (p1 << 4);   // exchange pairs 1 and 2
  const int s01 = p1 | (p0 << 2) | (p2 << 4);   // exchange pairs 0 and 1
  const int oXZY = p0 + 16 * p1 + 4 * p2;       // element held in layout (x,z,y)

  // ---- loads: the row's cells, the two row ends' outer x-neighbours, each
  // cell's z neighbours (x,y,z) and y neighbours (x,z,y).  All loads are
  // unconditional (a missing neighbour row reads the cells of zeros): one
  // basic block the compiler can schedule freely.
  const T* pc = u + (size_t)c0 * 64;
  const T* zc = zero_cells<T>();
  const T* pym = cy > 0 ? pc - (ptrdiff_t)n * 64 : zc;
  const T* pyp = cy < n - 1 ? pc + (ptrdiff_t)n * 64 : zc;
  const T* pzm = cz > 0 ? pc - (ptrdiff_t)nn * 64 : zc;
  const T* pzp = cz < n - 1 ? pc + (ptrdiff_t)nn * 64 : zc;
  double u0[CPW], uym[CPW], uyp[CPW], uzm[CPW], uzp[CPW], b0[CPW];
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    u0[q] = (double)pc[q * 64 + lane];
    uym[q] = (double)pym[q * 64 + oXZY];
    uyp[q] = (double)pyp[q * 64 + oXZY];
    uzm[q] = (double)pzm[q * 64 + lane];
    uzp[q] = (double)pzp[q * 64 + lane];
    b0[q] = RES ? (double)bv[(size_t)(c0 + q) * 64 + lane] : 0.0;
  }
  const double uxm0 = (double)(cx0 > 0 ? pc - 64 : zc)[lane];
  const double uxpE = (double)(cx0 + CPW < n ? pc + CPW * 64 : zc)[lane];

  // ---- matrix operands (uniform tables; the same registers serve as A and B)
  auto var = [&](int q) { return (q == 0 ? 1 : 0) | (q == n - 1 ? 2 : 0); };
  const double aM = a_operand(tab + lay.mass, lane);
  const double aLy = a_operand(tab + lay.lcell + var(cy) * 16, lane);
  const double aLz = a_operand(tab + lay.lcell + var(cz) * 16, lane);
  const double aRL = a_operand(tab + lay.rl, lane);  // coupling to the lower neighbour
  const double aLR = a_operand(tab + lay.lr, lane);  // coupling to the upper neighbour
  const double aLi = a_operand(tab + lay.lcell, lane);             // interior x block
  const double aL0 = a_operand(tab + lay.lcell + var(cx0) * 16, lane);
  const double aL1 = a_operand(tab + lay.lcell + var(cx0 + CPW - 1) * 16, lane);

  double ux[CPW + 2];  // the row in (y,z,x) with its outer neighbours
  ux[0] = gather(uxm0, sToX);
#pragma unroll
  for (int q = 0; q < CPW; ++q) ux[q + 1] = gather(u0[q], sToX);
  ux[CPW + 1] = gather(uxpE, sToX);

#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    // t3 = My Mx Lz~ u
    double w = mma(u0[q], aLz, 0.0);
    w = mma(uzm[q], aRL, w);
    w = mma(uzp[q], aLR, w);                           // (z,y,x)
    const double t3 = mma(gather(mma(aM, w, 0.0), s12), aM, 0.0);  // (y,x,z)
    // s1 = My Lx~ u
    const double aLx = (q == 0) ? aL0 : ((q == CPW - 1) ? aL1 : aLi);
    w = mma(ux[q + 1], aLx, 0.0);
    w = mma(ux[q], aRL, w);
    w = mma(ux[q + 2], aLR, w);                        // (x,z,y)
    double s = mma(w, aM, 0.0);                        // (y,z,x)
    // s2 = Mx Ly~ u
    w = mma(gather(u0[q], s12), aLy, 0.0);
    w = mma(uym[q], aRL, w);
    w = mma(uyp[q], aLR, w);                           // (y,z,x)
    s = mma(aM, w, s);
    // Mz (s1 + s2) + t3, back to (x,y,z)
    const double o = gather(mma(aM, gather(s, s12), t3), s01);
    T* dst = v + (size_t)(c0 + q) * 64 + lane;
    if (RES) *dst = (T)(b0[q] - h * o);
    else *dst = (T)(h * o);
  }
}

// ---------------------------------------------------------------------------
// Degree 7 (N = 8): 512 coefficients per cell, 8 per lane.  Each direction's
// index d = d_lo + 4 d_hi has d_lo in a lane-bit pair and d_hi in a register
// bit; register r holds (x_hi, y_hi, z_hi) = (r & 1, r >> 1 & 1, r >> 2) in
// every layout, and a layout (a, b, c) names the directions at lane bit pairs
// 0-1, 2-3 and 4-5.  An 8x8 matrix along the direction c is four 4x4 blocks:
// output half o of register r collects the blocks (o, 0) and (o, 1) applied
// to the two registers that differ from r in that direction's hi bit.
//
// Two forms of the product:
//   normal:  A = block, B = data (c at bits 4-5); the layout is unchanged.
//   swapped: A = data, B = block transposed; the result holds the new c index
//            at bits 0-1 and the old bits 0-1 direction at bits 4-5, so the
//            layout (a, b, c) becomes (c, b, a) at no cost.
// A block of a row-major matrix has the same lane pattern in both roles
// (lane 16k + 4b + i holds Q[i][k] as A, Q[j][k] as B for j = i).
//
// Global loads are fastest in the natural order (x, y, z): every cell is
// read that way and the other layouts are made in registers (ds_bpermute):
//   t3 = My Mx Lz~ u:  (x,y,z) -Lz~ swapped-> (z,y,x) -Mx-> (z,y,x)
//                       -permute-> (z,x,y) -My swapped-> (y,x,z)
//   s1 = My Lx~ u:      (x,y,z) -permute-> (y,z,x) -Lx~ swapped-> (x,z,y)
//                       -My swapped-> (y,z,x)
//   s2 = Mx Ly~ u:      (x,y,z) -permute-> (x,z,y) -Ly~ swapped-> (y,z,x) -Mx->
//   v  = h [Mz (s1 + s2) + t3]: (y,z,x) -permute-> (y,x,z) -Mz, plus t3->
//        (y,x,z) -permute-> (x,y,z), stored
// 224 products and nine layout changes per cell, one cell per wave.

// lane offset of the coefficient (lo bits only) for a layout whose lane bit
// pairs hold the directions with strides s0, s1, s2 (1, 8 or 64)
__device__ __forceinline__ int lane_off8(int lane, int s0, int s1, int s2) {
  return (lane & 3) * s0 + ((lane >> 2) & 3) * s1 + (lane >> 4) * s2;
}

// register offset of the hi bits: x_hi * 4 + y_hi * 32 + z_hi * 256
__host__ __device__ constexpr int reg_off8(int r) {
  return (r & 1) * 4 + ((r >> 1) & 1) * 32 + (r >> 2) * 256;
}

// block (o, i) of a row-major 8x8 matrix as an MFMA operand
__device__ __forceinline__ double blk8(const double* __restrict__ q, int o, int i, int lane) {
  return q[(4 * o + (lane & 3)) * 8 + 4 * i + (lane >> 4)];
}

// register r with the hi bit of direction bit `db` set to i
__host__ __device__ constexpr int with_hi(int r, int db, int i) {
  return (r & ~(1 << db)) | (i << db);
}

struct Op8 {
  double b[2][2];  // blocks (o, i)
};

__device__ __forceinline__ Op8 load_op8(const double* __restrict__ q, int lane) {
  Op8 m;
  m.b[0][0] = blk8(q, 0, 0, lane);
  m.b[0][1] = blk8(q, 0, 1, lane);
  m.b[1][0] = blk8(q, 1, 0, lane);
  m.b[1][1] = blk8(q, 1, 1, lane);
  return m;
}

// y[r] (+)= Q along direction bit DB, normal form (matrix is A)
template <int DB>
__device__ __forceinline__ void mul_normal(const Op8& Q, const double* x, double* y, bool acc) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int o = (r >> DB) & 1;
    double c = acc ? y[r] : 0.0;
    c = mma(Q.b[o][0], x[with_hi(r, DB, 0)], c);
    c = mma(Q.b[o][1], x[with_hi(r, DB, 1)], c);
    y[r] = c;
  }
}

// y[r] (+)= Q along direction bit DB, swapped form (data is A)
template <int DB>
__device__ __forceinline__ void mul_swapped(const Op8& Q, const double* x, double* y, bool acc) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int o = (r >> DB) & 1;
    double c = acc ? y[r] : 0.0;
    c = mma(x[with_hi(r, DB, 0)], Q.b[o][0], c);
    c = mma(x[with_hi(r, DB, 1)], Q.b[o][1], c);
    y[r] = c;
  }
}

// the 8 registers of a cell at q (layout offset included)
__device__ __forceinline__ void load8(const double* __restrict__ q, double* a) {
#pragma unroll
  for (int r = 0; r < 8; ++r) a[r] = q[reg_off8(r)];
}


__device__ __forceinline__ void permute8(const double* a, double* b, int src) {
#pragma unroll
  for (int r = 0; r < 8; ++r) b[r] = gather(a[r], src);
}

template <bool RES>
__global__ __launch_bounds__(kT) void apply_mfma8_kernel(Batch<double> B,
                                                       const double* __restrict__ tab,
                                                       TableLayout lay) {
  const int lane = threadIdx.x & 63;
  const int gi = __builtin_amdgcn_readfirstlane(blockIdx.x * (kT / 64) + (threadIdx.x >> 6));
  if (gi >= B.start[B.count]) return;  // wave-uniform; no barriers in this kernel
  const int pb = batch_find(B, gi);
  const double* __restrict__ u = B.d[pb].in;
  double* __restrict__ v = B.d[pb].out;
  const double* __restrict__ bv = B.d[pb].aux;
  const double h = B.d[pb].h;
  const int n = B.d[pb].n, nn = n * n;
  const int c = cell_of(gi - B.start[pb], n, B.d[pb].a2);
  const int cx = c % n, cy = (c / n) % n, cz = c / nn;
  auto var = [&](int q) { return (q == 0 ? 1 : 0) | (q == n - 1 ? 2 : 0); };

  const int oXYZ = lane_off8(lane, 1, 8, 64);
  // sources of the layout changes: (x,y,z) -> (y,z,x); exchange of pairs 1
  // and 2 (an involution); exchange of pairs 0 and 1
  const int p0 = lane & 3, p1 = (lane >> 2) & 3, p2 = lane >> 4;
  const int sToX = p2 | (p0 << 2) | (p1 << 4);
  const int s12 = p0 | (p2 << 2) | (p1 << 4);
  const int s01 = p1 | (p0 << 2) | (p2 << 4);
  const double* pc = u + (size_t)c * 512;
  const ptrdiff_t sx = 512, sy = (ptrdiff_t)n * 512, sz = (ptrdiff_t)nn * 512;

  const Op8 M = load_op8(tab + lay.mass, lane);
  const Op8 RL = load_op8(tab + lay.rl, lane);  // coupling to the lower neighbour
  const Op8 LR = load_op8(tab + lay.lr, lane);  // coupling to the upper neighbour

  // All loads are unconditional (a missing neighbour reads the cell itself
  // and is zeroed after the load), so they form one basic block that the
  // compiler may schedule ahead of the products.
  double u0[8], zm[8], zp[8], xm[8], xp[8], ym[8], yp[8];
  const double* zc = g_zero_cells;
  load8(pc + oXYZ, u0);
  load8((cz > 0 ? pc - sz : zc) + oXYZ, zm);
  load8((cz < n - 1 ? pc + sz : zc) + oXYZ, zp);
  load8((cx > 0 ? pc - sx : zc) + oXYZ, xm);
  load8((cx < n - 1 ? pc + sx : zc) + oXYZ, xp);
  load8((cy > 0 ? pc - sy : zc) + oXYZ, ym);
  load8((cy < n - 1 ? pc + sy : zc) + oXYZ, yp);

  double t3[8], w[8], s[8], a[8];
  {  // t3 = My Mx Lz~ u
    const Op8 Lz = load_op8(tab + lay.lcell + var(cz) * 64, lane);
    mul_swapped<2>(Lz, u0, w, false);
    mul_swapped<2>(RL, zm, w, true);
    mul_swapped<2>(LR, zp, w, true);  // (z, y, x)
    mul_normal<0>(M, w, a, false);    // Mx
    permute8(a, w, s12);              // (z, x, y)
    mul_swapped<1>(M, w, t3, false);  // My -> (y, x, z)
  }
  {  // s1 = My Lx~ u
    const Op8 Lx = load_op8(tab + lay.lcell + var(cx) * 64, lane);
    permute8(u0, a, sToX);            // (y, z, x)
    mul_swapped<0>(Lx, a, w, false);
    permute8(xm, a, sToX);
    mul_swapped<0>(RL, a, w, true);
    permute8(xp, a, sToX);
    mul_swapped<0>(LR, a, w, true);   // (x, z, y)
    mul_swapped<1>(M, w, s, false);   // My -> (y, z, x)
  }
  {  // s2 = Mx Ly~ u, added to s1
    const Op8 Ly = load_op8(tab + lay.lcell + var(cy) * 64, lane);
    permute8(u0, a, s12);             // (x, z, y)
    mul_swapped<1>(Ly, a, w, false);
    permute8(ym, a, s12);
    mul_swapped<1>(RL, a, w, true);
    permute8(yp, a, s12);
    mul_swapped<1>(LR, a, w, true);   // (y, z, x)
    mul_normal<0>(M, w, s, true);     // Mx
  }
  permute8(s, w, s12);                // (y, x, z)
  mul_normal<2>(M, w, t3, true);      // Mz, (y, x, z)
  double* dst = v + (size_t)c * 512 + oXYZ;
  const double* bsrc = RES ? bv + (size_t)c * 512 + oXYZ : nullptr;
  // the residual's b is read here, not with the other loads: holding it
  // through the products would cost a wave per SIMD
  if (RES) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const double o = h * gather(t3[r], s01);  // (x, y, z)
    if (RES) dst[reg_off8(r)] = bsrc[reg_off8(r)] - o;
    else dst[reg_off8(r)] = o;
  }
}

// ---------------------------------------------------------------------------
// Degree 7 with the mirror-pair (even-odd) split.  The GLL nodes are
// symmetric about the cell centre, so the reversal J of a direction maps the
// mass matrix and the interior cell block onto themselves and the coupling
// to the upper neighbour onto the one to the lower neighbour.  The register
// bit of a direction now selects a mirror half: node idx(h, lo) = h ? 7 - lo
// : lo (lo in the lane-bit pair), so J is an exchange of the two registers
// and the split E = v_0 + v_1, O = v_0 - v_1 is two vector additions per
// register pair.  In the split form a J-symmetric matrix acts on E and O with
// one 4 x 4 block each (one product per register instead of two); the two
// face couplings of a direction act through S = v_m + J v_p (its E part) and
// D = v_m - J v_p (its O part) with two blocks each, for both neighbours at
// once.  Per cell: 112 products (224 with the plain 8 x 8 blocks), about 140
// FP64 additions for the splits, the same nine layout changes; boundary
// cells add the boundary correction in the coupling form.  The chain is the
// one of apply_mfma8_kernel (layouts in the same order); every term reaches
// the split form in all three directions once, and three more splits at the
// end give 8 times the result (scaled by h / 8).

// (v_0, v_1) -> (v_0 + v_1, v_0 - v_1) along direction bit DB; applied to a
// split pair it gives twice the halves back
template <int DB>
__device__ __forceinline__ void split8(double* x) {
#pragma unroll
  for (int r = 0; r < 8; ++r)
    if (!((r >> DB) & 1)) {
      const int r1 = r | (1 << DB);
      const double a = x[r], b = x[r1];
      x[r] = a + b;
      x[r1] = a - b;
    }
}

// y[r] (+)= Q_p x[r] along direction bit DB for x split along DB (p = the
// register's bit: E block qe, O block qo); normal form or swapped (SW)
template <int DB, bool SW>
__device__ __forceinline__ void mul_sym(double qe, double qo, const double* x, double* y,
                                        bool acc) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const double q = ((r >> DB) & 1) ? qo : qe;
    const double c = acc ? y[r] : 0.0;
    y[r] = SW ? mma(x[r], q, c) : mma(q, x[r], c);
  }
}

// y[r] += c0 x[r, half 0] + c1 x[r, half 1] along DB for the registers of
// split part PAR (x in halves along DB)
template <int DB, bool SW, int PAR>
__device__ __forceinline__ void mul_cpl(double c0, double c1, const double* x, double* y) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (((r >> DB) & 1) != PAR) continue;
    double c = y[r];
    c = SW ? mma(x[with_hi(r, DB, 0)], c0, c) : mma(c0, x[with_hi(r, DB, 0)], c);
    c = SW ? mma(x[with_hi(r, DB, 1)], c1, c) : mma(c1, x[with_hi(r, DB, 1)], c);
    y[r] = c;
  }
}

// m <- m + J p, p <- m - J p along direction bit DB
template <int DB>
__device__ __forceinline__ void sum_diff8(double* m, double* p) {
  double sd[8], df[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    sd[r] = m[r] + p[r ^ (1 << DB)];
    df[r] = m[r] - p[r ^ (1 << DB)];
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    m[r] = sd[r];
    p[r] = df[r];
  }
}

// w += the boundary correction along direction bit DB in the coupling form
// (blocks 8-11 of the even-odd table), from the cell u0 itself (natural
// along DB, layout (x,y,z)); PERM: bring it to the layout of w first
template <int DB, bool PERM>
__device__ __forceinline__ void boundary8(const double* __restrict__ eo, int lane,
                                          const double* u0, bool lo_end, bool hi_end, int src,
                                          double* w) {
  const double Q0 = a_operand(eo + 128, lane), Q1 = a_operand(eo + 144, lane);
  const double Q2 = a_operand(eo + 160, lane), Q3 = a_operand(eo + 176, lane);
  double m[8], p[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    m[r] = lo_end ? u0[r] : 0.0;
    p[r] = hi_end ? u0[r] : 0.0;
  }
  sum_diff8<DB>(m, p);
  if (PERM) {
    double a[8];
    permute8(m, a, src);
    mul_cpl<DB, true, 0>(Q0, Q1, a, w);
    permute8(p, a, src);
    mul_cpl<DB, true, 1>(Q2, Q3, a, w);
  } else {
    mul_cpl<DB, true, 0>(Q0, Q1, m, w);
    mul_cpl<DB, true, 1>(Q2, Q3, p, w);
  }
}

// Three waves per SIMD: the kernel fits the 168-register budget without
// spills (left alone the compiler took 176-190 registers, two waves).
template <bool RES>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(3, 3)))
void apply_mfma8eo_kernel(Batch<double> B, const double* __restrict__ tab, TableLayout lay) {
  const int lane = threadIdx.x & 63;
  const int gi = __builtin_amdgcn_readfirstlane(blockIdx.x * (kT / 64) + (threadIdx.x >> 6));
  if (gi >= B.start[B.count]) return;  // wave-uniform; no barriers in this kernel
  const int pb = batch_find(B, gi);
  const double* __restrict__ u = B.d[pb].in;
  double* __restrict__ v = B.d[pb].out;
  const double* __restrict__ bv = B.d[pb].aux;
  const double h = B.d[pb].h;
  const int n = B.d[pb].n, nn = n * n;
  const int c = cell_of(gi - B.start[pb], n, B.d[pb].a2);
  const int cx = c % n, cy = (c / n) % n, cz = c / nn;

  // mirror-pair offsets of the layout (x, y, z): register r = (x_h, y_h, z_h)
  const int p0 = lane & 3, p1 = (lane >> 2) & 3, p2 = lane >> 4;
  int off[8];
#pragma unroll
  for (int r = 0; r < 8; ++r)
    off[r] = ((r & 1) ? 7 - p0 : p0) + 8 * (((r >> 1) & 1) ? 7 - p1 : p1) +
             64 * ((r >> 2) ? 7 - p2 : p2);
  const int sToX = p2 | (p0 << 2) | (p1 << 4);  // (x,y,z) -> (y,z,x)
  const int s12 = p0 | (p2 << 2) | (p1 << 4);   // exchange pairs 1 and 2
  const int s01 = p1 | (p0 << 2) | (p2 << 4);   // exchange pairs 0 and 1
  const double* pc = u + (size_t)c * 512;
  const ptrdiff_t sx = 512, sy = (ptrdiff_t)n * 512, sz = (ptrdiff_t)nn * 512;

  const double* eo = tab + lay.eo;
  const double Me = a_operand(eo + 0, lane), Mo = a_operand(eo + 16, lane);
  const double Le = a_operand(eo + 32, lane), Lo = a_operand(eo + 48, lane);
  const double R0 = a_operand(eo + 64, lane), R1 = a_operand(eo + 80, lane);
  const double R2 = a_operand(eo + 96, lane), R3 = a_operand(eo + 112, lane);

  // unconditional loads (a missing neighbour reads the cell of zeros)
  double u0[8], zm[8], zp[8], xm[8], xp[8], ym[8], yp[8];
  auto load = [&](const double* q, double* a) {
#pragma unroll
    for (int r = 0; r < 8; ++r) a[r] = q[off[r]];
  };
  const double* zc = g_zero_cells;
  load(pc, u0);
  load(cz > 0 ? pc - sz : zc, zm);
  load(cz < n - 1 ? pc + sz : zc, zp);
  load(cx > 0 ? pc - sx : zc, xm);
  load(cx < n - 1 ? pc + sx : zc, xp);

  double t3[8], w[8], s[8], a[8], b[8];
  {  // t3 = My Mx Lz~ u
#pragma unroll
    for (int r = 0; r < 8; ++r) b[r] = u0[r];
    split8<2>(b);
    mul_sym<2, true>(Le, Lo, b, w, false);  // (x,y,z) -> (z,y,x)
    sum_diff8<2>(zm, zp);
    mul_cpl<2, true, 0>(R0, R1, zm, w);
    mul_cpl<2, true, 1>(R2, R3, zp, w);
    if (cz == 0 || cz == n - 1) boundary8<2, false>(eo, lane, u0, cz == 0, cz == n - 1, 0, w);
    split8<0>(w);
    mul_sym<0, false>(Me, Mo, w, a, false);  // Mx
    permute8(a, w, s12);                     // (z,x,y)
    split8<1>(w);
    mul_sym<1, true>(Me, Mo, w, t3, false);  // My -> (y,x,z)
  }
  // the y neighbours are read after the z term: holding them through it
  // would not fit three waves per SIMD
  __builtin_amdgcn_sched_barrier(0);
  load(cy > 0 ? pc - sy : zc, ym);
  load(cy < n - 1 ? pc + sy : zc, yp);
  {  // s1 = My Lx~ u
#pragma unroll
    for (int r = 0; r < 8; ++r) b[r] = u0[r];
    split8<0>(b);
    permute8(b, a, sToX);                   // (y,z,x)
    mul_sym<0, true>(Le, Lo, a, w, false);  // -> (x,z,y)
    sum_diff8<0>(xm, xp);
    permute8(xm, a, sToX);
    mul_cpl<0, true, 0>(R0, R1, a, w);
    permute8(xp, a, sToX);
    mul_cpl<0, true, 1>(R2, R3, a, w);
    if (cx == 0 || cx == n - 1) boundary8<0, true>(eo, lane, u0, cx == 0, cx == n - 1, sToX, w);
    split8<1>(w);
    mul_sym<1, true>(Me, Mo, w, s, false);  // My -> (y,z,x)
  }
  {  // s2 = Mx Ly~ u, added to s1
#pragma unroll
    for (int r = 0; r < 8; ++r) b[r] = u0[r];
    split8<1>(b);
    permute8(b, a, s12);                    // (x,z,y)
    mul_sym<1, true>(Le, Lo, a, w, false);  // -> (y,z,x)
    sum_diff8<1>(ym, yp);
    permute8(ym, a, s12);
    mul_cpl<1, true, 0>(R0, R1, a, w);
    permute8(yp, a, s12);
    mul_cpl<1, true, 1>(R2, R3, a, w);
    if (cy == 0 || cy == n - 1) boundary8<1, true>(eo, lane, u0, cy == 0, cy == n - 1, s12, w);
    split8<0>(w);
    mul_sym<0, false>(Me, Mo, w, s, true);  // Mx, (y,z,x)
  }
  permute8(s, w, s12);                      // (y,x,z)
  split8<2>(w);
  mul_sym<2, false>(Me, Mo, w, t3, true);   // Mz, (y,x,z), split in all directions
  split8<0>(t3);
  split8<1>(t3);
  split8<2>(t3);                            // 8 x the halves
  const double hs = 0.125 * h;
  double* dst = v + (size_t)c * 512;
  const double* bsrc = RES ? bv + (size_t)c * 512 : nullptr;
  if (RES) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const double o = hs * gather(t3[r], s01);  // (x, y, z)
    if (RES) dst[off[r]] = bsrc[off[r]] - o;
    else dst[off[r]] = o;
  }
}

// ---------------------------------------------------------------------------
// Fast-diagonalization solve on the vertex patches of one colour for degree
// 3 (Sec. 7's smoother; exact inverse of the patch matrix):
//   x_P += (1/h) (Sz Sy Sx) diag(1 / (lx_i + ly_j + lz_l)) (Sz Sy Sx)^T r_P
// A patch is 2x2x2 cells, 8 nodes per direction: the degree-7 layout applies
// with the register index = the patch cell (dx, dy, dz) and the lane = the
// node inside the cell, so every register is one coalesced 512-byte line of
// a cell.  One patch per wave; 96 products and three layout changes:
//   (x,y,z) -Sz^T swapped-> (z,y,x) -Sx^T-> -permute-> (z,x,y) -Sy^T->
//   scale -Sy swapped-> (y,x,z) -Sz-> -permute-> (y,z,x) -Sx swapped->
//   (x,z,y) -permute-> (x,y,z)
// Patches of one colour share no cell, so the scatter-add needs no atomics.
// T is the vector type: FP32 vectors (the FP32 V-cycle) are widened on load
// and the update is rounded to FP32 on store; the products are FP64.

// blocks of the transpose of a row-major 8x8 matrix
__device__ __forceinline__ Op8 load_op8t(const double* __restrict__ q, int lane) {
  Op8 m;
#pragma unroll
  for (int o = 0; o < 2; ++o)
#pragma unroll
    for (int i = 0; i < 2; ++i) m.b[o][i] = q[(4 * i + (lane >> 4)) * 8 + 4 * o + (lane & 3)];
  return m;
}

template <typename T>
__global__ __launch_bounds__(kT) void patch_mfma4_kernel(Batch<T> B, const double* __restrict__ tab,
                                                         TableLayout lay, int bx, int by, int bz) {
  const int lane = threadIdx.x & 63;
  const int gi = __builtin_amdgcn_readfirstlane(blockIdx.x * (kT / 64) + (threadIdx.x >> 6));
  if (gi >= B.start[B.count]) return;  // wave-uniform; no barriers in this kernel
  const int pb = batch_find(B, gi);
  const T* __restrict__ r = B.d[pb].in;
  T* __restrict__ x = B.d[pb].out;
  const int n = B.d[pb].n, npx = B.d[pb].a0, npy = B.d[pb].a1, nn = n * n;
  const double h = B.d[pb].h;
  const int p = gi - B.start[pb];
  // the patch's vertex (interior vertices 1 .. n-1 of the colour's parity)
  const int vx = 2 * (p % npx) + (bx ? 1 : 2);
  const int vy = 2 * ((p / npx) % npy) + (by ? 1 : 2);
  const int vz = 2 * (p / (npx * npy)) + (bz ? 1 : 2);
  auto type = [&](int v) { return (v == 1 ? 1 : 0) | (v == n - 1 ? 2 : 0); };
  const int tx = type(vx), ty = type(vy), tz = type(vz);
  const T* pc = r + (size_t)((vx - 1) + n * (vy - 1) + nn * (vz - 1)) * 64 + lane;
  T* px = x + (size_t)((vx - 1) + n * (vy - 1) + nn * (vz - 1)) * 64 + lane;
  auto cell_off = [&](int q) { return (ptrdiff_t)((q & 1) + n * ((q >> 1) & 1) + nn * (q >> 2)) * 64; };

  double X[8], W[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) X[q] = (double)pc[cell_off(q)];
  const int p0 = lane & 3, p1 = (lane >> 2) & 3, p2 = lane >> 4;
  const int s12 = p0 | (p2 << 2) | (p1 << 4);  // exchange pairs 1 and 2
  const double* S = tab + lay.fd_s;
  const double* lam = tab + lay.fd_l;

  {  // forward: S^T along z, x, y
    const Op8 Tz = load_op8t(S + tz * 64, lane);
    const Op8 Tx = load_op8t(S + tx * 64, lane);
    const Op8 Ty = load_op8t(S + ty * 64, lane);
    mul_swapped<2>(Tz, X, W, false);  // (z, y, x)
    mul_normal<0>(Tx, W, X, false);
    permute8(X, W, s12);              // (z, x, y)
    mul_normal<1>(Ty, W, X, false);
  }
  // eigenvalue scaling; in (z, x, y) lane bit pairs hold z, x, y
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double l = lam[tx * 8 + p1 + 4 * (q & 1)] + lam[ty * 8 + p2 + 4 * ((q >> 1) & 1)] +
                     lam[tz * 8 + p0 + 4 * (q >> 2)];
    X[q] = X[q] / (h * l);
  }
  {  // backward: S along y, z, x
    const Op8 Sy = load_op8(S + ty * 64, lane);
    const Op8 Sz = load_op8(S + tz * 64, lane);
    const Op8 Sx = load_op8(S + tx * 64, lane);
    mul_swapped<1>(Sy, X, W, false);  // (y, x, z)
    mul_normal<2>(Sz, W, X, false);
    permute8(X, W, s12);              // (y, z, x)
    mul_swapped<0>(Sx, W, X, false);  // (x, z, y)
    permute8(X, W, s12);              // (x, y, z)
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) px[cell_off(q)] = (T)((double)px[cell_off(q)] + W[q]);
}

}  // namespace

namespace {

template <typename T>
hipError_t apply_mfma4(const ApplyJob* jobs, int count, const DevTab& t, hipStream_t s) {
  if (t.lay.N != 4 || count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
  Batch<T> B;
  const bool residual = jobs[0].b != nullptr;
  // cells per wave: 8 when every mesh of the launch allows it, else 4, 2 or 1
  int cpw = 8;
  for (int i = 0; i < count; ++i)
    while (cpw > 1 && jobs[i].n % cpw) cpw >>= 1;
  B.count = count;
  B.start[0] = 0;
  for (int i = 0; i < count; ++i) {
    const ApplyJob& j = jobs[i];
    if (j.n < 1 || j.n > 1024 || !j.u || !j.v || (j.b != nullptr) != residual)
      return hipErrorInvalidValue;
    Desc<T>& d = B.d[i];
    d.in = (const T*)j.u;
    d.out = (T*)j.v;
    d.aux = (const T*)j.b;
    d.h = (T)j.h;
    d.n = j.n;
    d.a0 = cpw;
    d.a1 = j.n / cpw;
    d.a2 = (j.order > 0 && j.n % j.order == 0) ? j.order : ((j.n % 8 == 0) ? 8 : 1);
    const int64_t items = (int64_t)j.n * j.n * (j.n / cpw);
    if (B.start[i] + items > 0x7fffffff) return hipErrorInvalidValue;
    B.start[i + 1] = B.start[i] + (int)items;
  }
  const int grid = (B.start[count] + kT / 64 - 1) / (kT / 64);
  if (grid == 0) return hipSuccess;
#define LAUNCH(RR, CC) \
  hipLaunchKernelGGL((apply_mfma4_kernel<T, RR, CC>), dim3(grid), dim3(kT), 0, s, B, t.tab, t.lay)
  if (cpw == 8) {
    if (residual) LAUNCH(true, 8); else LAUNCH(false, 8);
  } else if (cpw == 4) {
    if (residual) LAUNCH(true, 4); else LAUNCH(false, 4);
  } else if (cpw == 2) {
    if (residual) LAUNCH(true, 2); else LAUNCH(false, 2);
  } else {
    if (residual) LAUNCH(true, 1); else LAUNCH(false, 1);
  }
#undef LAUNCH
  return hipGetLastError();
}

}  // namespace

hipError_t launch_apply_mfma4_batch(int prec, const ApplyJob* jobs, int count, const DevTab& t,
                                    hipStream_t s) {
  return prec == 0 ? apply_mfma4<double>(jobs, count, t, s)
                   : apply_mfma4<float>(jobs, count, t, s);
}

}  // namespace sipg

namespace sipg {

hipError_t launch_apply_mfma8_batch(const ApplyJob* jobs, int count, const DevTab& t,
                                    hipStream_t s) {
  if (t.lay.N != 8 || count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
  Batch<double> B;
  const bool residual = jobs[0].b != nullptr;
  B.count = count;
  B.start[0] = 0;
  for (int i = 0; i < count; ++i) {
    const ApplyJob& j = jobs[i];
    if (j.n < 1 || j.n > 1024 || !j.u || !j.v || (j.b != nullptr) != residual)
      return hipErrorInvalidValue;
    Desc<double>& d = B.d[i];
    d.in = (const double*)j.u;
    d.out = (double*)j.v;
    d.aux = (const double*)j.b;
    d.h = j.h;
    d.n = j.n;
    d.a0 = 1;
    d.a1 = j.n;
    d.a2 = (j.order > 0 && j.n % j.order == 0) ? j.order : 1;
    const int64_t items = (int64_t)j.n * j.n * j.n;
    if (B.start[i] + items > 0x7fffffff) return hipErrorInvalidValue;
    B.start[i + 1] = B.start[i] + (int)items;
  }
  const int grid = (B.start[count] + kT / 64 - 1) / (kT / 64);
  if (grid == 0) return hipSuccess;
  if (t.lay.eo_ok) {  // the symmetries of the even-odd split hold (always, up to rounding)
    if (residual)
      hipLaunchKernelGGL((apply_mfma8eo_kernel<true>), dim3(grid), dim3(kT), 0, s, B, t.tab, t.lay);
    else
      hipLaunchKernelGGL((apply_mfma8eo_kernel<false>), dim3(grid), dim3(kT), 0, s, B, t.tab,
                         t.lay);
  } else if (residual) {
    hipLaunchKernelGGL((apply_mfma8_kernel<true>), dim3(grid), dim3(kT), 0, s, B, t.tab, t.lay);
  } else {
    hipLaunchKernelGGL((apply_mfma8_kernel<false>), dim3(grid), dim3(kT), 0, s, B, t.tab, t.lay);
  }
  return hipGetLastError();
}

}  // namespace sipg

namespace sipg {

namespace {

template <typename T>
hipError_t patch_mfma4(int colour, const PatchJob* jobs, int count, const DevTab& t,
                       hipStream_t s) {
  if (t.lay.N != 4 || count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
  const int bx = colour & 1, by = (colour >> 1) & 1, bz = (colour >> 2) & 1;
  Batch<T> B;
  B.count = count;
  B.start[0] = 0;
  for (int i = 0; i < count; ++i) {
    const PatchJob& j = jobs[i];
    if (j.n < 2 || j.n > 1024 || !j.r || !j.x) return hipErrorInvalidValue;
    // vertices in [1, n-1]: odd ones 1, 3, ..; even ones 2, 4, ..
    auto cnt = [&](int bit) { return bit ? j.n / 2 : (j.n - 1) / 2; };
    Desc<T>& d = B.d[i];
    d.in = (const T*)j.r;
    d.out = (T*)j.x;
    d.aux = nullptr;
    d.h = (T)j.h;
    d.n = j.n;
    d.a0 = cnt(bx);
    d.a1 = cnt(by);
    d.a2 = d.a0 * d.a1 * cnt(bz);
    if (B.start[i] + (int64_t)d.a2 > 0x7fffffff) return hipErrorInvalidValue;
    B.start[i + 1] = B.start[i] + d.a2;
  }
  const int grid = (B.start[count] + kT / 64 - 1) / (kT / 64);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(patch_mfma4_kernel<T>, dim3(grid), dim3(kT), 0, s, B, t.tab, t.lay, bx, by,
                     bz);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_patch_mfma4_batch(int prec, int colour, const PatchJob* jobs, int count,
                                    const DevTab& t, hipStream_t s) {
  return prec == 0 ? patch_mfma4<double>(colour, jobs, count, t, s)
                   : patch_mfma4<float>(colour, jobs, count, t, s);
}

}  // namespace sipg
