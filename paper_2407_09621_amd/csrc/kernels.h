// Launchers of the gfx950 kernels (host side).  Every launcher checks the
// shapes its grid assumes and returns hipErrorInvalidValue on a mismatch.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "batch.h"
#include "geometry.h"
#include "tables.h"

namespace sipg {

struct DevTab {
  const double* tab = nullptr;  // device copy of build_device_table()
  const float* tabf = nullptr;  // the same table rounded to FP32
  TableLayout lay;
};

// v = h * A_hat u (or r = b - h * A_hat u when b != nullptr); n cells per
// direction, cell-blocked vectors of n^3 N^3 doubles.
hipError_t launch_apply_f64(int N, const double* u, double* v, const double* b,
                            const DevTab& t, int n, double h, hipStream_t s);

hipError_t launch_apply_f32(int N, const float* u, float* v, const float* b, const DevTab& t,
                            int n, double h, hipStream_t s);
// The FP32 V-cycle's residual: FP32 vectors; at N = 4 on the FP64 matrix
// cores (widened on load, rounded on store), else as launch_apply_f32.
hipError_t launch_residual_f32(int N, const float* u, float* v, const float* b, const DevTab& t,
                               int n, double h, hipStream_t s);

// x_P += A_PP^{-1} r_P for all vertex patches of `colour`.
hipError_t launch_patch_fd_f64(int N, int colour, const double* r, double* x,
                               const DevTab& t, int n, double h, hipStream_t s);

hipError_t launch_patch_fd_f32(int N, int colour, const float* r, float* x, const DevTab& t,
                               int n, double h, hipStream_t s);

// out = in on the cells that no vertex patch of `colour` covers (the layers
// next to the domain boundary that the colour's vertices leave out); with
// the fused colour step (PatchJob.b set) this completes the new vector.
// prec 0 = FP64, 1 = FP32.
hipError_t launch_copy_uncovered(int prec, int N, int colour, const void* in, void* out, int n,
                                 hipStream_t s);

// Patch-wise evaluation: v_P += (patch operator) u_P for the vertex patches
// of `colour` (FP64, vector units); summed over the 8 colours v = A u.
hipError_t launch_patch_apply_f64(int N, int colour, const double* u, double* v, const DevTab& t,
                                  int n, double h, hipStream_t s);

// x = A_0^{-1} b on the n0^3-cell coarse level (overwrites x).
hipError_t launch_coarse_fd_f64(int N, int n0, const double* b, double* x,
                                const DevTab& t, double h, hipStream_t s);

hipError_t launch_coarse_fd_f32(int N, int n0, const float* b, float* x, const DevTab& t,
                                double h, hipStream_t s);

// rc = P^T rf (nc coarse cells per direction) and xf += P ec.
hipError_t launch_restrict_f64(int N, const double* rf, double* rc, const DevTab& t,
                               int nc, hipStream_t s);
hipError_t launch_prolongate_add_f64(int N, const double* ec, double* xf,
                                     const DevTab& t, int nc, hipStream_t s);
hipError_t launch_restrict_f32(int N, const float* rf, float* rc, const DevTab& t, int nc,
                               hipStream_t s);
hipError_t launch_prolongate_add_f32(int N, const float* ec, float* xf, const DevTab& t, int nc,
                                     hipStream_t s);

// Apply of degree 3 on the FP64 matrix cores (one wave per up to 8 cells of
// an x-row); same contract as launch_apply_batch with N = 4 (prec 0: FP64
// vectors, 1: FP32 vectors, widened on load, FP64 products).
hipError_t launch_apply_mfma4_batch(int prec, const ApplyJob* jobs, int count, const DevTab& t,
                                    hipStream_t s);
// FP64 apply of degree 7 on the matrix cores (one cell per wave); same
// contract as launch_apply_batch with prec 0 and N = 8.
hipError_t launch_apply_mfma8_batch(const ApplyJob* jobs, int count, const DevTab& t,
                                    hipStream_t s);
// Patch solve of degree 3 on the matrix cores (one patch per wave, FP64
// products); same contract as launch_patch_fd_batch with N = 4 (prec 0: FP64
// vectors, 1: FP32 vectors).
hipError_t launch_patch_mfma4_batch(int prec, int colour, const PatchJob* jobs, int count,
                                    const DevTab& t, hipStream_t s);

// Batched forms: up to kMaxBatch problems of one degree per launch.
// prec 0 = FP64 vectors (the apply on the matrix cores for N = 4 and 8),
// 1 = FP32 vectors (VALU arithmetic), 2 (apply only) = FP64 vectors on the
// vector units for every N, 3 (apply only) = FP32 vectors with FP64
// matrix-core products at N = 4 (else as 1).
hipError_t launch_apply_batch(int prec, int N, const ApplyJob* jobs, int count, const DevTab& t,
                              hipStream_t s);
hipError_t launch_patch_fd_batch(int prec, int N, int colour, const PatchJob* jobs, int count,
                                 const DevTab& t, hipStream_t s);
hipError_t launch_coarse_fd_batch(int prec, int N, const CoarseJob* jobs, int count,
                                  const DevTab& t, hipStream_t s);
hipError_t launch_transfer_batch(int prec, int N, bool restr, const TransferJob* jobs, int count,
                                 const DevTab& t, hipStream_t s);

// BLAS-1 helpers (FP64).  `partial` holds at least kDotBlocks * nv doubles.
constexpr int kDotBlocks = 1024;
hipError_t launch_mdot(const double* V, int64_t ld, int nv, const double* w, int64_t n,
                       double* partial, double* out, hipStream_t s);
// w -= sum_i coef[i] V[i] (coef on the device); if `acc` != nullptr also
// acc[i] += coef[i]
hipError_t launch_maxpy(const double* V, int64_t ld, int nv, const double* coef,
                        double* w, int64_t n, double* acc, double sign, hipStream_t s);
hipError_t launch_scale_copy(const double* src, double alpha, double* dst, int64_t n,
                             hipStream_t s);
hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t n, hipStream_t s);
hipError_t launch_fill(double* x, double value, int64_t n, hipStream_t s);
hipError_t launch_finite_check(const double* x, int64_t n, int* flag, hipStream_t s);
hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_to_f64(const float* src, double* dst, int64_t n, hipStream_t s);
hipError_t launch_zero_f32(float* x, int64_t n, hipStream_t s);

// Low-precision kernels: FP32 storage, FP16 (bf16 = false) or BF16 products
// on the matrix cores with FP32 accumulation; ec = 0 none, 1 both operands
// split (Alg. matmul), 2 only the matrix operand split.
hipError_t launch_apply_lp(int N, bool bf16, int ec, const float* u, float* v, const float* b,
                           const DevTab& t, int n, double h, hipStream_t s);
hipError_t launch_patch_fd_lp(int N, bool bf16, int ec, int colour, const float* r, float* x,
                              const DevTab& t, int n, double h, hipStream_t s);
hipError_t launch_apply_lp_batch(int N, bool bf16, int ec, const ApplyJob* jobs, int count,
                                 const DevTab& t, hipStream_t s);
hipError_t launch_patch_fd_lp_batch(int N, bool bf16, int ec, int colour, const PatchJob* jobs,
                                    int count, const DevTab& t, hipStream_t s);

// Manufactured right-hand side and L2 error (tables prepared on the host).
hipError_t launch_rhs_sines(int N, int n, int n_modes, const double* coef,
                            const double* bx, const double* by, const double* bz,
                            double* b, hipStream_t s);
hipError_t launch_l2_sines(int N, int nq, int n, int n_modes, const double* amps,
                           const double* sx, const double* sy, const double* sz,
                           const double* interp, const double* wq, double h,
                           const double* x, double* partial, double* out, hipStream_t s);

// Device address of the fixed workspace of the allocation-free L2 error on
// the current device (kL2ScratchDoubles doubles, 256-byte aligned; looked up
// once per device).  Calls that use it overlap-race on one device.
constexpr size_t kL2ScratchDoubles = 131072;  // 1 MiB
constexpr int kMaxDevices = 64;
hipError_t l2_scratch(double** out);

// General geometry (trilinear hexahedra): the device data of one level.
struct MappedLevel {
  const double* vert = nullptr;  // (n+1)^3 x 3 vertex positions, [vz][vy][vx][xyz]
  const double* gam = nullptr;   // n^3 x 6 face penalties, face 2 d + side
  int n = 0;
};
// v = A u (or v = b - A u when b != nullptr) on the trilinear cells of g;
// mtab is the device copy of mapped_table(k).  u and v must not alias.
hipError_t launch_apply_mapped(int N, const double* u, double* v, const double* b,
                               const MappedLevel& g, const double* mtab, hipStream_t s);
// the same on FP32 vectors (widened on load, FP64 arithmetic, rounded on
// store): the FP32 V-cycle's residuals on trilinear cells
hipError_t launch_apply_mapped_f32(int N, const float* u, float* v, const float* b,
                                   const MappedLevel& g, const double* mtab, hipStream_t s);
// b = int f phi on the trilinear cells, f a sum of nm sine modes (modes:
// [nm][coefficient, p, q, r]); qtab = quad_table(k, k + 2).
hipError_t launch_rhs_mapped(int N, const MappedLevel& g, int nm, const double* modes,
                             const double* qtab, double* b, hipStream_t s);
// out[0] = int (u - x)^2 over the trilinear cells, u a sum of nm sine modes
// (modes: [nm][amplitude, p, q, r]); qtab = quad_table(k, k + 3); partial
// holds max_blocks doubles.
hipError_t launch_l2_mapped(int N, const MappedLevel& g, int nm, const double* modes,
                            const double* qtab, const double* x, double* partial, int max_blocks,
                            double* out, hipStream_t s);

// ---- flexible GMRES of many problems with device-side scalars (krylov.hip)
// Per-problem state block (doubles, kStateStride per problem): g, Givens
// cosines and sines, flags, the triangular factor R (column-major, m x m),
// y and the residual history.
constexpr int kMaxKrylov = 32;
constexpr int kStateStride = 2048;
constexpr int kSG = 0, kSCs = 64, kSSn = 96;
constexpr int kSActive = 128, kSJd = 129, kSIts = 130, kSEst = 131, kSConv = 132, kSBad = 133,
              kSHist = 134;
constexpr int kFlagCount = 7;  // kSActive .. kSHist, the host's view
constexpr int kSInv = 140, kSNb = 141, kSTol = 142, kSMaxIts = 143;
constexpr int kSR = 256, kSY = 1280, kSHistory = 1536, kHistory = 128;
constexpr int kNormSlot = 160;  // small[] slot of the squared norms
struct KrylovDesc {
  double* V;        // Krylov basis, m + 1 vectors of n
  double* Z;        // preconditioned vectors, m vectors of n
  double* x;        // solution
  double* small;    // dot results: h at [0, 33), second pass at [80, 113), norm at kNormSlot
  double* partial;  // dot partial sums, 256 x 33 doubles
  double* st;       // state block
  int64_t n;
};
// small[off + i] = V_{first+i} . V_widx for i < nv (every problem of D[0..P))
hipError_t launch_krylov_dots(const KrylovDesc* D, int P, int first, int nv, int widx, int off,
                              hipStream_t s);
// V_widx -= sum_{i<nv} small[coef + i] V_i; small[acc + i] += coef (acc >= 0)
hipError_t launch_krylov_axpy(const KrylovDesc* D, int P, int64_t nmax, int nv, int widx,
                              int coef, int acc, hipStream_t s);
// V_widx *= st[kSInv]
hipError_t launch_krylov_scale(const KrylovDesc* D, int P, int64_t nmax, int widx, hipStream_t s);
// x += sum_{i<m} st[kSY + i] Z_i
hipError_t launch_krylov_update(const KrylovDesc* D, int P, int64_t nmax, int m, hipStream_t s);
// stage 0: cycle start; 1: Arnoldi step j; 2: cycle end (y, convergence);
// 3: copy the flags of every problem to flags[P x kFlagCount]
hipError_t launch_krylov_scalars(int stage, const KrylovDesc* D, int P, int j, int m,
                                 double* flags, hipStream_t s);

}  // namespace sipg
