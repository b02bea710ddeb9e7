/*
 * sipg.h - C ABI of the MI355X (gfx950) SIPG-DG Poisson library.
 *
 * The library evaluates the symmetric interior-penalty DG Laplacian on a
 * uniform Cartesian hexahedral mesh of the unit cube matrix-free by sum
 * factorization, and solves the Poisson problem with flexible GMRES
 * preconditioned by a geometric multigrid V-cycle with a multiplicative
 * vertex-patch smoother whose local solves use fast diagonalization.
 * Method: Cui, "Acceleration of Tensor-Product Operations with Tensor Cores",
 * arXiv 2407.09621 (Sec. 2, 2.1, 7).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh level l has n_l^3 cells of size h_l = 1/n_l; level 0 is the coarsest,
 * level L-1 the finest (n_{L-1} = n_cells), n_{l-1} = n_l / 2.
 * Degree k (1..7), N = k + 1 nodes per direction (Gauss-Lobatto points).
 * Vectors are cell-blocked: cell c = cx + n*cy + n*n*cz owns the N^3
 * contiguous entries c*N^3 + i + N*j + N*N*l (x fastest).  Every vector
 * argument is a DEVICE pointer owned by the caller, holding sipg_n_dofs()
 * entries, aligned to its element size (8 bytes FP64, 4 bytes FP32): the
 * kernels issue element-sized loads, so sub-views of larger tensors are
 * valid arguments; 256-byte alignment (what hipMalloc and torch return)
 * gives the coalescing the throughput figures assume.  Input and output
 * vectors of one call must not overlap unless the entry point says so.
 * Calls are asynchronous on the given HIP stream (NULL = default stream)
 * unless stated otherwise; the host arguments are read before return.
 * A handle is not thread-safe; different handles are independent.
 * Errors: a sipg_status is returned, and sipg_last_error() gives a
 * thread-local message for the last failing call.  No C++ exception crosses
 * the ABI.
 */
#ifndef SIPG_H
#define SIPG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SIPG_OK = 0,
  SIPG_ERR_ARG = 1,            /* bad size, degree, level, NULL pointer, alias */
  SIPG_ERR_UNSUPPORTED = 2,    /* valid request the library does not implement */
  SIPG_ERR_OOM = 3,            /* device allocation failed */
  SIPG_ERR_HIP = 4,            /* a HIP runtime call failed (text in last_error) */
  SIPG_ERR_NOT_CONVERGED = 5,  /* iteration limit reached; x holds the last iterate */
  SIPG_ERR_NONFINITE = 6       /* a NaN/Inf appeared and could not be recovered */
} sipg_status;

typedef enum {
  SIPG_F64 = 0,   /* FP64 storage and arithmetic */
  SIPG_F32 = 1,   /* FP32 storage and arithmetic */
  SIPG_F16 = 2,   /* FP32 storage, FP16 products with FP32 accumulation */
  SIPG_BF16 = 3   /* FP32 storage, BF16 products with FP32 accumulation */
} sipg_precision;

/* Device allocator callbacks: alloc returns `bytes` of device memory
 * aligned to 256 bytes (NULL on failure) usable on `stream`; dealloc
 * releases a block alloc returned.  `ctx` is passed through. */
typedef void* (*sipg_alloc_fn)(size_t bytes, hipStream_t stream, void* ctx);
typedef void (*sipg_dealloc_fn)(void* ptr, hipStream_t stream, void* ctx);

typedef struct {
  int k;                 /* polynomial degree, 1..7 */
  int n_cells;           /* cells per direction on the finest level */
  int n_levels;          /* 0: coarsen down to 1, 2 or 3 cells per direction */
  int mg_precision;      /* sipg_precision of the V-cycle (preconditioner) */
  int error_correction;  /* FP16/BF16 products: 0 none; 1 both operands split
                            into hi + 2^-s lo (Alg. matmul, s = 11 FP16, 8
                            BF16); 2 only the constant matrix operand split
                            (two products instead of three) */
  int nu_pre;            /* pre-smoothing sweeps (2 for V(2,2)) */
  int nu_post;           /* post-smoothing sweeps */
  int smoother;          /* 0: multiplicative vertex-patch smoother (colour by
                            colour, the paper's choice, Sec. 7.1): per colour a
                            residual launch, then the patch solves; 1: additive
                            (one residual per sweep, all patch corrections
                            summed and damped; FP64 V-cycles only); 2:
                            multiplicative with one fused launch per colour
                            step: the new patch values are the local solve
                            with the right-hand side minus the face couplings
                            of the outside neighbours, which equals
                            x_P + inv(A_PP) (b - A x)_P (same result as 0 to
                            rounding; FP64 / FP32 V-cycles, FP16 / BF16 take
                            form 0) */
  double damping;        /* additive smoother: x += damping * sum_P corrections
                            (0 means 1/8: every cell lies in 8 patches) */
  double penalty_scale;  /* penalty gamma = penalty_scale * k(k+1)(1/h+ + 1/h-)
                            (Sec. 2); 0 means 1.  Must lie in [1, 100]: below
                            1 the form need not stay coercive */
  sipg_alloc_fn alloc;   /* NULL: hipMalloc / hipFree.  Otherwise every block
                            of the handle's workspace comes from alloc (on the
                            stream given to sipg_create) and goes back through
                            dealloc, e.g. torch's caching allocator */
  sipg_dealloc_fn dealloc;
  void* alloc_ctx;
} sipg_config;

typedef struct sipg_problem sipg_problem;

/* Build the level hierarchy, 1D tables and workspace (Sec. 2.1, Sec. 7.1).
 * The penalty is gamma = k(k+1)(1/h+ + 1/h-) = 2k(k+1)/h on every face
 * (Sec. 2), times cfg->penalty_scale.  Requires n_cells = n0 * 2^(L-1); the
 * exact coarse solve needs n0 in {1, 2, 3}.  mg_precision SIPG_BF16 with
 * error_correction 0 is refused (SIPG_ERR_UNSUPPORTED) for k >= 5: with the
 * 1D operator rounded to 8 significand bits the preconditioned iteration
 * stalls there (use error_correction 1 or 2).  The additive smoother is
 * refused for mg_precision other than SIPG_F64.  The handle owns its workspace,
 * allocated on `stream` through cfg->alloc when given (freed by
 * sipg_destroy).  Synchronizes `stream`. */
sipg_status sipg_create(const sipg_config* cfg, hipStream_t stream, sipg_problem** out);

/* Free the handle and its workspace.  NULL-safe.  Synchronizes the device. */
void sipg_destroy(sipg_problem* p);

/* Number of levels and per-level sizes.  Return -1 on a bad argument. */
int sipg_num_levels(const sipg_problem* p);
int sipg_level_cells(const sipg_problem* p, int level);
int64_t sipg_n_dofs(const sipg_problem* p, int level);

/* v = A_l u in FP64 (Sec. 2.1 matrix-free loop with eq. tensorproduct_3d:
 * cell integrals by sum factorization, face integrals through neighbour
 * traces).  u, v: n_dofs(level) doubles, must not overlap. */
sipg_status sipg_apply(sipg_problem* p, int level, const double* u, double* v,
                       hipStream_t stream);

/* General geometry (Sec. 2 and Sec. 2.1: cells mapped from the reference
 * cube, A^K = G^T W G with per-point Jacobians).  Replaces the Cartesian
 * unit-cube mesh of every level by trilinear hexahedra through the given
 * vertex positions: `vertices` is a HOST array of (n+1)^3 * 3 doubles (n =
 * finest cells per direction), vertex (vx, vy, vz) at index
 * ((vz * (n+1) + vy) * (n+1) + vx) * 3 (x, y, z); level l takes every
 * 2^(L-1-l)-th vertex.  The caller keeps ownership; the library copies it.
 * Quadrature is N-point Gauss per direction on cells and N x N on faces;
 * the penalty of a face is k(k+1)(1/h- + 1/h+) times penalty_scale with h
 * the cell volume over the face area (boundary faces 2k(k+1)/h-).
 * Afterwards sipg_apply, sipg_residual, sipg_smooth, sipg_vcycle and
 * sipg_fgmres use the mapped operator; the smoother's patch solves and the
 * coarse solve keep the Cartesian fast diagonalization (an approximate
 * inverse on mapped cells; the outer FGMRES corrects for it).  NULL
 * restores the Cartesian mesh.  SIPG_ERR_UNSUPPORTED unless mg_precision is
 * SIPG_F64 or SIPG_F32 (the FP32 V-cycle's residuals then run on the
 * trilinear cells with FP32 vectors and FP64 arithmetic) and the smoother
 * is 0 or 1; while a geometry is set,
 * sipg_rhs_sines and sipg_l2_error_sines integrate over the mapped cells
 * (the same Gauss rules with det J at every point; the sine modes vanish on
 * the boundary only where it stays on the unit cube's faces), and
 * sipg_apply_units, sipg_apply_patchwise, sipg_apply_lp, sipg_autotune,
 * sipg_l2_error_sines_noalloc, the learned stage and the network training
 * return SIPG_ERR_UNSUPPORTED (they are Cartesian).  SIPG_ERR_ARG when a
 * cell has a non-positive Jacobian determinant at a Gauss point or corner
 * (the previous geometry is kept).  Synchronizes `stream`. */
sipg_status sipg_set_geometry(sipg_problem* p, const double* vertices, hipStream_t stream);

/* Execution units of the FP64 apply (the paper's comparison of tensor-core
 * and CUDA-core kernels, Sec. 4 and App. A, on gfx950's matrix and vector
 * units). */
typedef enum {
  SIPG_UNITS_AUTO = 0,    /* what sipg_apply uses: matrix cores for k = 3 and 7 */
  SIPG_UNITS_VECTOR = 1,  /* FP64 vector units (one 1D line per lane), every k */
  SIPG_UNITS_MATRIX = 2   /* FP64 matrix cores (v_mfma_f64_4x4x4f64); k = 3, 7 */
} sipg_units;

/* sipg_apply on the chosen execution units: the same v = A_l u (parity with
 * the oracle to rounding), computed by the kernel `units` names.
 * SIPG_ERR_UNSUPPORTED for SIPG_UNITS_MATRIX with k other than 3 and 7. */
sipg_status sipg_apply_units(sipg_problem* p, int level, const double* u, double* v, int units,
                             hipStream_t stream);

/* v = A_l u in FP64 evaluated patch by patch, the paper's form (Sec. 2.1,
 * Fig. patch_int): every interior vertex's patch of 2 x 2 x 2 cells applies
 * the Kronecker sum of its own 2N x 2N window matrices (mass and
 * stiffness-plus-face; each interior face integral in one window, the cell
 * integrals shared by the windows that contain the cell) to its (2N)^3
 * coefficients, and the patches' results are summed into v, colour by
 * colour (patches of one colour share no cell).  The same A u as sipg_apply
 * up to rounding, with about 8 times the products per DoF; for comparing
 * the two evaluations.  Needs n_level >= 2.  u, v must not overlap; v is
 * overwritten. */
sipg_status sipg_apply_patchwise(sipg_problem* p, int level, const double* u, double* v,
                                 hipStream_t stream);

/* v = A_l u with FP32 vectors in a reduced-precision arithmetic (Sec. 5,
 * Sec. 7.1): precision SIPG_F32 (FP32 throughout), SIPG_F16 or SIPG_BF16
 * (1D contractions on the matrix cores with FP16/BF16 operands and FP32
 * accumulation; FP16 lines are scaled by powers of two into range).  ec as
 * sipg_config.error_correction: 1 the split-operand error correction of
 * Alg. matmul, 2 only the matrix operand split (ignored for F32).
 * u, v: n_dofs(level) floats, must not overlap. */
sipg_status sipg_apply_lp(sipg_problem* p, int level, const float* u, float* v,
                          int precision, int ec, hipStream_t stream);

/* r = b - A_l x in FP64: the defect that Alg. v_cycle restricts to the
 * coarser level and the smoother (Sec. 7.1) corrects, with A_l the operator
 * of sipg_apply.  r must not overlap x or b. */
sipg_status sipg_residual(sipg_problem* p, int level, const double* b,
                          const double* x, double* r, hipStream_t stream);

/* Multiplicative vertex-patch smoother, FP64, in place on x (Sec. 7.1; the
 * paper's references for the smoother): for colours 0..7 in order,
 * r = b - A x, then every patch P of the colour (the 2x2x2 cells around an
 * interior vertex, colour = parity of the vertex coordinates) adds
 * A_PP^{-1} r_P, computed by fast diagonalization.  `sweeps` >= 0.
 * x and b must not overlap. */
sipg_status sipg_smooth(sipg_problem* p, int level, double* x, const double* b,
                        int sweeps, hipStream_t stream);

/* One colour step of the smoother, split for testing: for all patches of
 * `colour` (0..7) x_P += A_PP^{-1} r_P, with r given.  r and x must not
 * overlap. */
sipg_status sipg_patch_correct(sipg_problem* p, int level, int colour,
                               const double* r, double* x, hipStream_t stream);

/* The smoother and one colour step of it on FP32 vectors, in the handle's
 * reduced precision (mg_precision SIPG_F32, SIPG_F16 or SIPG_BF16 with its
 * error_correction; SIPG_ERR_ARG for an FP64 handle): the residual through
 * the kernels of sipg_apply_lp, the patch solves with the six 2N x 2N
 * eigenvector contractions of the fast diagonalization on the matrix cores
 * (FP32 vector arithmetic for SIPG_F32), FP32 accumulation (Sec. 5, 7.1).
 * Same contracts as sipg_smooth and sipg_patch_correct. */
sipg_status sipg_smooth_lp(sipg_problem* p, int level, float* x, const float* b, int sweeps,
                           hipStream_t stream);
sipg_status sipg_patch_correct_lp(sipg_problem* p, int level, int colour, const float* r,
                                  float* x, hipStream_t stream);

/* Level transfers (canonical embedding of nested spaces and its transpose;
 * Alg. v_cycle coarsen / coarse-grid correction).  `level` is the FINE
 * level (>= 1).  restrict: rc = P^T rf.  prolongate_add: xf += P ec. */
sipg_status sipg_restrict(sipg_problem* p, int level, const double* rf,
                          double* rc, hipStream_t stream);
sipg_status sipg_prolongate_add(sipg_problem* p, int level, const double* ec,
                                double* xf, hipStream_t stream);

/* x = A_0^{-1} b on the coarsest level, exactly, by fast diagonalization of
 * the Kronecker-sum coarse matrix (Alg. v_cycle, coarse grid solver). */
sipg_status sipg_coarse_solve(sipg_problem* p, const double* b, double* x,
                              hipStream_t stream);

/* x <- V-cycle_l(x, b) with nu_pre/nu_post sweeps (Alg. v_cycle), in the
 * handle's mg_precision (FP64 vectors in and out).  For mg_precision other
 * than SIPG_F64 the cycle runs on FP32 copies made at entry and converted
 * back at exit; residuals and patch solves then use the reduced-precision
 * kernels of sipg_apply_lp (with the handle's error_correction), transfers
 * and the coarse solve run in FP32.  x and b must not overlap. */
sipg_status sipg_vcycle(sipg_problem* p, int level, double* x, const double* b,
                        hipStream_t stream);

typedef enum {
  SIPG_FGMRES = 0,  /* flexible GMRES: keeps every preconditioned vector z_j and
                       forms x += Z y (Saad 1993; the paper's solver, Sec. 7) */
  SIPG_GMRES = 1    /* right-preconditioned GMRES: keeps only the Arnoldi basis
                       and forms x += M(V y) with one more V-cycle, which
                       assumes the same linear M in every step (the
                       comparison of Sec. 7.2, Fig. fgmres_vs_gmres) */
} sipg_krylov_variant;

typedef struct {
  double rtol;        /* stop when |Arnoldi residual| <= rtol * ||b||_2 */
  int restart;        /* Krylov dimension before restart (<= 64) */
  int max_iters;      /* total iteration limit */
  int use_learned;    /* 1: apply the attached network after each V-cycle */
  int log_history;    /* 1: record the residual estimate of every iteration */
  double stagnation;  /* learned stage: switch it off after an iteration whose
                         estimate falls by less than this factor (0: 0.9) */
  int variant;        /* sipg_krylov_variant (0: FGMRES) */
} sipg_solve_opts;

typedef struct {
  int iterations;
  int fell_back;           /* 1 if the learned stage was switched off during the
                              solve, or a non-finite preconditioner output was
                              replaced */
  double rel_res_est;      /* last Arnoldi estimate / ||b|| */
  double rel_res_true;     /* ||b - A x||_2 / ||b||_2, recomputed in FP64 */
  double seconds;          /* wall time of the solve */
  double history[128];     /* history[i] = estimate after i iterations (i <= 127) */
} sipg_solve_info;

/* Solve A x = b on the finest level with right-preconditioned flexible GMRES
 * (Saad 1993; Sec. 7.1-7.2), FP64 outer iteration and Gram-Schmidt
 * (classical, twice), preconditioner = one V-cycle from zero (opts->variant
 * SIPG_GMRES: the non-flexible form).  x is the initial guess on entry (pass
 * zeros for x0 = 0) and the solution on return.  A NaN or Inf in a
 * preconditioned vector switches that step to the plain V-cycle (learned
 * stage on) or to the identity (info->fell_back = 1).  Device scalars reach
 * the host through a pinned buffer by copies ordered on `stream`, which is
 * synchronized once per Krylov step.  Blocks until done.  Returns
 * SIPG_ERR_NOT_CONVERGED if max_iters is hit. */
sipg_status sipg_fgmres(sipg_problem* p, double* x, const double* b,
                        const sipg_solve_opts* opts, sipg_solve_info* info,
                        hipStream_t stream);

/* Manufactured data u = sum_m a_m sin(p_m pi x) sin(q_m pi y) sin(r_m pi z)
 * (Sec. 7.2 uses one mode with p = q = r = 1).  amps[n_modes] and
 * pqr[3*n_modes] are HOST arrays.
 * rhs_sines: b_I = int f phi_I with f = -Laplace u, (k+2)-point Gauss.
 * l2_error_sines: *err (HOST) = ||u - u_h||_L2 with (k+3)-point Gauss;
 * synchronizes the stream. */
sipg_status sipg_rhs_sines(sipg_problem* p, int level, int n_modes,
                           const double* amps, const int* pqr, double* b,
                           hipStream_t stream);
sipg_status sipg_l2_error_sines(sipg_problem* p, int level, int n_modes,
                                const double* amps, const int* pqr,
                                const double* x, double* err,
                                hipStream_t stream);

/* sipg_l2_error_sines without any allocation, for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid it):
 * the same result and kernels, with the tables, partial sums and result in a
 * fixed workspace of 1 MiB per device that the library holds in a static
 * device array (not in the handle, whose table buffer sipg_l2_error_sines
 * grows on demand).  Limit: n_modes * 3 * n_level * (k + 3) + n_modes +
 * (k + 3)(k + 2) <= 130,016 table entries (e.g. 4 modes up to 1,082 cells per
 * direction at k = 7); larger requests return SIPG_ERR_ARG.  Every call on a
 * device shares that device's workspace, so calls that overlap on one
 * device (from several host threads, or streams not ordered with each
 * other) race; host threads are serialized while the tables are staged.
 * Synchronizes the stream. */
sipg_status sipg_l2_error_sines_noalloc(sipg_problem* p, int level, int n_modes,
                                        const double* amps, const int* pqr,
                                        const double* x, double* err, hipStream_t stream);

/* Tile-order autotuner of the operator apply: times the apply on `level`
 * with each admissible tile-order block (1, 2, 4, 8 cells, dividing n) and
 * keeps the fastest for all later applies, residuals and smoother sweeps of
 * that level.  u, v: two distinct scratch vectors of the level (contents
 * irrelevant; v is overwritten).  *best (HOST, may be NULL) receives the
 * chosen block.  Synchronizes the stream. */
sipg_status sipg_autotune(sipg_problem* p, int level, const double* u, double* v,
                          int* best, hipStream_t stream);

/* ---- batches of independent problems (uneven sizes and degrees) ---------
 * A batch owns one problem handle per configuration.  All configurations
 * must share mg_precision, error_correction, nu_pre and nu_post, and reach
 * a coarsest level of 1, 2 or 3 cells.  Vector arguments are HOST arrays of
 * `count` DEVICE pointers (problem i uses sipg_n_dofs of its finest level).
 * Every stage of the batched V-cycle and FGMRES iteration is issued as
 * launches that each cover up to 16 problems of one degree. */
typedef struct sipg_batch sipg_batch;

/* Each problem is created as by sipg_create(&cfgs[i], stream, ...). */
sipg_status sipg_batch_create(const sipg_config* cfgs, int count, hipStream_t stream,
                              sipg_batch** out);
void sipg_batch_destroy(sipg_batch* b);
int sipg_batch_count(const sipg_batch* b);
/* Borrowed handle of problem i (owned by the batch; do not destroy). */
sipg_problem* sipg_batch_problem(sipg_batch* b, int i);
/* Run sipg_autotune on every level of one problem per (k, n) class and share
 * the result with the class.  Synchronizes. */
sipg_status sipg_batch_autotune(sipg_batch* b, hipStream_t stream);
/* v_i = A_i u_i on the finest levels (FP64). */
sipg_status sipg_batch_apply(sipg_batch* b, const double* const* u, double* const* v,
                             hipStream_t stream);
/* x_i <- V-cycle(x_i, b_i) on the finest levels, levels aligned by depth. */
sipg_status sipg_batch_vcycle(sipg_batch* b, double* const* x, const double* const* bvec,
                              hipStream_t stream);
/* FGMRES for all problems in lockstep, each with its own Hessenberg system,
 * stopping test and restarts.  use_graph = 0: batched launches, one host
 * synchronization per Krylov step for the whole batch; 1: the same with the
 * batched V-cycle of Krylov step j captured as a HIP graph on an internal
 * stream at its first use and replayed; 2: the FGMRES scalars on the device
 * (Gram-Schmidt, Arnoldi normalization, Givens rotations, stopping test and
 * the triangular solve in batched kernels), each whole Krylov step
 * (V-cycle, apply, Gram-Schmidt, update) one captured graph over all
 * problems; between steps the host reads only the problems' active flags
 * (one small copy) to decide whether to issue the next; restart <= 32.
 * Problems that stopped ride along with zero vectors.  Mode 2 allocates its
 * small device state (descriptors, a 16 KB state block per problem, flags)
 * with hipMalloc on first use; it is freed by sipg_batch_destroy.
 * infos[count] (HOST)
 * receive per-problem results; `seconds` is the batch wall time.  Blocks
 * until done.  SIPG_ERR_UNSUPPORTED if a problem has a geometry set. */
sipg_status sipg_batch_solve(sipg_batch* b, double* const* x, const double* const* bvec,
                             const sipg_solve_opts* opts, sipg_solve_info* infos,
                             int use_graph, hipStream_t stream);
/* Reference: sipg_fgmres on each problem in turn. */
sipg_status sipg_batch_solve_sequential(sipg_batch* b, double* const* x,
                                        const double* const* bvec,
                                        const sipg_solve_opts* opts,
                                        sipg_solve_info* infos, hipStream_t stream);

/* Thread-local text of the last error ("" if none). */
const char* sipg_last_error(void);

/* ---- learned correction stage (a project extension, not in the paper) ----
 * A 3D convolutional network 1 -> 32 -> 32 -> 32 -> 1 channels, 3x3x3
 * kernels, zero padding, ReLU between layers, FP16 weights and activations
 * with FP32 accumulation, on the G^3 grid of DG coefficients: node (i, j, l)
 * of cell (cx, cy, cz) sits at grid point (N cx + i, N cy + j, N cz + l),
 * G = n N, N = k + 1.  Grids are dense FP32 device arrays indexed
 * gx + G (gy + G gz), one after another for a batch; G must be a multiple of
 * 16.  The parameter vector (SIPG_CNN_PARAMS floats) is w1[32][27] b1[32]
 * w2[32][32][27] b2[32] w3[32][32][27] b3[32] w4[32][27] b4 with weights
 * indexed [c_out][c_in][9 (dz+1) + 3 (dy+1) + dx + 1] (cross-correlation).
 * The network output is multiplied by a power of two sigma (the output
 * scale, chosen from the first training pair when 0).
 * Stage: after the V-cycle z = V(v) the preconditioner forms the
 * correction c = s sigma net((v - A z) / s), s = 2^ceil(log2 max|v - A z|),
 * and adds alpha c with alpha = (rho . A c) / (A c . A c), rho = v - A z,
 * the factor minimising ||v - A (z + alpha c)||_2 (finest level).  sipg_fgmres (use_learned = 1) switches the stage off for the rest
 * of a solve once an iteration reduces the residual estimate by less than a
 * factor 0.9 or the corrected vector is not finite (that iteration then
 * uses the plain V-cycle); info->fell_back reports it.
 * A handle is used by one stream at a time. */
#define SIPG_CNN_PARAMS 57121
typedef struct sipg_cnn sipg_cnn;
int sipg_cnn_num_params(void);
/* All parameters zero, sigma 0 (no correction until trained or set). */
sipg_status sipg_cnn_create(sipg_cnn** out);
void sipg_cnn_destroy(sipg_cnn* c);
/* He-uniform weights from a splitmix64 stream seeded with `seed` (last
 * layer scaled by 0.1), zero biases, sigma 0, Adam state reset. */
sipg_status sipg_cnn_init(sipg_cnn* c, uint64_t seed);
/* HOST arrays of SIPG_CNN_PARAMS floats.  set resets the Adam state. */
sipg_status sipg_cnn_set_params(sipg_cnn* c, const float* params, float sigma);
sipg_status sipg_cnn_get_params(const sipg_cnn* c, float* params, float* sigma);
/* out = sigma * net(in) on `batch` device grids of side G (in is rounded
 * to FP16). */
sipg_status sipg_cnn_forward(sipg_cnn* c, int G, int batch, const float* in, float* out,
                             hipStream_t stream);
/* grad (device, SIPG_CNN_PARAMS floats) = gradient of the masked loss
 * L = sum m (sigma net(in) - target)^2 / sum m over the batch; *loss
 * (device float, may be NULL) = L.  mask m >= 0 per grid point. */
sipg_status sipg_cnn_gradient(sipg_cnn* c, int G, int batch, const float* in,
                              const float* target, const float* mask, float* grad,
                              float* loss, hipStream_t stream);
/* Residual-aware loss on the problem's finest level (the learned stage
 * should cancel the residual the V-cycle leaves, and A amplifies the
 * high-frequency part of any pointwise error in e): for the scaled residual
 * rho (device FP64 cell vector of the finest level, e.g. rho / s of a
 * training pair), c = sigma net(grid(rho)) mapped to cells, q = A c, the
 * stage's own step alpha = (rho . q) / (q . q) (0 if q = 0) and
 * r = rho - alpha q: L = ||r||^2 / ||rho||^2 (independent of sigma);
 * grad (device, SIPG_CNN_PARAMS floats) = dL/dparameters through
 * dL/dy = -2 sigma alpha grid(A r) / ||rho||^2; *loss (device float, may
 * be NULL) = L.  sigma must be set (> 0). */
sipg_status sipg_cnn_gradient_residual(sipg_cnn* c, sipg_problem* p, const double* rho,
                                       float* grad, float* loss, hipStream_t stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * device gradient `grad`. */
sipg_status sipg_cnn_adam_step(sipg_cnn* c, const float* grad, float lr, hipStream_t stream);
/* Training pairs generated by the solver on the finest level: starting
 * from x = x0 (device, not modified), each pair computes r = A x,
 * z = V-cycle(0, r), e = x - z, rho = r - A z, s = 2^ceil(log2 max|rho|),
 * writes grid(rho / s) and grid(e / s) into the next G^3 slot of rho_grids
 * and e_grids (device, count * G^3 floats each) and s into scales[j]
 * (HOST, may be NULL), then continues the chain with
 * x = e / 2^ceil(log2 max|e|).  Synchronizes the stream. */
sipg_status sipg_cnn_make_pairs(sipg_problem* p, const double* x0, int count,
                                float* rho_grids, float* e_grids, double* scales,
                                hipStream_t stream);
typedef struct {
  int n_chains;        /* right-hand sides (4 sine modes, a ~ U[-1,1], p,q,r ~ U{1..4}) */
  int chain_length;    /* pairs per right-hand side (one Adam step each) */
  int crops_per_pair;  /* random crops of side `crop` per step (1..16) */
  int crop;            /* crop side, a multiple of 16, <= G */
  float lr;            /* Adam learning rate */
  int log_every;       /* read the loss back every this many steps (0: first/last) */
  uint64_t seed;       /* seed of the draws (modes, crop offsets) */
  int loss;            /* 0: masked MSE on the error, on random crops (crop,
                          crops_per_pair); 1: the residual the correction leaves
                          after the stage's own step length, on the whole grid
                          (sipg_cnn_gradient_residual on rho/s) */
} sipg_cnn_train_opts;
typedef struct {
  int steps;
  float loss_first, loss_last;  /* masked MSE of the first and last step */
  float sigma;                  /* output scale in use */
  double seconds;               /* wall time of the training run */
  double seconds_pairs;         /* part spent generating pairs */
} sipg_cnn_train_info;
/* Train on the GPU with pairs made by the problem's own solver: per
 * right-hand side, x0 from three V-cycles on b, then chain_length pairs
 * (as in sipg_cnn_make_pairs), each giving one Adam step on crops_per_pair
 * random crops (loss masked to points at least 4 points from crop faces
 * inside the grid).  Runs on an internal stream; blocks until done. */
sipg_status sipg_cnn_train(sipg_problem* p, sipg_cnn* c, const sipg_cnn_train_opts* o,
                           sipg_cnn_train_info* info);
/* Parameters and output scale to / from a file: the 8 bytes "SIPGCNN1",
 * an int32 parameter count (SIPG_CNN_PARAMS), a float32 sigma, then the
 * parameters as float32, all little-endian.  load checks the magic and the
 * count (SIPG_ERR_ARG on a mismatch or a short file, SIPG_ERR_UNSUPPORTED on
 * an I/O error) and resets the Adam state.  Synchronous. */
sipg_status sipg_cnn_save(const sipg_cnn* c, const char* path);
sipg_status sipg_cnn_load(sipg_cnn* c, const char* path);
/* Use `c` as the problem's learned stage (NULL detaches).  The problem
 * borrows the handle: keep it alive while attached. */
sipg_status sipg_cnn_attach(sipg_problem* p, sipg_cnn* c);

#ifdef __cplusplus
}
#endif
#endif /* SIPG_H */
