// Internal state of a problem handle and helpers shared by the C-ABI
// translation units (not part of the public interface).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/sipg.h"
#include "kernels.h"
#include "tables.h"

namespace sipg {

extern thread_local std::string g_err;

inline sipg_status fail(sipg_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

template <typename T>
sipg_status dev_alloc(T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return SIPG_OK;
  hipError_t e = hipMalloc((void**)ptr, count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(SIPG_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return SIPG_OK;
}

}  // namespace sipg

#define SIPG_HIP(expr)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return ::sipg::fail(SIPG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define SIPG_TRY(expr)            \
  do {                            \
    sipg_status s_ = (expr);      \
    if (s_ != SIPG_OK) return s_; \
  } while (0)

struct sipg_problem {
  sipg_config cfg{};
  int k = 0, N = 0, L = 0, n0 = 0;
  std::vector<int> n;
  std::vector<int64_t> ndofs;
  sipg::DevTab tab;
  double* d_tab = nullptr;
  std::vector<double*> wx, wb, wr;  // per-level V-cycle vectors
  std::vector<double*> wc;          // additive smoother: summed patch corrections
  hipStream_t alloc_stream = nullptr;  // stream handed to the allocator callbacks
  int krylov_gen = 0;               // bumped whenever V / Z are reallocated
  double* h_pinned = nullptr;       // pinned host scalars (Hessenberg column, y)
  double* V = nullptr;              // Krylov basis, (restart + 1) vectors
  double* Z = nullptr;              // preconditioned vectors, restart vectors
  int restart_alloc = 0;
  double* d_partial = nullptr;      // kDotBlocks * 65 doubles
  double* d_small = nullptr;        // 512 doubles of scalars
  int* d_flag = nullptr;
  double* d_aux = nullptr;          // tables for rhs / l2 (grown on demand)
  size_t aux_size = 0;
  std::vector<double> l2_xq, l2_wq, l2_V;  // (k+3)-point Gauss rule, Lagrange values there
  // low-precision V-cycle (mg_precision != F64): FP32 level vectors
  int prec = SIPG_F64;
  int ec = 0;  // 0 none, 1 both operands split, 2 matrix operand split
  float* d_tabf = nullptr;
  std::vector<float*> fx, fb, fr;
  std::vector<int> order;  // tile order of the apply per level (autotuned; 0 = default)
  sipg_cnn* cnn = nullptr;  // learned correction stage (borrowed; see sipg_cnn_attach)
  double* stage_c = nullptr;  // the stage's correction and its image under A (finest level)
  double* stage_q = nullptr;
  // general geometry (sipg_set_geometry): per-level vertices and face penalties
  bool mapped = false;
  double* d_mtab = nullptr;
  std::vector<double*> geo_vert, geo_gam;
};

namespace sipg {
inline double level_h(const sipg_problem* p, int l) { return 1.0 / p->n[l]; }

inline sipg_status cartesian_only(const sipg_problem* p, const char* what) {
  if (p && p->mapped)
    return fail(SIPG_ERR_UNSUPPORTED, std::string(what) + " needs the Cartesian mesh (a geometry is set)");
  return SIPG_OK;
}

// Workspace of a problem handle: through the caller's allocator callbacks
// when the configuration names them, else hipMalloc / hipFree.
template <typename T>
sipg_status prob_alloc(sipg_problem* p, T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return SIPG_OK;
  const size_t bytes = count * sizeof(T);
  if (p->cfg.alloc) {
    *ptr = (T*)p->cfg.alloc(bytes, p->alloc_stream, p->cfg.alloc_ctx);
    if (!*ptr) return fail(SIPG_ERR_OOM, "allocator callback returned NULL");
    if (((uintptr_t)*ptr) & 255) {
      p->cfg.dealloc(*ptr, p->alloc_stream, p->cfg.alloc_ctx);
      *ptr = nullptr;
      return fail(SIPG_ERR_ARG, "allocator callback returned a block not aligned to 256 bytes");
    }
    return SIPG_OK;
  }
  return dev_alloc(ptr, count);
}
inline void prob_free(sipg_problem* p, void* ptr) {
  if (!ptr) return;
  if (p->cfg.dealloc) p->cfg.dealloc(ptr, p->alloc_stream, p->cfg.alloc_ctx);
  else hipFree(ptr);
}

sipg_status ensure_krylov(sipg_problem* p, int m);
// z += learned correction of the residual v - A z on the finest level
sipg_status cnn_stage(sipg_problem* p, const double* v, double* z, hipStream_t s);
}  // namespace sipg
