// C ABI of the library (include/sipg.h): the level hierarchy, the V-cycle
// (Alg. v_cycle) and the FP64 flexible GMRES outer iteration (Sec. 7.1) as
// host-side sequences of kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "problem.h"

using namespace sipg;

namespace sipg {
thread_local std::string g_err;
}  // namespace sipg

namespace {

sipg_status check_level(const sipg_problem* p, int level) {
  if (!p) return fail(SIPG_ERR_ARG, "NULL handle");
  if (level < 0 || level >= p->L) return fail(SIPG_ERR_ARG, "level out of range");
  return SIPG_OK;
}

int tile_order(const sipg_problem* p, int l) {
  return (l < (int)p->order.size()) ? p->order[l] : 0;
}

// the device geometry of level l (sipg_set_geometry)
MappedLevel mapped_level(const sipg_problem* p, int l) {
  MappedLevel g;
  g.vert = p->geo_vert[l];
  g.gam = p->geo_gam[l];
  g.n = p->n[l];
  return g;
}

// v = A_l u, or v = b - A_l u when b != nullptr: the Cartesian kernels, or the
// trilinear-cell kernel once a geometry is set
sipg_status op_apply(sipg_problem* p, int l, const double* u, double* v, const double* b,
                     hipStream_t s) {
  if (p->mapped) {
    SIPG_HIP(launch_apply_mapped(p->N, u, v, b, mapped_level(p, l), p->d_mtab, s));
    return SIPG_OK;
  }
  ApplyJob j{u, v, b, p->n[l], level_h(p, l), tile_order(p, l)};
  SIPG_HIP(launch_apply_batch(0, p->N, &j, 1, p->tab, s));
  return SIPG_OK;
}

sipg_status residual(sipg_problem* p, int l, const double* b, const double* x, double* r,
                     hipStream_t s) {
  return op_apply(p, l, x, r, b, s);
}

void free_geometry(sipg_problem* p) {
  for (auto q : p->geo_vert) prob_free(p, q);
  for (auto q : p->geo_gam) prob_free(p, q);
  p->geo_vert.clear();
  p->geo_gam.clear();
  prob_free(p, p->d_mtab);
  p->d_mtab = nullptr;
  p->mapped = false;
}

sipg_status smooth(sipg_problem* p, int l, double* x, const double* b, int sweeps,
                   hipStream_t s) {
  if (p->n[l] < 2) return SIPG_OK;
  if (p->cfg.smoother == 1) {  // additive: one residual, all patches, damped sum
    for (int sw = 0; sw < sweeps; ++sw) {
      SIPG_TRY(residual(p, l, b, x, p->wr[l], s));
      SIPG_HIP(launch_fill(p->wc[l], 0.0, p->ndofs[l], s));
      for (int colour = 0; colour < 8; ++colour)
        SIPG_HIP(launch_patch_fd_f64(p->N, colour, p->wr[l], p->wc[l], p->tab, p->n[l],
                                     level_h(p, l), s));
      SIPG_HIP(launch_axpy(p->cfg.damping, p->wc[l], x, p->ndofs[l], s));
    }
    return SIPG_OK;
  }
  if (p->cfg.smoother == 2) {  // fused colour steps, x and wr[l] in turn (8 per sweep)
    double* cur = x;
    double* other = p->wr[l];
    for (int sw = 0; sw < sweeps; ++sw)
      for (int colour = 0; colour < 8; ++colour) {
        PatchJob j{cur, other, p->n[l], level_h(p, l), b};
        SIPG_HIP(launch_patch_fd_batch(0, p->N, colour, &j, 1, p->tab, s));
        SIPG_HIP(launch_copy_uncovered(0, p->N, colour, cur, other, p->n[l], s));
        std::swap(cur, other);
      }
    return SIPG_OK;
  }
  for (int sw = 0; sw < sweeps; ++sw)
    for (int colour = 0; colour < 8; ++colour) {
      SIPG_TRY(residual(p, l, b, x, p->wr[l], s));
      SIPG_HIP(launch_patch_fd_f64(p->N, colour, p->wr[l], x, p->tab, p->n[l], level_h(p, l), s));
    }
  return SIPG_OK;
}

// ---- low-precision V-cycle on FP32 vectors
sipg_status residual_lp(sipg_problem* p, int l, const float* b, const float* x, float* r,
                        hipStream_t s) {
  if (p->prec == SIPG_F32 && p->mapped)
    SIPG_HIP(launch_apply_mapped_f32(p->N, x, r, b, mapped_level(p, l), p->d_mtab, s));
  else if (p->prec == SIPG_F32)
    SIPG_HIP(launch_residual_f32(p->N, x, r, b, p->tab, p->n[l], level_h(p, l), s));
  else
    SIPG_HIP(launch_apply_lp(p->N, p->prec == SIPG_BF16, p->ec, x, r, b, p->tab, p->n[l],
                             level_h(p, l), s));
  return SIPG_OK;
}

sipg_status patch_lp(sipg_problem* p, int l, int colour, const float* r, float* x,
                     hipStream_t s) {
  if (p->n[l] < 2) return SIPG_OK;
  if (p->prec == SIPG_F32)
    SIPG_HIP(launch_patch_fd_f32(p->N, colour, r, x, p->tab, p->n[l], level_h(p, l), s));
  else
    SIPG_HIP(launch_patch_fd_lp(p->N, p->prec == SIPG_BF16, p->ec, colour, r, x, p->tab,
                                p->n[l], level_h(p, l), s));
  return SIPG_OK;
}

sipg_status smooth_lp(sipg_problem* p, int l, float* x, const float* b, int sweeps,
                      hipStream_t s) {
  if (p->n[l] < 2) return SIPG_OK;
  if (p->prec == SIPG_F32 && p->cfg.smoother == 2) {  // fused colour steps (see smooth)
    float* cur = x;
    float* other = p->fr[l];
    for (int sw = 0; sw < sweeps; ++sw)
      for (int colour = 0; colour < 8; ++colour) {
        PatchJob j{cur, other, p->n[l], level_h(p, l), b};
        SIPG_HIP(launch_patch_fd_batch(1, p->N, colour, &j, 1, p->tab, s));
        SIPG_HIP(launch_copy_uncovered(1, p->N, colour, cur, other, p->n[l], s));
        std::swap(cur, other);
      }
    return SIPG_OK;
  }
  for (int sw = 0; sw < sweeps; ++sw)
    for (int colour = 0; colour < 8; ++colour) {
      SIPG_TRY(residual_lp(p, l, b, x, p->fr[l], s));
      SIPG_TRY(patch_lp(p, l, colour, p->fr[l], x, s));
    }
  return SIPG_OK;
}

sipg_status vcycle_lp(sipg_problem* p, int l, float* x, const float* b, hipStream_t s) {
  if (l == 0) {
    if (p->n0 > 3) return fail(SIPG_ERR_UNSUPPORTED, "coarsest level above 3 cells per direction");
    SIPG_HIP(launch_coarse_fd_f32(p->N, p->n0, b, x, p->tab, level_h(p, 0), s));
    return SIPG_OK;
  }
  SIPG_TRY(smooth_lp(p, l, x, b, p->cfg.nu_pre, s));
  SIPG_TRY(residual_lp(p, l, b, x, p->fr[l], s));
  SIPG_HIP(launch_restrict_f32(p->N, p->fr[l], p->fb[l - 1], p->tab, p->n[l - 1], s));
  if (l - 1 > 0) SIPG_HIP(launch_zero_f32(p->fx[l - 1], p->ndofs[l - 1], s));
  SIPG_TRY(vcycle_lp(p, l - 1, p->fx[l - 1], p->fb[l - 1], s));
  SIPG_HIP(launch_prolongate_add_f32(p->N, p->fx[l - 1], x, p->tab, p->n[l - 1], s));
  SIPG_TRY(smooth_lp(p, l, x, b, p->cfg.nu_post, s));
  return SIPG_OK;
}

sipg_status vcycle(sipg_problem* p, int l, double* x, const double* b, hipStream_t s);

// x <- V-cycle(x, b) in the handle's precision; FP64 in and out.  The
// low-precision cycle runs on FP32 copies (the format is converted at entry
// and exit of the V-cycle, Sec. 7.1).
sipg_status vcycle_any(sipg_problem* p, int l, double* x, const double* b, hipStream_t s) {
  if (p->prec == SIPG_F64) return vcycle(p, l, x, b, s);
  SIPG_HIP(launch_to_f32(b, p->fb[l], p->ndofs[l], s));
  SIPG_HIP(launch_to_f32(x, p->fx[l], p->ndofs[l], s));
  SIPG_TRY(vcycle_lp(p, l, p->fx[l], p->fb[l], s));
  SIPG_HIP(launch_to_f64(p->fx[l], x, p->ndofs[l], s));
  return SIPG_OK;
}

sipg_status vcycle(sipg_problem* p, int l, double* x, const double* b, hipStream_t s) {
  if (l == 0) {
    if (p->n0 > 3) return fail(SIPG_ERR_UNSUPPORTED, "coarsest level above 3 cells per direction");
    SIPG_HIP(launch_coarse_fd_f64(p->N, p->n0, b, x, p->tab, level_h(p, 0), s));
    return SIPG_OK;
  }
  SIPG_TRY(smooth(p, l, x, b, p->cfg.nu_pre, s));
  SIPG_TRY(residual(p, l, b, x, p->wr[l], s));
  SIPG_HIP(launch_restrict_f64(p->N, p->wr[l], p->wb[l - 1], p->tab, p->n[l - 1], s));
  if (l - 1 > 0) SIPG_HIP(launch_fill(p->wx[l - 1], 0.0, p->ndofs[l - 1], s));
  SIPG_TRY(vcycle(p, l - 1, p->wx[l - 1], p->wb[l - 1], s));
  SIPG_HIP(launch_prolongate_add_f64(p->N, p->wx[l - 1], x, p->tab, p->n[l - 1], s));
  SIPG_TRY(smooth(p, l, x, b, p->cfg.nu_post, s));
  return SIPG_OK;
}

// dot products of V[0..nv) with w; the result reaches the host through the
// handle's pinned buffer (stream-ordered copy, then a stream sync)
sipg_status mdot_host(sipg_problem* p, const double* V, int64_t ld, int nv, const double* w,
                      int64_t n, double* dev_out, double* host_out, hipStream_t s) {
  SIPG_HIP(launch_mdot(V, ld, nv, w, n, p->d_partial, dev_out, s));
  if (host_out) {
    SIPG_HIP(hipMemcpyAsync(p->h_pinned, dev_out, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
    SIPG_HIP(hipStreamSynchronize(s));
    std::memcpy(host_out, p->h_pinned, sizeof(double) * nv);
  }
  return SIPG_OK;
}

// An iteration whose residual estimate falls by less than this factor ends
// the learned stage for the rest of the solve.
constexpr double kStagnation = 0.9;

sipg_status ensure_aux(sipg_problem* p, size_t count) {
  if (count <= p->aux_size) return SIPG_OK;
  prob_free(p, p->d_aux);
  p->d_aux = nullptr;
  p->aux_size = 0;
  SIPG_TRY(prob_alloc(p, &p->d_aux, count));
  p->aux_size = count;
  return SIPG_OK;
}

// Sine modes and the nq-point quadrature table of the trilinear-cell RHS / L2
// error in the aux buffer: [n_modes][c, p, q, r] (c = amplitude, times
// pi^2 (p^2 + q^2 + r^2) for -Laplace u), then quad_table(k, nq).  Returns the
// offset of the quadrature table.
sipg_status upload_mapped_modes(sipg_problem* p, int n_modes, const double* amps, const int* pqr,
                                bool laplace, int nq, size_t* qoff, hipStream_t s) {
  std::vector<double> host((size_t)4 * n_modes);
  for (int m = 0; m < n_modes; ++m) {
    const double pp = pqr[3 * m], qq = pqr[3 * m + 1], rr = pqr[3 * m + 2];
    host[4 * m] = amps[m] * (laplace ? M_PI * M_PI * (pp * pp + qq * qq + rr * rr) : 1.0);
    host[4 * m + 1] = pp;
    host[4 * m + 2] = qq;
    host[4 * m + 3] = rr;
  }
  *qoff = host.size();
  const std::vector<double> qt = quad_table(p->k, nq);
  host.insert(host.end(), qt.begin(), qt.end());
  SIPG_TRY(ensure_aux(p, host.size()));
  SIPG_HIP(hipMemcpyAsync(p->d_aux, host.data(), host.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
  return SIPG_OK;
}

// Tables of the L2 error on a level of nl cells per direction with nq = k+3
// Gauss points: amps[n_modes], the mode values sin(p pi x) at every cell's
// points per direction [3][n_modes][nl][nq], the Lagrange values at the points
// [nq][N] and the weights [nq].
size_t l2_table_size(int n_modes, int nl, int nq, int N) {
  return (size_t)n_modes + 3 * (size_t)n_modes * nl * nq + (size_t)nq * N + nq;
}

void l2_fill_tables(const sipg_problem* p, int nl, int n_modes, const double* amps,
                    const int* pqr, double* host) {
  const int N = p->N, nq = p->k + 3;
  const double h = 1.0 / nl;
  const size_t tab = (size_t)n_modes * nl * nq;
  double* a = host;
  double* st[3] = {a + n_modes, a + n_modes + tab, a + n_modes + 2 * tab};
  double* ip = a + n_modes + 3 * tab;
  double* w = ip + (size_t)nq * N;
  for (int m = 0; m < n_modes; ++m) {
    a[m] = amps[m];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < nl; ++c)
        for (int q = 0; q < nq; ++q)
          st[d][((size_t)m * nl + c) * nq + q] =
              std::sin(pqr[3 * m + d] * M_PI * h * (c + p->l2_xq[q]));
  }
  for (int i = 0; i < nq * N; ++i) ip[i] = p->l2_V[i];
  for (int q = 0; q < nq; ++q) w[q] = p->l2_wq[q];
}

// sum over cells of the squared error into *out (device), tables at d
sipg_status l2_launch(const sipg_problem* p, int nl, int n_modes, const double* d,
                      const double* x, double* partial, double* out, hipStream_t s) {
  const int N = p->N, nq = p->k + 3;
  const size_t tab = (size_t)n_modes * nl * nq;
  SIPG_HIP(launch_l2_sines(N, nq, nl, n_modes, d, d + n_modes, d + n_modes + tab,
                           d + n_modes + 2 * tab, d + n_modes + 3 * tab,
                           d + n_modes + 3 * tab + (size_t)nq * N, 1.0 / nl, x, partial, out, s));
  return SIPG_OK;
}

}  // namespace

namespace sipg {
sipg_status ensure_krylov(sipg_problem* p, int m) {
  if (m <= p->restart_alloc) return SIPG_OK;
  const int64_t n = p->ndofs[p->L - 1];
  // the old blocks may still be read by queued work
  SIPG_HIP(hipDeviceSynchronize());
  prob_free(p, p->V);
  prob_free(p, p->Z);
  p->V = p->Z = nullptr;
  p->restart_alloc = 0;
  ++p->krylov_gen;  // anything that captured the old addresses is stale now
  SIPG_TRY(prob_alloc(p, &p->V, (size_t)(m + 1) * n));
  SIPG_TRY(prob_alloc(p, &p->Z, (size_t)m * n));
  p->restart_alloc = m;
  return SIPG_OK;
}
}  // namespace sipg

extern "C" {

const char* sipg_last_error(void) { return g_err.c_str(); }

sipg_status sipg_create(const sipg_config* cfg, hipStream_t stream, sipg_problem** out) {
  if (!cfg || !out) return fail(SIPG_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (cfg->k < 1 || cfg->k > 7) return fail(SIPG_ERR_ARG, "k must be in 1..7");
  if (cfg->n_cells < 1 || cfg->n_cells > 1024) return fail(SIPG_ERR_ARG, "n_cells must be in 1..1024");
  if (cfg->nu_pre < 0 || cfg->nu_post < 0 || cfg->nu_pre > 16 || cfg->nu_post > 16)
    return fail(SIPG_ERR_ARG, "smoothing steps must be in 0..16");
  if (cfg->mg_precision < SIPG_F64 || cfg->mg_precision > SIPG_BF16)
    return fail(SIPG_ERR_ARG, "mg_precision must be a sipg_precision");
  if (cfg->error_correction < 0 || cfg->error_correction > 2)
    return fail(SIPG_ERR_ARG, "error_correction must be 0, 1 or 2");
  const double pen = cfg->penalty_scale == 0.0 ? 1.0 : cfg->penalty_scale;
  if (!(pen >= 1.0 && pen <= 100.0)) return fail(SIPG_ERR_ARG, "penalty_scale must be 0 or in [1, 100]");
  if ((cfg->alloc == nullptr) != (cfg->dealloc == nullptr))
    return fail(SIPG_ERR_ARG, "alloc and dealloc must be given together");
  if (cfg->mg_precision == SIPG_BF16 && cfg->error_correction == 0 && cfg->k >= 5)
    return fail(SIPG_ERR_UNSUPPORTED,
                "BF16 V-cycle without error correction stalls for k >= 5 (the 1D operator "
                "rounded to 8 significand bits moves the lowest eigenvalues by many times their "
                "size); use error_correction 1 or 2");
  if (cfg->smoother < 0 || cfg->smoother > 2) return fail(SIPG_ERR_ARG, "smoother must be 0, 1 or 2");
  if (cfg->smoother == 1 && cfg->mg_precision != SIPG_F64)
    return fail(SIPG_ERR_UNSUPPORTED, "the additive smoother runs in FP64 only");
  if (cfg->damping < 0.0 || cfg->damping > 1.0) return fail(SIPG_ERR_ARG, "damping must be in [0, 1]");
  // Default hierarchy: halve while even and above 3 (coarsest 2 for powers of
  // two, 3 for three times a power of two); n_levels > 0 takes that many of
  // the finest levels of the full halving sequence (down to 1 cell).  A
  // coarsest level above 3 cells per direction is allowed for operator work;
  // its exact coarse solve then reports SIPG_ERR_UNSUPPORTED.
  std::vector<int> ns{cfg->n_cells};
  while (ns.back() % 2 == 0) ns.push_back(ns.back() / 2);
  std::vector<int> lv(ns.rbegin(), ns.rend());
  if (cfg->n_levels < 0) return fail(SIPG_ERR_ARG, "n_levels must be >= 0");
  if (cfg->n_levels > 0) {
    if (cfg->n_levels > (int)lv.size()) return fail(SIPG_ERR_ARG, "too many levels for n_cells");
    lv.erase(lv.begin(), lv.end() - cfg->n_levels);
  } else if (lv.size() > 1 && lv.front() == 1) {
    lv.erase(lv.begin());  // powers of two stop at 2 cells
  }
  auto* p = new sipg_problem();
  p->cfg = *cfg;
  p->cfg.penalty_scale = pen;
  if (p->cfg.damping == 0.0) p->cfg.damping = 0.125;
  p->alloc_stream = stream;
  p->k = cfg->k;
  p->N = cfg->k + 1;
  p->n = lv;
  p->L = (int)lv.size();
  p->n0 = lv.front();
  const int64_t N3 = (int64_t)p->N * p->N * p->N;
  for (int m : lv) p->ndofs.push_back((int64_t)m * m * m * N3);
  std::vector<double> tab;
  try {
    tab = build_device_table(p->k, p->n0, p->tab.lay, pen);
  } catch (const std::exception& e) {
    delete p;
    return fail(SIPG_ERR_ARG, e.what());
  }
  gauss_legendre(p->k + 3, p->l2_xq, p->l2_wq);  // L2 error rule
  lagrange_eval(make_tables_1d(p->k).nodes, p->l2_xq, p->l2_V, nullptr);
  std::vector<float> tf(tab.begin(), tab.end());  // FP32 copy (FP32 / FP16 / BF16 kernels)
  sipg_status st = prob_alloc(p, &p->d_tab, tab.size());
  if (st == SIPG_OK) st = prob_alloc(p, &p->d_tabf, tf.size());
  if (st == SIPG_OK && (hipMemcpyAsync(p->d_tab, tab.data(), tab.size() * sizeof(double),
                                       hipMemcpyHostToDevice, stream) != hipSuccess ||
                        hipMemcpyAsync(p->d_tabf, tf.data(), tf.size() * sizeof(float),
                                       hipMemcpyHostToDevice, stream) != hipSuccess ||
                        hipStreamSynchronize(stream) != hipSuccess))
    st = fail(SIPG_ERR_HIP, "table upload failed");
  p->tab.tab = p->d_tab;
  p->tab.tabf = p->d_tabf;
  p->wx.assign(p->L, nullptr);
  p->wb.assign(p->L, nullptr);
  p->wr.assign(p->L, nullptr);
  p->wc.assign(p->L, nullptr);
  for (int l = 0; l < p->L && st == SIPG_OK; ++l) {
    st = prob_alloc(p, &p->wr[l], p->ndofs[l]);
    if (st == SIPG_OK && cfg->smoother == 1) st = prob_alloc(p, &p->wc[l], p->ndofs[l]);
    if (st == SIPG_OK && l < p->L - 1) st = prob_alloc(p, &p->wx[l], p->ndofs[l]);
    if (st == SIPG_OK && l < p->L - 1) st = prob_alloc(p, &p->wb[l], p->ndofs[l]);
  }
  p->prec = cfg->mg_precision;
  p->ec = cfg->error_correction;
  p->fx.assign(p->L, nullptr);
  p->fb.assign(p->L, nullptr);
  p->fr.assign(p->L, nullptr);
  if (p->prec != SIPG_F64)
    for (int l = 0; l < p->L && st == SIPG_OK; ++l) {
      st = prob_alloc(p, &p->fx[l], p->ndofs[l]);
      if (st == SIPG_OK) st = prob_alloc(p, &p->fb[l], p->ndofs[l]);
      if (st == SIPG_OK) st = prob_alloc(p, &p->fr[l], p->ndofs[l]);
    }
  if (st == SIPG_OK) st = prob_alloc(p, &p->d_partial, (size_t)kDotBlocks * 65);
  if (st == SIPG_OK) st = prob_alloc(p, &p->d_small, 512);
  if (st == SIPG_OK) st = prob_alloc(p, &p->d_flag, 64);
  if (st == SIPG_OK && hipHostMalloc((void**)&p->h_pinned, 256 * sizeof(double)) != hipSuccess) {
    p->h_pinned = nullptr;
    st = fail(SIPG_ERR_HIP, "pinned host buffer allocation failed");
  }
  if (st != SIPG_OK) {
    std::string msg = g_err;
    sipg_destroy(p);
    return fail(st, msg);
  }
  *out = p;
  return SIPG_OK;
}

void sipg_destroy(sipg_problem* p) {
  if (!p) return;
  hipDeviceSynchronize();
  prob_free(p, p->d_tab);
  for (auto q : p->wx) prob_free(p, q);
  for (auto q : p->wb) prob_free(p, q);
  for (auto q : p->wr) prob_free(p, q);
  for (auto q : p->wc) prob_free(p, q);
  prob_free(p, p->V);
  prob_free(p, p->Z);
  prob_free(p, p->d_partial);
  prob_free(p, p->d_small);
  prob_free(p, p->d_flag);
  prob_free(p, p->d_aux);
  prob_free(p, p->d_tabf);
  for (auto q : p->fx) prob_free(p, q);
  for (auto q : p->fb) prob_free(p, q);
  for (auto q : p->fr) prob_free(p, q);
  prob_free(p, p->stage_c);
  prob_free(p, p->stage_q);
  free_geometry(p);
  if (p->h_pinned) hipHostFree(p->h_pinned);
  delete p;
}

int sipg_num_levels(const sipg_problem* p) { return p ? p->L : -1; }

int sipg_level_cells(const sipg_problem* p, int level) {
  if (!p || level < 0 || level >= p->L) return -1;
  return p->n[level];
}

int64_t sipg_n_dofs(const sipg_problem* p, int level) {
  if (!p || level < 0 || level >= p->L) return -1;
  return p->ndofs[level];
}

sipg_status sipg_apply(sipg_problem* p, int level, const double* u, double* v, hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (!u || !v) return fail(SIPG_ERR_ARG, "NULL vector");
  if (u == v) return fail(SIPG_ERR_ARG, "u and v must not alias");
  return op_apply(p, level, u, v, nullptr, s);
}

sipg_status sipg_set_geometry(sipg_problem* p, const double* vertices, hipStream_t s) {
  if (!p) return fail(SIPG_ERR_ARG, "NULL handle");
  if (!vertices) {
    SIPG_HIP(hipStreamSynchronize(s));
    free_geometry(p);
    return SIPG_OK;
  }
  if ((p->prec != SIPG_F64 && p->prec != SIPG_F32) || p->cfg.smoother == 2)
    return fail(SIPG_ERR_UNSUPPORTED,
                "general geometry needs mg_precision SIPG_F64 or SIPG_F32 and smoother 0 or 1");
  const int L = p->L, nf = p->n[L - 1];
  const size_t nf1 = (size_t)nf + 1;
  std::vector<std::vector<double>> verts(L), gams(L);
  for (int l = 0; l < L; ++l) {
    const int nl = p->n[l], stp = nf / nl;
    const size_t n1 = (size_t)nl + 1;
    std::vector<double>& V = verts[l];
    V.resize(n1 * n1 * n1 * 3);
    for (size_t z = 0; z < n1; ++z)
      for (size_t y = 0; y < n1; ++y)
        for (size_t x = 0; x < n1; ++x)
          for (int i = 0; i < 3; ++i)
            V[((z * n1 + y) * n1 + x) * 3 + i] =
                vertices[(((z * stp) * nf1 + y * stp) * nf1 + x * stp) * 3 + i];
    for (double d : V)
      if (!std::isfinite(d)) return fail(SIPG_ERR_ARG, "vertex positions must be finite");
    std::string err;
    if (!mapped_penalties(p->k, nl, V.data(), p->cfg.penalty_scale, gams[l], err))
      return fail(SIPG_ERR_ARG, "level " + std::to_string(l) + ": " + err);
  }
  SIPG_HIP(hipStreamSynchronize(s));
  free_geometry(p);
  const std::vector<double> mt = mapped_table(p->k);
  sipg_status st = prob_alloc(p, &p->d_mtab, mt.size());
  p->geo_vert.assign(L, nullptr);
  p->geo_gam.assign(L, nullptr);
  for (int l = 0; l < L && st == SIPG_OK; ++l) {
    st = prob_alloc(p, &p->geo_vert[l], verts[l].size());
    if (st == SIPG_OK) st = prob_alloc(p, &p->geo_gam[l], gams[l].size());
  }
  if (st != SIPG_OK) {
    std::string msg = g_err;
    free_geometry(p);
    return fail(st, msg);
  }
  bool ok = hipMemcpyAsync(p->d_mtab, mt.data(), mt.size() * sizeof(double),
                           hipMemcpyHostToDevice, s) == hipSuccess;
  for (int l = 0; l < L && ok; ++l)
    ok = hipMemcpyAsync(p->geo_vert[l], verts[l].data(), verts[l].size() * sizeof(double),
                        hipMemcpyHostToDevice, s) == hipSuccess &&
         hipMemcpyAsync(p->geo_gam[l], gams[l].data(), gams[l].size() * sizeof(double),
                        hipMemcpyHostToDevice, s) == hipSuccess;
  if (!ok || hipStreamSynchronize(s) != hipSuccess) {
    free_geometry(p);
    return fail(SIPG_ERR_HIP, "geometry upload failed");
  }
  p->mapped = true;
  return SIPG_OK;
}

sipg_status sipg_apply_units(sipg_problem* p, int level, const double* u, double* v, int units,
                             hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  SIPG_TRY(cartesian_only(p, "sipg_apply_units"));
  if (!u || !v) return fail(SIPG_ERR_ARG, "NULL vector");
  if (u == v) return fail(SIPG_ERR_ARG, "u and v must not alias");
  if (units < SIPG_UNITS_AUTO || units > SIPG_UNITS_MATRIX)
    return fail(SIPG_ERR_ARG, "units must be a sipg_units");
  const bool has_matrix = p->N == 4 || p->N == 8;
  if (units == SIPG_UNITS_MATRIX && !has_matrix)
    return fail(SIPG_ERR_UNSUPPORTED, "the FP64 matrix-core apply exists for k = 3 and 7 only");
  ApplyJob j{u, v, nullptr, p->n[level], level_h(p, level), tile_order(p, level)};
  SIPG_HIP(launch_apply_batch(units == SIPG_UNITS_VECTOR ? 2 : 0, p->N, &j, 1, p->tab, s));
  return SIPG_OK;
}

sipg_status sipg_apply_patchwise(sipg_problem* p, int level, const double* u, double* v,
                                 hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  SIPG_TRY(cartesian_only(p, "sipg_apply_patchwise"));
  if (!u || !v) return fail(SIPG_ERR_ARG, "NULL vector");
  if (u == v) return fail(SIPG_ERR_ARG, "u and v must not alias");
  if (p->n[level] < 2) return fail(SIPG_ERR_ARG, "patch-wise evaluation needs n >= 2 cells");
  SIPG_HIP(launch_fill(v, 0.0, p->ndofs[level], s));
  for (int colour = 0; colour < 8; ++colour)
    SIPG_HIP(launch_patch_apply_f64(p->N, colour, u, v, p->tab, p->n[level], level_h(p, level), s));
  return SIPG_OK;
}

sipg_status sipg_residual(sipg_problem* p, int level, const double* b, const double* x, double* r,
                          hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (!b || !x || !r) return fail(SIPG_ERR_ARG, "NULL vector");
  if (r == x || r == b) return fail(SIPG_ERR_ARG, "r must not alias x or b");
  return residual(p, level, b, x, r, s);
}

sipg_status sipg_smooth(sipg_problem* p, int level, double* x, const double* b, int sweeps,
                        hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (!x || !b) return fail(SIPG_ERR_ARG, "NULL vector");
  if (x == b) return fail(SIPG_ERR_ARG, "x and b must not alias");
  if (sweeps < 0) return fail(SIPG_ERR_ARG, "sweeps must be >= 0");
  return smooth(p, level, x, b, sweeps, s);
}

sipg_status sipg_patch_correct(sipg_problem* p, int level, int colour, const double* r, double* x,
                               hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (!x || !r) return fail(SIPG_ERR_ARG, "NULL vector");
  if (x == r) return fail(SIPG_ERR_ARG, "x and r must not alias");
  if (colour < 0 || colour > 7) return fail(SIPG_ERR_ARG, "colour must be in 0..7");
  if (p->n[level] < 2) return SIPG_OK;
  SIPG_HIP(launch_patch_fd_f64(p->N, colour, r, x, p->tab, p->n[level], level_h(p, level), s));
  return SIPG_OK;
}

sipg_status sipg_smooth_lp(sipg_problem* p, int level, float* x, const float* b, int sweeps,
                           hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (p->prec == SIPG_F64) return fail(SIPG_ERR_ARG, "the handle's mg_precision is FP64");
  if (!x || !b) return fail(SIPG_ERR_ARG, "NULL vector");
  if ((const void*)x == (const void*)b) return fail(SIPG_ERR_ARG, "x and b must not alias");
  if (sweeps < 0) return fail(SIPG_ERR_ARG, "sweeps must be >= 0");
  return smooth_lp(p, level, x, b, sweeps, s);
}

sipg_status sipg_patch_correct_lp(sipg_problem* p, int level, int colour, const float* r, float* x,
                                  hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (p->prec == SIPG_F64) return fail(SIPG_ERR_ARG, "the handle's mg_precision is FP64");
  if (!x || !r) return fail(SIPG_ERR_ARG, "NULL vector");
  if ((const void*)x == (const void*)r) return fail(SIPG_ERR_ARG, "x and r must not alias");
  if (colour < 0 || colour > 7) return fail(SIPG_ERR_ARG, "colour must be in 0..7");
  return patch_lp(p, level, colour, r, x, s);
}

sipg_status sipg_restrict(sipg_problem* p, int level, const double* rf, double* rc,
                          hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (level < 1) return fail(SIPG_ERR_ARG, "restrict needs a fine level >= 1");
  if (!rf || !rc) return fail(SIPG_ERR_ARG, "NULL vector");
  SIPG_HIP(launch_restrict_f64(p->N, rf, rc, p->tab, p->n[level - 1], s));
  return SIPG_OK;
}

sipg_status sipg_prolongate_add(sipg_problem* p, int level, const double* ec, double* xf,
                                hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (level < 1) return fail(SIPG_ERR_ARG, "prolongate needs a fine level >= 1");
  if (!ec || !xf) return fail(SIPG_ERR_ARG, "NULL vector");
  SIPG_HIP(launch_prolongate_add_f64(p->N, ec, xf, p->tab, p->n[level - 1], s));
  return SIPG_OK;
}

sipg_status sipg_coarse_solve(sipg_problem* p, const double* b, double* x, hipStream_t s) {
  if (!p) return fail(SIPG_ERR_ARG, "NULL handle");
  if (!b || !x) return fail(SIPG_ERR_ARG, "NULL vector");
  if (b == x) return fail(SIPG_ERR_ARG, "x and b must not alias");
  if (p->n0 > 3) return fail(SIPG_ERR_UNSUPPORTED, "coarsest level above 3 cells per direction");
  SIPG_HIP(launch_coarse_fd_f64(p->N, p->n0, b, x, p->tab, level_h(p, 0), s));
  return SIPG_OK;
}

sipg_status sipg_vcycle(sipg_problem* p, int level, double* x, const double* b, hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (!x || !b) return fail(SIPG_ERR_ARG, "NULL vector");
  if (x == b) return fail(SIPG_ERR_ARG, "x and b must not alias");
  return vcycle_any(p, level, x, b, s);
}

sipg_status sipg_autotune(sipg_problem* p, int level, const double* u, double* v, int* best,
                          hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  SIPG_TRY(cartesian_only(p, "sipg_autotune"));
  if (!u || !v || u == v) return fail(SIPG_ERR_ARG, "need two distinct vectors");
  const int nl = p->n[level];
  const int cand[4] = {1, 2, 4, 8};
  hipEvent_t e0, e1;
  SIPG_HIP(hipEventCreate(&e0));
  SIPG_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  int best_o = 0;
  for (int c : cand) {
    if (nl % c) continue;
    ApplyJob j{u, v, nullptr, nl, level_h(p, level), c};
    SIPG_HIP(launch_apply_batch(0, p->N, &j, 1, p->tab, s));  // warm-up
    SIPG_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 5; ++r) SIPG_HIP(launch_apply_batch(0, p->N, &j, 1, p->tab, s));
    SIPG_HIP(hipEventRecord(e1, s));
    SIPG_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    SIPG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best_o = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if ((int)p->order.size() < p->L) p->order.assign(p->L, 0);
  p->order[level] = best_o;
  if (best) *best = best_o;
  return SIPG_OK;
}

sipg_status sipg_apply_lp(sipg_problem* p, int level, const float* u, float* v, int precision,
                          int ec, hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  SIPG_TRY(cartesian_only(p, "sipg_apply_lp"));
  if (!u || !v) return fail(SIPG_ERR_ARG, "NULL vector");
  if (u == v) return fail(SIPG_ERR_ARG, "u and v must not alias");
  if (precision == SIPG_F32) {
    SIPG_HIP(launch_apply_f32(p->N, u, v, nullptr, p->tab, p->n[level], level_h(p, level), s));
  } else if (precision == SIPG_F16 || precision == SIPG_BF16) {
    if (ec < 0 || ec > 2) return fail(SIPG_ERR_ARG, "ec must be 0, 1 or 2");
    SIPG_HIP(launch_apply_lp(p->N, precision == SIPG_BF16, ec, u, v, nullptr, p->tab,
                             p->n[level], level_h(p, level), s));
  } else {
    return fail(SIPG_ERR_ARG, "precision must be SIPG_F32, SIPG_F16 or SIPG_BF16");
  }
  return SIPG_OK;
}

sipg_status sipg_fgmres(sipg_problem* p, double* x, const double* b, const sipg_solve_opts* o,
                        sipg_solve_info* info, hipStream_t s) {
  if (!p || !x || !b || !o || !info) return fail(SIPG_ERR_ARG, "NULL argument");
  if (x == b) return fail(SIPG_ERR_ARG, "x and b must not alias");
  if (o->restart < 1 || o->restart > 64) return fail(SIPG_ERR_ARG, "restart must be in 1..64");
  if (o->max_iters < 1) return fail(SIPG_ERR_ARG, "max_iters must be >= 1");
  if (!(o->rtol > 0.0)) return fail(SIPG_ERR_ARG, "rtol must be > 0");
  if (o->use_learned && !p->cnn) return fail(SIPG_ERR_ARG, "use_learned set but no network attached");
  if (o->use_learned) SIPG_TRY(cartesian_only(p, "the learned stage"));
  if (o->variant != SIPG_FGMRES && o->variant != SIPG_GMRES)
    return fail(SIPG_ERR_ARG, "variant must be SIPG_FGMRES or SIPG_GMRES");
  if (o->variant == SIPG_GMRES && o->use_learned)
    return fail(SIPG_ERR_ARG, "the learned stage needs the flexible variant");
  std::memset(info, 0, sizeof(*info));
  bool learned = o->use_learned != 0;
  const double stagnation = o->stagnation > 0.0 ? o->stagnation : kStagnation;
  const int m = o->restart;
  const int L = p->L - 1;
  const int64_t n = p->ndofs[L];
  SIPG_TRY(ensure_krylov(p, std::max(m, 2)));  // GMRES uses two Z slots as scratch
  SIPG_HIP(hipStreamSynchronize(s));
  const auto t0 = std::chrono::steady_clock::now();
  double* d_h = p->d_small;        // [0, 65)
  double* d_h2 = p->d_small + 80;  // [80, 145)
  double* d_nrm = p->d_small + 160;
  double nb2 = 0.0;
  SIPG_TRY(mdot_host(p, b, n, 1, b, n, d_nrm, &nb2, s));
  const double nb = std::sqrt(nb2);
  if (!std::isfinite(nb)) return fail(SIPG_ERR_NONFINITE, "right-hand side is not finite");
  if (nb == 0.0) {
    SIPG_HIP(launch_fill(x, 0.0, n, s));
    SIPG_HIP(hipStreamSynchronize(s));
    return SIPG_OK;
  }
  const double tol = o->rtol * nb;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  auto Hm = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  int it = 0, hist = 0;
  bool converged = false;
  double est = 1.0, prev_est = 1.0;
  auto record = [&](double v) {
    prev_est = est;
    est = v;
    if (o->log_history && hist < 128) info->history[hist] = v;
    ++hist;
  };
  const bool flexible = o->variant == SIPG_FGMRES;
  while (it < o->max_iters && !converged) {
    SIPG_TRY(residual(p, L, b, x, p->V, s));
    double beta2 = 0.0;
    SIPG_TRY(mdot_host(p, p->V, n, 1, p->V, n, d_nrm, &beta2, s));
    const double beta = std::sqrt(beta2);
    if (!std::isfinite(beta)) return fail(SIPG_ERR_NONFINITE, "residual is not finite");
    record(beta / nb);
    if (beta <= tol) {
      converged = true;
      break;
    }
    SIPG_HIP(launch_scale_copy(p->V, 1.0 / beta, p->V, n, s));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jd = 0;
    for (int j = 0; j < m; ++j) {
      double* Vj = p->V + (size_t)j * n;
      // FGMRES keeps every preconditioned vector; GMRES one scratch slot
      double* Zj = p->Z + (size_t)(flexible ? j : 0) * n;
      double* w = p->V + (size_t)(j + 1) * n;
      // 0: the configured preconditioner; 1: plain V-cycle after a non-finite
      // learned correction; 2: identity after a non-finite V-cycle
      int mode = 0;
      double hn = 0.0;
      while (true) {
        SIPG_HIP(launch_fill(Zj, 0.0, n, s));
        if (mode < 2) SIPG_TRY(vcycle_any(p, L, Zj, Vj, s));
        else SIPG_HIP(launch_scale_copy(Vj, 1.0, Zj, n, s));
        if (mode == 0 && learned) SIPG_TRY(cnn_stage(p, Vj, Zj, s));
        SIPG_TRY(op_apply(p, L, Zj, w, nullptr, s));
        // classical Gram-Schmidt, twice; the Hessenberg column and ||w||^2
        // come back in one stream-ordered copy (a NaN or Inf in z shows up
        // there, so no separate check is needed)
        SIPG_HIP(launch_mdot(p->V, n, j + 1, w, n, p->d_partial, d_h, s));
        SIPG_HIP(launch_maxpy(p->V, n, j + 1, d_h, w, n, nullptr, 1.0, s));
        SIPG_HIP(launch_mdot(p->V, n, j + 1, w, n, p->d_partial, d_h2, s));
        SIPG_HIP(launch_maxpy(p->V, n, j + 1, d_h2, w, n, d_h, 1.0, s));
        SIPG_HIP(launch_mdot(w, n, 1, w, n, p->d_partial, d_h + 70, s));
        SIPG_HIP(hipMemcpyAsync(p->h_pinned, d_h, sizeof(double) * 71, hipMemcpyDeviceToHost, s));
        SIPG_HIP(hipStreamSynchronize(s));
        hn = std::sqrt(p->h_pinned[70]);
        bool finite = std::isfinite(hn);
        for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(p->h_pinned[i]);
        if (finite) break;
        if (mode == 0 && learned) {  // the learned stage failed: plain V-cycle from here on
          learned = false;
          mode = 1;
        } else if (mode < 2) {       // the preconditioner broke down: identity for this step
          mode = 2;
        } else {
          return fail(SIPG_ERR_NONFINITE, "Arnoldi vector is not finite");
        }
        info->fell_back = 1;
      }
      for (int i = 0; i <= j; ++i) Hm(i, j) = p->h_pinned[i];
      Hm(j + 1, j) = hn;
      if (hn > 0.0) SIPG_HIP(launch_scale_copy(w, 1.0 / hn, w, n, s));
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hm(i, j) + sn[i] * Hm(i + 1, j);
        Hm(i + 1, j) = -sn[i] * Hm(i, j) + cs[i] * Hm(i + 1, j);
        Hm(i, j) = t;
      }
      const double den = std::hypot(Hm(j, j), Hm(j + 1, j));
      cs[j] = Hm(j, j) / den;
      sn[j] = Hm(j + 1, j) / den;
      Hm(j, j) = den;
      Hm(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      jd = j + 1;
      record(std::fabs(g[j + 1]) / nb);
      if (learned && !(est <= stagnation * prev_est)) {  // stagnation: drop the learned stage
        learned = false;
        info->fell_back = 1;
      }
      if (std::fabs(g[j + 1]) <= tol || it >= o->max_iters || den == 0.0) break;
    }
    for (int i = jd - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int c = i + 1; c < jd; ++c) sacc -= Hm(i, c) * y[c];
      y[i] = sacc / Hm(i, i);
    }
    std::memcpy(p->h_pinned + 128, y.data(), sizeof(double) * jd);
    SIPG_HIP(hipMemcpyAsync(p->d_small + 192, p->h_pinned + 128, sizeof(double) * jd,
                            hipMemcpyHostToDevice, s));
    if (flexible) {  // x += Z y
      SIPG_HIP(launch_maxpy(p->Z, n, jd, p->d_small + 192, x, n, nullptr, -1.0, s));
    } else {  // x += M (V y): one more preconditioner application
      double* t = p->Z + (size_t)n;
      SIPG_HIP(launch_fill(t, 0.0, n, s));
      SIPG_HIP(launch_maxpy(p->V, n, jd, p->d_small + 192, t, n, nullptr, -1.0, s));
      SIPG_HIP(launch_fill(p->Z, 0.0, n, s));
      SIPG_TRY(vcycle_any(p, L, p->Z, t, s));
      SIPG_HIP(launch_axpy(1.0, p->Z, x, n, s));
    }
    // the copy above reads the pinned buffer: let it finish before reuse
    SIPG_HIP(hipStreamSynchronize(s));
    if (std::fabs(g[jd]) <= tol) converged = true;
  }
  SIPG_TRY(residual(p, L, b, x, p->V, s));
  double rr = 0.0;
  SIPG_TRY(mdot_host(p, p->V, n, 1, p->V, n, d_nrm, &rr, s));
  const auto t1 = std::chrono::steady_clock::now();
  info->iterations = it;
  info->rel_res_est = est;
  info->rel_res_true = std::sqrt(rr) / nb;
  info->seconds = std::chrono::duration<double>(t1 - t0).count();
  if (!converged) return fail(SIPG_ERR_NOT_CONVERGED, "iteration limit reached");
  return SIPG_OK;
}

sipg_status sipg_rhs_sines(sipg_problem* p, int level, int n_modes, const double* amps,
                           const int* pqr, double* b, hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (n_modes < 1 || n_modes > 64 || !amps || !pqr || !b) return fail(SIPG_ERR_ARG, "bad modes");
  if (p->mapped) {  // trilinear cells: f at every quadrature point, det J weights
    size_t qoff = 0;
    SIPG_TRY(upload_mapped_modes(p, n_modes, amps, pqr, true, p->k + 2, &qoff, s));
    SIPG_HIP(launch_rhs_mapped(p->N, mapped_level(p, level), n_modes, p->d_aux, p->d_aux + qoff,
                               b, s));
    SIPG_HIP(hipStreamSynchronize(s));
    return SIPG_OK;
  }
  const int N = p->N, nl = p->n[level];
  const double h = 1.0 / nl;
  std::vector<double> nodes = make_tables_1d(p->k).nodes, xq, wq, V;
  gauss_legendre(p->k + 2, xq, wq);
  lagrange_eval(nodes, xq, V, nullptr);
  const int nq = p->k + 2;
  // coef, bx, by, bz
  std::vector<double> host((size_t)n_modes * (1 + 3 * nl * N));
  double* coef = host.data();
  double* bt[3] = {coef + n_modes, coef + n_modes + (size_t)n_modes * nl * N,
                   coef + n_modes + 2 * (size_t)n_modes * nl * N};
  for (int m = 0; m < n_modes; ++m) {
    const double lam = M_PI * M_PI * ((double)pqr[3 * m] * pqr[3 * m] +
                                      (double)pqr[3 * m + 1] * pqr[3 * m + 1] +
                                      (double)pqr[3 * m + 2] * pqr[3 * m + 2]);
    coef[m] = amps[m] * lam;
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < nl; ++c)
        for (int i = 0; i < N; ++i) {
          double acc = 0.0;
          for (int q = 0; q < nq; ++q)
            acc += wq[q] * std::sin(pqr[3 * m + d] * M_PI * h * (c + xq[q])) * V[q * N + i];
          bt[d][((size_t)m * nl + c) * N + i] = h * acc;
        }
  }
  SIPG_TRY(ensure_aux(p, host.size()));
  SIPG_HIP(hipMemcpyAsync(p->d_aux, host.data(), host.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
  const double* dc = p->d_aux;
  SIPG_HIP(launch_rhs_sines(N, nl, n_modes, dc, dc + n_modes, dc + n_modes + (size_t)n_modes * nl * N,
                            dc + n_modes + 2 * (size_t)n_modes * nl * N, b, s));
  SIPG_HIP(hipStreamSynchronize(s));
  return SIPG_OK;
}

sipg_status sipg_l2_error_sines(sipg_problem* p, int level, int n_modes, const double* amps,
                                const int* pqr, const double* x, double* err, hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  if (n_modes < 1 || n_modes > 64 || !amps || !pqr || !x || !err)
    return fail(SIPG_ERR_ARG, "bad modes");
  if (p->mapped) {
    size_t qoff = 0;
    SIPG_TRY(upload_mapped_modes(p, n_modes, amps, pqr, false, p->k + 3, &qoff, s));
    SIPG_HIP(launch_l2_mapped(p->N, mapped_level(p, level), n_modes, p->d_aux, p->d_aux + qoff,
                              x, p->d_partial, kDotBlocks, p->d_small + 300, s));
    double e2 = 0.0;
    SIPG_HIP(hipMemcpyAsync(&e2, p->d_small + 300, sizeof(double), hipMemcpyDeviceToHost, s));
    SIPG_HIP(hipStreamSynchronize(s));
    *err = std::sqrt(e2);
    return SIPG_OK;
  }
  const int N = p->N, nl = p->n[level], nq = p->k + 3;
  std::vector<double> host(l2_table_size(n_modes, nl, nq, N));
  l2_fill_tables(p, nl, n_modes, amps, pqr, host.data());
  SIPG_TRY(ensure_aux(p, host.size()));
  SIPG_HIP(hipMemcpyAsync(p->d_aux, host.data(), host.size() * sizeof(double),
                          hipMemcpyHostToDevice, s));
  SIPG_TRY(l2_launch(p, nl, n_modes, p->d_aux, x, p->d_partial, p->d_small + 300, s));
  double e2 = 0.0;
  SIPG_HIP(hipMemcpyAsync(&e2, p->d_small + 300, sizeof(double), hipMemcpyDeviceToHost, s));
  SIPG_HIP(hipStreamSynchronize(s));
  *err = std::sqrt(e2);
  return SIPG_OK;
}

sipg_status sipg_l2_error_sines_noalloc(sipg_problem* p, int level, int n_modes,
                                        const double* amps, const int* pqr, const double* x,
                                        double* err, hipStream_t s) {
  SIPG_TRY(check_level(p, level));
  SIPG_TRY(cartesian_only(p, "sipg_l2_error_sines_noalloc"));
  if (n_modes < 1 || n_modes > 64 || !amps || !pqr || !x || !err)
    return fail(SIPG_ERR_ARG, "bad modes");
  const int N = p->N, nl = p->n[level], nq = p->k + 3;
  // scratch: tables, then kDotBlocks partial sums and the result (256-byte aligned)
  const size_t tab = l2_table_size(n_modes, nl, nq, N);
  const size_t off_part = (tab + 31) / 32 * 32, off_out = off_part + kDotBlocks;
  if (off_out + 1 > kL2ScratchDoubles)
    return fail(SIPG_ERR_ARG, "sipg_l2_error_sines_noalloc: " + std::to_string(tab) +
                                  " table entries exceed the fixed workspace's " +
                                  std::to_string((kL2ScratchDoubles - kDotBlocks - 1) / 32 * 32) +
                                  " (use sipg_l2_error_sines)");
  double* scr = nullptr;
  SIPG_HIP(l2_scratch(&scr));
  // host staging: one fixed buffer (hipMemcpyAsync from pageable memory has
  // copied it out before it returns), serialized across host threads
  static std::mutex mu;
  static double host[kL2ScratchDoubles];
  std::lock_guard<std::mutex> lock(mu);
  l2_fill_tables(p, nl, n_modes, amps, pqr, host);
  SIPG_HIP(hipMemcpyAsync(scr, host, tab * sizeof(double), hipMemcpyHostToDevice, s));
  SIPG_TRY(l2_launch(p, nl, n_modes, scr, x, scr + off_part, scr + off_out, s));
  double e2 = 0.0;
  SIPG_HIP(hipMemcpyAsync(&e2, scr + off_out, sizeof(double), hipMemcpyDeviceToHost, s));
  SIPG_HIP(hipStreamSynchronize(s));
  *err = std::sqrt(e2);
  return SIPG_OK;
}

}  // extern "C"
