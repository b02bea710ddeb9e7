// Batched Poisson solves: many independent problems of uneven size and
// degree advanced together.  Every stage of the V-cycle (Alg. v_cycle) and
// of the flexible GMRES iteration (Sec. 7.1) is issued as batched launches
// that cover all problems of one degree (up to 16 per launch, see batch.h),
// levels aligned by depth below the finest level; the V-cycle launch
// sequence of an iteration is captured once as a HIP graph on an internal
// stream and replayed.  The one-problem-at-a-time loop over sipg_fgmres is
// provided as the reference for timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "problem.h"

using namespace sipg;

struct sipg_batch {
  std::vector<sipg_problem*> P;
  std::vector<int> nodes;          // distinct N values present
  int prec = SIPG_F64;
  int ec = 0;
  int nu_pre = 2, nu_post = 2;
  hipStream_t stream = nullptr;    // internal capture stream (default priority)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::map<int, hipGraphExec_t> graphs;  // Krylov index j -> captured V-cycle
  std::map<int, hipGraphExec_t> steps;   // Krylov index j -> captured whole step (device scalars)
  std::vector<int> graph_gen;            // krylov_gen of every problem at capture
  double* h_pinned = nullptr;            // host scalars of all problems
  // device-scalar FGMRES: descriptors, state blocks, flags (device and pinned)
  KrylovDesc* d_kd = nullptr;
  double* d_st = nullptr;
  double* d_flags = nullptr;
  double* h_flags = nullptr;             // 3 slots of P x kFlagCount
  hipEvent_t ev_flags[2] = {nullptr, nullptr};
};

namespace {

// ---- batched launch helpers ----------------------------------------------
// An item = (problem, level).  Items are grouped by N and split into
// launches of at most kMaxBatch problems.
struct Item {
  int p, l;
};

template <typename Fn>
sipg_status for_groups(sipg_batch* B, const std::vector<Item>& items, Fn&& fn) {
  for (int N : B->nodes) {
    std::vector<Item> g;
    for (const Item& it : items)
      if (B->P[it.p]->N == N) g.push_back(it);
    for (size_t s0 = 0; s0 < g.size(); s0 += kMaxBatch) {
      const size_t cnt = std::min<size_t>(kMaxBatch, g.size() - s0);
      SIPG_TRY(fn(N, &g[s0], (int)cnt));
    }
  }
  return SIPG_OK;
}

bool lowp(const sipg_batch* B) { return B->prec != SIPG_F64; }

// Captured V-cycles hold vector addresses and tile orders by value.
void drop_graphs(sipg_batch* B) {
  for (auto& kv : B->graphs) hipGraphExecDestroy(kv.second);
  B->graphs.clear();
  for (auto& kv : B->steps) hipGraphExecDestroy(kv.second);
  B->steps.clear();
}

sipg_status cartesian_batch(const sipg_batch* B) {
  for (const sipg_problem* q : B->P)
    if (q->mapped) return fail(SIPG_ERR_UNSUPPORTED, "batches run on Cartesian meshes (a problem has a geometry)");
  return SIPG_OK;
}

// level vectors: x, b, r of problem p at level l (the finest x/b are given)
struct Vecs {
  std::vector<void*> x, b;  // finest-level x and b per problem
};

void* X(const sipg_batch* B, const Vecs& v, int p, int l) {
  const sipg_problem* q = B->P[p];
  if (l == q->L - 1) return v.x[p];
  return lowp(B) ? (void*)q->fx[l] : (void*)q->wx[l];
}
void* Bv(const sipg_batch* B, const Vecs& v, int p, int l) {
  const sipg_problem* q = B->P[p];
  if (l == q->L - 1) return v.b[p];
  return lowp(B) ? (void*)q->fb[l] : (void*)q->wb[l];
}
void* R(const sipg_batch* B, int p, int l) {
  const sipg_problem* q = B->P[p];
  return lowp(B) ? (void*)q->fr[l] : (void*)q->wr[l];
}

sipg_status b_residual(sipg_batch* B, const Vecs& v, const std::vector<Item>& items,
                       hipStream_t s) {
  return for_groups(B, items, [&](int N, const Item* it, int cnt) -> sipg_status {
    ApplyJob jobs[kMaxBatch];
    for (int i = 0; i < cnt; ++i) {
      const sipg_problem* q = B->P[it[i].p];
      const int l = it[i].l;
      jobs[i] = ApplyJob{X(B, v, it[i].p, l), R(B, it[i].p, l), Bv(B, v, it[i].p, l), q->n[l],
                         level_h(q, l), l < (int)q->order.size() ? q->order[l] : 0};
    }
    const DevTab& t = B->P[it[0].p]->tab;
    if (B->prec == SIPG_F64) SIPG_HIP(launch_apply_batch(0, N, jobs, cnt, t, s));
    else if (B->prec == SIPG_F32) SIPG_HIP(launch_apply_batch(3, N, jobs, cnt, t, s));
    else SIPG_HIP(launch_apply_lp_batch(N, B->prec == SIPG_BF16, B->ec, jobs, cnt, t, s));
    return SIPG_OK;
  });
}

sipg_status b_patch(sipg_batch* B, const Vecs& v, const std::vector<Item>& items, int colour,
                    hipStream_t s) {
  return for_groups(B, items, [&](int N, const Item* it, int cnt) -> sipg_status {
    PatchJob jobs[kMaxBatch];
    int m = 0;
    for (int i = 0; i < cnt; ++i) {
      const sipg_problem* q = B->P[it[i].p];
      const int l = it[i].l;
      if (q->n[l] < 2) continue;
      jobs[m++] = PatchJob{R(B, it[i].p, l), X(B, v, it[i].p, l), q->n[l], level_h(q, l)};
    }
    if (m == 0) return SIPG_OK;
    const DevTab& t = B->P[it[0].p]->tab;
    if (B->prec == SIPG_F64) SIPG_HIP(launch_patch_fd_batch(0, N, colour, jobs, m, t, s));
    else if (B->prec == SIPG_F32) SIPG_HIP(launch_patch_fd_batch(1, N, colour, jobs, m, t, s));
    else SIPG_HIP(launch_patch_fd_lp_batch(N, B->prec == SIPG_BF16, B->ec, colour, jobs, m, t, s));
    return SIPG_OK;
  });
}

sipg_status b_smooth(sipg_batch* B, const Vecs& v, const std::vector<Item>& items, int sweeps,
                     hipStream_t s) {
  for (int sw = 0; sw < sweeps; ++sw)
    for (int c = 0; c < 8; ++c) {
      SIPG_TRY(b_residual(B, v, items, s));
      SIPG_TRY(b_patch(B, v, items, c, s));
    }
  return SIPG_OK;
}

sipg_status b_transfer(sipg_batch* B, const Vecs& v, const std::vector<Item>& items, bool restr,
                       hipStream_t s) {
  return for_groups(B, items, [&](int N, const Item* it, int cnt) -> sipg_status {
    TransferJob jobs[kMaxBatch];
    for (int i = 0; i < cnt; ++i) {
      const sipg_problem* q = B->P[it[i].p];
      const int l = it[i].l;  // fine level
      if (restr)
        jobs[i] = TransferJob{R(B, it[i].p, l), Bv(B, v, it[i].p, l - 1), q->n[l - 1]};
      else
        jobs[i] = TransferJob{X(B, v, it[i].p, l - 1), X(B, v, it[i].p, l), q->n[l - 1]};
    }
    SIPG_HIP(launch_transfer_batch(lowp(B) ? 1 : 0, N, restr, jobs, cnt, B->P[it[0].p]->tab, s));
    return SIPG_OK;
  });
}

// The coarse eigenvectors depend on the coarse mesh (1, 2 or 3 cells), so
// coarse solves are grouped by that size as well as by degree.
sipg_status b_coarse(sipg_batch* B, const Vecs& v, const std::vector<Item>& items,
                     hipStream_t s) {
  for (int n0 = 1; n0 <= 3; ++n0) {
    std::vector<Item> sub;
    for (const Item& it : items) {
      if (B->P[it.p]->n0 > 3) return fail(SIPG_ERR_UNSUPPORTED, "coarsest level above 3 cells");
      if (B->P[it.p]->n0 == n0) sub.push_back(it);
    }
    if (sub.empty()) continue;
    SIPG_TRY(for_groups(B, sub, [&](int N, const Item* it, int cnt) -> sipg_status {
      CoarseJob jobs[kMaxBatch];
      for (int i = 0; i < cnt; ++i) {
        const sipg_problem* q = B->P[it[i].p];
        jobs[i] = CoarseJob{Bv(B, v, it[i].p, 0), X(B, v, it[i].p, 0), q->n0, level_h(q, 0)};
      }
      SIPG_HIP(launch_coarse_fd_batch(lowp(B) ? 1 : 0, N, jobs, cnt, B->P[it[0].p]->tab, s));
      return SIPG_OK;
    }));
  }
  return SIPG_OK;
}

// V-cycle of all listed problems from their finest level, levels aligned by
// depth below the finest level.  x and b are the finest-level vectors in the
// V-cycle's storage precision.
sipg_status b_vcycle(sipg_batch* B, const Vecs& v, const std::vector<int>& probs,
                     hipStream_t s) {
  int dmax = 0;
  for (int p : probs) dmax = std::max(dmax, B->P[p]->L);
  auto at_depth = [&](int d, bool coarse) {
    std::vector<Item> it;
    for (int p : probs) {
      const int l = B->P[p]->L - 1 - d;
      if (l < 0) continue;
      if ((l == 0) == coarse) it.push_back(Item{p, l});
    }
    return it;
  };
  for (int d = 0; d < dmax; ++d) {
    std::vector<Item> fine = at_depth(d, false), coarse = at_depth(d, true);
    if (!fine.empty()) {
      SIPG_TRY(b_smooth(B, v, fine, B->nu_pre, s));
      SIPG_TRY(b_residual(B, v, fine, s));
      SIPG_TRY(b_transfer(B, v, fine, true, s));
      for (const Item& it : fine)
        if (it.l - 1 > 0) {
          const sipg_problem* q = B->P[it.p];
          if (lowp(B)) SIPG_HIP(launch_zero_f32(q->fx[it.l - 1], q->ndofs[it.l - 1], s));
          else SIPG_HIP(launch_fill(q->wx[it.l - 1], 0.0, q->ndofs[it.l - 1], s));
        }
    }
    if (!coarse.empty()) SIPG_TRY(b_coarse(B, v, coarse, s));
  }
  for (int d = dmax - 2; d >= 0; --d) {
    std::vector<Item> fine = at_depth(d, false);
    if (fine.empty()) continue;
    SIPG_TRY(b_transfer(B, v, fine, false, s));
    SIPG_TRY(b_smooth(B, v, fine, B->nu_post, s));
  }
  return SIPG_OK;
}

// z_p = V-cycle(0, v_p) for all listed problems; FP64 vectors in and out.
sipg_status b_precondition(sipg_batch* B, const std::vector<int>& probs,
                           const std::vector<const double*>& vin, const std::vector<double*>& zout,
                           hipStream_t s) {
  Vecs v;
  v.x.assign(B->P.size(), nullptr);
  v.b.assign(B->P.size(), nullptr);
  for (int p : probs) {
    sipg_problem* q = B->P[p];
    const int L = q->L - 1;
    if (lowp(B)) {
      SIPG_HIP(launch_to_f32(vin[p], q->fb[L], q->ndofs[L], s));
      SIPG_HIP(launch_zero_f32(q->fx[L], q->ndofs[L], s));
      v.x[p] = q->fx[L];
      v.b[p] = q->fb[L];
    } else {
      SIPG_HIP(launch_fill(zout[p], 0.0, q->ndofs[L], s));
      v.x[p] = zout[p];
      v.b[p] = (void*)vin[p];
    }
  }
  SIPG_TRY(b_vcycle(B, v, probs, s));
  if (lowp(B))
    for (int p : probs) {
      sipg_problem* q = B->P[p];
      SIPG_HIP(launch_to_f64(q->fx[q->L - 1], zout[p], q->ndofs[q->L - 1], s));
    }
  return SIPG_OK;
}

sipg_status b_apply64(sipg_batch* B, const std::vector<int>& probs,
                      const std::vector<const double*>& u, const std::vector<double*>& out,
                      const std::vector<const double*>& b, hipStream_t s) {
  std::vector<Item> items;
  for (int p : probs) items.push_back(Item{p, B->P[p]->L - 1});
  return for_groups(B, items, [&](int N, const Item* it, int cnt) -> sipg_status {
    ApplyJob jobs[kMaxBatch];
    for (int i = 0; i < cnt; ++i) {
      const sipg_problem* q = B->P[it[i].p];
      const int l = it[i].l;
      jobs[i] = ApplyJob{u[it[i].p], out[it[i].p], b.empty() ? nullptr : b[it[i].p], q->n[l],
                         level_h(q, l), l < (int)q->order.size() ? q->order[l] : 0};
    }
    SIPG_HIP(launch_apply_batch(0, N, jobs, cnt, B->P[it[0].p]->tab, s));
    return SIPG_OK;
  });
}

// FGMRES(m) of every problem with its scalars on the device (krylov.hip):
// each Krylov step (V-cycle, apply, Gram-Schmidt twice, Arnoldi and Givens
// update, scaling) is one captured graph over all problems; after a step
// the host reads only the problems' active flags (one small copy) to decide
// whether to issue the next one.  (Issuing ahead and reading the flags one
// step behind was measured slower: the step issued after the last problem
// stopped costs more than the flag round trip saves.)
sipg_status device_krylov(sipg_batch* B, double* const* x, const double* const* b,
                          const sipg_solve_opts* o, const std::vector<double>& nb,
                          const std::vector<double>& tol, std::vector<int>& conv,
                          std::vector<int>& its, sipg_solve_info* infos, hipStream_t s) {
  const int P = (int)B->P.size(), m = o->restart;
  if (m > kMaxKrylov) return fail(SIPG_ERR_ARG, "device-scalar FGMRES needs restart <= 32");
  if (!B->d_kd) {
    KrylovDesc* kd = nullptr;
    double *st = nullptr, *fl = nullptr, *hf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool ok =
        hipMalloc((void**)&kd, sizeof(KrylovDesc) * P) == hipSuccess &&
        hipMalloc((void**)&st, sizeof(double) * kStateStride * P) == hipSuccess &&
        hipMalloc((void**)&fl, sizeof(double) * kFlagCount * P) == hipSuccess &&
        hipHostMalloc((void**)&hf, sizeof(double) * 3 * kFlagCount * P) == hipSuccess &&
        hipEventCreateWithFlags(&e0, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&e1, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      if (kd) hipFree(kd);
      if (st) hipFree(st);
      if (fl) hipFree(fl);
      if (hf) hipHostFree(hf);
      if (e0) hipEventDestroy(e0);
      if (e1) hipEventDestroy(e1);
      return fail(SIPG_ERR_OOM, "device-scalar FGMRES workspace allocation failed");
    }
    B->d_kd = kd;
    B->d_st = st;
    B->d_flags = fl;
    B->h_flags = hf;
    B->ev_flags[0] = e0;
    B->ev_flags[1] = e1;
  }
  auto n_of = [&](int p) { return B->P[p]->ndofs[B->P[p]->L - 1]; };
  auto Vj = [&](int p, int j) { return B->P[p]->V + (size_t)j * n_of(p); };
  auto Zj = [&](int p, int j) { return B->P[p]->Z + (size_t)j * n_of(p); };
  int64_t nmax = 1;
  std::vector<KrylovDesc> kd(P);
  std::vector<double> st0((size_t)kStateStride * P, 0.0);
  for (int p = 0; p < P; ++p) {
    sipg_problem* q = B->P[p];
    kd[p] = KrylovDesc{q->V, q->Z, x[p], q->d_small, q->d_partial, B->d_st + (size_t)p * kStateStride,
                       n_of(p)};
    nmax = std::max(nmax, n_of(p));
    double* t = st0.data() + (size_t)p * kStateStride;
    t[kSNb] = nb[p];
    t[kSTol] = tol[p];
    t[kSMaxIts] = o->max_iters;
    t[kSConv] = conv[p];
  }
  SIPG_HIP(hipMemcpyAsync(B->d_kd, kd.data(), sizeof(KrylovDesc) * P, hipMemcpyHostToDevice, s));
  SIPG_HIP(hipMemcpyAsync(B->d_st, st0.data(), sizeof(double) * st0.size(), hipMemcpyHostToDevice,
                          s));
  SIPG_HIP(hipStreamSynchronize(s));
  std::vector<int> all(P);
  for (int p = 0; p < P; ++p) all[p] = p;
  auto step = [&](int j) -> sipg_status {
    std::vector<const double*> vin(P), u(P);
    std::vector<double*> zout(P), out(P);
    for (int p = 0; p < P; ++p) {
      vin[p] = Vj(p, j);
      zout[p] = Zj(p, j);
      u[p] = Zj(p, j);
      out[p] = Vj(p, j + 1);
    }
    SIPG_TRY(b_precondition(B, all, vin, zout, s));
    SIPG_TRY(b_apply64(B, all, u, out, {}, s));
    SIPG_HIP(launch_krylov_dots(B->d_kd, P, 0, j + 1, j + 1, 0, s));
    SIPG_HIP(launch_krylov_axpy(B->d_kd, P, nmax, j + 1, j + 1, 0, -1, s));
    SIPG_HIP(launch_krylov_dots(B->d_kd, P, 0, j + 1, j + 1, 80, s));
    SIPG_HIP(launch_krylov_axpy(B->d_kd, P, nmax, j + 1, j + 1, 80, 0, s));
    SIPG_HIP(launch_krylov_dots(B->d_kd, P, j + 1, 1, j + 1, kNormSlot, s));
    SIPG_HIP(launch_krylov_scalars(1, B->d_kd, P, j, m, nullptr, s));
    SIPG_HIP(launch_krylov_scale(B->d_kd, P, nmax, j + 1, s));
    return SIPG_OK;
  };
  const size_t fbytes = sizeof(double) * kFlagCount * P;
  auto hflags = [&](int slot) { return B->h_flags + (size_t)slot * kFlagCount * P; };
  std::vector<int> bad(P, 0);
  while (true) {
    bool any = false;
    for (int p = 0; p < P; ++p) any = any || (!conv[p] && its[p] < o->max_iters);
    if (!any) break;
    {  // cycle start: V_0 = b - A x, its norm, g and the scale of V_0
      std::vector<const double*> u(P), bb(P);
      std::vector<double*> out(P);
      for (int p = 0; p < P; ++p) {
        u[p] = x[p];
        bb[p] = b[p];
        out[p] = Vj(p, 0);
      }
      SIPG_TRY(b_apply64(B, all, u, out, bb, s));
      SIPG_HIP(launch_krylov_dots(B->d_kd, P, 0, 1, 0, kNormSlot, s));
      SIPG_HIP(launch_krylov_scalars(0, B->d_kd, P, 0, m, nullptr, s));
      SIPG_HIP(launch_krylov_scale(B->d_kd, P, nmax, 0, s));
    }
    int issued = 0;
    for (int j = 0; j < m; ++j) {
      const int key = m * 64 + j;
      auto it = B->steps.find(key);
      if (it == B->steps.end()) {
        hipGraph_t gr;
        SIPG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        sipg_status stc = step(j);
        hipError_t ee = hipStreamEndCapture(s, &gr);
        if (stc != SIPG_OK) return stc;
        SIPG_HIP(ee);
        hipGraphExec_t ex;
        hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        hipGraphDestroy(gr);
        SIPG_HIP(ei);
        it = B->steps.emplace(key, ex).first;
      }
      SIPG_HIP(hipGraphLaunch(it->second, s));
      issued = j + 1;
      if (j + 1 == m) break;
      // the active flags after step j decide whether step j + 1 is issued
      SIPG_HIP(launch_krylov_scalars(3, B->d_kd, P, 0, m, B->d_flags, s));
      SIPG_HIP(hipMemcpyAsync(hflags(j & 1), B->d_flags, fbytes, hipMemcpyDeviceToHost, s));
      SIPG_HIP(hipEventRecord(B->ev_flags[j & 1], s));
      SIPG_HIP(hipEventSynchronize(B->ev_flags[j & 1]));
      const double* f = hflags(j & 1);
      bool live = false;
      for (int p = 0; p < P; ++p) live = live || f[(size_t)p * kFlagCount] != 0.0;
      if (!live) break;
    }
    // cycle end: y = R^{-1} g, x += Z y over the steps issued, flags to the host
    SIPG_HIP(launch_krylov_scalars(2, B->d_kd, P, 0, m, nullptr, s));
    SIPG_HIP(launch_krylov_update(B->d_kd, P, nmax, issued, s));
    SIPG_HIP(launch_krylov_scalars(3, B->d_kd, P, 0, m, B->d_flags, s));
    SIPG_HIP(hipMemcpyAsync(hflags(2), B->d_flags, fbytes, hipMemcpyDeviceToHost, s));
    SIPG_HIP(hipStreamSynchronize(s));
    const double* f = hflags(2);
    for (int p = 0; p < P; ++p) {
      conv[p] = f[(size_t)p * kFlagCount + (kSConv - kSActive)] != 0.0;
      its[p] = (int)f[(size_t)p * kFlagCount + (kSIts - kSActive)];
      bad[p] = f[(size_t)p * kFlagCount + (kSBad - kSActive)] != 0.0;
      if (bad[p]) return fail(SIPG_ERR_NONFINITE, "Arnoldi vector is not finite");
    }
  }
  std::vector<double> stv((size_t)kStateStride * P);
  SIPG_HIP(hipMemcpyAsync(stv.data(), B->d_st, sizeof(double) * stv.size(), hipMemcpyDeviceToHost,
                          s));
  SIPG_HIP(hipStreamSynchronize(s));
  for (int p = 0; p < P; ++p) {
    const double* t = stv.data() + (size_t)p * kStateStride;
    infos[p].rel_res_est = t[kSEst];
    if (o->log_history) {
      const int h = std::min((int)t[kSHist], kHistory);
      for (int i = 0; i < h; ++i) infos[p].history[i] = t[kSHistory + i];
    }
  }
  return SIPG_OK;
}

}  // namespace

extern "C" {

sipg_status sipg_batch_create(const sipg_config* cfgs, int count, hipStream_t stream,
                              sipg_batch** out) {
  if (!cfgs || !out || count < 1 || count > 4096) return fail(SIPG_ERR_ARG, "bad batch");
  *out = nullptr;
  for (int i = 1; i < count; ++i)
    if (cfgs[i].mg_precision != cfgs[0].mg_precision ||
        cfgs[i].error_correction != cfgs[0].error_correction ||
        cfgs[i].nu_pre != cfgs[0].nu_pre || cfgs[i].nu_post != cfgs[0].nu_post)
      return fail(SIPG_ERR_ARG, "all problems of a batch share precision and smoothing steps");
  for (int i = 0; i < count; ++i)
    if (cfgs[i].smoother != 0)
      return fail(SIPG_ERR_UNSUPPORTED, "batches use the multiplicative smoother");
  auto* B = new sipg_batch();
  B->prec = cfgs[0].mg_precision;
  B->ec = cfgs[0].error_correction;
  B->nu_pre = cfgs[0].nu_pre;
  B->nu_post = cfgs[0].nu_post;
  for (int i = 0; i < count; ++i) {
    sipg_problem* q = nullptr;
    sipg_status st = sipg_create(&cfgs[i], stream, &q);
    if (st != SIPG_OK) {
      std::string msg = g_err;
      sipg_batch_destroy(B);
      return fail(st, "problem " + std::to_string(i) + ": " + msg);
    }
    if (q->n0 > 3) {
      sipg_destroy(q);
      sipg_batch_destroy(B);
      return fail(SIPG_ERR_UNSUPPORTED, "batch problems need a coarsest level of <= 3 cells");
    }
    B->P.push_back(q);
    if (std::find(B->nodes.begin(), B->nodes.end(), q->N) == B->nodes.end())
      B->nodes.push_back(q->N);
  }
  std::sort(B->nodes.begin(), B->nodes.end());
  if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void**)&B->h_pinned, sizeof(double) * 128 * (size_t)count) != hipSuccess) {
    sipg_batch_destroy(B);
    return fail(SIPG_ERR_HIP, "stream / event / pinned buffer creation failed");
  }
  *out = B;
  return SIPG_OK;
}

void sipg_batch_destroy(sipg_batch* B) {
  if (!B) return;
  hipDeviceSynchronize();
  drop_graphs(B);
  for (sipg_problem* q : B->P) sipg_destroy(q);
  if (B->stream) hipStreamDestroy(B->stream);
  if (B->ev_in) hipEventDestroy(B->ev_in);
  if (B->ev_out) hipEventDestroy(B->ev_out);
  if (B->h_pinned) hipHostFree(B->h_pinned);
  if (B->h_flags) hipHostFree(B->h_flags);
  if (B->d_kd) hipFree(B->d_kd);
  if (B->d_st) hipFree(B->d_st);
  if (B->d_flags) hipFree(B->d_flags);
  for (hipEvent_t e : B->ev_flags)
    if (e) hipEventDestroy(e);
  delete B;
}

int sipg_batch_count(const sipg_batch* B) { return B ? (int)B->P.size() : -1; }

sipg_problem* sipg_batch_problem(sipg_batch* B, int i) {
  if (!B || i < 0 || i >= (int)B->P.size()) return nullptr;
  return B->P[i];
}

sipg_status sipg_batch_autotune(sipg_batch* B, hipStream_t s) {
  if (!B) return fail(SIPG_ERR_ARG, "NULL batch");
  drop_graphs(B);
  // one timing per (degree, mesh) class; the result is shared by the class
  std::map<std::pair<int, int>, std::vector<int>> done;
  for (sipg_problem* q : B->P) {
    const auto key = std::make_pair(q->k, q->n.back());
    auto it = done.find(key);
    if (it != done.end()) {
      q->order = it->second;
      continue;
    }
    double* tmp = nullptr;
    SIPG_TRY(prob_alloc(q, &tmp, q->ndofs[q->L - 1]));
    q->order.assign(q->L, 0);
    sipg_status st = SIPG_OK;
    for (int l = 0; l < q->L && st == SIPG_OK; ++l) {
      if (q->n[l] < 8) continue;  // small levels keep the default order
      if (launch_fill(q->wr[l], 0.0, q->ndofs[l], s) != hipSuccess) st = SIPG_ERR_HIP;
      int best = 0;
      if (st == SIPG_OK) st = sipg_autotune(q, l, q->wr[l], tmp, &best, s);
    }
    hipStreamSynchronize(s);
    prob_free(q, tmp);
    if (st != SIPG_OK) return st;
    done[key] = q->order;
  }
  return SIPG_OK;
}

sipg_status sipg_batch_apply(sipg_batch* B, const double* const* u, double* const* v,
                             hipStream_t s) {
  if (!B || !u || !v) return fail(SIPG_ERR_ARG, "NULL argument");
  SIPG_TRY(cartesian_batch(B));
  std::vector<int> all(B->P.size());
  std::vector<const double*> uu(B->P.size());
  std::vector<double*> vv(B->P.size());
  for (size_t i = 0; i < B->P.size(); ++i) {
    all[i] = (int)i;
    if (!u[i] || !v[i] || u[i] == v[i]) return fail(SIPG_ERR_ARG, "bad vector pointer");
    uu[i] = u[i];
    vv[i] = v[i];
  }
  return b_apply64(B, all, uu, vv, {}, s);
}

sipg_status sipg_batch_vcycle(sipg_batch* B, double* const* x, const double* const* b,
                              hipStream_t s) {
  if (!B || !x || !b) return fail(SIPG_ERR_ARG, "NULL argument");
  SIPG_TRY(cartesian_batch(B));
  std::vector<int> all(B->P.size());
  Vecs v;
  v.x.assign(B->P.size(), nullptr);
  v.b.assign(B->P.size(), nullptr);
  for (size_t i = 0; i < B->P.size(); ++i) {
    all[i] = (int)i;
    sipg_problem* q = B->P[i];
    const int L = q->L - 1;
    if (!x[i] || !b[i] || (const void*)x[i] == (const void*)b[i])
      return fail(SIPG_ERR_ARG, "bad vector pointer");
    if (lowp(B)) {
      SIPG_HIP(launch_to_f32(b[i], q->fb[L], q->ndofs[L], s));
      SIPG_HIP(launch_to_f32(x[i], q->fx[L], q->ndofs[L], s));
      v.x[i] = q->fx[L];
      v.b[i] = q->fb[L];
    } else {
      v.x[i] = x[i];
      v.b[i] = (void*)b[i];
    }
  }
  SIPG_TRY(b_vcycle(B, v, all, s));
  if (lowp(B))
    for (size_t i = 0; i < B->P.size(); ++i) {
      sipg_problem* q = B->P[i];
      SIPG_HIP(launch_to_f64(q->fx[q->L - 1], x[i], q->ndofs[q->L - 1], s));
    }
  return SIPG_OK;
}

sipg_status sipg_batch_solve(sipg_batch* B, double* const* x, const double* const* b,
                             const sipg_solve_opts* o, sipg_solve_info* infos, int use_graph,
                             hipStream_t s_user) {
  if (!B || !x || !b || !o || !infos) return fail(SIPG_ERR_ARG, "NULL argument");
  if (o->restart < 1 || o->restart > 64) return fail(SIPG_ERR_ARG, "restart must be in 1..64");
  if (use_graph < 0 || use_graph > 2) return fail(SIPG_ERR_ARG, "use_graph must be 0, 1 or 2");
  SIPG_TRY(cartesian_batch(B));
  if (o->max_iters < 1 || !(o->rtol > 0.0)) return fail(SIPG_ERR_ARG, "bad options");
  if (o->use_learned) return fail(SIPG_ERR_UNSUPPORTED, "learned stage not available in batches");
  if (o->variant != SIPG_FGMRES) return fail(SIPG_ERR_UNSUPPORTED, "batches run FGMRES");
  const int P = (int)B->P.size();
  const int m = o->restart;
  for (int p = 0; p < P; ++p) {
    if (!x[p] || !b[p] || (const void*)x[p] == (const void*)b[p])
      return fail(SIPG_ERR_ARG, "bad vector pointer");
    SIPG_TRY(ensure_krylov(B->P[p], m));
    std::memset(&infos[p], 0, sizeof(sipg_solve_info));
  }
  // Captured V-cycles hold Krylov addresses: they are stale once any problem
  // reallocated its Krylov space (here or in sipg_fgmres through a borrowed
  // handle), whether or not the new block landed at the old address.
  {
    std::vector<int> gen(P);
    for (int p = 0; p < P; ++p) gen[p] = B->P[p]->krylov_gen;
    if (gen != B->graph_gen) {
      drop_graphs(B);
      B->graph_gen = gen;
    }
  }
  // work on the internal stream, ordered after the caller's stream; on every
  // exit from here on the caller's stream waits for that work
  hipStream_t s = B->stream;
  SIPG_HIP(hipEventRecord(B->ev_in, s_user));
  SIPG_HIP(hipStreamWaitEvent(s, B->ev_in, 0));
  struct Join {
    sipg_batch* B;
    hipStream_t s, user;
    ~Join() {
      if (hipEventRecord(B->ev_out, s) == hipSuccess) hipStreamWaitEvent(user, B->ev_out, 0);
    }
  } join{B, s, s_user};
  SIPG_HIP(hipStreamSynchronize(s));
  const auto t0 = std::chrono::steady_clock::now();
  double* hp = B->h_pinned;
  auto n_of = [&](int p) { return B->P[p]->ndofs[B->P[p]->L - 1]; };
  auto Vj = [&](int p, int j) { return B->P[p]->V + (size_t)j * n_of(p); };
  auto Zj = [&](int p, int j) { return B->P[p]->Z + (size_t)j * n_of(p); };

  // ||b||
  std::vector<double> nb(P), tol(P);
  for (int p = 0; p < P; ++p) {
    SIPG_HIP(launch_mdot(b[p], n_of(p), 1, b[p], n_of(p), B->P[p]->d_partial,
                         B->P[p]->d_small + 160, s));
    SIPG_HIP(hipMemcpyAsync(hp + 128 * p, B->P[p]->d_small + 160, sizeof(double),
                            hipMemcpyDeviceToHost, s));
  }
  SIPG_HIP(hipStreamSynchronize(s));
  std::vector<int> conv(P, 0), its(P, 0), hist(P, 0);
  for (int p = 0; p < P; ++p) {
    nb[p] = std::sqrt(hp[128 * p]);
    if (!std::isfinite(nb[p])) return fail(SIPG_ERR_NONFINITE, "right-hand side is not finite");
    tol[p] = o->rtol * nb[p];
    if (nb[p] == 0.0) {
      SIPG_HIP(launch_fill(x[p], 0.0, n_of(p), s));
      conv[p] = 1;
    }
  }
  auto record = [&](int p, double v) {
    infos[p].rel_res_est = v;
    if (o->log_history && hist[p] < 128) infos[p].history[hist[p]] = v;
    ++hist[p];
  };
  std::vector<std::vector<double>> H(P, std::vector<double>((size_t)(m + 1) * m)),
      cs(P, std::vector<double>(m)), sn(P, std::vector<double>(m)),
      g(P, std::vector<double>(m + 1));
  bool graphs_ok = use_graph != 0;
  int total_it = 0;
  if (use_graph == 2) SIPG_TRY(device_krylov(B, x, b, o, nb, tol, conv, its, infos, s));
  while (use_graph != 2) {
    std::vector<int> act;
    for (int p = 0; p < P; ++p)
      if (!conv[p] && its[p] < o->max_iters) act.push_back(p);
    if (act.empty()) break;
    // restart: r = b - A x into V_0, beta
    {
      std::vector<const double*> u(P), bb(P);
      std::vector<double*> out(P);
      for (int p : act) {
        u[p] = x[p];
        bb[p] = b[p];
        out[p] = Vj(p, 0);
      }
      SIPG_TRY(b_apply64(B, act, u, out, bb, s));
      for (int p : act) {
        SIPG_HIP(launch_mdot(Vj(p, 0), n_of(p), 1, Vj(p, 0), n_of(p), B->P[p]->d_partial,
                             B->P[p]->d_small + 160, s));
        SIPG_HIP(hipMemcpyAsync(hp + 128 * p, B->P[p]->d_small + 160, sizeof(double),
                                hipMemcpyDeviceToHost, s));
      }
      SIPG_HIP(hipStreamSynchronize(s));
    }
    std::vector<int> cyc;
    for (int p : act) {
      const double beta = std::sqrt(hp[128 * p]);
      if (!std::isfinite(beta)) return fail(SIPG_ERR_NONFINITE, "residual is not finite");
      record(p, beta / nb[p]);
      if (beta <= tol[p]) {
        conv[p] = 1;
        continue;
      }
      SIPG_HIP(launch_scale_copy(Vj(p, 0), 1.0 / beta, Vj(p, 0), n_of(p), s));
      std::fill(g[p].begin(), g[p].end(), 0.0);
      g[p][0] = beta;
      cyc.push_back(p);
    }
    if (cyc.empty()) break;
    // the graph of Krylov step j is valid for the full problem set only
    const bool full = (int)cyc.size() == P;
    std::vector<int> jd(P, 0), live(cyc);
    for (int j = 0; j < m && !live.empty(); ++j) {
      std::vector<const double*> vin(P);
      std::vector<double*> zout(P);
      for (int p : live) {
        vin[p] = Vj(p, j);
        zout[p] = Zj(p, j);
      }
      if (graphs_ok && full && (int)live.size() == P) {
        auto it = B->graphs.find(j);
        if (it == B->graphs.end()) {
          hipGraph_t gr;
          SIPG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
          sipg_status st = b_precondition(B, live, vin, zout, s);
          hipError_t ee = hipStreamEndCapture(s, &gr);
          if (st != SIPG_OK) return st;
          SIPG_HIP(ee);
          hipGraphExec_t ex;
          SIPG_HIP(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
          hipGraphDestroy(gr);
          it = B->graphs.emplace(j, ex).first;
        }
        SIPG_HIP(hipGraphLaunch(it->second, s));
      } else {
        SIPG_TRY(b_precondition(B, live, vin, zout, s));
      }
      // w = A z_j into V_{j+1}
      {
        std::vector<const double*> u(P);
        std::vector<double*> out(P);
        for (int p : live) {
          u[p] = Zj(p, j);
          out[p] = Vj(p, j + 1);
        }
        SIPG_TRY(b_apply64(B, live, u, out, {}, s));
      }
      // classical Gram-Schmidt twice, per problem; one host sync for all
      for (int p : live) {
        sipg_problem* q = B->P[p];
        double* w = Vj(p, j + 1);
        const int64_t n = n_of(p);
        SIPG_HIP(launch_mdot(q->V, n, j + 1, w, n, q->d_partial, q->d_small, s));
        SIPG_HIP(launch_maxpy(q->V, n, j + 1, q->d_small, w, n, nullptr, 1.0, s));
        SIPG_HIP(launch_mdot(q->V, n, j + 1, w, n, q->d_partial, q->d_small + 80, s));
        SIPG_HIP(launch_maxpy(q->V, n, j + 1, q->d_small + 80, w, n, q->d_small, 1.0, s));
        SIPG_HIP(launch_mdot(w, n, 1, w, n, q->d_partial, q->d_small + 160, s));
        SIPG_HIP(hipMemcpyAsync(hp + 128 * p, q->d_small, sizeof(double) * (j + 1),
                                hipMemcpyDeviceToHost, s));
        SIPG_HIP(hipMemcpyAsync(hp + 128 * p + 100, q->d_small + 160, sizeof(double),
                                hipMemcpyDeviceToHost, s));
      }
      SIPG_HIP(hipStreamSynchronize(s));
      std::vector<int> next;
      for (int p : live) {
        auto Hm = [&](int i, int c) -> double& { return H[p][(size_t)i * m + c]; };
        const double hn = std::sqrt(hp[128 * p + 100]);
        if (!std::isfinite(hn)) return fail(SIPG_ERR_NONFINITE, "Arnoldi vector is not finite");
        for (int i = 0; i <= j; ++i) Hm(i, j) = hp[128 * p + i];
        Hm(j + 1, j) = hn;
        if (hn > 0.0) SIPG_HIP(launch_scale_copy(Vj(p, j + 1), 1.0 / hn, Vj(p, j + 1), n_of(p), s));
        for (int i = 0; i < j; ++i) {
          const double t = cs[p][i] * Hm(i, j) + sn[p][i] * Hm(i + 1, j);
          Hm(i + 1, j) = -sn[p][i] * Hm(i, j) + cs[p][i] * Hm(i + 1, j);
          Hm(i, j) = t;
        }
        const double den = std::hypot(Hm(j, j), Hm(j + 1, j));
        cs[p][j] = Hm(j, j) / den;
        sn[p][j] = Hm(j + 1, j) / den;
        Hm(j, j) = den;
        Hm(j + 1, j) = 0.0;
        g[p][j + 1] = -sn[p][j] * g[p][j];
        g[p][j] = cs[p][j] * g[p][j];
        ++its[p];
        ++total_it;
        jd[p] = j + 1;
        record(p, std::fabs(g[p][j + 1]) / nb[p]);
        if (!(std::fabs(g[p][j + 1]) <= tol[p] || its[p] >= o->max_iters || den == 0.0))
          next.push_back(p);
      }
      live = next;
    }
    // x += Z y
    for (int p : cyc) {
      const int J = jd[p];
      std::vector<double> y(J);
      auto Hm = [&](int i, int c) -> double { return H[p][(size_t)i * m + c]; };
      for (int i = J - 1; i >= 0; --i) {
        double a = g[p][i];
        for (int c = i + 1; c < J; ++c) a -= Hm(i, c) * y[c];
        y[i] = a / Hm(i, i);
      }
      // y goes through this problem's pinned slots (H and the norm were consumed)
      std::copy(y.begin(), y.end(), hp + 128 * p);
      SIPG_HIP(hipMemcpyAsync(B->P[p]->d_small + 192, hp + 128 * p, sizeof(double) * J,
                              hipMemcpyHostToDevice, s));
      SIPG_HIP(launch_maxpy(B->P[p]->Z, n_of(p), J, B->P[p]->d_small + 192, x[p], n_of(p),
                            nullptr, -1.0, s));
      if (std::fabs(g[p][J]) <= tol[p]) conv[p] = 1;
    }
  }
  // true residuals
  {
    std::vector<int> all(P);
    std::vector<const double*> u(P), bb(P);
    std::vector<double*> out(P);
    for (int p = 0; p < P; ++p) {
      all[p] = p;
      u[p] = x[p];
      bb[p] = b[p];
      out[p] = Vj(p, 0);
    }
    SIPG_TRY(b_apply64(B, all, u, out, bb, s));
    for (int p = 0; p < P; ++p) {
      SIPG_HIP(launch_mdot(Vj(p, 0), n_of(p), 1, Vj(p, 0), n_of(p), B->P[p]->d_partial,
                           B->P[p]->d_small + 160, s));
      SIPG_HIP(hipMemcpyAsync(hp + 128 * p, B->P[p]->d_small + 160, sizeof(double),
                              hipMemcpyDeviceToHost, s));
    }
    SIPG_HIP(hipStreamSynchronize(s));
  }
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool all_conv = true;
  for (int p = 0; p < P; ++p) {
    infos[p].iterations = its[p];
    infos[p].rel_res_true = nb[p] > 0 ? std::sqrt(hp[128 * p]) / nb[p] : 0.0;
    infos[p].seconds = secs;
    all_conv = all_conv && conv[p];
  }
  if (!all_conv) return fail(SIPG_ERR_NOT_CONVERGED, "iteration limit reached");
  return SIPG_OK;
}

sipg_status sipg_batch_solve_sequential(sipg_batch* B, double* const* x, const double* const* b,
                                        const sipg_solve_opts* o, sipg_solve_info* infos,
                                        hipStream_t s) {
  if (!B || !x || !b || !o || !infos) return fail(SIPG_ERR_ARG, "NULL argument");
  sipg_status worst = SIPG_OK;
  for (size_t p = 0; p < B->P.size(); ++p) {
    sipg_status st = sipg_fgmres(B->P[p], x[p], b[p], o, &infos[p], s);
    if (st != SIPG_OK && st != SIPG_ERR_NOT_CONVERGED) return st;
    if (st != SIPG_OK) worst = st;
  }
  return worst;
}

}  // extern "C"
