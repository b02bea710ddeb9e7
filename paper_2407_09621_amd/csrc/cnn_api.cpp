// C ABI of the learned correction stage (include/sipg.h): network handle,
// forward and gradient on device grids, Adam, solver-generated training
// pairs, the training loop, and the stage inside the flexible GMRES
// preconditioner.  The stage and its training are a project extension;
// the paper has no learned component.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "cnn.h"
#include "problem.h"

using namespace sipg;
namespace C = sipg::cnn;

struct sipg_cnn {
  float* prm = nullptr;        // FP32 master parameters
  float* am = nullptr;         // Adam first moments
  float* av = nullptr;         // Adam second moments
  float* grad = nullptr;
  _Float16* packed = nullptr;  // 4 * kPacked FP16 fragments (layers 2, 3; fwd, bwd)
  float* part = nullptr;       // weight-gradient block partials
  float* lpart = nullptr;      // loss partials
  float* sums = nullptr;       // [loss, mask sum]
  float sigma = 0.0f;          // output scale (0 = not yet chosen)
  int adam_t = 0;
  // activation workspace
  int64_t ws_points = 0;
  bool ws_train = false;
  _Float16 *x16 = nullptr, *a1 = nullptr, *a2 = nullptr, *a3 = nullptr;
  _Float16 *g1 = nullptr, *g2 = nullptr, *g3 = nullptr;
  _Float16 *ot = nullptr, *os = nullptr;  // weight-gradient octet copies (np * 32, 3 np * 32)
  float *y = nullptr, *g4 = nullptr, *xin = nullptr, *tgt = nullptr, *msk = nullptr;
};

namespace {

void free_ws(sipg_cnn* c) {
  for (_Float16** p : {&c->x16, &c->a1, &c->a2, &c->a3, &c->g1, &c->g2, &c->g3, &c->ot, &c->os}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  for (float** p : {&c->y, &c->g4, &c->xin, &c->tgt, &c->msk}) {
    if (*p) hipFree(*p);
    *p = nullptr;
  }
  c->ws_points = 0;
  c->ws_train = false;
}

sipg_status ensure_ws(sipg_cnn* c, int64_t points, bool train) {
  if (points <= c->ws_points && (!train || c->ws_train)) return SIPG_OK;
  const int64_t np = points > c->ws_points ? points : c->ws_points;
  const bool tr = train || c->ws_train;
  free_ws(c);
  const size_t pc = (size_t)np * C::kC;
  SIPG_TRY(dev_alloc(&c->x16, (size_t)np));
  SIPG_TRY(dev_alloc(&c->a1, pc));
  SIPG_TRY(dev_alloc(&c->a2, pc));
  SIPG_TRY(dev_alloc(&c->a3, pc));
  SIPG_TRY(dev_alloc(&c->y, (size_t)np));
  if (tr) {
    SIPG_TRY(dev_alloc(&c->g1, pc));
    SIPG_TRY(dev_alloc(&c->g2, pc));
    SIPG_TRY(dev_alloc(&c->g3, pc));
    SIPG_TRY(dev_alloc(&c->ot, pc));
    SIPG_TRY(dev_alloc(&c->os, 3 * pc));
    SIPG_TRY(dev_alloc(&c->g4, (size_t)np));
    SIPG_TRY(dev_alloc(&c->xin, (size_t)np));
    SIPG_TRY(dev_alloc(&c->tgt, (size_t)np));
    SIPG_TRY(dev_alloc(&c->msk, (size_t)np));
  }
  c->ws_points = np;
  c->ws_train = tr;
  return SIPG_OK;
}

sipg_status check_grid(int G, int ns) {
  if (G < C::kTile || G % C::kTile) return fail(SIPG_ERR_ARG, "grid side must be a multiple of 16");
  if (ns < 1) return fail(SIPG_ERR_ARG, "batch must be >= 1");
  return SIPG_OK;
}

// a1..a3 and y = scale * net(x) from x16 (FP16 input already in c->x16)
sipg_status forward(sipg_cnn* c, int G, int ns, float* y, float scale, hipStream_t s) {
  SIPG_HIP(C::launch_in_fwd(c->x16, G, ns, c->prm, c->a1, s));
  SIPG_HIP(C::launch_mid(0, c->a1, c->packed, c->prm + C::kB2, nullptr, c->a2, G, ns, s));
  SIPG_HIP(C::launch_mid(0, c->a2, c->packed + C::kPacked, c->prm + C::kB3, nullptr, c->a3, G, ns,
                         s));
  if (y) SIPG_HIP(C::launch_out_fwd(c->a3, G, ns, c->prm, scale, y, s));
  return SIPG_OK;
}

// parameter gradient from the output gradient in c->g4 (scaled as
// launch_loss leaves it, with the matching normalisation in c->sums[1])
sipg_status backward_from_output(sipg_cnn* c, int G, int ns, float* grad, hipStream_t s) {
  const float sig = c->sigma > 0.0f ? c->sigma : 1.0f;
  SIPG_HIP(C::launch_out_bwd(c->g4, c->a3, G, ns, c->prm, c->g3, s));
  const C::WgradBufs wb{c->ot, c->os};
  SIPG_HIP(C::launch_out_wgrad(c->a3, c->g4, G, ns, wb, c->part, s));
  SIPG_HIP(C::launch_reduce_rows(c->part, C::kSegOut, c->sums, sig, grad + C::kW4, s));
  SIPG_HIP(C::launch_mid_wgrad(c->a2, c->g3, G, ns, wb, c->part, s));
  SIPG_HIP(C::launch_reduce_rows(c->part, C::kSegMid, c->sums, sig, grad + C::kW3, s));
  SIPG_HIP(C::launch_mid(1, c->g3, c->packed + 3 * C::kPacked, nullptr, c->a2, c->g2, G, ns, s));
  SIPG_HIP(C::launch_mid_wgrad(c->a1, c->g2, G, ns, wb, c->part, s));
  SIPG_HIP(C::launch_reduce_rows(c->part, C::kSegMid, c->sums, sig, grad + C::kW2, s));
  SIPG_HIP(C::launch_mid(1, c->g2, c->packed + 2 * C::kPacked, nullptr, c->a1, c->g1, G, ns, s));
  SIPG_HIP(C::launch_in_wgrad(c->x16, c->g1, G, ns, wb, c->part, s));
  SIPG_HIP(C::launch_reduce_rows(c->part, C::kSegIn, c->sums, sig, grad + C::kW1, s));
  return SIPG_OK;
}

// gradient of the masked loss on x16 / tgt / msk into `grad`; loss in c->sums[0]
sipg_status backward(sipg_cnn* c, int G, int ns, float* grad, hipStream_t s) {
  const int64_t np = (int64_t)ns * G * G * G;
  const float sig = c->sigma > 0.0f ? c->sigma : 1.0f;
  SIPG_TRY(forward(c, G, ns, c->y, 1.0f, s));
  SIPG_HIP(C::launch_loss(c->y, c->tgt, c->msk, np, sig, c->g4, c->lpart, c->sums, s));
  return backward_from_output(c, G, ns, grad, s);
}

// Residual-aware loss on the problem's finest level for the scaled residual
// rho_s (FP64 cell vector): c = sigma net(grid(rho_s)), q = A c, the stage's
// step alpha = (rho_s . q) / (q . q), r = rho_s - alpha q,
// L = ||r||^2 / ||rho_s||^2 into c->sums[0] and dL/dparameters into grad,
// through dL/dy = -2 sigma alpha grid(A r) / ||rho_s||^2 (A symmetric; the
// derivative in alpha vanishes at the minimising alpha).  wc, wq: two cell
// vectors of workspace; p->d_small[440..445] hold device scalars.
sipg_status residual_backward(sipg_cnn* c, sipg_problem* p, const double* rho_s, double* wc,
                              double* wq, float* grad, hipStream_t s) {
  const int L = p->L - 1;
  const int n = p->n[L], N = p->N, G = n * N;
  const int64_t nd = p->ndofs[L];
  const float sig = c->sigma > 0.0f ? c->sigma : 1.0f;
  double* one = p->d_small + 440;
  double* rr = p->d_small + 441;
  double* pp = p->d_small + 442;
  double* S = p->d_small + 443;
  double* ab = p->d_small + 444;  // [rho . q, q . q]
  SIPG_HIP(launch_fill(one, 1.0, 1, s));
  SIPG_HIP(C::launch_gather_f16(rho_s, n, N, one, c->x16, s));
  SIPG_TRY(forward(c, G, 1, nullptr, 0.0f, s));
  SIPG_HIP(launch_fill(wc, 0.0, nd, s));
  SIPG_HIP(C::launch_out_scatter(c->a3, n, N, c->prm, sig, one, wc, s));  // c
  SIPG_TRY(sipg_apply(p, L, wc, wq, s));                                   // q = A c
  SIPG_HIP(launch_mdot(rho_s, nd, 1, wq, nd, p->d_partial, ab, s));
  SIPG_HIP(launch_mdot(wq, nd, 1, wq, nd, p->d_partial, ab + 1, s));
  SIPG_HIP(launch_scale_copy(rho_s, -1.0, wc, nd, s));
  SIPG_HIP(C::launch_axpy_ratio(ab, ab + 1, wq, wc, nd, s));              // -r = alpha q - rho
  SIPG_HIP(launch_mdot(wc, nd, 1, wc, nd, p->d_partial, rr, s));
  SIPG_HIP(launch_mdot(rho_s, nd, 1, rho_s, nd, p->d_partial, pp, s));
  SIPG_TRY(sipg_apply(p, L, wc, wq, s));                                   // -A r
  SIPG_HIP(C::launch_pow2_absmax(wq, nd, p->d_partial, S, s));
  SIPG_HIP(C::launch_gather_f32(wq, n, N, S, c->g4, s));                  // -grid(A r) / S
  SIPG_HIP(C::launch_residual_sums(rr, pp, S, ab, sig, c->sums, s));
  return backward_from_output(c, G, 1, grad, s);
}

sipg_status adam(sipg_cnn* c, const float* grad, float lr, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  ++c->adam_t;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, c->adam_t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, c->adam_t)));
  SIPG_HIP(C::launch_adam(c->prm, c->am, c->av, grad, C::kParams, lr, (float)b1, (float)b2, 1e-8f,
                          c1, c2, s));
  SIPG_HIP(C::launch_pack(c->prm, c->packed, s));
  return SIPG_OK;
}

// splitmix64 (Steele, Lea, Flood 2014) for the training loop's draws
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  int below(int m) { return (int)(uniform() * m); }
};

// One pair of the chain (see sipg_cnn_make_pairs); x is advanced in place.
struct PairBufs {
  double *r = nullptr, *z = nullptr, *e = nullptr, *rho = nullptr, *scale = nullptr;
};

sipg_status make_pair(sipg_problem* p, double* x, PairBufs& w, float* rho_g, float* e_g,
                      double* s_rho, hipStream_t s) {
  const int L = p->L - 1;
  const int64_t n = p->ndofs[L];
  SIPG_TRY(sipg_apply(p, L, x, w.r, s));                     // r = A x
  SIPG_HIP(launch_fill(w.z, 0.0, n, s));
  SIPG_TRY(sipg_vcycle(p, L, w.z, w.r, s));                  // z = V(r)
  SIPG_HIP(launch_scale_copy(x, 1.0, w.e, n, s));
  SIPG_HIP(launch_axpy(-1.0, w.z, w.e, n, s));               // e = x - z
  SIPG_TRY(sipg_residual(p, L, w.r, w.z, w.rho, s));         // rho = r - A z
  SIPG_HIP(C::launch_pow2_absmax(w.rho, n, p->d_partial, w.scale, s));
  SIPG_HIP(C::launch_gather_f32(w.rho, p->n[L], p->N, w.scale, rho_g, s));
  SIPG_HIP(C::launch_gather_f32(w.e, p->n[L], p->N, w.scale, e_g, s));
  SIPG_HIP(C::launch_pow2_absmax(w.e, n, p->d_partial, w.scale + 1, s));
  SIPG_HIP(C::launch_div_scale(w.e, w.scale + 1, x, n, s));  // next x of the chain
  if (s_rho) {  // the scales are checked on the host only when asked for
    double hs[2];
    SIPG_HIP(hipMemcpyAsync(hs, w.scale, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    SIPG_HIP(hipStreamSynchronize(s));
    if (!(hs[0] > 0.0) || !(hs[1] > 0.0) || !std::isfinite(hs[0]) || !std::isfinite(hs[1]))
      return fail(SIPG_ERR_NONFINITE, "degenerate training pair (zero or non-finite error)");
    *s_rho = hs[0];
  }
  return SIPG_OK;
}

sipg_status alloc_pair_bufs(sipg_problem* p, PairBufs& w) {
  const int64_t n = p->ndofs[p->L - 1];
  SIPG_TRY(dev_alloc(&w.r, n));
  SIPG_TRY(dev_alloc(&w.z, n));
  SIPG_TRY(dev_alloc(&w.e, n));
  SIPG_TRY(dev_alloc(&w.rho, n));
  SIPG_TRY(dev_alloc(&w.scale, 2));
  return SIPG_OK;
}

void free_pair_bufs(PairBufs& w) {
  for (double* q : {w.r, w.z, w.e, w.rho, w.scale})
    if (q) hipFree(q);
  w = PairBufs();
}

sipg_status check_problem_grid(const sipg_problem* p) {
  SIPG_TRY(cartesian_only(p, "the learned stage"));
  const int G = p->n[p->L - 1] * p->N;
  if (G % C::kTile) return fail(SIPG_ERR_UNSUPPORTED, "n (k+1) must be a multiple of 16");
  return SIPG_OK;
}

}  // namespace

namespace sipg {

// The learned stage applied after the V-cycle inside the preconditioner:
// rho = v - A z, s = 2^ceil(log2 max|rho|), c = s sigma net(rho / s),
// q = A c and z += alpha c with alpha = (rho . q) / (q . q), the factor that
// minimises ||v - A (z + alpha c)||_2 (0 when q = 0).
sipg_status cnn_stage(sipg_problem* p, const double* v, double* z, hipStream_t s) {
  sipg_cnn* c = p->cnn;
  const int L = p->L - 1;
  const int n = p->n[L], N = p->N, G = n * N;
  const int64_t nd = p->ndofs[L];
  SIPG_TRY(ensure_ws(c, (int64_t)G * G * G, false));
  if (!p->stage_c) SIPG_TRY(prob_alloc(p, &p->stage_c, nd));
  if (!p->stage_q) SIPG_TRY(prob_alloc(p, &p->stage_q, nd));
  double* rho = p->wr[L];
  double* scale = p->d_small + 400;
  double* dots = p->d_small + 408;  // [rho . q, q . q]
  SIPG_TRY(sipg_residual(p, L, v, z, rho, s));
  SIPG_HIP(C::launch_pow2_absmax(rho, nd, p->d_partial, scale, s));
  SIPG_HIP(C::launch_gather_f16(rho, n, N, scale, c->x16, s));
  SIPG_TRY(forward(c, G, 1, nullptr, 0.0f, s));
  SIPG_HIP(launch_fill(p->stage_c, 0.0, nd, s));
  SIPG_HIP(C::launch_out_scatter(c->a3, n, N, c->prm, c->sigma, scale, p->stage_c, s));
  SIPG_TRY(sipg_apply(p, L, p->stage_c, p->stage_q, s));
  SIPG_HIP(launch_mdot(rho, nd, 1, p->stage_q, nd, p->d_partial, dots, s));
  SIPG_HIP(launch_mdot(p->stage_q, nd, 1, p->stage_q, nd, p->d_partial, dots + 1, s));
  SIPG_HIP(C::launch_axpy_ratio(dots, dots + 1, p->stage_c, z, nd, s));
  return SIPG_OK;
}

}  // namespace sipg

extern "C" {

int sipg_cnn_num_params(void) { return C::kParams; }

sipg_status sipg_cnn_create(sipg_cnn** out) {
  if (!out) return fail(SIPG_ERR_ARG, "NULL argument");
  *out = nullptr;
  auto* c = new sipg_cnn();
  sipg_status st = SIPG_OK;
  if (st == SIPG_OK) st = dev_alloc(&c->prm, C::kParams);
  if (st == SIPG_OK) st = dev_alloc(&c->am, C::kParams);
  if (st == SIPG_OK) st = dev_alloc(&c->av, C::kParams);
  if (st == SIPG_OK) st = dev_alloc(&c->grad, C::kParams);
  if (st == SIPG_OK) st = dev_alloc(&c->packed, 4 * (size_t)C::kPacked);
  if (st == SIPG_OK) st = dev_alloc(&c->part, (size_t)C::kWgradRows * C::kSegMid);
  if (st == SIPG_OK) st = dev_alloc(&c->lpart, 2 * 1024);
  if (st == SIPG_OK) st = dev_alloc(&c->sums, 2);
  if (st == SIPG_OK) {
    std::vector<float> zero(C::kParams, 0.0f);
    if (hipMemcpy(c->prm, zero.data(), sizeof(float) * C::kParams, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->am, zero.data(), sizeof(float) * C::kParams, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->av, zero.data(), sizeof(float) * C::kParams, hipMemcpyHostToDevice) !=
            hipSuccess ||
        C::launch_pack(c->prm, c->packed, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
      st = fail(SIPG_ERR_HIP, "network initialisation failed");
  }
  if (st != SIPG_OK) {
    std::string msg = g_err;
    sipg_cnn_destroy(c);
    return fail(st, msg);
  }
  *out = c;
  return SIPG_OK;
}

void sipg_cnn_destroy(sipg_cnn* c) {
  if (!c) return;
  hipDeviceSynchronize();
  free_ws(c);
  for (float* p : {c->prm, c->am, c->av, c->grad, c->part, c->lpart, c->sums})
    if (p) hipFree(p);
  if (c->packed) hipFree(c->packed);
  delete c;
}

sipg_status sipg_cnn_set_params(sipg_cnn* c, const float* params, float sigma) {
  if (!c || !params) return fail(SIPG_ERR_ARG, "NULL argument");
  if (!(sigma >= 0.0f) || !std::isfinite(sigma)) return fail(SIPG_ERR_ARG, "sigma must be >= 0");
  std::vector<float> zero(C::kParams, 0.0f);
  SIPG_HIP(hipMemcpy(c->prm, params, sizeof(float) * C::kParams, hipMemcpyHostToDevice));
  SIPG_HIP(hipMemcpy(c->am, zero.data(), sizeof(float) * C::kParams, hipMemcpyHostToDevice));
  SIPG_HIP(hipMemcpy(c->av, zero.data(), sizeof(float) * C::kParams, hipMemcpyHostToDevice));
  SIPG_HIP(C::launch_pack(c->prm, c->packed, nullptr));
  SIPG_HIP(hipDeviceSynchronize());
  c->sigma = sigma;
  c->adam_t = 0;
  return SIPG_OK;
}

sipg_status sipg_cnn_get_params(const sipg_cnn* c, float* params, float* sigma) {
  if (!c) return fail(SIPG_ERR_ARG, "NULL argument");
  SIPG_HIP(hipDeviceSynchronize());
  if (params)
    SIPG_HIP(hipMemcpy(params, c->prm, sizeof(float) * C::kParams, hipMemcpyDeviceToHost));
  if (sigma) *sigma = c->sigma;
  return SIPG_OK;
}

// File format: "SIPGCNN1", int32 parameter count, float32 sigma, float32
// parameters, little-endian (the byte order of the host; gfx950 hosts are
// x86-64 or AArch64 little-endian).
static const char kCnnMagic[8] = {'S', 'I', 'P', 'G', 'C', 'N', 'N', '1'};

sipg_status sipg_cnn_save(const sipg_cnn* c, const char* path) {
  if (!c || !path) return fail(SIPG_ERR_ARG, "NULL argument");
  std::vector<float> prm(C::kParams);
  float sigma = 0.0f;
  SIPG_TRY(sipg_cnn_get_params(c, prm.data(), &sigma));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(SIPG_ERR_UNSUPPORTED, std::string("cannot open for writing: ") + path);
  const int32_t count = C::kParams;
  bool ok = std::fwrite(kCnnMagic, 1, 8, f) == 8 && std::fwrite(&count, 4, 1, f) == 1 &&
            std::fwrite(&sigma, 4, 1, f) == 1 &&
            std::fwrite(prm.data(), 4, prm.size(), f) == prm.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(SIPG_ERR_UNSUPPORTED, std::string("write failed: ") + path);
  return SIPG_OK;
}

sipg_status sipg_cnn_load(sipg_cnn* c, const char* path) {
  if (!c || !path) return fail(SIPG_ERR_ARG, "NULL argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(SIPG_ERR_UNSUPPORTED, std::string("cannot open: ") + path);
  char magic[8] = {0};
  int32_t count = 0;
  float sigma = 0.0f;
  std::vector<float> prm(C::kParams);
  const bool head = std::fread(magic, 1, 8, f) == 8 && std::fread(&count, 4, 1, f) == 1 &&
                    std::fread(&sigma, 4, 1, f) == 1;
  const bool body = head && std::memcmp(magic, kCnnMagic, 8) == 0 && count == C::kParams &&
                    std::fread(prm.data(), 4, prm.size(), f) == prm.size();
  std::fclose(f);
  if (!head || std::memcmp(magic, kCnnMagic, 8) != 0)
    return fail(SIPG_ERR_ARG, std::string("not a network file: ") + path);
  if (count != C::kParams)
    return fail(SIPG_ERR_ARG, "parameter count " + std::to_string(count) + " does not match");
  if (!body) return fail(SIPG_ERR_ARG, std::string("short file: ") + path);
  return sipg_cnn_set_params(c, prm.data(), sigma);
}

sipg_status sipg_cnn_init(sipg_cnn* c, uint64_t seed) {
  if (!c) return fail(SIPG_ERR_ARG, "NULL argument");
  // He-uniform weights (bound sqrt(6 / fan_in)), zero biases; the last
  // layer starts 10x smaller so the untrained correction is small
  Rng rng{seed};
  std::vector<float> w(C::kParams, 0.0f);
  auto fill = [&](int off, int count, int fan_in, double gain) {
    const double bound = gain * std::sqrt(6.0 / fan_in);
    for (int i = 0; i < count; ++i) w[off + i] = (float)((2.0 * rng.uniform() - 1.0) * bound);
  };
  fill(C::kW1, C::kC * 27, 27, 1.0);
  fill(C::kW2, C::kC * C::kC * 27, C::kC * 27, 1.0);
  fill(C::kW3, C::kC * C::kC * 27, C::kC * 27, 1.0);
  fill(C::kW4, C::kC * 27, C::kC * 27, 0.1);
  return sipg_cnn_set_params(c, w.data(), 0.0f);
}

sipg_status sipg_cnn_forward(sipg_cnn* c, int G, int batch, const float* in, float* out,
                             hipStream_t s) {
  if (!c || !in || !out) return fail(SIPG_ERR_ARG, "NULL argument");
  SIPG_TRY(check_grid(G, batch));
  const int64_t np = (int64_t)batch * G * G * G;
  SIPG_TRY(ensure_ws(c, np, false));
  SIPG_HIP(C::launch_f32_to_f16(in, c->x16, np, s));
  return forward(c, G, batch, out, c->sigma, s);
}

sipg_status sipg_cnn_gradient(sipg_cnn* c, int G, int batch, const float* in,
                              const float* target, const float* mask, float* grad, float* loss,
                              hipStream_t s) {
  if (!c || !in || !target || !mask || !grad) return fail(SIPG_ERR_ARG, "NULL argument");
  SIPG_TRY(check_grid(G, batch));
  const int64_t np = (int64_t)batch * G * G * G;
  SIPG_TRY(ensure_ws(c, np, true));
  SIPG_HIP(C::launch_f32_to_f16(in, c->x16, np, s));
  SIPG_HIP(hipMemcpyAsync(c->tgt, target, sizeof(float) * np, hipMemcpyDeviceToDevice, s));
  SIPG_HIP(hipMemcpyAsync(c->msk, mask, sizeof(float) * np, hipMemcpyDeviceToDevice, s));
  SIPG_TRY(backward(c, G, batch, grad, s));
  if (loss) SIPG_HIP(hipMemcpyAsync(loss, c->sums, sizeof(float), hipMemcpyDeviceToDevice, s));
  return SIPG_OK;
}

sipg_status sipg_cnn_gradient_residual(sipg_cnn* c, sipg_problem* p, const double* rho,
                                       float* grad, float* loss, hipStream_t s) {
  if (!c || !p || !rho || !grad) return fail(SIPG_ERR_ARG, "NULL argument");
  SIPG_TRY(check_problem_grid(p));
  const int L = p->L - 1;
  const int G = p->n[L] * p->N;
  const int64_t nd = p->ndofs[L];
  SIPG_TRY(ensure_ws(c, (int64_t)G * G * G, true));
  if (!p->stage_c) SIPG_TRY(prob_alloc(p, &p->stage_c, nd));
  if (!p->stage_q) SIPG_TRY(prob_alloc(p, &p->stage_q, nd));
  SIPG_TRY(residual_backward(c, p, rho, p->stage_c, p->stage_q, grad, s));
  if (loss) SIPG_HIP(hipMemcpyAsync(loss, c->sums, sizeof(float), hipMemcpyDeviceToDevice, s));
  return SIPG_OK;
}

sipg_status sipg_cnn_adam_step(sipg_cnn* c, const float* grad, float lr, hipStream_t s) {
  if (!c || !grad) return fail(SIPG_ERR_ARG, "NULL argument");
  if (!(lr > 0.0f)) return fail(SIPG_ERR_ARG, "lr must be > 0");
  return adam(c, grad, lr, s);
}

sipg_status sipg_cnn_make_pairs(sipg_problem* p, const double* x0, int count, float* rho_grids,
                                float* e_grids, double* scales, hipStream_t s) {
  if (!p || !x0 || !rho_grids || !e_grids) return fail(SIPG_ERR_ARG, "NULL argument");
  if (count < 1) return fail(SIPG_ERR_ARG, "count must be >= 1");
  SIPG_TRY(cartesian_only(p, "the learned stage"));
  const int L = p->L - 1;
  const int64_t n = p->ndofs[L];
  PairBufs w;
  double* x = nullptr;
  sipg_status st = alloc_pair_bufs(p, w);
  if (st == SIPG_OK) st = dev_alloc(&x, n);
  if (st == SIPG_OK && launch_scale_copy(x0, 1.0, x, n, s) != hipSuccess)
    st = fail(SIPG_ERR_HIP, "copy failed");
  for (int j = 0; j < count && st == SIPG_OK; ++j) {
    double sr = 0.0;
    st = make_pair(p, x, w, rho_grids + j * n, e_grids + j * n, &sr, s);
    if (scales) scales[j] = sr;
  }
  hipStreamSynchronize(s);
  free_pair_bufs(w);
  if (x) hipFree(x);
  return st;
}

sipg_status sipg_cnn_train(sipg_problem* p, sipg_cnn* c, const sipg_cnn_train_opts* o,
                           sipg_cnn_train_info* info) {
  if (!p || !c || !o || !info) return fail(SIPG_ERR_ARG, "NULL argument");
  SIPG_TRY(check_problem_grid(p));
  const int L = p->L - 1;
  const int G = p->n[L] * p->N;
  const int64_t n = p->ndofs[L];
  if (o->n_chains < 1 || o->chain_length < 1) return fail(SIPG_ERR_ARG, "empty training run");
  if (o->loss != 0 && o->loss != 1) return fail(SIPG_ERR_ARG, "loss must be 0 or 1");
  const bool resid = o->loss == 1;
  if (!resid && (o->crops_per_pair < 1 || o->crops_per_pair > 16))
    return fail(SIPG_ERR_ARG, "crops_per_pair must be in 1..16");
  if (!resid && (o->crop < C::kTile || o->crop % C::kTile || o->crop > G))
    return fail(SIPG_ERR_ARG, "crop must be a multiple of 16 and <= n (k+1)");
  if (!(o->lr > 0.0f)) return fail(SIPG_ERR_ARG, "lr must be > 0");
  std::memset(info, 0, sizeof(*info));
  hipStream_t s = nullptr;
  SIPG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  const auto t0 = std::chrono::steady_clock::now();
  PairBufs w;
  double *b = nullptr, *x = nullptr;
  float *rho_g = nullptr, *e_g = nullptr;
  const int cr = o->crop, nc = o->crops_per_pair;
  sipg_status st = alloc_pair_bufs(p, w);
  if (st == SIPG_OK) st = dev_alloc(&b, n);
  if (st == SIPG_OK) st = dev_alloc(&x, n);
  if (st == SIPG_OK) st = dev_alloc(&rho_g, n);
  if (st == SIPG_OK) st = dev_alloc(&e_g, n);
  if (st == SIPG_OK)
    st = ensure_ws(c, resid ? (int64_t)G * G * G : (int64_t)nc * cr * cr * cr, true);
  Rng rng{o->seed};
  double gen = 0.0;
  for (int ch = 0; ch < o->n_chains && st == SIPG_OK; ++ch) {
    // smooth right-hand side: 4 sine modes, a ~ U[-1, 1], p, q, r ~ U{1..4}
    double amps[4];
    int pqr[12];
    for (int m = 0; m < 4; ++m) {
      amps[m] = 2.0 * rng.uniform() - 1.0;
      for (int a = 0; a < 3; ++a) pqr[3 * m + a] = 1 + rng.below(4);
    }
    st = sipg_rhs_sines(p, L, 4, amps, pqr, b, s);
    if (st == SIPG_OK && launch_fill(x, 0.0, n, s) != hipSuccess) st = fail(SIPG_ERR_HIP, "fill");
    for (int it = 0; it < 3 && st == SIPG_OK; ++it) st = sipg_vcycle(p, L, x, b, s);
    for (int j = 0; j < o->chain_length && st == SIPG_OK; ++j) {
      const auto g1 = std::chrono::steady_clock::now();
      st = make_pair(p, x, w, rho_g, e_g, nullptr, s);
      gen += std::chrono::duration<double>(std::chrono::steady_clock::now() - g1).count();
      if (st != SIPG_OK) break;
      if (!(c->sigma > 0.0f)) {  // output scale from the first pair: mean |e| / mean |rho|
        std::vector<float> hr(n), he(n);
        // the pair was made on the non-blocking stream s: finish it before the
        // (null-stream) copies read the grids
        if (hipStreamSynchronize(s) != hipSuccess ||
            hipMemcpy(hr.data(), rho_g, sizeof(float) * n, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(he.data(), e_g, sizeof(float) * n, hipMemcpyDeviceToHost) != hipSuccess) {
          st = fail(SIPG_ERR_HIP, "copy failed");
          break;
        }
        double sr = 0.0, se = 0.0;
        for (int64_t i = 0; i < n; ++i) {
          sr += std::fabs(hr[i]);
          se += std::fabs(he[i]);
        }
        c->sigma = (float)std::ldexp(1.0, (int)std::lround(std::log2(se / sr)));
      }
      if (resid) {  // the whole grid: rho / s into w.e (free after make_pair)
        if (C::launch_div_scale(w.rho, w.scale, w.e, n, s) != hipSuccess) {
          st = fail(SIPG_ERR_HIP, "scale launch failed");
          break;
        }
        st = residual_backward(c, p, w.e, w.r, w.z, c->grad, s);
      } else {
        C::CropJob job{};
        job.count = nc;
        for (int k = 0; k < nc; ++k)
          for (int a = 0; a < 3; ++a) job.off[k][a] = rng.below(G - cr + 1);
        if (C::launch_crops(rho_g, e_g, G, cr, job, c->x16, c->tgt, c->msk, s) != hipSuccess) {
          st = fail(SIPG_ERR_HIP, "crop launch failed");
          break;
        }
        st = backward(c, cr, nc, c->grad, s);
      }
      if (st == SIPG_OK) st = adam(c, c->grad, o->lr, s);
      if (st != SIPG_OK) break;
      const bool first = info->steps == 0;
      ++info->steps;
      const bool last = ch == o->n_chains - 1 && j == o->chain_length - 1;
      if (first || last || (o->log_every > 0 && info->steps % o->log_every == 0)) {
        float lv = 0.0f;
        if (hipMemcpyAsync(&lv, c->sums, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
          st = fail(SIPG_ERR_HIP, "loss copy failed");
          break;
        }
        if (first) info->loss_first = lv;
        info->loss_last = lv;
        if (!std::isfinite(lv)) st = fail(SIPG_ERR_NONFINITE, "training loss is not finite");
      }
    }
  }
  hipStreamSynchronize(s);
  info->sigma = c->sigma;
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  info->seconds_pairs = gen;
  free_pair_bufs(w);
  for (double* q : {b, x})
    if (q) hipFree(q);
  for (float* q : {rho_g, e_g})
    if (q) hipFree(q);
  hipStreamDestroy(s);
  return st;
}

sipg_status sipg_cnn_attach(sipg_problem* p, sipg_cnn* c) {
  if (!p) return fail(SIPG_ERR_ARG, "NULL handle");
  if (c) SIPG_TRY(check_problem_grid(p));
  p->cnn = c;
  return SIPG_OK;
}

}  // extern "C"
