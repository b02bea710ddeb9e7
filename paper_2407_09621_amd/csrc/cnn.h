// Learned correction stage (a project extension; the paper has no learned
// part): a 3D convolutional network 1 -> 32 -> 32 -> 32 -> 1 channels with
// 3x3x3 kernels, zero padding and ReLU between layers, on the G^3 grid of DG
// coefficients.  FP16 weights and activations, FP32 accumulation.
//
// Parameter vector (FP32 master copy, also the C-ABI order):
//   w1[co][27] b1[32] w2[co][ci][27] b2[32] w3[co][ci][27] b3[32] w4[ci][27] b4
// with the 27 offsets ordered d = 9 (dz+1) + 3 (dy+1) + (dx+1).
// Activations are channel-last FP16 arrays act[sample][p][32],
// p = gx + G (gy + G gz).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace sipg {
namespace cnn {

constexpr int kC = 32;
constexpr int kW1 = 0, kB1 = kW1 + kC * 27, kW2 = kB1 + kC, kB2 = kW2 + kC * kC * 27;
constexpr int kW3 = kB2 + kC, kB3 = kW3 + kC * kC * 27, kW4 = kB3 + kC, kB4 = kW4 + kC * 27;
constexpr int kParams = kB4 + 1;
constexpr int kPacked = 27 * 2 * 64 * 8;  // FP16 weight fragments of one 32 -> 32 layer
constexpr int kTile = 16;                 // grids must be multiples of this size

// Partial-sum rows of the weight-gradient kernels: one row per block, each
// row the contiguous parameter segment [w_l, b_l] of its layer.
constexpr int kSegIn = kC * 27 + kC, kSegMid = kC * kC * 27 + kC, kSegOut = kC * 27 + 1;
constexpr int kWgradRows = 1024;

// Workspace of the weight gradients for np grid points: ot holds np * 32
// FP16 values (a channel-octet copy), os 3 * np * 32 (three x-shifted
// copies; the one-channel layers use 3 * np of it).
struct WgradBufs {
  _Float16* ot;
  _Float16* os;
};

// ---- inference / forward ----------------------------------------------------
// a1 = ReLU(conv1(x)): x FP16 [ns][G^3], a1 FP16 [ns][G^3][32]
hipError_t launch_in_fwd(const _Float16* x, int G, int ns, const float* prm, _Float16* a1,
                         hipStream_t s);
// 32 -> 32 layer on the matrix cores.  mode 0: out = ReLU(conv(in) + b);
// mode 1 (data gradient): out = conv_flip(in) * [act_prev > 0].
// `packed` holds the layer's FP16 fragments (see launch_pack).
hipError_t launch_mid(int mode, const _Float16* in, const _Float16* packed, const float* bias,
                      const _Float16* act_prev, _Float16* out, int G, int ns, hipStream_t s);
// y = scale * (conv4(a3) + b4): FP32 grid [ns][G^3]
hipError_t launch_out_fwd(const _Float16* a3, int G, int ns, const float* prm, float scale,
                          float* y, hipStream_t s);
// z[cell(p)] += scale * sigma * conv4(a3)[p] on the cell-blocked FP64 vector
// of n^3 cells of N^3 nodes (G = n N); scale read from the device.
hipError_t launch_out_scatter(const _Float16* a3, int n, int N, const float* prm, float sigma,
                              const double* scale, double* z, hipStream_t s);
// FP16 fragments of layers 2 and 3, forward (dst[0], dst[1]) and flipped /
// transposed for the data gradient (dst[2], dst[3]).
hipError_t launch_pack(const float* prm, _Float16* packed4, hipStream_t s);

// ---- grid mapping -------------------------------------------------------------
// scale = 2^ceil(log2 max|v|) (0 if v = 0); partial holds >= 1024 doubles
hipError_t launch_pow2_absmax(const double* v, int64_t n, double* partial, double* scale,
                              hipStream_t s);
// x[p] = v[cell(p)] / scale as FP16 (0 if scale = 0)
hipError_t launch_gather_f16(const double* v, int n, int N, const double* scale, _Float16* x,
                             hipStream_t s);
// g[p] = v[cell(p)] / scale as FP32
hipError_t launch_gather_f32(const double* v, int n, int N, const double* scale, float* g,
                             hipStream_t s);
hipError_t launch_f32_to_f16(const float* a, _Float16* b, int64_t n, hipStream_t s);
// y += (num[0] / den[0]) x (nothing if den[0] = 0); scalars on the device
hipError_t launch_axpy_ratio(const double* num, const double* den, const double* x, double* y,
                             int64_t n, hipStream_t s);

// out = v / scale[0] (0 if scale[0] = 0), scale on the device
hipError_t launch_div_scale(const double* v, const double* scale, double* out, int64_t n,
                            hipStream_t s);

// ---- training -----------------------------------------------------------------
// Residual loss: sums[0] = rr / pp, sums[1] = sigma pp b / (2 a S) for the
// output gradient g4 = -grid(A r) / S, r = rho - (a / b) q (device scalars
// rr = ||r||^2, pp = ||rho||^2, ab = [rho . q, q . q]; sums[1] = 0 when
// a = 0 or b = 0: no gradient)
hipError_t launch_residual_sums(const double* rr, const double* pp, const double* S,
                                const double* ab, float sigma, float* sums, hipStream_t s);
// Loss L = sum m (sigma y - t)^2 / sum m.  g4 = 2 m (y - t / sigma), which is
// dL/dy times sum(m) / sigma^2 (kept O(1) for the FP16 backward pass);
// sums[0] = L, sums[1] = sum m (two-pass, partial holds >= 2 * 1024 floats)
hipError_t launch_loss(const float* y, const float* t, const float* m, int64_t n, float sigma,
                       float* g4, float* partial, float* sums, hipStream_t s);
// g3 = [a3 > 0] * conv4^T(g4) (FP16)
hipError_t launch_out_bwd(const float* g4, const _Float16* a3, int G, int ns, const float* prm,
                          _Float16* g3, hipStream_t s);
// Block partials (kWgradRows rows as above) of the weight gradients on the
// matrix cores, through the octet copies in `w` (see cnn.hip)
hipError_t launch_out_wgrad(const _Float16* a3, const float* g4, int G, int ns,
                            const WgradBufs& w, float* part, hipStream_t s);
hipError_t launch_mid_wgrad(const _Float16* a, const _Float16* g, int G, int ns,
                            const WgradBufs& w, float* part, hipStream_t s);
hipError_t launch_in_wgrad(const _Float16* x, const _Float16* g1, int G, int ns,
                           const WgradBufs& w, float* part, hipStream_t s);
// grad[i] = sigma^2 sum_b part[b][i] / sums[1] for i < seg
hipError_t launch_reduce_rows(const float* part, int seg, const float* sums, float sigma,
                              float* grad, hipStream_t s);
// Adam step on the master parameters; c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
hipError_t launch_adam(float* prm, float* m, float* v, const float* grad, int n, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, hipStream_t s);
// crops of side c at (z, y, x) offsets of full FP32 grids of side G:
// x16 (input, FP16), t (target), m (mask of the receptive radius)
struct CropJob {
  int count;
  int off[16][3];
};
hipError_t launch_crops(const float* in, const float* target, int G, int c, const CropJob& j,
                        _Float16* x16, float* t, float* m, hipStream_t s);

}  // namespace cnn
}  // namespace sipg
