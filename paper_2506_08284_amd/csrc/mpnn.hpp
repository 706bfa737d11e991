// Learned initial guess for P^(e): message-passing network on the level-0
// pattern entries (forward, backward and Adam on the GPU).
#pragma once
#include "amg.hpp"

namespace hc {

constexpr int kNF = 16;      // input features per pattern entry
constexpr int kHD = 64;      // hidden width
constexpr int kNL = 3;       // message-passing layers
constexpr int kKZ = 3 * kHD; // [h, mean_row, mean_col]
constexpr int64_t kOffWin = 0;
constexpr int64_t kOffBin = kNF * kHD;
constexpr int64_t kOffW0 = kOffBin + kHD;
constexpr int64_t kLayerStride = (int64_t)kKZ * kHD + kHD;
constexpr int64_t kOffWout = kOffW0 + kNL * kLayerStride;
constexpr int64_t kOffBout = kOffWout + kHD;
constexpr int64_t kNParam = kOffBout + 1;
inline int64_t off_W(int l) { return kOffW0 + l * kLayerStride; }
inline int64_t off_b(int l) { return off_W(l) + (int64_t)kKZ * kHD; }

struct Net {
  Ctx ctx;
  DBuf<float> w, m, v, g;  // FP32 master weights, Adam moments, gradient
  DBuf<uint16_t> wt_in;    // W_in^T (64 x 16) bf16
  DBuf<uint16_t> wt[kNL];  // W_l^T (64 x 192) bf16, forward products
  DBuf<uint16_t> wr[kNL];  // W_l   (192 x 64) bf16, input-gradient products
  bool fp32_products = false;  // debug: FP32-operand products (hcurl_mpnn_set_fp32_products)
  void refresh_bf16(Ctx& c);
};

// Graph and features of one level-0 pattern (a training sample, or the
// inference input inside setup).
struct Sample {
  hipStream_t s = nullptr;
  int64_t E = 0;
  int nrow = 0, ncol = 0;
  DBuf<int> rowptr, row_of, col_of, colptr, colidx;
  DBuf<float> X;  // E x 16
  DBuf<double> p0, target;
  // activations kept for the backward pass
  DBuf<float> h[kNL + 1], u[kNL + 1], mr[kNL], mc[kNL];
  DBuf<float> dh, du, dz, mdr, mdc;
  // inference: BF16 activations (alternating) and means
  DBuf<uint16_t> hb[2], mrb, mcb;
  DBuf<double> delta;
  // activations are transient: released after every forward / training step
  void release_workspace() {
    for (auto& b : h) b.release();
    for (auto& b : u) b.release();
    for (auto& b : mr) b.release();
    for (auto& b : mc) b.release();
    dh.release(); du.release(); dz.release(); mdr.release(); mdc.release();
    for (auto& b : hb) b.release();
    mrb.release(); mcb.release();
  }
};

// Builds graph and features from level 0 (L0) and its coarse gradient (L1's
// edges), with the plain initial values p0plain and min-norm values pmin.
void mpnn_build_sample(Hierarchy& H, Level& L0, const Level& L1, const double* p0plain, const double* pmin, Sample& S);
// delta (device, E doubles) = network correction for the sample
void mpnn_forward(Net& net, Sample& S, Ctx& c, bool keep);
// loss and gradient into net.g
double mpnn_loss_grad(Net& net, Sample& S, Ctx& c);
void mpnn_adam(Net& net, float lr, float b1, float b2, float eps, int step, Ctx& c);

}  // namespace hc

struct hcurl_mpnn_s {
  hc::Net net;
};
struct hcurl_mpnn_sample_s {
  hc::Ctx ctx;
  hc::Sample S;
};
