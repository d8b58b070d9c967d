// Learned warm start network: shapes, parameter layout and launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "flash_device.h"

namespace flash {

constexpr int kFeat = 16;      // per-contact input features
constexpr int kHidden = 128;   // width of the three hidden layers
constexpr int kOut = 3;        // (n, t1, t2) multiplier prediction
constexpr int kNorm = 2 * kFeat + kOut;   // feature means, feature inverse scales, label scales

// Parameters packed as W1, b1, W2, b2, W3, b3, W4, b4; W row-major (out x in).
struct MlpLayout {
  static constexpr long w1 = 0;
  static constexpr long b1 = w1 + (long)kHidden * kFeat;
  static constexpr long w2 = b1 + kHidden;
  static constexpr long b2 = w2 + (long)kHidden * kHidden;
  static constexpr long w3 = b2 + kHidden;
  static constexpr long b3 = w3 + (long)kHidden * kHidden;
  static constexpr long w4 = b3 + kHidden;
  static constexpr long b4 = w4 + (long)kOut * kHidden;
  static constexpr long total = b4 + kOut;
};
static_assert(MlpLayout::total == 35587, "parameter count");

// C = act(op(A) op(B) + bias) with bf16 operands and FP32 accumulation.
struct GemmArgs {
  const float* A; long sam, sak;
  const float* B; long sbk, sbn;
  float* C; long scm, scn;
  const float* bias;
  long M; int N, K;
  int relu, accumulate;
  float* work;      // optional split-K scratch (nullptr: no split); work_cap floats
  long work_cap;
  int kslice;       // set by launch_gemm
};

// Device buffers of an inference pass over the contact slots of a batch.
struct MlpBuffers {
  const float* W;      // FP32 copy of the bf16 weights (exactly representable)
  const float* norm;   // [kNorm]
  float* feat;         // [rows * kFeat] raw features
  int* need;           // [rows] 1: active contact without a previous-step multiplier
  float* Y;            // [rows * kOut]
  double* lam_ml;      // [rows * 3] cone-projected candidate multipliers
};

void launch_gemm(const GemmArgs& g, hipStream_t s);
// Raises the dynamic LDS limit of the fused forward kernel (call once before its first launch).
void prepare_mlp();
// Fused forward pass on the matrix cores: Y = network(X).  norm != nullptr: X holds raw
// features; need != nullptr: 32-row tiles without a flagged row are skipped; H1..H3 != nullptr:
// hidden activations stored for the backward pass.
void launch_mlp_fused(const float* W, const float* norm, const float* X, long rows, const int* need, float* Y,
                      float* H1, float* H2, float* H3, hipStream_t s);
void mlp_backward(const float* W, const float* X, long n, const float* H1, const float* H2, const float* H3,
                  float* dY, float* dA, float* dB, float* G, float* work, long work_cap, hipStream_t s);
void mlp_loss(const float* Y, const float* Lab, long n, float* dY, double* partial, float* loss, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, int t, hipStream_t s);
void launch_gather_batch(const float* feat, const float* lab, const int* idx, int B, const float* norm, float* X,
                         float* Y, hipStream_t s);
void launch_col_moments(const float* X, long rows, int cols, double* out, hipStream_t s);

template <class T> void launch_ws_features(const DevBatch<T>& B, const T* mu_env, float* feat, int* need,
                                          hipStream_t s);
// labels of the first contact solve of a step (launched right after it)
template <class T> void launch_ws_labels(const DevBatch<T>& B, const float* feat, float* lab, hipStream_t s);
template <class T> void launch_ws_infer(const DevBatch<T>& B, const T* mu_env, const MlpBuffers& M, hipStream_t s);
// Appends the active contact slots' rows (feature, label) in env order; base = rows already stored.
// coff: device scratch of n_envs + 1 ints; coff[n_envs] receives the number of rows appended.
template <class T> void launch_ws_compact(const DevBatch<T>& B, const float* feat, const float* lab, float* out_feat,
                                         float* out_lab, long base, int* coff, hipStream_t s);

}  // namespace flash
