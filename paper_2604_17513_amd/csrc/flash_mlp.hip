// Learned warm start: a 16 -> 128 -> 128 -> 128 -> 3 ReLU MLP that predicts the
// contact multipliers of a step from local features.  Every GEMM runs on the
// CDNA matrix cores (v_mfma_f32_32x32x8bf16_1k): operands are rounded to
// bfloat16 (round to nearest even), products accumulate in FP32.  Training
// keeps FP32 master weights and Adam moments; bias gradients and losses use
// fixed-order reductions, so a training run is deterministic.
#include <algorithm>

#include "flash_device.h"
#include "flash_launch.h"
#include "flash_mlp.h"

namespace flash {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// C(m, n) = act(sum_k A(m, k) B(k, n) + bias[n]) (+ C if accumulate).
// A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn]; one wave per
// 32 x 32 tile of C; 32x32x8 lane layout: A row = lane % 32, k = 4 (lane / 32) + t;
// B column = lane % 32, same k; D row = 8 (r / 4) + 4 (lane / 32) + r % 4, column = lane % 32.
// blockIdx.z selects a K slice of g.kslice rows when the product is split over K: the
// slice's partial sums go to g.work[z][M][N] and a second kernel adds the slices in order.
__global__ void __launch_bounds__(64) k_gemm_bf16(GemmArgs g) {
  const int l = threadIdx.x;
  const long m0 = (long)blockIdx.x * 32, n0 = (long)blockIdx.y * 32;
  const long i = m0 + (l & 31), j = n0 + (l & 31);
  const int kq = 4 * (l >> 5);
  const int kb = g.work ? (int)blockIdx.z * g.kslice : 0;
  const int ke = g.work ? min(g.K, kb + g.kslice) : g.K;
  floatx16 c = {};
  for (int k0 = kb; k0 < ke; k0 += 8) {
    bf16x4 a, b;
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + kq + t;
      const float av = (i < g.M && k < ke) ? g.A[i * g.sam + (long)k * g.sak] : 0.f;
      const float bv = (j < g.N && k < ke) ? g.B[(long)k * g.sbk + j * g.sbn] : 0.f;
      a[t] = f2bf(av);
      b[t] = f2bf(bv);
    }
    c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
  }
  if (g.work) {
    float* wk = g.work + (size_t)blockIdx.z * g.M * g.N;
    for (int r = 0; r < 16; ++r) {
      const long ii = m0 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
      const long jj = n0 + (l & 31);
      if (ii < g.M && jj < g.N) wk[ii * g.N + jj] = c[r];
    }
    return;
  }
  for (int r = 0; r < 16; ++r) {
    const long ii = m0 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
    const long jj = n0 + (l & 31);
    if (ii < g.M && jj < g.N) {
      float v = c[r];
      if (g.bias) v += g.bias[jj];
      if (g.relu) v = fmaxf(v, 0.f);
      float* dst = g.C + ii * g.scm + jj * g.scn;
      *dst = g.accumulate ? *dst + v : v;
    }
  }
}

// sum of the K slices in slice order, then the epilogue of the plain kernel
__global__ void k_splitk_reduce(GemmArgs g, int slices) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.M * g.N) return;
  const long ii = idx / g.N, jj = idx - ii * g.N;
  float v = 0.f;
  for (int z = 0; z < slices; ++z) v += g.work[(size_t)z * g.M * g.N + idx];
  if (g.bias) v += g.bias[jj];
  if (g.relu) v = fmaxf(v, 0.f);
  float* dst = g.C + ii * g.scm + jj * g.scn;
  *dst = g.accumulate ? *dst + v : v;
}

void launch_gemm(const GemmArgs& g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0) return;
  GemmArgs g = g0;
  dim3 grid((unsigned)((g.M + 31) / 32), (unsigned)((g.N + 31) / 32));
  const long tiles = (long)grid.x * grid.y;
  // few output tiles over a long K (weight gradients): split K so that the chip fills
  int slices = 1;
  if (g.work && tiles < 512 && g.K > 256) {
    slices = (int)std::min<long>((g.K + 127) / 128, std::max<long>(1, 1024 / tiles));
    slices = std::min<long>(slices, g.work_cap / (g.M * g.N));
  }
  if (slices <= 1) {
    g.work = nullptr;
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(64), 0, s, g);
    return;
  }
  g.kslice = ((g.K + slices - 1) / slices + 7) / 8 * 8;
  slices = (g.K + g.kslice - 1) / g.kslice;
  grid.z = (unsigned)slices;
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(64), 0, s, g);
  const long mn = g.M * g.N;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, g, slices);
}

// dH <- dH * (H > 0)
__global__ void k_relu_grad(float* dH, const float* H, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(H[i] > 0.f)) dH[i] = 0.f;
}

// dY = 2 (Y - L) / (rows * 3); per-block partial sums of (Y - L)^2 in fixed order
__global__ void k_mse(const float* Y, const float* L, long n, float* dY, double* partial) {
  __shared__ double sh[256];
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  double e2 = 0.0;
  if (i < n) {
    const float d = Y[i] - L[i];
    dY[i] = 2.f * d / (float)n;
    e2 = (double)d * d;
  }
  sh[threadIdx.x] = e2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_sum_partials(const double* partial, int nb, long n, float* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    *loss = (float)(s / (double)n);
  }
}

// out[c] = sum_r X[r * ld + c], one block per column, fixed tree order
__global__ void k_colsum(const float* X, long rows, int ld, float* out) {
  __shared__ float sh[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (long r = threadIdx.x; r < rows; r += 256) s += X[r * ld + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = sh[0];
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// minibatch gather with feature / label normalisation
__global__ void k_gather_batch(const float* feat, const float* lab, const int* idx, int B, const float* norm,
                               float* X, float* Y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= B) return;
  const long s = idx[r];
  for (int k = 0; k < kFeat; ++k) X[r * kFeat + k] = (feat[s * kFeat + k] - norm[k]) * norm[kFeat + k];
  for (int k = 0; k < 3; ++k) Y[r * 3 + k] = lab[s * 3 + k] * norm[2 * kFeat + k];
}

// ---------------------------------------------------------------------------
// forward / backward of the network on row-major activations
// ---------------------------------------------------------------------------
void mlp_forward(const float* W, const float* X, long n, float* H1, float* H2, float* H3, float* Y, hipStream_t s) {
  const MlpLayout L;
  auto lin = [&](const float* in, int nin, const float* w, const float* b, int nout, float* out, int relu) {
    GemmArgs g{};
    g.M = n; g.N = nout; g.K = nin;
    g.A = in; g.sam = nin; g.sak = 1;
    g.B = w; g.sbk = 1; g.sbn = nin;    // B(k, n) = W[n][k]
    g.C = out; g.scm = nout; g.scn = 1;
    g.bias = b; g.relu = relu; g.accumulate = 0;
    launch_gemm(g, s);
  };
  lin(X, kFeat, W + L.w1, W + L.b1, kHidden, H1, 1);
  lin(H1, kHidden, W + L.w2, W + L.b2, kHidden, H2, 1);
  lin(H2, kHidden, W + L.w3, W + L.b3, kHidden, H3, 1);
  lin(H3, kHidden, W + L.w4, W + L.b4, 3, Y, 0);
}

// grads of the mean-squared loss; dY holds dLoss/dY on entry (overwritten scratch: dA, dB)
void mlp_backward(const float* W, const float* X, long n, const float* H1, const float* H2, const float* H3,
                  float* dY, float* dA, float* dB, float* G, float* work, long work_cap, hipStream_t s) {
  const MlpLayout L;
  // dW = dZ^T * Hin  (nout x nin), db = colsum(dZ)
  auto wgrad = [&](const float* dZ, int nout, const float* Hin, int nin, float* dW, float* db) {
    GemmArgs g{};
    g.M = nout; g.N = nin; g.K = (int)n;
    g.A = dZ; g.sam = 1; g.sak = nout;   // A(m, k) = dZ[k][m]
    g.B = Hin; g.sbk = nin; g.sbn = 1;   // B(k, n) = Hin[k][n]
    g.C = dW; g.scm = nin; g.scn = 1;
    g.work = work; g.work_cap = work_cap;
    launch_gemm(g, s);
    hipLaunchKernelGGL(k_colsum, dim3(nout), dim3(256), 0, s, dZ, n, nout, db);
  };
  // dHin = dZ * W (n x nin)
  auto dgrad = [&](const float* dZ, int nout, const float* w, int nin, float* dH) {
    GemmArgs g{};
    g.M = n; g.N = nin; g.K = nout;
    g.A = dZ; g.sam = nout; g.sak = 1;
    g.B = w; g.sbk = nin; g.sbn = 1;     // B(k, n) = W[k][n]
    g.C = dH; g.scm = nin; g.scn = 1;
    launch_gemm(g, s);
  };
  const long nh = n * kHidden;
  const unsigned gb = (unsigned)((nh + 255) / 256);
  wgrad(dY, 3, H3, kHidden, G + L.w4, G + L.b4);
  dgrad(dY, 3, W + L.w4, kHidden, dA);
  hipLaunchKernelGGL(k_relu_grad, dim3(gb), dim3(256), 0, s, dA, H3, nh);
  wgrad(dA, kHidden, H2, kHidden, G + L.w3, G + L.b3);
  dgrad(dA, kHidden, W + L.w3, kHidden, dB);
  hipLaunchKernelGGL(k_relu_grad, dim3(gb), dim3(256), 0, s, dB, H2, nh);
  wgrad(dB, kHidden, H1, kHidden, G + L.w2, G + L.b2);
  dgrad(dB, kHidden, W + L.w2, kHidden, dA);
  hipLaunchKernelGGL(k_relu_grad, dim3(gb), dim3(256), 0, s, dA, H1, nh);
  wgrad(dA, kHidden, X, kFeat, G + L.w1, G + L.b1);
}

void mlp_loss(const float* Y, const float* Lab, long n, float* dY, double* partial, float* loss, hipStream_t s) {
  const long m = 3 * n;
  const int nb = (int)((m + 255) / 256);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, Y, Lab, m, dY, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1), 0, s, partial, nb, m, loss);
}

void launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, int t, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, 1e-8f, c1, c2);
}

void launch_gather_batch(const float* feat, const float* lab, const int* idx, int B, const float* norm, float* X,
                         float* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_batch, dim3((B + 255) / 256), dim3(256), 0, s, feat, lab, idx, B, norm, X, Y);
}

// ---------------------------------------------------------------------------
// per-contact features and labels (one thread per contact slot of every env)
// features: d0/dc, n.u~/dc, (h v - dobs).{n,t1,t2}/dc, s lambda0/dc (3), had-warm-start,
// mu, log10(Gbar_vv m_v), log10(m_v / 1 g), contacts on the vertex, (g.n) h^2/dc,
// (dobs.n)/dc, 1.
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_ws_features(DevBatch<T> B, const T* mu_env, float* feat) {
  const long slot = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= (long)B.n_envs * B.cap) return;
  const int e = (int)(slot / B.cap), jj = (int)(slot - (long)e * B.cap);
  float* f = feat + slot * kFeat;
  if (jj >= B.ccount[e]) {
    for (int k = 0; k < kFeat; ++k) f[k] = 0.f;
    return;
  }
  const double dc = B.margin > 0 ? B.margin : 1e-3;
  const int vloc = B.cvert[slot];
  const int vi = B.voff[e] + vloc;
  const T* F = B.cframe + 9 * slot;
  const int o = e * kMaxObs + B.cobs[slot];
  double dob[3];
  for (int k = 0; k < 3; ++k) dob[k] = B.obs_move[o] != 0 ? B.h * B.obs_vel[3 * o + k] : 0.0;
  double ut[3], hv[3];
  for (int k = 0; k < 3; ++k) {
    ut[k] = (double)B.ut[(size_t)k * B.NV + vi];
    hv[k] = B.h * (double)B.v[(size_t)k * B.NV + vi] - dob[k];
  }
  const double m = (double)B.mass[vi];
  const double s = B.h * B.h / m;
  const T* G = B.G + B.goff[e];
  const double gvv = (double)G[(size_t)vloc * B.gld[e] + vloc];
  auto dotF = [&](int a, const double* w) {
    return (double)F[3 * a] * w[0] + (double)F[3 * a + 1] * w[1] + (double)F[3 * a + 2] * w[2];
  };
  int nc = 1;
  if (jj > 0 && B.cvert[slot - 1] == vloc) ++nc;
  if (jj + 1 < B.ccount[e] && B.cvert[slot + 1] == vloc) ++nc;
  const double g[3] = {B.g[0], B.g[1], B.g[2]};
  f[0] = (float)(B.cd0d[slot] / dc);
  f[1] = (float)(dotF(0, ut) / dc);
  f[2] = (float)(dotF(0, hv) / dc);
  f[3] = (float)(dotF(1, hv) / dc);
  f[4] = (float)(dotF(2, hv) / dc);
  f[5] = (float)(s * B.clam[3 * slot] / dc);
  f[6] = (float)(s * B.clam[3 * slot + 1] / dc);
  f[7] = (float)(s * B.clam[3 * slot + 2] / dc);
  f[8] = B.cnew[slot] ? 0.f : 1.f;
  f[9] = (float)mu_env[e];
  f[10] = (float)log10(fmax(gvv * m, 1e-30));
  f[11] = (float)log10(m / 1e-3);
  f[12] = (float)nc;
  f[13] = (float)(dotF(0, g) * B.h * B.h / dc);
  f[14] = (float)(dotF(0, dob) / dc);
  f[15] = 1.f;
}

// label: s (lambda - lambda_ws) / dc, the first contact solve's change of each
// contact's multipliers from its previous-step warm start (features 5..7 hold s lambda_ws / dc)
template <class T>
__global__ void k_ws_labels(DevBatch<T> B, const float* feat, float* lab) {
  const long slot = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= (long)B.n_envs * B.cap) return;
  const int e = (int)(slot / B.cap), jj = (int)(slot - (long)e * B.cap);
  float* y = lab + slot * 3;
  if (jj >= B.ccount[e]) { y[0] = y[1] = y[2] = 0.f; return; }
  const double dc = B.margin > 0 ? B.margin : 1e-3;
  const int vi = B.voff[e] + B.cvert[slot];
  const double s = B.h * B.h / (double)B.mass[vi];
  for (int k = 0; k < 3; ++k) y[k] = (float)(s * B.clam[3 * slot + k] / dc - (double)feat[slot * kFeat + 5 + k]);
}

// network output -> candidate multipliers (cone-projected) for the contact solve
template <class T>
__global__ void k_ws_candidates(DevBatch<T> B, const T* mu_env, const float* feat, const float* Y, const float* norm,
                                double* lam_ml) {
  const long slot = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= (long)B.n_envs * B.cap) return;
  const int e = (int)(slot / B.cap), jj = (int)(slot - (long)e * B.cap);
  if (jj >= B.ccount[e]) return;
  const double dc = B.margin > 0 ? B.margin : 1e-3;
  const int vi = B.voff[e] + B.cvert[slot];
  const double s = B.h * B.h / (double)B.mass[vi];
  double l[3];
  for (int k = 0; k < 3; ++k)
    l[k] = ((double)feat[slot * kFeat + 5 + k] + (double)Y[slot * 3 + k] / (double)norm[2 * kFeat + k]) * dc / s;
  // a non-finite prediction stays non-finite: the solve's merit test then rejects it
  l[0] = l[0] > 0.0 ? l[0] : (l[0] == l[0] ? 0.0 : l[0]);
  const double lt = sqrt(l[1] * l[1] + l[2] * l[2]), rho = (double)mu_env[e] * l[0];
  if (lt > rho) { const double f = lt > 0 ? rho / lt : 0.0; l[1] *= f; l[2] *= f; }
  for (int k = 0; k < 3; ++k) lam_ml[3 * slot + k] = l[k];
}

// per-column sum and sum of squares (FP64, fixed order), one block per column
__global__ void k_col_moments(const float* X, long rows, int cols, double* out) {
  __shared__ double s1[256], s2[256];
  const int c = blockIdx.x;
  double a = 0.0, q = 0.0;
  for (long r = threadIdx.x; r < rows; r += 256) {
    const double v = X[r * cols + c];
    a += v;
    q += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = q;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) { s1[threadIdx.x] += s1[threadIdx.x + k]; s2[threadIdx.x] += s2[threadIdx.x + k]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[2 * c] = s1[0]; out[2 * c + 1] = s2[0]; }
}

void launch_col_moments(const float* X, long rows, int cols, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_col_moments, dim3(cols), dim3(256), 0, s, X, rows, cols, out);
}

// coff[e] = number of active contacts in envs before e (coff[n_envs] = total)
__global__ void k_count_offsets(const int* ccount, int n_envs, int cap, int* coff) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int s = 0;
    for (int e = 0; e < n_envs; ++e) {
      coff[e] = s;
      const int c = ccount[e];
      s += c < cap ? c : cap;
    }
    coff[n_envs] = s;
  }
}

template <class T>
__global__ void k_ws_compact(DevBatch<T> B, const int* coff, const float* feat, const float* lab, float* out_feat,
                             float* out_lab, long base) {
  const long slot = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= (long)B.n_envs * B.cap) return;
  const int e = (int)(slot / B.cap), jj = (int)(slot - (long)e * B.cap);
  if (jj >= B.ccount[e]) return;
  const long row = base + coff[e] + jj;
  for (int k = 0; k < kFeat; ++k) out_feat[row * kFeat + k] = feat[slot * kFeat + k];
  for (int k = 0; k < kOut; ++k) out_lab[row * kOut + k] = lab[slot * kOut + k];
}

__global__ void k_normalize_rows(const float* feat, long n, const float* norm, float* X) {
  const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int k = 0; k < kFeat; ++k) X[r * kFeat + k] = (feat[r * kFeat + k] - norm[k]) * norm[kFeat + k];
}

template <class T>
void launch_ws_features(const DevBatch<T>& B, const T* mu_env, float* feat, hipStream_t s) {
  const long n = (long)B.n_envs * B.cap;
  hipLaunchKernelGGL(k_ws_features<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, mu_env, feat);
}
template <class T>
void launch_ws_labels(const DevBatch<T>& B, const float* feat, float* lab, hipStream_t s) {
  const long n = (long)B.n_envs * B.cap;
  hipLaunchKernelGGL(k_ws_labels<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, feat, lab);
}
template <class T>
void launch_ws_infer(const DevBatch<T>& B, const T* mu_env, const MlpBuffers& M, hipStream_t s) {
  const long n = (long)B.n_envs * B.cap;
  hipLaunchKernelGGL(k_normalize_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, M.feat, n, M.norm, M.X);
  mlp_forward(M.W, M.X, n, M.H1, M.H2, M.H3, M.Y, s);
  hipLaunchKernelGGL(k_ws_candidates<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, mu_env, M.feat, M.Y,
                     M.norm, M.lam_ml);
}

template <class T>
void launch_ws_compact(const DevBatch<T>& B, const float* feat, const float* lab, float* out_feat, float* out_lab,
                       long base, int* coff, hipStream_t s) {
  const long n = (long)B.n_envs * B.cap;
  hipLaunchKernelGGL(k_count_offsets, dim3(1), dim3(64), 0, s, B.ccount, B.n_envs, B.cap, coff);
  hipLaunchKernelGGL(k_ws_compact<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, coff, feat, lab,
                     out_feat, out_lab, base);
}

#define INSTW(T)                                                                           \
  template void launch_ws_features<T>(const DevBatch<T>&, const T*, float*, hipStream_t); \
  template void launch_ws_labels<T>(const DevBatch<T>&, const float*, float*, hipStream_t);             \
  template void launch_ws_infer<T>(const DevBatch<T>&, const T*, const MlpBuffers&, hipStream_t); \
  template void launch_ws_compact<T>(const DevBatch<T>&, const float*, const float*, float*, float*, long, int*, \
                                     hipStream_t);
INSTW(float)
INSTW(double)

}  // namespace flash
