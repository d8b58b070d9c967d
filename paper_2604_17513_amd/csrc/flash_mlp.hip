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
// A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn].  One workgroup of 4 waves per
// 64 x 64 tile of C, each wave a 32 x 32 quadrant on v_mfma_f32_32x32x8bf16_1k (A row = lane % 32,
// k = 4 (lane / 32) + t; B column = lane % 32, same k; D row = 8 (r / 4) + 4 (lane / 32) + r % 4,
// column = lane % 32).  K runs in chunks of kKc staged in LDS as bf16, each element rounded once
// and loaded along whichever of its two indices is contiguous; B is staged transposed so that every
// MFMA operand is one 8-byte LDS read.  Every quadrant accumulates over k in steps of 8 from the
// slice start, so the result does not depend on the chunking.
// blockIdx.z selects a K slice of g.kslice rows when the product is split over K: the slice's
// partial sums go to g.work[z][M][N] and a second kernel adds the slices in order.
constexpr int kKc = 32;
constexpr int kKp = kKc + 4;   // padded LDS row (shorts): rows 72 bytes apart

__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
  __shared__ short As[64 * kKp];   // [m][k]
  __shared__ short Bs[64 * kKp];   // [n][k]
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const long m0 = (long)blockIdx.x * 64, n0 = (long)blockIdx.y * 64;
  const int wm = 32 * (w & 1), wn = 32 * (w >> 1);
  const int kb = g.work ? (int)blockIdx.z * g.kslice : 0;
  const int ke = g.work ? min(g.K, kb + g.kslice) : g.K;
  const bool a_mfast = g.sam == 1, b_nfast = g.sbn == 1;
  floatx16 c = {};
  for (int k0 = kb; k0 < ke; k0 += kKc) {
    // stage: 64 x kKc of A and of B (8 elements per thread each)
#pragma unroll
    for (int q = 0; q < 64 * kKc / 256; ++q) {
      const int e = tid + 256 * q;
      const int am = a_mfast ? (e & 63) : (e / kKc), ak = a_mfast ? (e >> 6) : (e % kKc);
      const long gm = m0 + am;
      const int gk = k0 + ak;
      const float av = (gm < g.M && gk < ke) ? g.A[gm * g.sam + (long)gk * g.sak] : 0.f;
      As[am * kKp + ak] = f2bf(av);
      const int bn = b_nfast ? (e & 63) : (e / kKc), bk = b_nfast ? (e >> 6) : (e % kKc);
      const long gn = n0 + bn;
      const int gk2 = k0 + bk;
      const float bv = (gn < g.N && gk2 < ke) ? g.B[(long)gk2 * g.sbk + gn * g.sbn] : 0.f;
      Bs[bn * kKp + bk] = f2bf(bv);
    }
    __syncthreads();
    const int kend = min(kKc, ke - k0);
    for (int kk = 0; kk < kend; kk += 8) {
      const int ko = kk + 4 * (l >> 5);
      const bf16x4 a = *reinterpret_cast<const bf16x4*>(&As[(wm + (l & 31)) * kKp + ko]);
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(&Bs[(wn + (l & 31)) * kKp + ko]);
      c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
    }
    __syncthreads();
  }
  const long jj = n0 + wn + (l & 31);
  if (g.work) {
    float* wk = g.work + (size_t)blockIdx.z * g.M * g.N;
    for (int r = 0; r < 16; ++r) {
      const long ii = m0 + wm + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
      if (ii < g.M && jj < g.N) wk[ii * g.N + jj] = c[r];
    }
    return;
  }
  for (int r = 0; r < 16; ++r) {
    const long ii = m0 + wm + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
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
  dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64));
  // few output tiles over a long K (weight gradients): split K so that the chip fills.  The slice
  // count is the one chosen for 32 x 32 tiles, so the slices (hence the bits) are those of that
  // tiling.
  const long tiles32 = ((g.M + 31) / 32) * (long)((g.N + 31) / 32);
  int slices = 1;
  if (g.work && tiles32 < 512 && g.K > 256) {
    slices = (int)std::min<long>((g.K + 127) / 128, std::max<long>(1, 1024 / tiles32));
    slices = std::min<long>(slices, g.work_cap / (g.M * g.N));
  }
  if (slices <= 1) {
    g.work = nullptr;
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
    return;
  }
  g.kslice = ((g.K + slices - 1) / slices + 7) / 8 * 8;
  slices = (g.K + g.kslice - 1) / g.kslice;
  grid.z = (unsigned)slices;
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, g);
  const long mn = g.M * g.N;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, g, slices);
}

// ---------------------------------------------------------------------------
// Fused forward pass on v_mfma_f32_32x32x16_bf16.  Lane layout of that
// instruction: A(m, k) from lane m + 32 (k / 8), element k % 8; B(k, n) from
// lane n + 32 (k / 8), element k % 8; D(i, j) in lane j + 32 ((i / 4) % 2),
// register 4 (i / 8) + i % 4.  The network runs transposed (H^T = W X^T):
// rows of a D tile are neurons, columns are 32 samples, so the registers a
// lane holds for one output tile are exactly the B operand of the next layer
// once the 16 inputs of each K step are visited in the order neuron(k) =
// 8 ((k % 8) / 4) + 4 (k / 8) + k % 4.  The weights are staged in LDS as
// bf16 with the columns of each 16-block permuted to that order (bits 2 and
// 3 of the input index swapped), so every A operand is one 16-byte read.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kLd1 = 24;    // LDS row stride of W1 (bf16): 48 B keeps 16-byte reads conflict-free
constexpr int kLdH = 136;   // LDS row stride of W2, W3, W4 (bf16): 272 B
constexpr int kWaves = 4;

struct FusedSmem {
  __bf16 w1[kHidden * kLd1];
  __bf16 w2[kHidden * kLdH];
  __bf16 w3[kHidden * kLdH];
  __bf16 w4[kOut * kLdH];
  float b[3 * kHidden + 4];
  float nrm[2 * kFeat];
};
constexpr size_t kFusedSmem = sizeof(FusedSmem);

__device__ __forceinline__ int perm16(int c) { return (c & ~12) | ((c & 4) << 1) | ((c & 8) >> 1); }

__device__ __forceinline__ __bf16 to_bf(float f) { return __builtin_bit_cast(__bf16, f2bf(f)); }

// one hidden layer: hn = relu(W h + b) on the 4 x 16 register tile of a wave
__device__ __forceinline__ void fused_hidden(const __bf16* w, const float* bias, const float (&h)[4][16],
                                             float (&hn)[4][16], int l) {
  bf16x8 bop[4][2];
  for (int mt = 0; mt < 4; ++mt)
    for (int p = 0; p < 2; ++p)
      for (int t = 0; t < 8; ++t) bop[mt][p][t] = to_bf(h[mt][8 * p + t]);
  for (int mt = 0; mt < 4; ++mt) {
    const __bf16* wrow = w + (32 * mt + (l & 31)) * kLdH + 8 * (l >> 5);
    floatx16 acc = {};
    for (int q = 0; q < 4; ++q)
      for (int p = 0; p < 2; ++p) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(wrow + 32 * q + 16 * p);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bop[q][p], acc, 0, 0, 0);
      }
    for (int r = 0; r < 16; ++r)
      hn[mt][r] = fmaxf(acc[r] + bias[32 * mt + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3)], 0.f);
  }
}

__device__ __forceinline__ void fused_store(float* H, long row, long rows, const float (&h)[4][16], int l) {
  if (row >= rows) return;
  for (int mt = 0; mt < 4; ++mt)
    for (int q = 0; q < 4; ++q) {
      float4 v = make_float4(h[mt][4 * q], h[mt][4 * q + 1], h[mt][4 * q + 2], h[mt][4 * q + 3]);
      *reinterpret_cast<float4*>(H + row * kHidden + 32 * mt + 8 * q + 4 * (l >> 5)) = v;
    }
}

// Y = network(X) for `rows` rows.  norm != nullptr: X holds raw features, normalised on load.
// need != nullptr: 32-row tiles without a flagged row are skipped (their Y is left as is).
// H1 != nullptr: the hidden activations are stored for the backward pass.
__global__ void __launch_bounds__(64 * kWaves) k_mlp_fused(const float* W, const float* norm, const float* X,
                                                           long rows, const int* need, float* Y, float* H1,
                                                           float* H2, float* H3) {
  extern __shared__ __align__(16) unsigned char fsm_raw[];
  FusedSmem& S = *reinterpret_cast<FusedSmem*>(fsm_raw);
  const MlpLayout L;
  const int tid = threadIdx.x;
  for (int i = tid; i < kHidden * kFeat; i += blockDim.x) {
    const int r = i / kFeat, c = i - r * kFeat;
    S.w1[r * kLd1 + c] = to_bf(W[L.w1 + i]);
  }
  for (int i = tid; i < kHidden * kHidden; i += blockDim.x) {
    const int r = i / kHidden, c = i - r * kHidden;
    S.w2[r * kLdH + perm16(c)] = to_bf(W[L.w2 + i]);
    S.w3[r * kLdH + perm16(c)] = to_bf(W[L.w3 + i]);
  }
  for (int i = tid; i < kOut * kHidden; i += blockDim.x) {
    const int r = i / kHidden, c = i - r * kHidden;
    S.w4[r * kLdH + perm16(c)] = to_bf(W[L.w4 + i]);
  }
  for (int i = tid; i < kHidden; i += blockDim.x) {
    S.b[i] = W[L.b1 + i];
    S.b[kHidden + i] = W[L.b2 + i];
    S.b[2 * kHidden + i] = W[L.b3 + i];
  }
  if (tid < kOut) S.b[3 * kHidden + tid] = W[L.b4 + tid];
  if (tid < 2 * kFeat) S.nrm[tid] = norm ? norm[tid] : (tid < kFeat ? 0.f : 1.f);
  __syncthreads();

  const int l = tid & 63, wave = tid >> 6;
  const int h = l >> 5;
  const long ntiles = (rows + 31) / 32;
  for (long tile = (long)blockIdx.x * kWaves + wave; tile < ntiles; tile += (long)gridDim.x * kWaves) {
    const long row = tile * 32 + (l & 31);
    if (need) {
      const bool mine = row < rows && need[row] != 0;
      if (__ballot(mine) == 0) continue;
    }
    // layer 1: B operand = 8 features of this lane's sample
    bf16x8 xb;
    for (int t = 0; t < 8; ++t) {
      const int k = 8 * h + t;
      const float v = row < rows ? X[row * kFeat + k] : 0.f;
      xb[t] = to_bf((v - S.nrm[k]) * S.nrm[kFeat + k]);
    }
    float ha[4][16], hb[4][16];
    for (int mt = 0; mt < 4; ++mt) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(S.w1 + (32 * mt + (l & 31)) * kLd1 + 8 * h);
      floatx16 acc = {};
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xb, acc, 0, 0, 0);
      for (int r = 0; r < 16; ++r) ha[mt][r] = fmaxf(acc[r] + S.b[32 * mt + 8 * (r >> 2) + 4 * h + (r & 3)], 0.f);
    }
    if (H1) fused_store(H1, row, rows, ha, l);
    fused_hidden(S.w2, S.b + kHidden, ha, hb, l);
    if (H2) fused_store(H2, row, rows, hb, l);
    fused_hidden(S.w3, S.b + 2 * kHidden, hb, ha, l);
    if (H3) fused_store(H3, row, rows, ha, l);
    // output layer: rows 0..2 of a zero-padded 32-row tile
    bf16x8 bop[4][2];
    for (int mt = 0; mt < 4; ++mt)
      for (int p = 0; p < 2; ++p)
        for (int t = 0; t < 8; ++t) bop[mt][p][t] = to_bf(ha[mt][8 * p + t]);
    floatx16 acc = {};
    const int m = l & 31;
    for (int q = 0; q < 4; ++q)
      for (int p = 0; p < 2; ++p) {
        bf16x8 a;
        if (m < kOut) a = *reinterpret_cast<const bf16x8*>(S.w4 + m * kLdH + 8 * h + 32 * q + 16 * p);
        else for (int t = 0; t < 8; ++t) a[t] = __builtin_bit_cast(__bf16, (short)0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bop[q][p], acc, 0, 0, 0);
      }
    if (h == 0 && row < rows)
      for (int k = 0; k < kOut; ++k) Y[row * kOut + k] = acc[k] + S.b[3 * kHidden + k];
  }
}

void prepare_mlp() {
  (void)hipFuncSetAttribute((const void*)k_mlp_fused, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedSmem);
}

void launch_mlp_fused(const float* W, const float* norm, const float* X, long rows, const int* need, float* Y,
                      float* H1, float* H2, float* H3, hipStream_t s) {
  if (rows <= 0) return;
  const long ntiles = (rows + 31) / 32;
  const long blocks = std::min<long>((ntiles + kWaves - 1) / kWaves, 1024);
  hipLaunchKernelGGL(k_mlp_fused, dim3((unsigned)blocks), dim3(64 * kWaves), kFusedSmem, s, W, norm, X, rows, need, Y,
                     H1, H2, H3);
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
__global__ void k_ws_features(DevBatch<T> B, const T* mu_env, float* feat, int* need) {
  const long slot = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= (long)B.n_envs * B.cap) return;
  const int e = (int)(slot / B.cap), jj = (int)(slot - (long)e * B.cap);
  float* f = feat + slot * kFeat;
  // empty slots and attachment rows (bilateral, no prediction) get no features
  if (jj >= B.ccount[e] || B.cobs[slot] >= kMaxObs) {
    for (int k = 0; k < kFeat; ++k) f[k] = 0.f;
    if (need) need[slot] = 0;
    return;
  }
  if (need) need[slot] = B.cnew[slot];
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
  if (jj >= B.ccount[e] || B.cobs[slot] >= kMaxObs) { y[0] = y[1] = y[2] = 0.f; return; }
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
  if (B.cobs[slot] >= kMaxObs) {   // attachment rows keep the plain start
    for (int k = 0; k < 3; ++k) lam_ml[3 * slot + k] = B.clam[3 * slot + k];
    return;
  }
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

template <class T>
void launch_ws_features(const DevBatch<T>& B, const T* mu_env, float* feat, int* need, hipStream_t s) {
  const long n = (long)B.n_envs * B.cap;
  hipLaunchKernelGGL(k_ws_features<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, mu_env, feat, need);
}
template <class T>
void launch_ws_labels(const DevBatch<T>& B, const float* feat, float* lab, hipStream_t s) {
  const long n = (long)B.n_envs * B.cap;
  hipLaunchKernelGGL(k_ws_labels<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, feat, lab);
}
template <class T>
void launch_ws_infer(const DevBatch<T>& B, const T* mu_env, const MlpBuffers& M, hipStream_t s) {
  const long n = (long)B.n_envs * B.cap;
  launch_mlp_fused(M.W, M.norm, M.feat, n, M.need, M.Y, nullptr, nullptr, nullptr, s);
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
  template void launch_ws_features<T>(const DevBatch<T>&, const T*, float*, int*, hipStream_t); \
  template void launch_ws_labels<T>(const DevBatch<T>&, const float*, float*, hipStream_t);             \
  template void launch_ws_infer<T>(const DevBatch<T>&, const T*, const MlpBuffers&, hipStream_t); \
  template void launch_ws_compact<T>(const DevBatch<T>&, const float*, const float*, float*, float*, long, int*, \
                                     hipStream_t);
INSTW(float)
INSTW(double)

}  // namespace flash
