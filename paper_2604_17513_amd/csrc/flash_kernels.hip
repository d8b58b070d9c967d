// Step kernels: local projection, assembly gather, the explicit-inverse global
// apply, the contact-space non-smooth Newton solve and the position update.
//
// Working variable: the per-step displacement u = q - x_t (x_t = positions at
// the step start).  With A = M + h^2 sum_e w_e G_e^T G_e (Eq. 4) the assembled
// system A q = b + h^2 H^T lambda becomes
//     A u = M u~ + h^2 sum_e w_e G_e^T (p_e - G_e x_t) + h^2 H^T lambda,
// u~ = h v + h^2 g, which keeps FP32 relative precision on small quantities.
#include <algorithm>
#include <type_traits>

#include "flash_contact.h"
#include "flash_device.h"
#include "flash_launch.h"

namespace flash {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

template <class T>
__device__ T wave_sum(T v) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}
template <class T>
__device__ T wave_max(T v) {
  for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  return v;
}

// Block-wide reductions (every thread gets the result).  sh: >= kBlock/64 doubles.
__device__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) sh[wave_id()] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
  return t;
}
__device__ double block_max(double v, double* sh) {
  v = wave_max(v);
  __syncthreads();
  if (lane_id() == 0) sh[wave_id()] = v;
  __syncthreads();
  double t = sh[0];
  for (int w = 1; w < kBlock / 64; ++w) t = fmax(t, sh[w]);
  return t;
}
__device__ int block_excl_scan_i(int v, int* sh, int* total) {
  int lane = lane_id(), wid = wave_id();
  int incl = v;
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  __syncthreads();
  if (lane == 63) sh[wid] = incl;
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    int s = sh[w];
    if (w < wid) off += s;
    tot += s;
  }
  *total = tot;
  return off + incl - v;
}

// ---------------------------------------------------------------------------
// 3x3 helpers (row-major)
// ---------------------------------------------------------------------------
template <class T>
__device__ void cof3(const T* X, T* C, T* det) {
  C[0] = X[4] * X[8] - X[5] * X[7];
  C[1] = X[5] * X[6] - X[3] * X[8];
  C[2] = X[3] * X[7] - X[4] * X[6];
  C[3] = X[2] * X[7] - X[1] * X[8];
  C[4] = X[0] * X[8] - X[2] * X[6];
  C[5] = X[1] * X[6] - X[0] * X[7];
  C[6] = X[1] * X[5] - X[2] * X[4];
  C[7] = X[2] * X[3] - X[0] * X[5];
  C[8] = X[0] * X[4] - X[1] * X[3];
  *det = X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
}

// Closest rotation of a well-conditioned F (det F > 0): orthogonal polar factor
// by the scaled Newton iteration X <- (g X + X^-T / g) / 2, g = |det X|^-1/3.
template <class T>
__device__ void polar_newton(const T* F, T* R) {
  T X[9], C[9], det;
  for (int k = 0; k < 9; ++k) X[k] = F[k];
  const T tol = sizeof(T) == 4 ? T(1e-6) : T(1e-13);
  for (int it = 0; it < 20; ++it) {
    cof3(X, C, &det);
    T g = it < 8 ? T(1) / cbrt(det) : T(1);
    T a = T(0.5) * g, bcoef = T(0.5) / (g * det);
    T diff = 0;
    for (int k = 0; k < 9; ++k) {
      T xn = a * X[k] + bcoef * C[k];
      T d = xn - X[k];
      diff += d * d;
      X[k] = xn;
    }
    if (diff < tol * tol) break;
  }
  for (int k = 0; k < 9; ++k) R[k] = X[k];
}

// FP64 closest rotation for any F (inverted or near-degenerate):
// F^T F = V S^2 V^T by cyclic Jacobi, sigma descending, det V = +1;
// u1 = F v1 / |F v1|, u2 = F v2 orthogonalised against u1, R = [u1 u2 u1 x u2] V^T.
__device__ void polar_svd64(const double* F, double* R) {
  double A[9], V[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      A[3 * r + c] = F[r] * F[c] + F[3 + r] * F[3 + c] + F[6 + r] * F[6 + c];
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    double dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off <= 1e-32 * dia || off == 0.0) break;
    for (int pq = 0; pq < 3; ++pq) {
      int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      double apq = A[3 * p + q];
      if (apq == 0.0) continue;
      double th = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
      double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
      double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      // A <- J^T A J, V <- V J with J = I except J_pp = J_qq = c, J_pq = s, J_qp = -s
      for (int k = 0; k < 3; ++k) {
        double akp = A[3 * k + p], akq = A[3 * k + q];
        A[3 * k + p] = c * akp - s * akq;
        A[3 * k + q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {
        double apk = A[3 * p + k], aqk = A[3 * q + k];
        A[3 * p + k] = c * apk - s * aqk;
        A[3 * q + k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {
        double vkp = V[3 * k + p], vkq = V[3 * k + q];
        V[3 * k + p] = c * vkp - s * vkq;
        V[3 * k + q] = s * vkp + c * vkq;
      }
    }
  }
  // sort eigenpairs descending
  double ev[3] = {A[0], A[4], A[8]};
  int o[3] = {0, 1, 2};
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j)
      if (ev[o[j]] > ev[o[i]]) { int t = o[i]; o[i] = o[j]; o[j] = t; }
  double v1[3], v2[3], v3[3];
  for (int k = 0; k < 3; ++k) { v1[k] = V[3 * k + o[0]]; v2[k] = V[3 * k + o[1]]; v3[k] = V[3 * k + o[2]]; }
  double dv = v1[0] * (v2[1] * v3[2] - v2[2] * v3[1]) - v1[1] * (v2[0] * v3[2] - v2[2] * v3[0]) +
              v1[2] * (v2[0] * v3[1] - v2[1] * v3[0]);
  if (dv < 0) { v3[0] = -v3[0]; v3[1] = -v3[1]; v3[2] = -v3[2]; }
  double u1[3], u2[3], u3[3];
  for (int r = 0; r < 3; ++r) {
    u1[r] = F[3 * r] * v1[0] + F[3 * r + 1] * v1[1] + F[3 * r + 2] * v1[2];
    u2[r] = F[3 * r] * v2[0] + F[3 * r + 1] * v2[1] + F[3 * r + 2] * v2[2];
  }
  double n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
  if (n1 > 0) { u1[0] /= n1; u1[1] /= n1; u1[2] /= n1; }
  else { u1[0] = v1[0]; u1[1] = v1[1]; u1[2] = v1[2]; }
  double dp = u1[0] * u2[0] + u1[1] * u2[1] + u1[2] * u2[2];
  for (int r = 0; r < 3; ++r) u2[r] -= dp * u1[r];
  double n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  if (n2 > 1e-300) { u2[0] /= n2; u2[1] /= n2; u2[2] /= n2; }
  else {
    // any unit vector orthogonal to u1
    int k = fabs(u1[0]) <= fabs(u1[1]) ? (fabs(u1[0]) <= fabs(u1[2]) ? 0 : 2) : (fabs(u1[1]) <= fabs(u1[2]) ? 1 : 2);
    double e[3] = {0, 0, 0};
    e[k] = 1;
    u2[0] = e[1] * u1[2] - e[2] * u1[1];
    u2[1] = e[2] * u1[0] - e[0] * u1[2];
    u2[2] = e[0] * u1[1] - e[1] * u1[0];
    double l = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
    u2[0] /= l; u2[1] /= l; u2[2] /= l;
  }
  u3[0] = u1[1] * u2[2] - u1[2] * u2[1];
  u3[1] = u1[2] * u2[0] - u1[0] * u2[2];
  u3[2] = u1[0] * u2[1] - u1[1] * u2[0];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) R[3 * r + c] = u1[r] * v1[c] + u2[r] * v2[c] + u3[r] * v3[c];
}

// ---------------------------------------------------------------------------
// local projection (Eq. 3) and per-tet vertex forces w (p - F(x_t)) gradN_a
// ---------------------------------------------------------------------------
// Closest matrix with orthonormal columns to a 3x2 F in FP64: eigenvectors v1, v2 of
// S = F^T F (2x2, closed form), u_i = F v_i / sigma_i, and for a rank-deficient F a unit u2
// orthogonal to u1; R = u1 v1^T + u2 v2^T.
__device__ void ortho_cols64(const double* F, double* R) {
  const double s00 = F[0] * F[0] + F[2] * F[2] + F[4] * F[4];
  const double s01 = F[0] * F[1] + F[2] * F[3] + F[4] * F[5];
  const double s11 = F[1] * F[1] + F[3] * F[3] + F[5] * F[5];
  const double hd = 0.5 * (s00 - s11), rt = sqrt(hd * hd + s01 * s01);
  const double l1 = 0.5 * (s00 + s11) + rt;
  double v1[2];
  if (rt > 0) {
    // eigenvector of the larger eigenvalue, from the better-conditioned row
    if (hd >= 0) { v1[0] = hd + rt; v1[1] = s01; } else { v1[0] = s01; v1[1] = rt - hd; }
    const double nv = sqrt(v1[0] * v1[0] + v1[1] * v1[1]);
    v1[0] /= nv; v1[1] /= nv;
  } else { v1[0] = 1.0; v1[1] = 0.0; }
  const double v2[2] = {-v1[1], v1[0]};
  double u1[3], u2[3];
  for (int r = 0; r < 3; ++r) {
    u1[r] = F[2 * r] * v1[0] + F[2 * r + 1] * v1[1];
    u2[r] = F[2 * r] * v2[0] + F[2 * r + 1] * v2[1];
  }
  double n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
  if (!(n1 > 0)) { u1[0] = 1.0; u1[1] = 0.0; u1[2] = 0.0; n1 = 1.0; }
  for (int r = 0; r < 3; ++r) u1[r] /= n1;
  // Gram-Schmidt against u1; a vanishing remainder takes any direction orthogonal to u1
  double d = u1[0] * u2[0] + u1[1] * u2[1] + u1[2] * u2[2];
  for (int r = 0; r < 3; ++r) u2[r] -= d * u1[r];
  double n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  if (!(n2 > 1e-12 * sqrt(fmax(l1, 0.0)))) {
    const int k = (fabs(u1[0]) <= fabs(u1[1]) && fabs(u1[0]) <= fabs(u1[2])) ? 0 : (fabs(u1[1]) <= fabs(u1[2]) ? 1 : 2);
    double ek[3] = {0.0, 0.0, 0.0};
    ek[k] = 1.0;
    u2[0] = u1[1] * ek[2] - u1[2] * ek[1];
    u2[1] = u1[2] * ek[0] - u1[0] * ek[2];
    u2[2] = u1[0] * ek[1] - u1[1] * ek[0];
    n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
  }
  for (int r = 0; r < 3; ++r) u2[r] /= n2;
  for (int r = 0; r < 3; ++r) {
    R[2 * r] = u1[r] * v1[0] + u2[r] * v2[0];
    R[2 * r + 1] = u1[r] * v1[1] + u2[r] * v2[1];
  }
}

// Membrane triangle: F = [x1 - x0 | x2 - x0] B (3x2, B = D_m^-1 2x2 in tet_B entries 0..3),
// p = the closest matrix with orthonormal columns, F S^-1/2 with S = F^T F in closed form
// (sqrt S = (S + sqrt(det S) I) / sqrt(tr S + 2 sqrt(det S))); nearly rank-deficient F
// (det S < 1e-4 (tr S / 2)^2) goes to the FP64 eigen path.  Forces w (p - F_x) gradN_a.
// Inputs of an element's local step, all loaded before any of its arithmetic, so that a loop
// over elements can load the next element while it computes the current one.
template <class T>
struct ElemIn {
  int tri;               // 1: membrane triangle (vertices 0..2)
  int slot[4];           // incidence slots of the element's vertices
  T dx[3][3], du[3][3];  // x and u of vertices 1.. minus those of vertex 0 (a triangle uses two)
  T Bm[9];               // D_m^-1 (a triangle uses the first 4 entries)
  T w;
};

template <class T>
__device__ __forceinline__ void elem_ids(const DevBatch<T>& B, int t, int id[4]) {
  for (int a = 0; a < 4; ++a) id[a] = B.tet_idx[a * B.NT + t];
}

template <class T>
__device__ __forceinline__ void elem_load(const DevBatch<T>& B, int t, const int id[4], ElemIn<T>& in) {
  const int NT = B.NT, NV = B.NV;
  in.tri = id[3] < 0 ? 1 : 0;
  const int ne = in.tri ? 2 : 3, nb = in.tri ? 4 : 9;
  T X0[3], U0[3];
  for (int k = 0; k < 3; ++k) { X0[k] = B.x[k * NV + id[0]]; U0[k] = B.u[k * NV + id[0]]; }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      in.dx[a][k] = a < ne ? B.x[k * NV + id[a + 1]] - X0[k] : T(0);
      in.du[a][k] = a < ne ? B.u[k * NV + id[a + 1]] - U0[k] : T(0);
    }
#pragma unroll
  for (int k = 0; k < 9; ++k) in.Bm[k] = k < nb ? B.tet_B[k * NT + t] : T(0);
  in.w = B.tet_w[t];
#pragma unroll
  for (int a = 0; a < 4; ++a) in.slot[a] = a <= ne ? B.slot[4 * (size_t)t + a] : 0;
}

template <class T>
__device__ __forceinline__ void project_tri(const DevBatch<T>& B, int t, const ElemIn<T>& in) {
  const T(&dx)[3][3] = in.dx;
  const T(&du)[3][3] = in.du;
  const T* Bm = in.Bm;
  T F[6], Fx[6];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 2; ++c) {
      T f = 0, fx = 0;
      for (int a = 0; a < 2; ++a) {
        fx += dx[a][r] * Bm[2 * a + c];
        f += (dx[a][r] + du[a][r]) * Bm[2 * a + c];
      }
      F[2 * r + c] = f;
      Fx[2 * r + c] = fx;
    }
  const T s00 = F[0] * F[0] + F[2] * F[2] + F[4] * F[4];
  const T s01 = F[0] * F[1] + F[2] * F[3] + F[4] * F[5];
  const T s11 = F[1] * F[1] + F[3] * F[3] + F[5] * F[5];
  const T det = s00 * s11 - s01 * s01, tr = s00 + s11;
  T R[6];
  if (det > T(1e-4) * T(0.25) * tr * tr) {
    const T r = sqrt(det), dsq = sqrt(tr + T(2) * r);
    // inverse of (S + r I) / dsq
    const T a00 = s00 + r, a11 = s11 + r;
    const T idet = dsq / (a00 * a11 - s01 * s01);
    const T i00 = a11 * idet, i01 = -s01 * idet, i11 = a00 * idet;
    for (int q = 0; q < 3; ++q) {
      R[2 * q] = F[2 * q] * i00 + F[2 * q + 1] * i01;
      R[2 * q + 1] = F[2 * q] * i01 + F[2 * q + 1] * i11;
    }
  } else {
    double Fd[6], Rd[6];
    for (int k = 0; k < 6; ++k) Fd[k] = (double)F[k];
    ortho_cols64(Fd, Rd);
    for (int k = 0; k < 6; ++k) R[k] = (T)Rd[k];
    atomicAdd(&B.fp64_polar[B.tet_env[t]], 1);
  }
  const T w = in.w;
  T P[6];
  for (int k = 0; k < 6; ++k) P[k] = w * (R[k] - Fx[k]);
  T f0[3] = {0, 0, 0};
  for (int a = 0; a < 2; ++a) {
    T* dst = B.fel + 3 * (size_t)in.slot[a + 1];
    for (int r = 0; r < 3; ++r) {
      const T fa = P[2 * r] * Bm[2 * a] + P[2 * r + 1] * Bm[2 * a + 1];
      dst[r] = fa;
      f0[r] -= fa;
    }
  }
  T* dst0 = B.fel + 3 * (size_t)in.slot[0];
  for (int r = 0; r < 3; ++r) dst0[r] = f0[r];
}

// Local step of element t (tet or membrane triangle) from its loaded inputs: projection and
// its slot forces.
template <class T>
__device__ __forceinline__ void elem_compute(const DevBatch<T>& B, int t, const ElemIn<T>& in) {
  if (in.tri) { project_tri(B, t, in); return; }
  const T(&dx)[3][3] = in.dx;
  const T(&du)[3][3] = in.du;
  const T* Bm = in.Bm;
  // F = D_s B with D_s[:, a] = dx_a + du_a ; F_x = D_x B
  T F[9], Fx[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      T f = 0, fx = 0;
      for (int a = 0; a < 3; ++a) {
        fx += dx[a][r] * Bm[3 * a + c];
        f += (dx[a][r] + du[a][r]) * Bm[3 * a + c];
      }
      F[3 * r + c] = f;
      Fx[3 * r + c] = fx;
    }
  T C[9], det;
  cof3(F, C, &det);
  T fn2 = 0;
  for (int k = 0; k < 9; ++k) fn2 += F[k] * F[k];
  // quality det F / (|F|_F / sqrt 3)^3; degenerate or inverted -> FP64 path
  T q3 = fn2 * (T)(1.0 / 3.0);
  T quality = det / (q3 * sqrt(q3));
  T R[9];
  if (det > T(0) && quality >= T(1e-2)) {
    polar_newton(F, R);
  } else {
    double Fd[9], Rd[9];
    for (int k = 0; k < 9; ++k) Fd[k] = (double)F[k];
    polar_svd64(Fd, Rd);
    for (int k = 0; k < 9; ++k) R[k] = (T)Rd[k];
    atomicAdd(&B.fp64_polar[B.tet_env[t]], 1);
  }
  const T w = in.w;
  T P[9];
  for (int k = 0; k < 9; ++k) P[k] = w * (R[k] - Fx[k]);
  // vertex forces go to their slots in the vertex-ordered incidence list
  T f0[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) {
    T* dst = B.fel + 3 * (size_t)in.slot[a + 1];
    for (int r = 0; r < 3; ++r) {
      T fa = P[3 * r] * Bm[3 * a] + P[3 * r + 1] * Bm[3 * a + 1] + P[3 * r + 2] * Bm[3 * a + 2];
      dst[r] = fa;
      f0[r] -= fa;
    }
  }
  T* dst0 = B.fel + 3 * (size_t)in.slot[0];
  for (int r = 0; r < 3; ++r) dst0[r] = f0[r];
}

// Local step of one element t: its inputs, then its projection and slot forces.
template <class T>
__device__ __forceinline__ void project_element(const DevBatch<T>& B, int t) {
  int id[4];
  elem_ids(B, t, id);
  ElemIn<T> in;
  elem_load(B, t, id, in);
  elem_compute(B, t, in);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_project(DevBatch<T> B) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t < B.NT) project_element(B, t);
}

// Bending hinges have the target p = 0, so in displacement form each contributes the
// constant (per step) force w_h G_h^T (0 - G_h x) = -w_h alpha_a (sum_b alpha_b x_b) to its
// four vertices; written once per step into the hinge slots that the assembly gathers.
template <class T>
__global__ void __launch_bounds__(kBlock) k_hinge(DevBatch<T> B) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= B.NH) return;
  const int NV = B.NV, NH = B.NH;
  int id[4];
  T al[4];
  for (int a = 0; a < 4; ++a) { id[a] = B.hinge_idx[a * NH + q]; al[a] = B.hinge_alpha[a * NH + q]; }
  T gx[3];
  for (int k = 0; k < 3; ++k) {
    T sum = 0;
    for (int a = 0; a < 4; ++a) sum += al[a] * B.x[k * NV + id[a]];
    gx[k] = sum;
  }
  const T w = B.hinge_w[q];
  for (int a = 0; a < 4; ++a) {
    T* dst = B.fel + 3 * (size_t)B.hinge_slot[a * NH + q];
    for (int k = 0; k < 3; ++k) dst[k] = -w * al[a] * gx[k];
  }
}

template <class T>
void launch_hinge(const DevBatch<T>& B, hipStream_t s) {
  if (B.NH == 0) return;
  hipLaunchKernelGGL(k_hinge<T>, dim3((B.NH + kBlock - 1) / kBlock), dim3(kBlock), 0, s, B);
}

// b = M u~ + h^2 sum over incident tets (fixed incidence order; the forces of
// vertex i occupy the contiguous slots inc_off[i] .. inc_off[i+1]-1).
constexpr int kAsmChunk = 1024;   // incidence slots staged per pass (3 values each)

// Right-hand side of the vertices vbeg .. vend-1 (at most kBlock, one per thread):
// their incidence slots form one contiguous range, staged through LDS (s_f: 3 *
// kAsmChunk values) in coalesced chunks; each thread then sums its own slots in slot
// order (the same order, hence the same bits, as a direct per-vertex loop).  Every
// thread of the workgroup must call it.
template <class T>
__device__ __forceinline__ void assemble_vertices(const DevBatch<T>& B, int vbeg, int vend, T* s_f) {
  constexpr int CH = kAsmChunk;
  const int i = vbeg + threadIdx.x;
  const int pb = B.inc_off[vbeg], pe = B.inc_off[vend];
  int my0 = 0, my1 = 0;
  if (i < vend) { my0 = B.inc_off[i]; my1 = B.inc_off[i + 1]; }
  T s0 = 0, s1 = 0, s2 = 0;
  for (int c0 = pb; c0 < pe; c0 += CH) {
    const int c1 = min(c0 + CH, pe);
    __syncthreads();
    {
      // every load of the chunk in flight before the LDS stores
      constexpr int NQ = 3 * CH / kBlock;
      const int nq = 3 * (c1 - c0);
      T tv[NQ];
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const int q = (int)threadIdx.x + u * kBlock;
        if (q < nq) tv[u] = B.fel[3 * (size_t)c0 + q];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < NQ; ++u) {
        const int q = (int)threadIdx.x + u * kBlock;
        if (q < nq) s_f[q] = tv[u];
      }
    }
    __syncthreads();
    const int a = max(my0, c0), b = min(my1, c1);
    for (int p = a; p < b; ++p) {
      const T* f = s_f + 3 * (p - c0);
      s0 += f[0];
      s1 += f[1];
      s2 += f[2];
    }
  }
  if (i >= vend) return;
  const int NV = B.NV;
  const T hh = (T)(B.h * B.h);
  const T m = B.mass[i];
  B.b[i] = m * B.ut[i] + hh * s0;
  B.b[NV + i] = m * B.ut[NV + i] + hh * s1;
  B.b[2 * NV + i] = m * B.ut[2 * NV + i] + hh * s2;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_assemble(DevBatch<T> B) {
  __shared__ T s_f[3 * kAsmChunk];
  const int vbeg = blockIdx.x * kBlock;
  if (vbeg >= B.NV) return;
  assemble_vertices(B, vbeg, min(vbeg + kBlock, B.NV), s_f);
}

// ---------------------------------------------------------------------------
// Explicit-inverse products.  Gbar is symmetric, so row j of Gbar is also
// column j: out[:, i] = sum_r Gbar[row_r, i] * vec_r, read along rows
// (coalesced, 16-byte vectors, 4 waves split the rows, fixed-order LDS
// reduction).  ROWS = false: rows are 0..n-1 and vec = b (z = Gbar b).
// ROWS = true: rows are the contact vertices and vec = their world forces;
// out = z + h^2 * sum (u = z + h^2 Gbar H^T lambda).
// ---------------------------------------------------------------------------
constexpr int kChunk = 1024;

// VW columns per lane (TILE = 64 VW per workgroup), UNROLL rows in flight per wave.
// A workgroup takes one (env, first column) work item; the item list holds only the
// column tiles that exist, largest envs first.  Neither parameter changes the
// arithmetic: every column is summed over the same rows in the same order by the same
// wave, so all schedules give the same bits.
template <class T, int VW>
struct alignas(VW * sizeof(T) >= 16 ? 16 : VW * sizeof(T)) GVec {
  T v[VW];
};

// Row segment of the explicit inverse, streamed with the non-temporal hint: the inverse is
// read once per product, and keeping it out of the caches' working set leaves them to the
// contact solve's matrices (in the fused loop this took the solve from 20.1 to 17.6 ms per
// env-step on the squeeze workload).
template <class T, int VW>
__device__ __forceinline__ GVec<T, VW> load_gvec(const T* p) {
  constexpr int PER = (int)(16 / sizeof(T));   // values per 16-byte load
  typedef T v4 __attribute__((ext_vector_type(16 / sizeof(T))));
  GVec<T, VW> g;
  if constexpr (VW >= PER) {
#pragma unroll
    for (int i = 0; i < VW / PER; ++i) {
      const v4 x = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p) + i);
#pragma unroll
      for (int k = 0; k < PER; ++k) g.v[i * PER + k] = x[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < VW; ++k) g.v[k] = __builtin_nontemporal_load(p + k);
  }
  return g;
}

// One column tile (columns tile0 .. tile0 + 64 VW - 1) of env e's product with the
// workgroup: z = Gbar b (ROWS = false) or u = z + h^2 Gbar[:, contacts] (F lambda)
// (ROWS = true).  LDS: s_vec 3 * kChunk values, s_row kChunk ints, s_red
// 3 * 3 * 64 VW values.  Every thread of the workgroup must call it.
template <class T, bool ROWS, int VW, int UNROLL>
__device__ __forceinline__ void gemv_tile(const DevBatch<T>& B, int e, int tile0, T* s_vec, int* s_row, T* s_red) {
  constexpr int TILE = 64 * VW;
  const int v0 = B.voff[e];
  const int n = B.voff[e + 1] - v0;
  const int ld = B.gld[e];
  const T* G = B.G + B.goff[e];
  const int nrows = ROWS ? B.ccount[e] : n;
  const int lane = lane_id(), wid = wave_id();
  const int col0 = tile0 + lane * VW;
  const bool active = col0 < ld;
  T acc[VW][3];
  for (int q = 0; q < VW; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0;
  for (int r0 = 0; r0 < nrows; r0 += kChunk) {
    const int nr = min(kChunk, nrows - r0);
    __syncthreads();
    for (int r = threadIdx.x; r < nr; r += kBlock) {
      if (ROWS) {
        const int j = e * B.cap + r0 + r;
        s_row[r] = B.cvert[j];
        s_vec[r] = B.cforce[3 * j];
        s_vec[kChunk + r] = B.cforce[3 * j + 1];
        s_vec[2 * kChunk + r] = B.cforce[3 * j + 2];
      } else {
        s_row[r] = r0 + r;
        s_vec[r] = B.b[v0 + r0 + r];
        s_vec[kChunk + r] = B.b[B.NV + v0 + r0 + r];
        s_vec[2 * kChunk + r] = B.b[2 * B.NV + v0 + r0 + r];
      }
    }
    __syncthreads();
    if (active) {
      // UNROLL rows per batch: every load of the batch is issued before the first use (the
      // scheduling barrier keeps the compiler from interleaving them with the products, which
      // it does under the register pressure of the fused loop); rows are still summed in
      // increasing order
      constexpr int WS = kBlock / 64;
      for (int rb = wid; rb < nr; rb += WS * UNROLL) {
        GVec<T, VW> g[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int r = rb + WS * u;
          if (r < nr) g[u] = load_gvec<T, VW>(G + (size_t)s_row[r] * ld + col0);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int r = rb + WS * u;
          if (r < nr) {
            const T b0 = s_vec[r], b1 = s_vec[kChunk + r], b2 = s_vec[2 * kChunk + r];
            for (int q = 0; q < VW; ++q) {
              acc[q][0] += g[u].v[q] * b0;
              acc[q][1] += g[u].v[q] * b1;
              acc[q][2] += g[u].v[q] * b2;
            }
          }
        }
      }
    }
  }
  // fixed-order reduction over the 4 waves
  __syncthreads();
  if (wid > 0)
    for (int q = 0; q < VW; ++q)
      for (int k = 0; k < 3; ++k) s_red[((wid - 1) * 3 + k) * TILE + lane * VW + q] = acc[q][k];
  __syncthreads();
  if (wid == 0) {
    const T hh = (T)(B.h * B.h);
    for (int q = 0; q < VW; ++q) {
      const int col = col0 + q;
      if (col >= n) continue;
      for (int k = 0; k < 3; ++k) {
        T s = acc[q][k];
        for (int w = 0; w < kBlock / 64 - 1; ++w) s += s_red[(w * 3 + k) * TILE + lane * VW + q];
        const size_t o = (size_t)k * B.NV + v0 + col;
        if (ROWS) B.u[o] = B.z[o] + hh * s;
        else B.z[o] = s;
      }
    }
  }
}

template <class T, bool ROWS, int VW, int UNROLL>
__global__ void __launch_bounds__(kBlock) k_gemv(DevBatch<T> B, const int2* items, const int* skip) {
  __shared__ T s_vec[3 * kChunk];
  __shared__ int s_row[kChunk];
  __shared__ T s_red[(kBlock / 64 - 1) * 3 * 64 * VW];
  const int2 item = items[blockIdx.x];
  if (skip && skip[item.x]) return;
  gemv_tile<T, ROWS, VW, UNROLL>(B, item.x, item.y, s_vec, s_row, s_red);
}

// Gbar restricted to the contacts of each env: Gc[j][k] = Gbar[v_j][v_k]
// (stored in the contact-solve precision CT).
template <class T, class CT>
__global__ void __launch_bounds__(kBlock) k_gather(DevBatch<T> B) {
  const int e = blockIdx.x;
  const int c = B.ccount[e];
  const T* G = B.G + B.goff[e];
  const int ld = B.gld[e];
  CT* Gc = static_cast<CT*>(B.Gc) + (size_t)e * B.cap * B.cap;
  const int* cv = B.cvert + (size_t)e * B.cap;
  for (int idx = threadIdx.x; idx < c * c; idx += kBlock) {
    const int j = idx / c, k = idx - j * c;
    Gc[idx] = (CT)G[(size_t)cv[j] * ld + cv[k]];
  }
}

// ---------------------------------------------------------------------------
// Workgroup-cooperative dense kernels for the contact solve.  Panels of kBK
// columns; pivot blocks are staged in LDS; trailing updates use 4x4 register
// tiles and read the panels from global memory (L1/L2 resident).
// ---------------------------------------------------------------------------
// kBK (panel width of the blocked factorisations) lives in flash_device.h

// Runs use(k, load(k)) for k = k0, k0 + 1, ..., n - 1 in that order, with the loads of
// BATCH consecutive terms issued before the first of them is used: under the contact
// solve's register pressure the compiler otherwise waits for every load before issuing
// the next (one global round trip per term).  The order of the uses, hence of any sums
// they form, is unchanged.
template <int BATCH, class LoadF, class UseF>
__device__ __forceinline__ void batched_terms(int k0, int n, LoadF load, UseF use) {
  using V = decltype(load(0));
  typedef V vec __attribute__((ext_vector_type(BATCH)));   // a register value, never scratch
  for (int kb = k0; kb < n; kb += BATCH) {
    vec v = (V)0;
#pragma unroll
    for (int u = 0; u < BATCH; ++u)
      if (kb + u < n) v[u] = load(kb + u);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < BATCH; ++u)
      if (kb + u < n) use(kb + u, (V)v[u]);
  }
}

// In-place inverse of a symmetric positive definite n x n matrix (ld n) by
// blocked Gauss-Jordan sweeps.  CP: global scratch of n x kBK; P: LDS kBK x kBK;
// v: LDS 2 * kBK.  lds (lds_cap values, or nullptr): when 2 kBK n values fit, the
// panel column copy and the new row panel live there, so that the trailing update reads
// memory only for the entries it updates.
template <class T>
__device__ __forceinline__ void wg_spd_inverse(T* M, int n, T* CP, T* P, T* v, T* lds, int lds_cap) {
  const int tid = threadIdx.x;
  const bool in_lds = lds && 2 * kBK * n <= lds_cap;
  T* rp = in_lds ? lds + (size_t)kBK * n : nullptr;   // new row panel, rp[t * n + j]
  if (in_lds) CP = lds;
  for (int k0 = 0; k0 < n; k0 += kBK) {
    const int kb = min(kBK, n - k0);
    __syncthreads();
    for (int idx = tid; idx < kb * kb; idx += kBlock) {
      const int i = idx / kb, j = idx - i * kb;
      P[i * kBK + j] = M[(size_t)(k0 + i) * n + k0 + j];
    }
    __syncthreads();
    if (tid < 64) {
      // Gauss-Jordan on the pivot block by one wave (lane l owns rows l, l + 16 ... of column l % 16)
      for (int k = 0; k < kb; ++k) {
        const T piv = P[k * kBK + k];
        const T colv = tid < kb ? P[tid * kBK + k] : T(0);
        const T rowv = tid < kb ? P[k * kBK + tid] / piv : T(0);
        __builtin_amdgcn_wave_barrier();
        for (int idx = tid; idx < kb * kb; idx += 64) {
          const int i = idx / kb, j = idx - i * kb;
          const T ci = __shfl(colv, i, 64);
          const T rj = __shfl(rowv, j, 64);
          T val;
          if (i == k) val = (j == k) ? T(1) / piv : rj;
          else val = (j == k) ? -ci / piv : P[i * kBK + j] - ci * rj;
          P[i * kBK + j] = val;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    {
      const int cnt = (n * kb - tid + kBlock - 1) / kBlock;   // this thread's elements
      batched_terms<8>(0, cnt, [&](int k) {
        const int idx = tid + k * kBlock, i = idx / kb, t = idx - i * kb;
        return M[(size_t)i * n + k0 + t];
      }, [&](int k, T v) {
        const int idx = tid + k * kBlock, i = idx / kb, t = idx - i * kb;
        CP[(size_t)i * kBK + t] = v;
      });
    }
    __syncthreads();
    // row panel: M[k0+t][j] <- sum_s Pinv[t][s] M[k0+s][j] for j outside the block
    for (int j = tid; j < n; j += kBlock) {
      if (j >= k0 && j < k0 + kb) continue;
      T col[kBK];
#pragma unroll
      for (int s2 = 0; s2 < kBK; ++s2) col[s2] = s2 < kb ? M[(size_t)(k0 + s2) * n + j] : T(0);
      __builtin_amdgcn_sched_barrier(0);
      for (int t = 0; t < kb; ++t) {
        T acc = 0;
#pragma unroll
        for (int s2 = 0; s2 < kBK; ++s2)
          if (s2 < kb) acc += P[t * kBK + s2] * col[s2];
        M[(size_t)(k0 + t) * n + j] = acc;
        if (in_lds) rp[t * n + j] = acc;
      }
    }
    if (in_lds)   // the block's own columns of the row panel enter only discarded products
      for (int idx = tid; idx < kb * kb; idx += kBlock) rp[(idx / kb) * n + k0 + idx % kb] = T(0);
    __syncthreads();
    // trailing update M[i][j] -= sum_t M_old[i][k0+t] * M_new[k0+t][j]
    const int nt = (n + 3) / 4;
    if (in_lds) {
      for (int tile = tid; tile < nt * nt; tile += kBlock) {
        const int i0 = (tile / nt) * 4, j0 = (tile - (tile / nt) * nt) * 4;
        T mv[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = i0 + p, j = j0 + q;
            const bool upd = i < n && j < n && !(i >= k0 && i < k0 + kb) && !(j >= k0 && j < k0 + kb);
            mv[p][q] = upd ? M[(size_t)i * n + j] : T(0);
          }
        __builtin_amdgcn_sched_barrier(0);
        T acc[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p][q] = 0;
        for (int t = 0; t < kb; ++t) {
          T a[4], r[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            a[q] = (i0 + q < n) ? CP[(size_t)(i0 + q) * kBK + t] : T(0);
            r[q] = (j0 + q < n) ? rp[t * n + j0 + q] : T(0);
          }
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * r[q];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = i0 + p, j = j0 + q;
            if (i < n && j < n && !(i >= k0 && i < k0 + kb) && !(j >= k0 && j < k0 + kb))
              M[(size_t)i * n + j] = mv[p][q] - acc[p][q];
          }
      }
    } else
    for (int tile = tid; tile < nt * nt; tile += kBlock) {
      const int i0 = (tile / nt) * 4, j0 = (tile - (tile / nt) * nt) * 4;
      T acc[4][4];
      for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) acc[p][q] = 0;
      // panel columns and rows in batches of 8, every load of a batch issued before the products
      for (int t0 = 0; t0 < kb; t0 += 8) {
        T av[8][4], rv[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            av[u][q] = (t0 + u < kb && i0 + q < n) ? CP[(size_t)(i0 + q) * kBK + t0 + u] : T(0);
            rv[u][q] = (t0 + u < kb && j0 + q < n) ? M[(size_t)(k0 + t0 + u) * n + j0 + q] : T(0);
          }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (t0 + u < kb)
            for (int p = 0; p < 4; ++p)
              for (int q = 0; q < 4; ++q) acc[p][q] += av[u][p] * rv[u][q];
      }
      for (int p = 0; p < 4; ++p) {
        const int i = i0 + p;
        if (i >= n || (i >= k0 && i < k0 + kb)) continue;
        for (int q = 0; q < 4; ++q) {
          const int j = j0 + q;
          if (j >= n || (j >= k0 && j < k0 + kb)) continue;
          M[(size_t)i * n + j] -= acc[p][q];
        }
      }
    }
    // column panel: M[i][k0+t] <- -sum_s M_old[i][k0+s] Pinv[s][t]
    for (int i = tid; i < n; i += kBlock) {
      if (i >= k0 && i < k0 + kb) continue;
      T cp[kBK];
#pragma unroll
      for (int s2 = 0; s2 < kBK; ++s2) cp[s2] = s2 < kb ? CP[(size_t)i * kBK + s2] : T(0);
      __builtin_amdgcn_sched_barrier(0);
      for (int t = 0; t < kb; ++t) {
        T acc = 0;
#pragma unroll
        for (int s2 = 0; s2 < kBK; ++s2)
          if (s2 < kb) acc += cp[s2] * P[s2 * kBK + t];
        M[(size_t)i * n + k0 + t] = -acc;
      }
    }
    __syncthreads();
    for (int idx = tid; idx < kb * kb; idx += kBlock) {
      const int i = idx / kb, j = idx - i * kb;
      M[(size_t)(k0 + i) * n + k0 + j] = P[i * kBK + j];
    }
  }
  __syncthreads();
}

// Factors a general n x n matrix A (ld n, overwritten) by a blocked
// right-looking LU with partial pivoting: rows are swapped across the whole
// matrix (ties to the lowest row) and the pivot row of step k is stored in
// piv[k].  Each kBK-column panel is factored in LDS (pan: n * (kBK + 1) values; with lds_cap > 0
// values available from pan on, the panel's U12 block is kept beside it when it fits).
template <class T>
__device__ __forceinline__ void wg_lu_factor(T* A, int n, int* piv, int* perm, T* L11, T* pan, int lds_cap, double* sh_red,
                                             int* sh_i, int* sh_piv) {
  const int tid = threadIdx.x;
  constexpr int PS = kBK + 1;   // odd panel row stride: column accesses spread over the LDS banks
  __shared__ T sh_ui[kBK * kBK];
  for (int k0 = 0; k0 < n; k0 += kBK) {
    const int kb = min(kBK, n - k0);
    const int pr_rows = n - k0;
    __syncthreads();
    {
      const int cnt = (pr_rows * kb - tid + kBlock - 1) / kBlock;   // this thread's elements
      batched_terms<8>(0, cnt, [&](int k) {
        const int idx = tid + k * kBlock, i = idx / kb, t = idx - i * kb;
        return A[(size_t)(k0 + i) * n + k0 + t];
      }, [&](int k, T v) {
        const int idx = tid + k * kBlock, i = idx / kb, t = idx - i * kb;
        pan[i * PS + t] = v;
      });
    }
    __syncthreads();
    if (tid < 64) {
      // panel factorisation by one wave: lane l owns panel rows l, l + 64, ...
      for (int t = 0; t < kb; ++t) {
        double best = -1.0;
        int bi = pr_rows;
        for (int i = t + tid; i < pr_rows; i += 64) {
          const double a = fabs((double)pan[i * PS + t]);
          if (a > best) { best = a; bi = i; }
        }
        for (int d = 32; d > 0; d >>= 1) {
          const double ob = __shfl_xor(best, d, 64);
          const int oi = __shfl_xor(bi, d, 64);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const int pr = bi < pr_rows ? bi : t;
        if (tid == 0) piv[k0 + t] = k0 + pr;
        if (pr != t && tid < kb) {
          const T t0 = pan[t * PS + tid];
          pan[t * PS + tid] = pan[pr * PS + tid];
          pan[pr * PS + tid] = t0;
        }
        __builtin_amdgcn_wave_barrier();
        const T pv = pan[t * PS + t];
        // the pivot row right of the diagonal, in registers (fixed-size loops, so that the array is
        // never indexed dynamically and stays out of scratch)
        T urow[kBK];
#pragma unroll
        for (int q = 0; q < kBK; ++q) urow[q] = (t + 1 + q < kb) ? pan[t * PS + t + 1 + q] : T(0);
        for (int i = t + 1 + tid; i < pr_rows; i += 64) {
          const T l = pv != T(0) ? pan[i * PS + t] / pv : T(0);
          pan[i * PS + t] = l;
#pragma unroll
          for (int q = 0; q < kBK; ++q)
            if (t + 1 + q < kb) pan[i * PS + t + 1 + q] -= l * urow[q];
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    // The diagonal block is stored as the inverses of its factors (strictly lower part: the
    // unit lower inverse, upper part: the upper inverse), so that every triangular solve with
    // it (U12 below, wg_lu_apply) is a small matrix-vector product instead of a serial
    // substitution.  Lane cc forms column cc of both inverses by substitution; a zero pivot
    // gives a zero row (the solve then sets that unknown to zero).
    if (tid < kb) {
      const int cc = tid;
      T* LI = L11;      // unit lower inverse, kept for U12
      T* UI = sh_ui;
      for (int i = 0; i < kb; ++i) {
        T v = (i == cc) ? T(1) : T(0);
        for (int s2 = 0; s2 < i; ++s2) v -= pan[i * PS + s2] * LI[s2 * kBK + cc];
        LI[i * kBK + cc] = v;
      }
      for (int i = kb - 1; i >= 0; --i) {
        T v = (i == cc) ? T(1) : T(0);
        for (int s2 = i + 1; s2 < kb; ++s2) v -= pan[i * PS + s2] * UI[s2 * kBK + cc];
        const T d = pan[i * PS + i];
        UI[i * kBK + cc] = d != T(0) ? v / d : T(0);
      }
      for (int i = 0; i < kb; ++i)
        A[(size_t)(k0 + i) * n + k0 + cc] = (cc < i) ? LI[i * kBK + cc] : UI[i * kBK + cc];
    }
    // write the rest of the factored panel back; apply the block's row swaps to the other columns
    for (int idx = kb * kb + tid; idx < pr_rows * kb; idx += kBlock) {
      const int i = idx / kb, t = idx - i * kb;
      A[(size_t)(k0 + i) * n + k0 + t] = pan[i * PS + t];
    }
    for (int j = tid; j < n; j += kBlock) {
      if (j >= k0 && j < k0 + kb) continue;
      for (int t = 0; t < kb; ++t) {
        const int pr = piv[k0 + t];
        if (pr != k0 + t) {
          const T t0 = A[(size_t)(k0 + t) * n + j];
          A[(size_t)(k0 + t) * n + j] = A[(size_t)pr * n + j];
          A[(size_t)pr * n + j] = t0;
        }
      }
    }
    __syncthreads();
    // U12 = L11^-1 A12 with the unit lower inverse in L11 (rows taken last to first, so that
    // col[s < t] still holds the input).  When it fits beside the panel in LDS (lds_cap values
    // from pan on), U12 is also kept there for the trailing update.
    const int m0 = k0 + kb, mm = n - m0;
    T* u12 = pan + pr_rows * PS;
    const bool u12_lds = lds_cap > 0 && pr_rows * PS + kb * mm <= lds_cap;
    for (int j = k0 + kb + tid; j < n; j += kBlock) {
      T col[kBK];
      for (int t = 0; t < kb; ++t) col[t] = A[(size_t)(k0 + t) * n + j];
      for (int t = kb - 1; t > 0; --t) {
        T v = col[t];
        for (int s2 = 0; s2 < t; ++s2) v += L11[t * kBK + s2] * col[s2];
        col[t] = v;
      }
      for (int t = 0; t < kb; ++t) {
        A[(size_t)(k0 + t) * n + j] = col[t];
        if (u12_lds) u12[t * mm + (j - m0)] = col[t];
      }
    }
    __syncthreads();
    // A22 -= L21 U12 (L21 read from the LDS panel) in 4 x 4 tiles
    if (mm > 0) {
      const int nt = (mm + 3) / 4;
      if (u12_lds) {
        // both operands in LDS: the tile's 16 entries of A22 are loaded together before the
        // products, one round trip per tile
        auto tile_origin = [&](int tile, int& ti, int& tj) {
          ti = m0 + (tile / nt) * 4;
          tj = m0 + (tile - (tile / nt) * nt) * 4;
        };
        auto load_tile = [&](int ti, int tj, T (&v)[4][4]) {
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[p][q] = (ti + p < n && tj + q < n) ? A[(size_t)(ti + p) * n + tj + q] : T(0);
        };
        auto update_tile = [&](int ti, int tj, const T (&v)[4][4]) {
          T acc[4][4];
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p][q] = 0;
          for (int t = 0; t < kb; ++t) {
            T a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              a[q] = (ti + q < n) ? pan[(ti + q - k0) * PS + t] : T(0);
              b[q] = (tj + q < n) ? u12[t * mm + (tj + q - m0)] : T(0);
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
              for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
          }
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (ti + p < n && tj + q < n) A[(size_t)(ti + p) * n + tj + q] = v[p][q] - acc[p][q];
        };
        for (int tile = tid; tile < nt * nt; tile += kBlock) {
          int ti, tj;
          tile_origin(tile, ti, tj);
          T v[4][4];
          load_tile(ti, tj, v);
          __builtin_amdgcn_sched_barrier(0);
          update_tile(ti, tj, v);
        }
      } else {
        for (int tile = tid; tile < nt * nt; tile += kBlock) {
          const int ti0 = m0 + (tile / nt) * 4, tj0 = m0 + (tile - (tile / nt) * nt) * 4;
          T acc[4][4];
          for (int p = 0; p < 4; ++p)
            for (int q = 0; q < 4; ++q) acc[p][q] = 0;
          // U12 rows in batches of 8, every load of a batch issued before the products
          for (int t0 = 0; t0 < kb; t0 += 8) {
            T bv[8][4];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
              for (int q = 0; q < 4; ++q)
                bv[u][q] = (t0 + u < kb && tj0 + q < n) ? A[(size_t)(k0 + t0 + u) * n + tj0 + q] : T(0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              if (t0 + u < kb) {
                T a[4];
                for (int q = 0; q < 4; ++q) a[q] = (ti0 + q < n) ? pan[(ti0 + q - k0) * PS + t0 + u] : T(0);
                for (int p = 0; p < 4; ++p)
                  for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * bv[u][q];
              }
            }
          }
          for (int p = 0; p < 4; ++p) {
            if (ti0 + p >= n) continue;
            for (int q = 0; q < 4; ++q)
              if (tj0 + q < n) A[(size_t)(ti0 + p) * n + tj0 + q] -= acc[p][q];
          }
        }
      }
    }
  }
  __syncthreads();
  // the row swaps as one gather: applying them to the identity gives perm, so that
  // (P y)[q] = y[perm[q]]; built in the panel scratch, then copied out in parallel
  int* pw = reinterpret_cast<int*>(pan);
  for (int q = tid; q < n; q += kBlock) pw[q] = q;
  __syncthreads();
  if (tid == 0)
    for (int k = 0; k < n; ++k) {
      const int pr = piv[k];
      if (pr != k) { const int t0 = pw[k]; pw[k] = pw[pr]; pw[pr] = t0; }
    }
  __syncthreads();
  for (int q = tid; q < n; q += kBlock) perm[q] = pw[q];
  __syncthreads();
}

// Solves A y = r with the factors of wg_lu_factor.  r[16 q + 6] holds the
// right-hand side; the solution goes to r[16 q + 7].  perm: the row gather of the
// pivoting; ys: scratch of n values.  The diagonal blocks hold the inverses of their
// factors, so each block step is a 16-lane matrix-vector product followed by the update
// of the remaining rows.  dstage (LDS of 16 n values, or nullptr): the diagonal blocks are
// first staged there in one pass, so that the sequential block steps read them from LDS.
template <class T>
__device__ __forceinline__ void wg_lu_apply(const T* A, int n, const int* perm, T* r, T* ys, T* dstage) {
  const int tid = threadIdx.x;
  const int nblk = (n + kBK - 1) / kBK;
  __syncthreads();
  for (int q = tid; q < n; q += kBlock) ys[q] = r[16 * perm[q] + 6];
  if (dstage) {
    const int cnt = (nblk * kBK * kBK - tid + kBlock - 1) / kBlock;   // this thread's entries
    batched_terms<8>(0, cnt, [&](int k) {
      const int idx = tid + k * kBlock, b = idx / (kBK * kBK), ii = (idx / kBK) % kBK, jj = idx % kBK;
      const int k0 = b * kBK, kb = min(kBK, n - k0);
      return (ii < kb && jj < kb) ? A[(size_t)(k0 + ii) * n + k0 + jj] : T(0);
    }, [&](int k, T v) { dstage[tid + k * kBlock] = v; });
  }
  __syncthreads();
  // diagonal-block row tid of block b (kb columns), from LDS or memory
  auto drow = [&](int b, int k0) -> const T* {
    return dstage ? dstage + (size_t)b * kBK * kBK + tid * kBK : A + (size_t)(k0 + tid) * n + k0;
  };
  // Each thread's first row of the next block step is loaded one step ahead (the loads do not
  // depend on the solution), so that they complete under the current step's barriers; further
  // rows of a thread (systems above kBlock + kBK rows) are loaded when used.
  T pre[kBK];
  auto prefetch = [&](int row, int k0n, int kbn) {
#pragma unroll
    for (int t = 0; t < kBK; ++t) pre[t] = (row < n && t < kbn) ? A[(size_t)row * n + k0n + t] : T(0);
  };
  // forward substitution with the unit lower factor
  prefetch(min(kBK, n) + tid, 0, min(kBK, n));
  for (int k0 = 0; k0 < n; k0 += kBK) {
    const int kb = min(kBK, n - k0);
    T v = 0;
    if (tid < kb) {
      const T* Ar = drow(k0 / kBK, k0);
      v = ys[k0 + tid];
      for (int s2 = 0; s2 < tid; ++s2) v += Ar[s2] * ys[k0 + s2];
    }
    __syncthreads();
    if (tid < kb) ys[k0 + tid] = v;
    __syncthreads();
    {
      const int i = k0 + kb + tid;
      if (i < n) {
        T acc = 0;
#pragma unroll
        for (int t = 0; t < kBK; ++t)
          if (t < kb) acc += pre[t] * ys[k0 + t];
        ys[i] -= acc;
      }
      const int k0n = k0 + kBK, kbn = min(kBK, n - k0n);
      if (k0n < n) prefetch(k0n + kbn + tid, k0n, kbn);
    }
    for (int i = k0 + kb + kBlock + tid; i < n; i += kBlock) {
      T acc = 0;
      const T* Ar = A + (size_t)i * n + k0;
      batched_terms<8>(0, kb, [&](int t) { return Ar[t]; }, [&](int t, T a) { acc += a * ys[k0 + t]; });
      ys[i] -= acc;
    }
    __syncthreads();
  }
  // back substitution with the upper factor
  if (nblk > 1) prefetch(tid < (nblk - 1) * kBK ? tid : n, (nblk - 1) * kBK, min(kBK, n - (nblk - 1) * kBK));
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int k0 = bk * kBK, kb = min(kBK, n - k0);
    T v = 0;
    if (tid < kb) {
      const T* Ar = drow(bk, k0);
      for (int s2 = tid; s2 < kb; ++s2) v += Ar[s2] * ys[k0 + s2];
    }
    __syncthreads();
    if (tid < kb) ys[k0 + tid] = v;
    __syncthreads();
    {
      const int i = tid;
      if (i < k0) {
        T acc = 0;
#pragma unroll
        for (int t = 0; t < kBK; ++t)
          if (t < kb) acc += pre[t] * ys[k0 + t];
        ys[i] -= acc;
      }
      if (bk > 0) prefetch(tid < k0 - kBK ? tid : n, k0 - kBK, kBK);
    }
    for (int i = kBlock + tid; i < k0; i += kBlock) {
      T acc = 0;
      const T* Ar = A + (size_t)i * n + k0;
      batched_terms<8>(0, kb, [&](int t) { return Ar[t]; }, [&](int t, T a) { acc += a * ys[k0 + t]; });
      ys[i] -= acc;
    }
    __syncthreads();
  }
  for (int q = tid; q < n; q += kBlock) r[16 * q + 7] = ys[q];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Contact subproblem (Eq. 2b with Eq. 4 at fixed projections): find lambda
// with Phi(lambda) = 0 for Y(lambda) = y_free + W lambda,
// W = h^2 F^T (Gc (x) I3) F the exact Delassus operator of the env.
// Semismooth Newton on Phi with the Delassus diagonal as proximal scale; the
// Newton system Z = K W + E is solved exactly by the Woodbury identity around
// the explicit inverse of W on the coupled contacts (rows of Z that are not
// plain W rows form the capacitance system, LU with partial pivoting).
// The stopping test uses the residual scale s = h^2 / m_v in FP64.
// ---------------------------------------------------------------------------
template <class T>
struct CspSmem {
  double* lam;                                 // [3*cap] multipliers, FP64
  T *Y, *dl, *Wd, *rv, *x0, *fw, *ph, *tmp;    // [3*cap]
  T *sp, *kap, *yh0, *yh1;                    // [cap]
  T *pan, *ys;                                // [rlds*(kBK+1)], [rlds]
  int *cls, *pos, *bas;                       // [cap]
};

// The lightweight update (flash_contact.h) of one env's contact subproblem by one workgroup with
// the env's contact data in LDS; the contact displacement follows lambda through the contact-space
// Delassus operator W = h^2 F^T Gbar[contacts] F.
template <class T, class CT>
__device__ __forceinline__ void csp_env_lite(const DevBatch<T>& B, const T* mu_env, int first_lg, int e,
                                             unsigned char* smem_raw, bool own_cost) {
  const unsigned long long t_start = (own_cost && B.cost && threadIdx.x == 0) ? wall_clock64() : 0ull;
  const int c = B.ccount[e];
  if (c == 0) {
    if (first_lg && B.ws_state && threadIdx.x == 0) B.ws_state[e] &= ~5;
    return;
  }
  const int cap = B.cap;
  double* lam = reinterpret_cast<double*>(smem_raw);
  CT* Y = reinterpret_cast<CT*>(lam + 3 * cap);
  CT* fw = Y + 3 * cap;
  CT* dl = fw + 3 * cap;
  CT* d0s = dl + 3 * cap;
  CT* dobs = d0s + cap;
  __shared__ double sh_red[kBlock / 64];
  const size_t cb = (size_t)e * cap;
  const CT* Gc = static_cast<const CT*>(B.Gc) + cb * cap;
  const int v0 = B.voff[e];
  const CT hh = (CT)(B.h * B.h);
  const CT mu = mu_env[e];
  const double dmaxf = B.max_force;
  const CT* Fr;
  if constexpr (std::is_same<CT, T>::value) Fr = B.cframe + 9 * cb;
  else Fr = B.cframe64 + 9 * cb;
  CT* yfg = static_cast<CT*>(B.cyf) + 3 * cb;
  const int* cv = B.cvert + cb;
  const int* cobs = B.cobs + cb;
  const int tid = threadIdx.x;
  for (int j = tid; j < c; j += kBlock) {
    const CT* F = Fr + 9 * j;
    const int vi = v0 + cv[j];
    const CT zw0 = B.z[vi], zw1 = B.z[B.NV + vi], zw2 = B.z[2 * B.NV + vi];
    for (int a = 0; a < 3; ++a) {
      yfg[3 * j + a] = F[3 * a] * zw0 + F[3 * a + 1] * zw1 + F[3 * a + 2] * zw2;
      lam[3 * j + a] = B.clam[3 * (cb + j) + a];
    }
    d0s[j] = B.cd0[cb + j];
    dobs[2 * j] = B.cdob[2 * (cb + j)];
    dobs[2 * j + 1] = B.cdob[2 * (cb + j) + 1];
  }
  __syncthreads();
  // Y = y_free + W lambda with W = h^2 F^T Gbar[contacts] F (Gc symmetric: coalesced column reads)
  auto update_Y = [&]() {
    for (int j = tid; j < c; j += kBlock) {
      const CT* F = Fr + 9 * j;
      const CT l0 = (CT)lam[3 * j], l1 = (CT)lam[3 * j + 1], l2 = (CT)lam[3 * j + 2];
      for (int k = 0; k < 3; ++k) fw[3 * j + k] = F[k] * l0 + F[3 + k] * l1 + F[6 + k] * l2;
    }
    __syncthreads();
    for (int j = tid; j < c; j += kBlock) {
      CT g0 = 0, g1 = 0, g2 = 0;
      batched_terms<16>(0, c, [&](int k) { return Gc[(size_t)k * c + j]; }, [&](int k, CT g) {
        g0 += g * fw[3 * k]; g1 += g * fw[3 * k + 1]; g2 += g * fw[3 * k + 2];
      });
      const CT* F = Fr + 9 * j;
      for (int a = 0; a < 3; ++a)
        Y[3 * j + a] = yfg[3 * j + a] + hh * (F[3 * a] * g0 + F[3 * a + 1] * g1 + F[3 * a + 2] * g2);
    }
    __syncthreads();
  };
  update_Y();
  const int maxit = B.max_newton;
  int it = 0;
  double r = 0.0;
  for (;; ++it) {
    // residual at the residual scale s = h^2 / m_v (FP64), the same scale as the update's
    double rloc = 0.0;
    for (int j = tid; j < c; j += kBlock) {
      const double s = (double)B.cs[cb + j];
      const double ld0 = lam[3 * j], ld1 = lam[3 * j + 1], ld2 = lam[3 * j + 2];
      const double cnd = B.cd0d[cb + j] + (double)Y[3 * j];
      const double ut1 = (double)Y[3 * j + 1] - (double)dobs[2 * j], ut2 = (double)Y[3 * j + 2] - (double)dobs[2 * j + 1];
      const bool att = cobs[j] >= kMaxObs;
      const double pn = att ? cnd : fmin(cnd, s * ld0);
      const double z1 = ld1 - ut1 / s, z2 = ld2 - ut2 / s;
      const double nz = sqrt(z1 * z1 + z2 * z2);
      const double rh = (double)mu * fmax(ld0, 0.0);
      double q1 = z1, q2 = z2;
      if (!att && nz > rh) { const double f = nz > 0 ? rh / nz : 0.0; q1 = f * z1; q2 = f * z2; }
      const double t1 = s * (ld1 - q1), t2 = s * (ld2 - q2);
      double rj = fmax(fabs(pn), sqrt(t1 * t1 + t2 * t2));
      if (!(rj == rj)) rj = INFINITY;
      rloc = fmax(rloc, rj);
    }
    r = block_max(rloc, sh_red);
    if (r <= B.tol || it >= maxit) break;
    // one update per vertex group (contacts are listed by vertex, so a group is contiguous)
    for (int j = tid; j < c; j += kBlock) {
      if (j > 0 && cv[j - 1] == cv[j]) continue;
      int m = 1;
      while (j + m < c && cv[j + m] == cv[j] && m < kCacheSlots) ++m;
      const CT sp = (CT)B.cs[cb + j];
      if (m == 1) {
        CT ph[3], K[3][3], E[3][3];
        lite_contact(sp, mu, d0s[j], dobs[2 * j], dobs[2 * j + 1], Y + 3 * j, lam + 3 * j, cobs[j] >= kMaxObs, ph, K,
                     E);
        // Z = sp K + E = [sp 0 0; E_tn sp I]
        const CT dn = -ph[0] / sp;
        dl[3 * j] = dn;
        dl[3 * j + 1] = (-ph[1] - E[1][0] * dn) / sp;
        dl[3 * j + 2] = (-ph[2] - E[2][0] * dn) / sp;
      } else {
        lite_group_solve<CT>(m, sp, mu, Fr + 9 * j, d0s + j, dobs + 2 * j, Y + 3 * j, lam + 3 * j, cobs + j,
                             dl + 3 * j);
      }
    }
    __syncthreads();
    for (int q = tid; q < 3 * c; q += kBlock) lam[q] = fmin(fmax(lam[q] + (double)dl[q], -dmaxf), dmaxf);
    __syncthreads();
    update_Y();
  }
  for (int j = tid; j < c; j += kBlock) {
    const CT* F = Fr + 9 * j;
    const CT l0 = (CT)lam[3 * j], l1 = (CT)lam[3 * j + 1], l2 = (CT)lam[3 * j + 2];
    for (int a = 0; a < 3; ++a) B.clam[3 * (cb + j) + a] = lam[3 * j + a];
    for (int k = 0; k < 3; ++k) B.cforce[3 * (cb + j) + k] = (T)(F[k] * l0 + F[3 + k] * l1 + F[6 + k] * l2);
  }
  if (tid == 0) {
    B.iters[e] += it;
    if (B.phase) {
      unsigned long long* cnt = B.phase + (size_t)B.n_envs * 8 + 8 * e;
      cnt[3] += (r > B.tol) ? 1 : 0;
      cnt[6] += it;
      cnt[7] += 1;
    }
    if (r > B.tol) B.flags[e] |= 2; else B.flags[e] &= ~2;
    if (own_cost && B.cost) B.cost[e] += wall_clock64() - t_start;
    if (first_lg && B.ws_state) B.ws_state[e] &= ~5;
  }
}

// The contact subproblem of env e by the whole workgroup; smem_raw: csp_smem_bytes<CT>
// of LDS.  own_cost: add the solve's wall-clock time to the env's scheduling cost.
template <class T, class CT, bool LITE = false>
__device__ __forceinline__ void csp_env(const DevBatch<T>& B, const T* mu_env, int first_lg, int e, unsigned char* smem_raw,
                        bool own_cost) {
  if constexpr (LITE) {
    csp_env_lite<T, CT>(B, mu_env, first_lg, e, smem_raw, own_cost);
    return;
  }
  const unsigned long long t_start = (own_cost && B.cost && threadIdx.x == 0) ? wall_clock64() : 0ull;
  const int c = B.ccount[e];
  if (c == 0) {
    if (first_lg && B.ws_state && threadIdx.x == 0) B.ws_state[e] &= ~5;
    return;
  }
  const int cap = B.cap;
  CspSmem<CT> S;
  {
    S.lam = reinterpret_cast<double*>(smem_raw);
    CT* p = reinterpret_cast<CT*>(S.lam + 3 * cap);
    S.Y = p; p += 3 * cap; S.dl = p; p += 3 * cap;
    S.Wd = p; p += 3 * cap; S.rv = p; p += 3 * cap; S.x0 = p; p += 3 * cap; S.fw = p; p += 3 * cap;
    S.ph = p; p += 3 * cap; S.tmp = p; p += 3 * cap;
    S.sp = p; p += cap; S.kap = p; p += cap; S.yh0 = p; p += cap; S.yh1 = p; p += cap;
    S.pan = p; p += (size_t)B.rlds * (kBK + 1); S.ys = p; p += B.rlds;
    int* ip = reinterpret_cast<int*>(p);
    S.cls = ip; ip += cap; S.pos = ip; ip += cap; S.bas = ip; ip += cap;
  }
  __shared__ double sh_red[kBlock / 64];
  __shared__ int sh_i[kBlock / 64];
  __shared__ int sh_nb, sh_nR, sh_piv;
  __shared__ CT sh_blk[kBK * kBK];
  __shared__ CT sh_vv[2 * kBK];

  const size_t cb = (size_t)e * cap;
  const CT* Gc = static_cast<const CT*>(B.Gc) + cb * cap;   // ld c
  CT* Ginv = static_cast<CT*>(B.Ginv) + cb * cap;            // ld nb
  CT* Cm = static_cast<CT*>(B.Cm) + (size_t)e * B.rmax * B.rmax;
  const int v0 = B.voff[e];
  const CT hh = (CT)(B.h * B.h), ihh = CT(1) / hh;
  const CT mu = mu_env[e];
  const double dmaxf = B.max_force;
  // contact frames in the solve's precision: FP32 frames are orthonormal only to ~1e-7, and the
  // Woodbury step applies the base inverse as F^T (.) F, which amplifies that by the condition
  // of the contact-space operator (~1e5 for stiff bending against light vertices)
  const CT* Fr;
  if constexpr (std::is_same<CT, T>::value) Fr = B.cframe + 9 * cb;
  else Fr = B.cframe64 + 9 * cb;
  CT* yfg = static_cast<CT*>(B.cyf) + 3 * cb;     // free displacement y_free in contact frames
  const int tid = threadIdx.x;
  // per-phase wall-clock accounting (thread 0, when enabled)
  unsigned long long t_mark = (B.phase && tid == 0) ? wall_clock64() : 0ull;
  auto mark = [&](int ph) {
    if (B.phase && tid == 0) {
      const unsigned long long now = wall_clock64();
      B.phase[(size_t)e * 8 + ph] += now - t_mark;
      t_mark = now;
    }
  };

  // per-R-row data in global scratch (after the rmax*rmax matrices):
  // vR(3) uR(3) rhs y Krow(3) Erow(3) -- 16 values per row
  CT* Rv = static_cast<CT*>(B.Cm) + (size_t)B.n_envs * B.rmax * B.rmax + (size_t)e * B.rmax * 16;
  int* Rj = reinterpret_cast<int*>(static_cast<CT*>(B.Cm) + (size_t)B.n_envs * B.rmax * B.rmax + (size_t)B.n_envs * B.rmax * 16) +
            (size_t)e * B.rmax * 4;
  int* RjF = Rj + B.rmax;      // row list of the stored factorisation
  int* piv = Rj + 2 * B.rmax;  // its pivots
  int* perm = Rj + 3 * B.rmax; // and the equivalent row gather
  int* lust = B.lust + 4 * e;  // valid, nR, base version at factorisation, current base version

  // ---- load state ----
  if (tid == 0) sh_nb = B.nbase[e];
  __syncthreads();
  int nb = sh_nb;
  for (int j = tid; j < c; j += kBlock) {
    S.pos[j] = -1;
    const CT* F = Fr + 9 * j;
    const int vi = v0 + B.cvert[cb + j];
    CT zw0 = B.z[vi], zw1 = B.z[B.NV + vi], zw2 = B.z[2 * B.NV + vi];
    for (int a = 0; a < 3; ++a) {
      yfg[3 * j + a] = F[3 * a] * zw0 + F[3 * a + 1] * zw1 + F[3 * a + 2] * zw2;
      S.lam[3 * j + a] = B.clam[3 * (cb + j) + a];
    }
    S.sp[j] = hh * Gc[(size_t)j * c + j];
  }
  __syncthreads();
  for (int p = tid; p < nb; p += kBlock) {
    int j = B.base[cb + p];
    S.bas[p] = j;
    S.pos[j] = p;
  }
  __syncthreads();

  // Y = y_free + W lambda (fw = F lambda world; Gc symmetric -> coalesced column reads)
  auto apply_W = [&](const auto* vin, CT* vout) {
    for (int j = tid; j < c; j += kBlock) {
      const CT* F = Fr + 9 * j;
      const CT l0 = (CT)vin[3 * j], l1 = (CT)vin[3 * j + 1], l2 = (CT)vin[3 * j + 2];
      for (int k = 0; k < 3; ++k) S.fw[3 * j + k] = F[k] * l0 + F[3 + k] * l1 + F[6 + k] * l2;
    }
    __syncthreads();
    for (int j = tid; j < c; j += kBlock) {
      CT d0 = 0, d1 = 0, d2 = 0;
      batched_terms<16>(0, c, [&](int k) { return Gc[(size_t)k * c + j]; }, [&](int k, CT g) {
        d0 += g * S.fw[3 * k]; d1 += g * S.fw[3 * k + 1]; d2 += g * S.fw[3 * k + 2];
      });
      const CT* F = Fr + 9 * j;
      for (int a = 0; a < 3; ++a) vout[3 * j + a] = hh * (F[3 * a] * d0 + F[3 * a + 1] * d1 + F[3 * a + 2] * d2);
    }
    __syncthreads();
  };

  // previous-iterate start: the multipliers in clam (the previous-step warm start
  // in the first local-global iteration), new contacts get a Jacobi estimate of lambda_n
  auto load_prev = [&](bool reload) {
    if (reload) {
      for (int j = tid; j < c; j += kBlock)
        for (int a = 0; a < 3; ++a) S.lam[3 * j + a] = B.clam[3 * (cb + j) + a];
      __syncthreads();
    }
    apply_W(S.lam, S.Y);
    for (int j = tid; j < c; j += kBlock)
      for (int a = 0; a < 3; ++a) S.Y[3 * j + a] += yfg[3 * j + a];
    __syncthreads();
    if (first_lg) {
      int any = 0;
      for (int j = tid; j < c; j += kBlock) {
        if (B.cnew[cb + j]) {
          const CT cn = B.cd0[cb + j] + S.Y[3 * j];
          const bool att = B.cobs[cb + j] >= kMaxObs;   // attachment rows start from zero
          S.lam[3 * j] = (cn < CT(0) && !att) ? (double)(-cn / S.sp[j]) : 0.0;
          S.lam[3 * j + 1] = 0;
          S.lam[3 * j + 2] = 0;
          any = 1;
        }
      }
      if (block_max((double)any, sh_red) > 0) {
        apply_W(S.lam, S.Y);
        for (int j = tid; j < c; j += kBlock)
          for (int a = 0; a < 3; ++a) S.Y[3 * j + a] += yfg[3 * j + a];
        __syncthreads();
      }
    }
  };
  load_prev(false);

  // learned warm start: contacts without a previous-step multiplier (new contacts, or
  // every contact after a reset) take the network's prediction instead of the Jacobi
  // estimate when that lowers the merit 0.5 |Phi|^2 of the start (inner scale);
  // non-finite predictions never win
  bool learned = false;
  if (first_lg && B.lam_ml && (B.ws_state[e] & 0xff00) < (kWsMaxFail << 8)) {
    int anynew = 0;
    for (int j = tid; j < c; j += kBlock) anynew |= B.cnew[cb + j];
    if (block_max((double)anynew, sh_red) > 0) {
      auto merit = [&](const auto* L, const CT* Yv) {
        double ps = 0.0;
        for (int j = tid; j < c; j += kBlock) {
          const CT sp = S.sp[j];
          const CT l0 = (CT)L[3 * j], l1 = (CT)L[3 * j + 1], l2 = (CT)L[3 * j + 2];
          const CT cn = B.cd0[cb + j] + Yv[3 * j];
          const CT ut1 = Yv[3 * j + 1] - B.cdob[2 * (cb + j)], ut2 = Yv[3 * j + 2] - B.cdob[2 * (cb + j) + 1];
          const bool att = B.cobs[cb + j] >= kMaxObs;
          const CT phn = att ? cn : fmin(cn, sp * l0);
          const CT y1 = l1 - ut1 / sp, y2 = l2 - ut2 / sp;
          const CT rho = mu * fmax(l0, CT(0));
          const CT ny = sqrt(y1 * y1 + y2 * y2);
          CT p1 = 0, p2 = 0;
          if (att) { p1 = y1; p2 = y2; }
          else if (rho > CT(0)) {
            if (ny <= rho) { p1 = y1; p2 = y2; }
            else { p1 = rho * y1 / ny; p2 = rho * y2 / ny; }
          }
          const CT ph1 = sp * (l1 - p1), ph2 = sp * (l2 - p2);
          double q = (double)phn * phn + (double)ph1 * ph1 + (double)ph2 * ph2;
          if (!(q == q)) q = INFINITY;
          ps += q;
        }
        return 0.5 * block_sum(ps, sh_red);
      };
      const double psi_prev = merit(S.lam, S.Y);
      for (int j = tid; j < c; j += kBlock) {
        const bool take = B.cnew[cb + j] != 0;
        for (int a = 0; a < 3; ++a)
          S.dl[3 * j + a] = (CT)(take ? B.lam_ml[3 * (cb + j) + a] : S.lam[3 * j + a]);
      }
      __syncthreads();
      apply_W(S.dl, S.tmp);
      for (int j = tid; j < c; j += kBlock)
        for (int a = 0; a < 3; ++a) S.tmp[3 * j + a] += yfg[3 * j + a];
      __syncthreads();
      if (merit(S.dl, S.tmp) < psi_prev) {
        learned = true;
        for (int j = tid; j < c; j += kBlock) {
          if (B.cnew[cb + j])
            for (int a = 0; a < 3; ++a) S.lam[3 * j + a] = B.lam_ml[3 * (cb + j) + a];
          for (int a = 0; a < 3; ++a) S.Y[3 * j + a] = S.tmp[3 * j + a];
        }
        __syncthreads();
      }
    }
  }
  bool learned_failed = false;

  int it = 0, nref = 0, nfact = 0, nreuse = 0, nlsfail = 0, max_nr = 0;
  long sum_nr = 0;
  const int maxit = B.max_newton;
  double r = 0.0;
  mark(0);
  int it0 = 0;
  // stall recovery: after kStallRun consecutive failed line searches the solve starts once more
  // from the zero start (Jacobi estimates of the normal multipliers) with a fresh iteration budget
  constexpr int kStallRun = 8;
  int ls_run = 0;
  bool zero_restarted = false;
restart:
  for (;; ++it) {
    // ---- Phi (inner scale), classification, residual (residual scale, FP64) ----
    double rloc = 0.0, psil = 0.0;
    for (int j = tid; j < c; j += kBlock) {
      const CT sp = S.sp[j];
      const double ld0 = S.lam[3 * j], ld1 = S.lam[3 * j + 1], ld2 = S.lam[3 * j + 2];
      const CT l0 = (CT)ld0, l1 = (CT)ld1, l2 = (CT)ld2;
      const CT cn = B.cd0[cb + j] + S.Y[3 * j];
      const CT ut1 = S.Y[3 * j + 1] - B.cdob[2 * (cb + j)], ut2 = S.Y[3 * j + 2] - B.cdob[2 * (cb + j) + 1];
      // attachment rows (bilateral): Phi = Y - d, always active and sticking, no cone
      const bool att = B.cobs[cb + j] >= kMaxObs;
      const CT phn = att ? cn : fmin(cn, sp * l0);
      const CT y1 = l1 - ut1 / sp, y2 = l2 - ut2 / sp;
      const CT rho = mu * fmax(l0, CT(0));
      const CT ny = sqrt(y1 * y1 + y2 * y2);
      int cls = (att || cn <= sp * l0) ? 1 : 0;
      CT p1 = y1, p2 = y2, kap = 0, yh0 = 0, yh1 = 0;
      if (att) cls |= 2;
      else if (rho > CT(0)) {
        if (ny <= rho) cls |= 2;
        else {
          cls |= 4;
          kap = rho / ny; yh0 = y1 / ny; yh1 = y2 / ny;
          p1 = rho * yh0; p2 = rho * yh1;
        }
      } else { p1 = 0; p2 = 0; }
      const CT ph1 = sp * (l1 - p1), ph2 = sp * (l2 - p2);
      S.ph[3 * j] = phn; S.ph[3 * j + 1] = ph1; S.ph[3 * j + 2] = ph2;
      S.cls[j] = cls; S.kap[j] = kap; S.yh0[j] = yh0; S.yh1[j] = yh1;
      psil += (double)phn * phn + (double)ph1 * ph1 + (double)ph2 * ph2;
      // residual scale
      const double s = (double)B.cs[cb + j];
      const double cnd = B.cd0d[cb + j] + (double)S.Y[3 * j];
      const double pn = att ? cnd : fmin(cnd, s * ld0);
      const double z1 = ld1 - (double)ut1 / s, z2 = ld2 - (double)ut2 / s;
      const double nz = sqrt(z1 * z1 + z2 * z2);
      const double rh = (double)mu * fmax(ld0, 0.0);
      double q1 = z1, q2 = z2;
      if (!att && nz > rh) { double f = nz > 0 ? rh / nz : 0.0; q1 = f * z1; q2 = f * z2; }
      const double t1 = s * (ld1 - q1), t2 = s * (ld2 - q2);
      double rj = fmax(fabs(pn), sqrt(t1 * t1 + t2 * t2));
      if (!(rj == rj)) rj = INFINITY;
      rloc = fmax(rloc, rj);
    }
    r = block_max(rloc, sh_red);
    const double psi = 0.5 * block_sum(psil, sh_red);
    mark(1);
    if (r <= B.tol || it - it0 >= maxit) break;

    // ---- base set: refactor when a coupled contact lies outside it ----
    int need = 0;
    for (int j = tid; j < c; j += kBlock)
      if ((S.cls[j] & 7) && S.pos[j] < 0) need = 1;
    if (block_max((double)need, sh_red) > 0) {
      // base = coupled contacts in index order
      for (int j0 = 0; j0 < c; j0 += kBlock) {
        const int j = j0 + tid;
        const int f = (j < c && (S.cls[j] & 7)) ? 1 : 0;
        int tot;
        const int off = block_excl_scan_i(f, sh_i, &tot);
        const int basep = j0 == 0 ? 0 : sh_nb;
        __syncthreads();
        if (j < c) S.pos[j] = f ? basep + off : -1;
        if (f) S.bas[basep + off] = j;
        __syncthreads();
        if (tid == 0) sh_nb = basep + tot;
        __syncthreads();
      }
      nb = sh_nb;
      // Ginv = inverse of Gc[base, base] (+1e-4 relative on repeated vertices), Gauss-Jordan
      {
        const int cnt = (nb * nb - tid + kBlock - 1) / kBlock;   // this thread's entries
        batched_terms<8>(0, cnt, [&](int k) {
          const int idx = tid + k * kBlock, p = idx / nb, q = idx - p * nb;
          return Gc[(size_t)S.bas[p] * c + S.bas[q]];
        }, [&](int k, CT g) {
          const int idx = tid + k * kBlock, p = idx / nb, q = idx - p * nb;
          if (p == q && p > 0 && B.cvert[cb + S.bas[p]] == B.cvert[cb + S.bas[p - 1]]) g *= CT(1.0001);
          Ginv[idx] = g;
        });
      }
      wg_spd_inverse(Ginv, nb, static_cast<CT*>(B.scr) + cb * kBK, sh_blk, sh_vv, S.pan, B.rlds * (kBK + 2));
      if (tid == 0) lust[3] += 1;
      __syncthreads();
      ++nref;
    }

    mark(2);
    // ---- decoupled contacts (outside the base): local rows E = sp I ----
    int anydec = 0;
    for (int j = tid; j < c; j += kBlock) {
      if (S.pos[j] < 0) {
        const CT isp = CT(1) / S.sp[j];
        for (int a = 0; a < 3; ++a) {
          S.dl[3 * j + a] = -S.ph[3 * j + a] * isp;
          anydec |= S.dl[3 * j + a] != CT(0) ? 1 : 0;
        }
      } else {
        for (int a = 0; a < 3; ++a) S.dl[3 * j + a] = 0;
      }
    }
    __syncthreads();
    if (block_max((double)anydec, sh_red) > 0) {
      apply_W(S.dl, S.Wd);   // W * (decoupled part)
    } else {                 // no decoupled update: the product is exactly zero
      for (int q = tid; q < 3 * c; q += kBlock) S.Wd[q] = 0;
      __syncthreads();
    }
    // rhs on base rows: r = -Phi - K (W dl_D)
    for (int j = tid; j < c; j += kBlock) {
      if (S.pos[j] < 0) continue;
      CT K[3][3], E[3][3];
      contact_KE(S.cls[j], S.sp[j], mu, S.kap[j], S.yh0[j], S.yh1[j], K, E);
      CT w0 = S.Wd[3 * j], w1 = S.Wd[3 * j + 1], w2 = S.Wd[3 * j + 2];
      for (int a = 0; a < 3; ++a)
        S.rv[3 * j + a] = -S.ph[3 * j + a] - (K[a][0] * w0 + K[a][1] * w1 + K[a][2] * w2);
    }
    __syncthreads();

    mark(3);
    // ---- capacitance rows R: base rows whose (K, E) differ from (I, 0) ----
    if (tid == 0) sh_nR = 0;
    __syncthreads();
    {
      for (int p0 = 0; p0 < nb; p0 += kBlock) {
        const int p = p0 + tid;
        int cnt = 0, cl = 0;
        if (p < nb) {
          cl = S.cls[S.bas[p]];
          cnt = ((cl & 1) ? 0 : 1) + ((cl & 2) ? 0 : 2);
        }
        int tot;
        const int off = block_excl_scan_i(cnt, sh_i, &tot);
        const int base_r = p0 == 0 ? 0 : sh_nR;
        __syncthreads();
        if (p < nb) {
          int o = base_r + off;
          const int j = S.bas[p];
          for (int a = 0; a < 3; ++a) {
            const bool mod = a == 0 ? !(cl & 1) : !(cl & 2);
            if (!mod) continue;
            if (o < B.rmax) Rj[o] = 3 * j + a;
            ++o;
          }
        }
        __syncthreads();
        if (tid == 0) sh_nR = base_r + tot;
        __syncthreads();
      }
    }
    const int nR = min(sh_nR, B.rmax);
    if (sh_nR > B.rmax && tid == 0) B.flags[e] |= 8;   // capacity exceeded: inexact direction
    // LU panel and solve vector: LDS for systems up to rlds rows, global scratch above
    CT* gpan = static_cast<CT*>(B.lupan) + (size_t)e * B.rmax * (kBK + 2);
    CT* gys = gpan + (size_t)B.rmax * (kBK + 1);
    const bool big = nR > B.rlds;
    bool reused = false;
    if (nR > 0) {
      // reuse the stored factorisation when its row set and base are unchanged
      int diff = 0;
      if (B.reuse && lust[0] && lust[1] == nR && lust[2] == lust[3]) {
        for (int q = tid; q < nR; q += kBlock) diff |= Rj[q] != RjF[q];
      } else {
        diff = 1;
      }
      reused = block_max((double)diff, sh_red) == 0.0;
      if (!reused) {
        // per-row vectors: vR = F E^CT[:, a] (world), uR = F[:, a], K and E rows (contact frame)
        for (int q = tid; q < nR; q += kBlock) {
          const int ja = Rj[q], j = ja / 3, a = ja - 3 * (ja / 3);
          CT K[3][3], E[3][3];
          contact_KE(S.cls[j], S.sp[j], mu, S.kap[j], S.yh0[j], S.yh1[j], K, E);
          const CT* F = Fr + 9 * j;
          CT* rv = Rv + 16 * q;
          for (int k = 0; k < 3; ++k) {
            rv[k] = E[a][0] * F[k] + E[a][1] * F[3 + k] + E[a][2] * F[6 + k];
            rv[3 + k] = F[3 * a + k];
            rv[8 + k] = K[a][k];
            rv[11 + k] = E[a][k];
          }
          RjF[q] = ja;
          if (!big) {
            // also staged in the (still free) LDS panel for the build below: vR, uR, K row;
            // contact, component and base position
            CT* sv = S.pan + 9 * q;
            int* si = reinterpret_cast<int*>(S.pan + 9 * nR) + 3 * q;
            for (int k = 0; k < 6; ++k) sv[k] = rv[k];
            for (int k = 0; k < 3; ++k) sv[6 + k] = K[a][k];
            si[0] = j;
            si[1] = a;
            si[2] = S.pos[j];
          }
        }
        __syncthreads();
        // C[q][s] = [same contact] K[a][b] + h^-2 Ginv[pj][pk] (vR_q . uR_s)
        if (!big) {
          // each entry reads memory once (its Ginv gather, batched)
          const CT* sv = S.pan;
          const int* si = reinterpret_cast<const int*>(S.pan + 9 * nR);
          const int cnt = (nR * nR - tid + kBlock - 1) / kBlock;   // this thread's entries
          batched_terms<8>(0, cnt, [&](int k) {
            const int idx = tid + k * kBlock, q = idx / nR, s2 = idx - q * nR;
            return Ginv[(size_t)si[3 * q + 2] * nb + si[3 * s2 + 2]];
          }, [&](int k, CT g) {
            const int idx = tid + k * kBlock, q = idx / nR, s2 = idx - q * nR;
            const CT* vq = sv + 9 * q;
            const CT* us = sv + 9 * s2 + 3;
            CT v = ihh * g * (vq[0] * us[0] + vq[1] * us[1] + vq[2] * us[2]);
            if (si[3 * q] == si[3 * s2]) v += vq[6 + si[3 * s2 + 1]];
            Cm[idx] = v;
          });
        } else {
          for (int idx = tid; idx < nR * nR; idx += kBlock) {
            const int q = idx / nR, s2 = idx - q * nR;
            const int jaq = Rj[q], jas = Rj[s2];
            const int jq = jaq / 3, js = jas / 3, as = jas - 3 * js;
            const CT* vq = Rv + 16 * q;
            const CT* us = Rv + 16 * s2 + 3;
            CT v = ihh * Ginv[(size_t)S.pos[jq] * nb + S.pos[js]] * (vq[0] * us[0] + vq[1] * us[1] + vq[2] * us[2]);
            if (jq == js) v += vq[8 + as];
            Cm[idx] = v;
          }
        }
        __syncthreads();
        mark(4);
        if (big) wg_lu_factor(Cm, nR, piv, perm, sh_blk, gpan, 0, sh_red, sh_i, &sh_piv);
        else wg_lu_factor(Cm, nR, piv, perm, sh_blk, S.pan, B.rlds * (kBK + 2), sh_red, sh_i, &sh_piv);
        if (tid == 0) { lust[0] = 1; lust[1] = nR; lust[2] = lust[3]; ++nfact; sum_nr += nR; max_nr = max(max_nr, nR); }
      } else if (tid == 0) {
        ++nreuse;
      }
    }

    // Woodbury solve on the base rows with the stored factorisation:
    // dout_B = W_B^-1 rin - W_B^-1 U C^-1 (K_R rin - rin_R + E_R W_B^-1 rin)
    auto wsolve = [&](const CT* rin, CT* dout) {
      for (int p = tid; p < nb; p += kBlock) {
        const int j = S.bas[p];
        const CT* F = Fr + 9 * j;
        const CT r0 = rin[3 * j], r1 = rin[3 * j + 1], r2 = rin[3 * j + 2];
        for (int k = 0; k < 3; ++k) S.fw[3 * p + k] = F[k] * r0 + F[3 + k] * r1 + F[6 + k] * r2;
      }
      __syncthreads();
      for (int p = tid; p < nb; p += kBlock) {
        CT w0 = 0, w1 = 0, w2 = 0;
        batched_terms<16>(0, nb, [&](int q) { return Ginv[(size_t)q * nb + p]; }, [&](int q, CT g) {
          w0 += g * S.fw[3 * q]; w1 += g * S.fw[3 * q + 1]; w2 += g * S.fw[3 * q + 2];
        });
        const int j = S.bas[p];
        const CT* F = Fr + 9 * j;
        for (int a = 0; a < 3; ++a) S.x0[3 * j + a] = ihh * (F[3 * a] * w0 + F[3 * a + 1] * w1 + F[3 * a + 2] * w2);
      }
      __syncthreads();
      if (nR > 0) {
        for (int q = tid; q < nR; q += kBlock) {
          const int ja = Rj[q], j = ja / 3, a = ja - 3 * (ja / 3);
          CT* rv = Rv + 16 * q;
          CT rr = -rin[3 * j + a];
          for (int b = 0; b < 3; ++b) rr += rv[8 + b] * rin[3 * j + b] + rv[11 + b] * S.x0[3 * j + b];
          rv[6] = rr;
        }
        if (big) wg_lu_apply(Cm, nR, perm, Rv, gys, static_cast<CT*>(nullptr));
        else {
          // the LDS panel (rlds (kBK + 1) values) is free during the solve; it holds the staged
          // diagonal blocks unless the system is too small for a whole block to fit
          const bool fits = ((nR + kBK - 1) / kBK) * kBK * kBK <= B.rlds * (kBK + 1);
          wg_lu_apply(Cm, nR, perm, Rv, S.ys, fits ? S.pan : static_cast<CT*>(nullptr));
        }
        if (!big) {
          // the rows' solution y_s, vectors u_s and base positions staged in the (now free)
          // LDS panel and solve vector, so that only the Ginv gathers go to memory
          CT* st = S.pan;
          int* spos = reinterpret_cast<int*>(S.ys);
          for (int q = tid; q < nR; q += kBlock) {
            const CT* rv = Rv + 16 * q;
            st[4 * q] = rv[7]; st[4 * q + 1] = rv[3]; st[4 * q + 2] = rv[4]; st[4 * q + 3] = rv[5];
            spos[q] = S.pos[Rj[q] / 3];
          }
          __syncthreads();
          for (int p = tid; p < nb; p += kBlock) {
            CT w0 = 0, w1 = 0, w2 = 0;
            batched_terms<16>(0, nR, [&](int s2) { return Ginv[(size_t)spos[s2] * nb + p]; }, [&](int s2, CT gi) {
              const CT g = gi * st[4 * s2];
              w0 += g * st[4 * s2 + 1]; w1 += g * st[4 * s2 + 2]; w2 += g * st[4 * s2 + 3];
            });
            const int j = S.bas[p];
            const CT* F = Fr + 9 * j;
            for (int a = 0; a < 3; ++a)
              dout[3 * j + a] = S.x0[3 * j + a] - ihh * (F[3 * a] * w0 + F[3 * a + 1] * w1 + F[3 * a + 2] * w2);
          }
        } else {
          for (int p = tid; p < nb; p += kBlock) {
            CT w0 = 0, w1 = 0, w2 = 0;
            for (int s2 = 0; s2 < nR; ++s2) {
              const int js = Rj[s2] / 3;
              const CT g = Ginv[(size_t)S.pos[js] * nb + p] * Rv[16 * s2 + 7];
              const CT* us = Rv + 16 * s2 + 3;
              w0 += g * us[0]; w1 += g * us[1]; w2 += g * us[2];
            }
            const int j = S.bas[p];
            const CT* F = Fr + 9 * j;
            for (int a = 0; a < 3; ++a)
              dout[3 * j + a] = S.x0[3 * j + a] - ihh * (F[3 * a] * w0 + F[3 * a + 1] * w1 + F[3 * a + 2] * w2);
          }
        }
      } else {
        for (int p = tid; p < nb; p += kBlock) {
          const int j = S.bas[p];
          for (int a = 0; a < 3; ++a) dout[3 * j + a] = S.x0[3 * j + a];
        }
      }
      __syncthreads();
    };
    wsolve(S.rv, S.dl);
    mark(5);
    // one step of iterative refinement against the current Jacobian (exact W products):
    // res_B = -Phi_B - K (W dl) - E dl_B ; dl_B += Z^-1 res_B.  It is needed even right after a
    // factorisation: on stiff sheets the Woodbury direction alone loses too many digits (an FP64
    // cloth drop missed the oracle by 1e-3 m without it)
    apply_W(S.dl, S.Wd);
    double rloc_b = 0.0, ploc_b = 0.0;
    for (int j = tid; j < c; j += kBlock) {
      if (S.pos[j] < 0) continue;
      CT K[3][3], E[3][3];
      contact_KE(S.cls[j], S.sp[j], mu, S.kap[j], S.yh0[j], S.yh1[j], K, E);
      const CT w0 = S.Wd[3 * j], w1 = S.Wd[3 * j + 1], w2 = S.Wd[3 * j + 2];
      const CT d0 = S.dl[3 * j], d1 = S.dl[3 * j + 1], d2 = S.dl[3 * j + 2];
      for (int a = 0; a < 3; ++a) {
        S.rv[3 * j + a] = -S.ph[3 * j + a] - (K[a][0] * w0 + K[a][1] * w1 + K[a][2] * w2) -
                          (E[a][0] * d0 + E[a][1] * d1 + E[a][2] * d2);
        rloc_b = fmax(rloc_b, fabs((double)S.rv[3 * j + a]));
        ploc_b = fmax(ploc_b, fabs((double)S.ph[3 * j + a]));
      }
    }
    // the refinement runs where the direction solves its linear system to fewer than 6 digits
    // (relative to Phi on the base rows, max norms); otherwise W dl is already the line search's
    const double rres = block_max(rloc_b, sh_red);
    const double rphi = block_max(ploc_b, sh_red);
    if (!(rres <= 1e-6 * rphi)) {
      wsolve(S.rv, S.tmp);
      for (int p = tid; p < nb; p += kBlock) {
        const int j = S.bas[p];
        for (int a = 0; a < 3; ++a) S.dl[3 * j + a] += S.tmp[3 * j + a];
      }
      __syncthreads();
      apply_W(S.dl, S.Wd);
    }

    mark(6);
    // ---- backtracking line search on 1/2 |Phi|^2 (inner scale) ----
    CT alpha = 1;
    bool ok = false;
    double psit = psi;
    for (int ls = 0; ls < 30; ++ls) {
      double pl = 0.0;
      for (int j = tid; j < c; j += kBlock) {
        const CT sp = S.sp[j];
        const CT l0 = (CT)fmin(fmax(S.lam[3 * j] + (double)(alpha * S.dl[3 * j]), -dmaxf), dmaxf);
        const CT l1 = (CT)fmin(fmax(S.lam[3 * j + 1] + (double)(alpha * S.dl[3 * j + 1]), -dmaxf), dmaxf);
        const CT l2 = (CT)fmin(fmax(S.lam[3 * j + 2] + (double)(alpha * S.dl[3 * j + 2]), -dmaxf), dmaxf);
        const CT cn = B.cd0[cb + j] + S.Y[3 * j] + alpha * S.Wd[3 * j];
        const CT ut1 = S.Y[3 * j + 1] + alpha * S.Wd[3 * j + 1] - B.cdob[2 * (cb + j)];
        const CT ut2 = S.Y[3 * j + 2] + alpha * S.Wd[3 * j + 2] - B.cdob[2 * (cb + j) + 1];
        const bool att = B.cobs[cb + j] >= kMaxObs;
        const CT phn = att ? cn : fmin(cn, sp * l0);
        const CT y1 = l1 - ut1 / sp, y2 = l2 - ut2 / sp;
        const CT rho = mu * fmax(l0, CT(0));
        const CT ny = sqrt(y1 * y1 + y2 * y2);
        CT p1 = 0, p2 = 0;
        if (att) { p1 = y1; p2 = y2; }
        else if (rho > CT(0)) {
          if (ny <= rho) { p1 = y1; p2 = y2; }
          else { p1 = rho * y1 / ny; p2 = rho * y2 / ny; }
        }
        const CT ph1 = sp * (l1 - p1), ph2 = sp * (l2 - p2);
        pl += (double)phn * phn + (double)ph1 * ph1 + (double)ph2 * ph2;
      }
      psit = 0.5 * block_sum(pl, sh_red);
      if (psit <= (1.0 - 2e-4 * (double)alpha) * psi) { ok = true; break; }
      alpha *= CT(0.5);
    }
    if (!ok) alpha = alpha * CT(2);   // smallest tried step: keep moving
    if (tid == 0) {
      if (!ok) ++nlsfail;
      // a chord step on frozen capacitance rows must at least halve |Phi|; otherwise refactor next
      if (reused && (!ok || alpha < CT(1))) lust[0] = 0;
    }
    for (int j = tid; j < c; j += kBlock)
      for (int a = 0; a < 3; ++a) {
        S.lam[3 * j + a] = fmin(fmax(S.lam[3 * j + a] + (double)(alpha * S.dl[3 * j + a]), -dmaxf), dmaxf);
        S.Y[3 * j + a] += alpha * S.Wd[3 * j + a];
      }
    __syncthreads();
    mark(7);
    if ((it & 7) == 7) {   // refresh Y from lambda to stop drift
      apply_W(S.lam, S.Y);
      for (int j = tid; j < c; j += kBlock)
        for (int a = 0; a < 3; ++a) S.Y[3 * j + a] += yfg[3 * j + a];
      __syncthreads();
    }
    ls_run = ok ? 0 : ls_run + 1;
    if (ls_run >= kStallRun && !zero_restarted) {
      zero_restarted = true;
      ls_run = 0;
      for (int j = tid; j < c; j += kBlock) {
        const CT cn = B.cd0[cb + j] + yfg[3 * j];
        const bool att = B.cobs[cb + j] >= kMaxObs;
        S.lam[3 * j] = (cn < CT(0) && !att) ? (double)(-cn / S.sp[j]) : 0.0;
        S.lam[3 * j + 1] = 0;
        S.lam[3 * j + 2] = 0;
      }
      __syncthreads();
      apply_W(S.lam, S.Y);
      for (int j = tid; j < c; j += kBlock)
        for (int a = 0; a < 3; ++a) S.Y[3 * j + a] += yfg[3 * j + a];
      if (tid == 0) lust[0] = 0;
      __syncthreads();
      it0 = it + 1;
    }
  }
  mark(7);
  if (learned && !learned_failed && r > B.tol) {
    // the solve from the prediction did not converge: start again from the previous iterate
    learned_failed = true;
    load_prev(true);
    if (tid == 0) lust[0] = 0;
    __syncthreads();
    it0 = it;
    goto restart;
  }
  // ---- write back ----
  for (int j = tid; j < c; j += kBlock) {
    const CT* F = Fr + 9 * j;
    const CT l0 = (CT)S.lam[3 * j], l1 = (CT)S.lam[3 * j + 1], l2 = (CT)S.lam[3 * j + 2];
    for (int a = 0; a < 3; ++a) B.clam[3 * (cb + j) + a] = S.lam[3 * j + a];
    for (int k = 0; k < 3; ++k) B.cforce[3 * (cb + j) + k] = (T)(F[k] * l0 + F[3 + k] * l1 + F[6 + k] * l2);
  }
  for (int p = tid; p < nb; p += kBlock) B.base[cb + p] = S.bas[p];
  if (tid == 0) {
    B.nbase[e] = nb;
    B.iters[e] += it;
    B.refac[e] += nref;
    if (B.phase) {
      unsigned long long* cnt = B.phase + (size_t)B.n_envs * 8 + 8 * e;
      cnt[0] += nfact;
      cnt[1] += nreuse;
      cnt[2] += nlsfail;
      cnt[3] += (r > B.tol) ? 1 : 0;
      cnt[4] += sum_nr;
      cnt[5] = max((unsigned long long)max_nr, cnt[5]);
      cnt[6] += it;
      cnt[7] += 1;
    }
    if (r > B.tol) B.flags[e] |= 2; else B.flags[e] &= ~2;
    if (own_cost && B.cost) B.cost[e] += wall_clock64() - t_start;
    if (first_lg && B.ws_state) {
      int w = B.ws_state[e] & ~5;
      if (learned && !learned_failed) w |= 1;
      if (learned_failed) w |= 4;
      if (learned_failed && (w & 0xff00) < (kWsMaxFail << 8)) w += 1 << 8;
      if ((w & 0xff00) >= (kWsMaxFail << 8)) w |= 2;   // previous-iterate start only from now on
      B.ws_state[e] = w;
    }
  }
}

template <class T, class CT, bool LITE>
__global__ void __launch_bounds__(kBlock) k_csp(DevBatch<T> B, const T* mu_env, int first_lg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // workgroups take envs in the order of the last step's solve times, longest first
  const int e = B.order ? B.order[blockIdx.x] : blockIdx.x;
  csp_env<T, CT, LITE>(B, mu_env, first_lg, e, smem_raw, true);
}

// ---------------------------------------------------------------------------
// The whole local-global loop of a step (Alg. 1: K x (project, assemble, global
// apply, contact solve, position update)) with one workgroup per env.  Each phase
// runs the same device code, on the same data, as its batched kernel, so results
// are bitwise those of the kernel-per-phase step; what changes is that an env
// never waits for the slowest env of the batch between phases.  Envs never couple,
// and every phase of env e reads only what earlier phases of env e wrote (made
// visible within the workgroup by its barriers).  Workgroups take envs longest
// first by the previous step's whole-loop times.
template <class T, int VW>
constexpr size_t fused_gemv_lds() {
  return 3 * kChunk * sizeof(T) + kChunk * sizeof(int) + (size_t)(kBlock / 64 - 1) * 3 * 64 * VW * sizeof(T);
}

template <class T, class CT, int VW, int UNROLL, bool LITE>
__global__ void __launch_bounds__(kBlock) k_lg_fused(DevBatch<T> B, const T* mu_env) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int TILE = 64 * VW;
  const int e = B.order ? B.order[blockIdx.x] : blockIdx.x;
  const unsigned long long t_start = (B.cost && threadIdx.x == 0) ? wall_clock64() : 0ull;
  const int v0 = B.voff[e], v1 = B.voff[e + 1], t0 = B.toff[e], t1 = B.toff[e + 1];
  T* s_vec = reinterpret_cast<T*>(smem_raw);
  int* s_row = reinterpret_cast<int*>(s_vec + 3 * kChunk);
  T* s_red = reinterpret_cast<T*>(s_row + kChunk);
  for (int k = 0; k < B.lg_iterations; ++k) {
    {
      // the next element's indices are loaded while the current element computes
      int t = t0 + (int)threadIdx.x;
      int idn[4];
      if (t < t1) elem_ids(B, t, idn);
      for (; t < t1; t += kBlock) {
        ElemIn<T> cur;
        elem_load(B, t, idn, cur);
        if (t + kBlock < t1) elem_ids(B, t + kBlock, idn);
        elem_compute(B, t, cur);
      }
    }
    __syncthreads();
    for (int vb = v0; vb < v1; vb += kBlock) assemble_vertices(B, vb, min(vb + kBlock, v1), s_vec);
    __syncthreads();
    for (int c0 = 0; c0 < v1 - v0; c0 += TILE) gemv_tile<T, false, VW, UNROLL>(B, e, c0, s_vec, s_row, s_red);
    __syncthreads();
    csp_env<T, CT, LITE>(B, mu_env, k == 0 ? 1 : 0, e, smem_raw, false);
    __syncthreads();
    for (int c0 = 0; c0 < v1 - v0; c0 += TILE) gemv_tile<T, true, VW, UNROLL>(B, e, c0, s_vec, s_row, s_red);
    __syncthreads();
  }
  if (B.cost && threadIdx.x == 0) B.cost[e] += wall_clock64() - t_start;
}

// columns per lane of the fused loop's products (32 bytes per lane) and rows in flight per
// wave (16 measured no faster than 8)
template <class T>
constexpr int fused_vw() { return (int)(32 / sizeof(T)); }
constexpr int kFusedUnroll = 8;

template <class T, class CT>
size_t fused_smem_bytes(const DevBatch<T>& B) {
  size_t a = csp_smem_bytes<CT>(B.cap, B.rlds);
  a = std::max(a, fused_gemv_lds<T, fused_vw<T>()>());
  a = std::max(a, (size_t)3 * kAsmChunk * sizeof(T));
  return a;
}

template <class T>
void launch_lg_fused(const DevBatch<T>& B, const T* mu_env, hipStream_t s) {
  constexpr int VW = fused_vw<T>();
  const dim3 g(B.n_envs), blk(kBlock);
  if (B.csp64) {
    const size_t sm = fused_smem_bytes<T, double>(B);
    if (B.lite) hipLaunchKernelGGL((k_lg_fused<T, double, VW, kFusedUnroll, true>), g, blk, sm, s, B, mu_env);
    else hipLaunchKernelGGL((k_lg_fused<T, double, VW, kFusedUnroll, false>), g, blk, sm, s, B, mu_env);
  } else {
    const size_t sm = fused_smem_bytes<T, T>(B);
    if (B.lite) hipLaunchKernelGGL((k_lg_fused<T, T, VW, kFusedUnroll, true>), g, blk, sm, s, B, mu_env);
    else hipLaunchKernelGGL((k_lg_fused<T, T, VW, kFusedUnroll, false>), g, blk, sm, s, B, mu_env);
  }
}

// ---------------------------------------------------------------------------
template <class T>
void launch_gather(const DevBatch<T>& B, hipStream_t s) {
  if (B.csp64) hipLaunchKernelGGL((k_gather<T, double>), dim3(B.n_envs), dim3(kBlock), 0, s, B);
  else hipLaunchKernelGGL((k_gather<T, T>), dim3(B.n_envs), dim3(kBlock), 0, s, B);
}
template <class T>
void launch_project(const DevBatch<T>& B, hipStream_t s) {
  hipLaunchKernelGGL(k_project<T>, dim3((B.NT + kBlock - 1) / kBlock), dim3(kBlock), 0, s, B);
}
template <class T>
void launch_assemble(const DevBatch<T>& B, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble<T>, dim3((B.NV + kBlock - 1) / kBlock), dim3(kBlock), 0, s, B);
}
// columns per lane of schedule variant vw (0, 1, 2): 8, 16, 32 bytes per lane
template <class T>
constexpr int gemv_vw(int vw) { return (int)((8 << vw) / sizeof(T)); }

template <class T, bool ROWS>
static void launch_gemv(const DevBatch<T>& B, const GemvSchedule& S, hipStream_t s, const int* skip) {
  const dim3 grid((unsigned)S.n_items), blk(kBlock);
  const int2* it = S.items;
  const int key = S.vw * 2 + (S.unroll == 8 ? 1 : 0);
  switch (key) {
    case 0: hipLaunchKernelGGL((k_gemv<T, ROWS, gemv_vw<T>(0), 4>), grid, blk, 0, s, B, it, skip); break;
    case 1: hipLaunchKernelGGL((k_gemv<T, ROWS, gemv_vw<T>(0), 8>), grid, blk, 0, s, B, it, skip); break;
    case 2: hipLaunchKernelGGL((k_gemv<T, ROWS, gemv_vw<T>(1), 4>), grid, blk, 0, s, B, it, skip); break;
    case 3: hipLaunchKernelGGL((k_gemv<T, ROWS, gemv_vw<T>(1), 8>), grid, blk, 0, s, B, it, skip); break;
    case 4: hipLaunchKernelGGL((k_gemv<T, ROWS, gemv_vw<T>(2), 4>), grid, blk, 0, s, B, it, skip); break;
    default: hipLaunchKernelGGL((k_gemv<T, ROWS, gemv_vw<T>(2), 8>), grid, blk, 0, s, B, it, skip); break;
  }
}

template <class T>
void launch_apply(const DevBatch<T>& B, const GemvSchedule& S, hipStream_t s) {
  launch_gemv<T, false>(B, S, s, nullptr);
}
template <class T>
void launch_correct(const DevBatch<T>& B, const GemvSchedule& S, hipStream_t s, const int* skip) {
  launch_gemv<T, true>(B, S, s, skip);
}
// Longest-processing-time order of the contact-solve workgroups: envs sorted by the
// solve time they took in the previous step (descending; ties by env index), by a
// bitonic sort in one workgroup; the accumulated times are then cleared.  Scheduling
// only: the order never changes what a workgroup computes.
constexpr int kOrderMax = 4096;
__global__ void __launch_bounds__(1024) k_order(int n_envs, unsigned long long* cost, int* order) {
  __shared__ unsigned long long key[kOrderMax];
  __shared__ int val[kOrderMax];
  int N = 1;
  while (N < n_envs) N <<= 1;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    // larger cost first; the env index breaks ties (smaller first) through the low bits
    key[i] = i < n_envs ? ((min(cost[i], 0xFFFFFFFFull) << 32) | (unsigned)(0x7FFFFFFF - i)) : 0ull;
    val[i] = i;
  }
  __syncthreads();
  for (int k = 2; k <= N; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool desc = (i & k) == 0;
          const unsigned long long a = key[i], b = key[l];
          if (desc ? (a < b) : (a > b)) {
            key[i] = b; key[l] = a;
            const int t = val[i]; val[i] = val[l]; val[l] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n_envs; i += blockDim.x) {
    order[i] = val[i];
    cost[i] = 0ull;
  }
}

template <class T>
void launch_order(const DevBatch<T>& B, hipStream_t s) {
  if (!B.order || !B.cost || B.n_envs > kOrderMax) return;
  hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, s, B.n_envs, B.cost, B.order);
}

template <class T>
void launch_csp(const DevBatch<T>& B, const T* mu_env, int first_lg, hipStream_t s) {
  const dim3 g(B.n_envs), blk(kBlock);
  if (B.csp64) {
    size_t sm = csp_smem_bytes<double>(B.cap, B.rlds);
    if (B.lite) hipLaunchKernelGGL((k_csp<T, double, true>), g, blk, sm, s, B, mu_env, first_lg);
    else hipLaunchKernelGGL((k_csp<T, double, false>), g, blk, sm, s, B, mu_env, first_lg);
  } else {
    size_t sm = csp_smem_bytes<T>(B.cap, B.rlds);
    if (B.lite) hipLaunchKernelGGL((k_csp<T, T, true>), g, blk, sm, s, B, mu_env, first_lg);
    else hipLaunchKernelGGL((k_csp<T, T, false>), g, blk, sm, s, B, mu_env, first_lg);
  }
}

template <class T>
hipError_t prepare_csp(size_t* static_lds) {
  constexpr int VW = fused_vw<T>();
  const void* kernels[8] = {(const void*)k_csp<T, double, false>, (const void*)k_csp<T, T, false>,
                            (const void*)k_lg_fused<T, double, VW, kFusedUnroll, false>,
                            (const void*)k_lg_fused<T, T, VW, kFusedUnroll, false>,
                            (const void*)k_csp<T, double, true>, (const void*)k_csp<T, T, true>,
                            (const void*)k_lg_fused<T, double, VW, kFusedUnroll, true>,
                            (const void*)k_lg_fused<T, T, VW, kFusedUnroll, true>};
  size_t most = 0;
  for (const void* k : kernels) {
    hipFuncAttributes fa;
    hipError_t err = hipFuncGetAttributes(&fa, k);
    if (err != hipSuccess) return err;
    most = std::max(most, (size_t)fa.sharedSizeBytes);
    err = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsBytes - kCspStaticLds));
    if (err != hipSuccess) return err;
  }
  if (static_lds) *static_lds = most;
  return hipSuccess;
}

#define INST(T)                                                          \
  template hipError_t prepare_csp<T>(size_t*);                           \
  template void launch_gather<T>(const DevBatch<T>&, hipStream_t);       \
  template void launch_hinge<T>(const DevBatch<T>&, hipStream_t);        \
  template void launch_order<T>(const DevBatch<T>&, hipStream_t);        \
  template void launch_project<T>(const DevBatch<T>&, hipStream_t);      \
  template void launch_assemble<T>(const DevBatch<T>&, hipStream_t);     \
  template void launch_apply<T>(const DevBatch<T>&, const GemvSchedule&, hipStream_t);   \
  template void launch_correct<T>(const DevBatch<T>&, const GemvSchedule&, hipStream_t, const int*); \
  template void launch_csp<T>(const DevBatch<T>&, const T*, int, hipStream_t);      \
  template void launch_lg_fused<T>(const DevBatch<T>&, const T*, hipStream_t);
INST(float)
INST(double)

}  // namespace flash
