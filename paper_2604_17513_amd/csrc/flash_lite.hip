// Lightweight contact update in global memory (Alg. 1 with the inertia-only metric of Eq. 10)
// for contact counts beyond what one CU's LDS holds.
//
// Each update reads the current displacement u = z + h^2 Gbar H^T lambda (the position update
// of Alg. 1, formed by the explicit-inverse product over the contact rows), evaluates Phi and its
// generalized-Jacobian blocks at Y = F^T u per contact, and takes lambda <- lambda + delta with
// (K W~ + E) delta = -Phi per vertex, W~ = h^2 H M^-1 H^T.  The metric couples only the contacts
// of one vertex, so every vertex group is updated by one thread from global memory; the env's
// residual is reduced over chunks of contacts first (one launch), then the update decides and
// updates (a second launch), both spread over (chunks, envs).  The contact displacement follows lambda through
// the global apply instead of the contact-space Delassus operator, so no cap x cap matrix exists.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "flash_contact.h"
#include "flash_device.h"
#include "flash_launch.h"

namespace flash {

namespace {

__device__ __forceinline__ double wg_max(double v, double* sh) {
  for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = sh[0];
  for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, sh[w]);
  __syncthreads();
  return m;
}

// Residual of contact j at (u, lambda), FP64, at the residual scale s = h^2 / m_v.
template <class T, class CT>
__device__ __forceinline__ double lite_residual(const DevBatch<T>& B, size_t cb, int j, const CT* Fr, int v0, CT mu) {
  const int NV = B.NV;
  const CT* F = Fr + 9 * j;
  const int vi = v0 + B.cvert[cb + j];
  const double uw0 = (double)B.u[vi], uw1 = (double)B.u[NV + vi], uw2 = (double)B.u[2 * NV + vi];
  double Y[3];
  for (int a = 0; a < 3; ++a) Y[a] = (double)F[3 * a] * uw0 + (double)F[3 * a + 1] * uw1 + (double)F[3 * a + 2] * uw2;
  const double s = (double)B.cs[cb + j];
  const double* lj = B.clam + 3 * (cb + j);
  const double cnd = B.cd0d[cb + j] + Y[0];
  const double ut1 = Y[1] - (double)B.cdob[2 * (cb + j)], ut2 = Y[2] - (double)B.cdob[2 * (cb + j) + 1];
  const bool att = B.cobs[cb + j] >= kMaxObs;
  const double pn = att ? cnd : fmin(cnd, s * lj[0]);
  const double z1 = lj[1] - ut1 / s, z2 = lj[2] - ut2 / s;
  const double nz = sqrt(z1 * z1 + z2 * z2);
  const double rh = (double)mu * fmax(lj[0], 0.0);
  double q1 = z1, q2 = z2;
  if (!att && nz > rh) { const double f = nz > 0 ? rh / nz : 0.0; q1 = f * z1; q2 = f * z2; }
  const double t1 = s * (lj[1] - q1), t2 = s * (lj[2] - q2);
  const double rj = fmax(fabs(pn), sqrt(t1 * t1 + t2 * t2));
  return rj == rj ? rj : INFINITY;
}

template <class T, class CT>
__device__ __forceinline__ const CT* lite_frames(const DevBatch<T>& B, size_t cb) {
  if constexpr (std::is_same<CT, T>::value) return B.cframe + 9 * cb;
  else return B.cframe64 + 9 * cb;
}

// Once per step, after detection: world forces F lambda of the warm start (the first position
// update reads them); the env's residual slots cleared; its iteration not stopped.  Grid: (chunks of
// kBlock contacts, envs).
template <class T, class CT>
__global__ void __launch_bounds__(kBlock) k_lite_prepare(DevBatch<T> B) {
  const int e = blockIdx.y;
  const int c = B.ccount[e];
  const size_t cb = (size_t)e * B.cap;
  const CT* Fr = lite_frames<T, CT>(B, cb);
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j < c) {
    const CT* F = Fr + 9 * j;
    const double* lj = B.clam + 3 * (cb + j);
    const CT l0 = (CT)lj[0], l1 = (CT)lj[1], l2 = (CT)lj[2];
    for (int k = 0; k < 3; ++k) B.cforce[3 * (cb + j) + k] = (T)(F[k] * l0 + F[3 + k] * l1 + F[6 + k] * l2);
  }
  if (blockIdx.x == 0) {
    const int ns = B.lg_iterations * (B.max_newton + 1);
    for (int q = threadIdx.x; q < ns; q += kBlock) B.lite_r[(size_t)e * ns + q] = 0ull;
    if (threadIdx.x == 0) B.lite_done[e] = 0;
  }
}

// The env's residual at (u, lambda): each workgroup reduces one chunk of kBlock contacts and folds
// its maximum into the env's slot for this update (non-negative doubles order like their bits, so an
// integer atomic maximum gives the exact maximum whatever the order).
template <class T, class CT>
__global__ void __launch_bounds__(kBlock) k_lite_residual(DevBatch<T> B, const T* mu_env, int slot, int it) {
  __shared__ double sh_red[kBlock / 64];
  const int e = blockIdx.y;
  if (it > 0 && B.lite_done[e]) return;
  const int c = B.ccount[e];
  const int j0 = blockIdx.x * kBlock;
  if (j0 >= c) return;
  const size_t cb = (size_t)e * B.cap;
  const CT* Fr = lite_frames<T, CT>(B, cb);
  const int v0 = B.voff[e];
  const CT mu = (CT)mu_env[e];
  const int j = j0 + threadIdx.x;
  const double rloc = j < c ? lite_residual<T, CT>(B, cb, j, Fr, v0, mu) : 0.0;
  const double r = wg_max(rloc, sh_red);
  if (threadIdx.x == 0) {
    const int ns = B.lg_iterations * (B.max_newton + 1);
    atomicMax(&B.lite_r[(size_t)e * ns + slot], (unsigned long long)__double_as_longlong(r));
  }
}

// Decision and update: the env's iteration stops (done flag, counters, not-converged flag) when its
// residual is at inner_tol or `it` reached the budget; otherwise every vertex group whose first
// contact lies in this workgroup's chunk takes one update.
template <class T, class CT>
__global__ void __launch_bounds__(kBlock) k_lite_apply(DevBatch<T> B, const T* mu_env, int slot, int it, int first_lg) {
  const int e = blockIdx.y;
  if (it > 0 && B.lite_done[e]) return;
  const int c = B.ccount[e];
  const int ns = B.lg_iterations * (B.max_newton + 1);
  const double r = __longlong_as_double((long long)B.lite_r[(size_t)e * ns + slot]);
  const int tid = threadIdx.x;
  if (r <= B.tol || it >= B.max_newton) {
    if (blockIdx.x == 0 && tid == 0) {
      B.lite_done[e] = 1;
      B.iters[e] += it;
      if (B.phase) {
        unsigned long long* cnt = B.phase + (size_t)B.n_envs * 8 + 8 * e;
        cnt[3] += (r > B.tol) ? 1 : 0;
        cnt[6] += it;
        cnt[7] += 1;
      }
      if (c > 0 && r > B.tol) B.flags[e] |= 2; else B.flags[e] &= ~2;
      if (first_lg && B.ws_state) B.ws_state[e] &= ~5;
    }
    return;
  }
  if (it == 0 && blockIdx.x == 0 && tid == 0) B.lite_done[e] = 0;
  const int j = blockIdx.x * kBlock + tid;
  if (j >= c) return;
  const size_t cb = (size_t)e * B.cap;
  const int* cv = B.cvert + cb;
  if (j > 0 && cv[j - 1] == cv[j]) return;   // not the first contact of its vertex
  const CT* Fr = lite_frames<T, CT>(B, cb);
  const int* cobs = B.cobs + cb;
  const int v0 = B.voff[e];
  const int NV = B.NV;
  const CT mu = (CT)mu_env[e];
  const double dmaxf = B.max_force;
  int m = 1;
  while (j + m < c && cv[j + m] == cv[j] && m < kCacheSlots) ++m;
  const int vi = v0 + cv[j];
  const CT uw0 = (CT)B.u[vi], uw1 = (CT)B.u[NV + vi], uw2 = (CT)B.u[2 * NV + vi];
  CT Y[3 * kCacheSlots], d0[kCacheSlots], dob[2 * kCacheSlots], dl[3 * kCacheSlots];
  double lam[3 * kCacheSlots];
  for (int q = 0; q < m; ++q) {
    const CT* F = Fr + 9 * (j + q);
    for (int a = 0; a < 3; ++a) {
      Y[3 * q + a] = F[3 * a] * uw0 + F[3 * a + 1] * uw1 + F[3 * a + 2] * uw2;
      lam[3 * q + a] = B.clam[3 * (cb + j + q) + a];
    }
    d0[q] = (CT)B.cd0[cb + j + q];
    dob[2 * q] = (CT)B.cdob[2 * (cb + j + q)];
    dob[2 * q + 1] = (CT)B.cdob[2 * (cb + j + q) + 1];
  }
  const CT sp = (CT)B.cs[cb + j];
  if (m == 1) {
    CT ph[3], K[3][3], E[3][3];
    lite_contact(sp, mu, d0[0], dob[0], dob[1], Y, lam, cobs[j] >= kMaxObs, ph, K, E);
    // Z = sp K + E = [sp 0 0; E_tn sp I]
    const CT dn = -ph[0] / sp;
    dl[0] = dn;
    dl[1] = (-ph[1] - E[1][0] * dn) / sp;
    dl[2] = (-ph[2] - E[2][0] * dn) / sp;
  } else {
    lite_group_solve<CT>(m, sp, mu, Fr + 9 * j, d0, dob, Y, lam, cobs + j, dl);
  }
  for (int q = 0; q < m; ++q) {
    const CT* F = Fr + 9 * (j + q);
    double ln[3];
    for (int a = 0; a < 3; ++a) {
      ln[a] = fmin(fmax(lam[3 * q + a] + (double)dl[3 * q + a], -dmaxf), dmaxf);
      B.clam[3 * (cb + j + q) + a] = ln[a];
    }
    const CT l0 = (CT)ln[0], l1 = (CT)ln[1], l2 = (CT)ln[2];
    for (int k = 0; k < 3; ++k) B.cforce[3 * (cb + j + q) + k] = (T)(F[k] * l0 + F[3 + k] * l1 + F[6 + k] * l2);
  }
}

// Partial sums of one row split of env e's explicit-inverse product for one column tile.
// ROWS = false: rows 0..n-1 with the right-hand side b (z = Gbar b); ROWS = true: the contact
// rows with their world forces (u = z + h^2 Gbar H^T lambda).  Gbar is symmetric, so rows are
// read along their length (16-byte vectors, non-temporal: each row is read once per product).
template <class T, bool ROWS>
__global__ void __launch_bounds__(kBlock) k_gemv_split(DevBatch<T> B, const int4* items, const int* skip,
                                                       T* partial, const int64_t* poff) {
  constexpr int VW = (int)(16 / sizeof(T));
  constexpr int TILE = 64 * VW;
  constexpr int UNROLL = 4;
  constexpr int WS = kBlock / 64;
  typedef T vec_t __attribute__((ext_vector_type(VW)));
  __shared__ T s_vec[3 * kSplitRows];
  __shared__ int s_row[kSplitRows];
  __shared__ T s_red[(WS - 1) * 3 * TILE];
  const int4 item = items[blockIdx.x];
  const int e = item.x, tile0 = item.y, split = item.z;
  if (e < 0 || (skip && skip[e])) return;   // padding item, or an env whose iteration stopped
  const int v0 = B.voff[e];
  const int n = B.voff[e + 1] - v0;
  const int ld = B.gld[e];
  const int nrows = ROWS ? B.ccount[e] : n;
  const int R = split_rows(split_cover(n, B.cap));
  const int r0 = split * R;
  if (r0 >= nrows) return;   // the merge reads only the splits that hold rows
  const int r1 = min(r0 + R, nrows);
  const T* G = B.G + B.goff[e];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col0 = tile0 + lane * VW;
  T acc[VW][3];
  for (int q = 0; q < VW; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0;
  // the split's rows in chunks of kSplitRows staged in LDS, summed in row order per wave
  for (int c0 = r0; c0 < r1; c0 += kSplitRows) {
  const int nr = min(kSplitRows, r1 - c0);
  __syncthreads();
  for (int r = threadIdx.x; r < nr; r += kBlock) {
    if (ROWS) {
      const size_t j = (size_t)e * B.cap + c0 + r;
      s_row[r] = B.cvert[j];
      s_vec[r] = B.cforce[3 * j];
      s_vec[kSplitRows + r] = B.cforce[3 * j + 1];
      s_vec[2 * kSplitRows + r] = B.cforce[3 * j + 2];
    } else {
      s_row[r] = c0 + r;
      s_vec[r] = B.b[v0 + c0 + r];
      s_vec[kSplitRows + r] = B.b[B.NV + v0 + c0 + r];
      s_vec[2 * kSplitRows + r] = B.b[2 * B.NV + v0 + c0 + r];
    }
  }
  __syncthreads();
  if (col0 < ld) {   // ld is a multiple of 32 columns: a lane's VW columns lie inside the row
    for (int rb = wid; rb < nr; rb += WS * UNROLL) {
      vec_t g[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int r = rb + WS * u;
        if (r < nr) g[u] = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(G + (size_t)s_row[r] * ld + col0));
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int r = rb + WS * u;
        if (r < nr) {
          const T b0 = s_vec[r], b1 = s_vec[kSplitRows + r], b2 = s_vec[2 * kSplitRows + r];
#pragma unroll
          for (int q = 0; q < VW; ++q) {
            acc[q][0] += g[u][q] * b0;
            acc[q][1] += g[u][q] * b1;
            acc[q][2] += g[u][q] * b2;
          }
        }
      }
    }
  }
  }
  // fixed-order reduction over the waves
  if (wid > 0)
    for (int q = 0; q < VW; ++q)
      for (int k = 0; k < 3; ++k) s_red[((wid - 1) * 3 + k) * TILE + lane * VW + q] = acc[q][k];
  __syncthreads();
  if (wid == 0) {
    T* P = partial + poff[e];
    for (int q = 0; q < VW; ++q) {
      const int col = col0 + q;
      if (col >= n) continue;
      for (int k = 0; k < 3; ++k) {
        T s = acc[q][k];
        for (int w = 0; w < WS - 1; ++w) s += s_red[(w * 3 + k) * TILE + lane * VW + q];
        P[((size_t)split * 3 + k) * n + col] = s;
      }
    }
  }
}

// Adds each env's row-split partials in split order: z = sum (ROWS = false) or u = z + h^2 sum.
template <class T, bool ROWS>
__global__ void __launch_bounds__(kBlock) k_gemv_merge(DevBatch<T> B, const int* skip, const T* partial,
                                                       const int64_t* poff) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= B.NV) return;
  const int e = B.vert_env[i];
  if (skip && skip[e]) return;
  const int v0 = B.voff[e];
  const int n = B.voff[e + 1] - v0, col = i - v0;
  const int nrows = ROWS ? B.ccount[e] : n;
  const int R = split_rows(split_cover(n, B.cap));
  const int ns = (nrows + R - 1) / R;
  const T* P = partial + poff[e];
  const T hh = (T)(B.h * B.h);
  for (int k = 0; k < 3; ++k) {
    T s = 0;
    for (int sp = 0; sp < ns; ++sp) s += P[((size_t)sp * 3 + k) * n + col];
    const size_t o = (size_t)k * B.NV + i;
    if (ROWS) B.u[o] = B.z[o] + hh * s;
    else B.z[o] = s;
  }
}

}  // namespace

template <class T>
void launch_split_apply(const DevBatch<T>& B, const SplitSchedule& S, hipStream_t s) {
  T* P = static_cast<T*>(S.partial);
  hipLaunchKernelGGL((k_gemv_split<T, false>), dim3((unsigned)S.n_items), dim3(kBlock), 0, s, B, S.items,
                     (const int*)nullptr, P, S.poff);
  hipLaunchKernelGGL((k_gemv_merge<T, false>), dim3((unsigned)((B.NV + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, B,
                     (const int*)nullptr, (const T*)P, S.poff);
}

template <class T>
void launch_split_correct(const DevBatch<T>& B, const SplitSchedule& S, const int* skip, hipStream_t s) {
  T* P = static_cast<T*>(S.partial);
  hipLaunchKernelGGL((k_gemv_split<T, true>), dim3((unsigned)S.n_items), dim3(kBlock), 0, s, B, S.items, skip, P,
                     S.poff);
  hipLaunchKernelGGL((k_gemv_merge<T, true>), dim3((unsigned)((B.NV + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, B,
                     skip, (const T*)P, S.poff);
}

template void launch_split_apply<float>(const DevBatch<float>&, const SplitSchedule&, hipStream_t);
template void launch_split_apply<double>(const DevBatch<double>&, const SplitSchedule&, hipStream_t);
template void launch_split_correct<float>(const DevBatch<float>&, const SplitSchedule&, const int*, hipStream_t);
template void launch_split_correct<double>(const DevBatch<double>&, const SplitSchedule&, const int*, hipStream_t);

template <class T>
void launch_lite_update(const DevBatch<T>& B, const T* mu_env, int k, int it, int first_lg, hipStream_t s) {
  const dim3 g((unsigned)((B.cap + kBlock - 1) / kBlock), (unsigned)B.n_envs), blk(kBlock);
  if (it < 0) {
    if (B.csp64) hipLaunchKernelGGL((k_lite_prepare<T, double>), g, blk, 0, s, B);
    else hipLaunchKernelGGL((k_lite_prepare<T, T>), g, blk, 0, s, B);
    return;
  }
  const int slot = k * (B.max_newton + 1) + it;
  if (B.csp64) {
    hipLaunchKernelGGL((k_lite_residual<T, double>), g, blk, 0, s, B, mu_env, slot, it);
    hipLaunchKernelGGL((k_lite_apply<T, double>), g, blk, 0, s, B, mu_env, slot, it, first_lg);
  } else {
    hipLaunchKernelGGL((k_lite_residual<T, T>), g, blk, 0, s, B, mu_env, slot, it);
    hipLaunchKernelGGL((k_lite_apply<T, T>), g, blk, 0, s, B, mu_env, slot, it, first_lg);
  }
}

template void launch_lite_update<float>(const DevBatch<float>&, const float*, int, int, int, hipStream_t);
template void launch_lite_update<double>(const DevBatch<double>&, const double*, int, int, int, hipStream_t);

}  // namespace flash
