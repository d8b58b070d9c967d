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
  typedef T f4_t __attribute__((ext_vector_type(4)));
  __shared__ f4_t s_vec[kSplitRows];   // (b0, b1, b2, 0) per staged row
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
    f4_t f;
    if (ROWS) {
      const size_t j = (size_t)e * B.cap + c0 + r;
      s_row[r] = B.cvert[j];
      f[0] = B.cforce[3 * j]; f[1] = B.cforce[3 * j + 1]; f[2] = B.cforce[3 * j + 2];
    } else {
      s_row[r] = c0 + r;
      f[0] = B.b[v0 + c0 + r]; f[1] = B.b[B.NV + v0 + c0 + r]; f[2] = B.b[2 * B.NV + v0 + c0 + r];
    }
    f[3] = 0;
    s_vec[r] = f;
  }
  __syncthreads();
  if (col0 < ld) {   // ld is a multiple of 32 columns: a lane's VW columns lie inside the row
    // Row indices are the same over the wave (scalar registers): the UNROLL loads go out
    // together, and the next UNROLL rows' loads before this iteration's FMAs (double buffer);
    // rows past the staged ones load the last staged row, unused.
    const int wsc = __builtin_amdgcn_readfirstlane(wid);
    auto load_rows = [&](int rb, vec_t* g) {
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int q = __builtin_amdgcn_readfirstlane(s_row[min(rb + WS * u, nr - 1)]);
        g[u] = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(G + (size_t)q * ld + col0));
      }
    };
    vec_t gn[UNROLL];
    if (wsc < nr) load_rows(wsc, gn);
    for (int rb = wsc; rb < nr; rb += WS * UNROLL) {
      vec_t g[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) g[u] = gn[u];
      if (rb + WS * UNROLL < nr) load_rows(rb + WS * UNROLL, gn);
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int r = rb + WS * u;
        if (r < nr) {
          const f4_t b = s_vec[r];
#pragma unroll
          for (int q = 0; q < VW; ++q) {
            acc[q][0] += g[u][q] * b[0];
            acc[q][1] += g[u][q] * b[1];
            acc[q][2] += g[u][q] * b[2];
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

// k_gemv_split for a chunk of up to kTwinChunk envs that share one inverse.  A lane's inverse row
// vector, loaded once, serves every env of the chunk that reads that row at that position of the
// split: all of them in the apply, and in the position update wherever their contact rows
// coincide (identical envs in identical states); where they differ, each env loads its own row.
// Rows are staged kTwinRows at a time, a multiple of the wave count, so every row stays on the wave
// k_gemv_split gives it; with its per-wave row order and its fixed-order reduction over the waves,
// every env gets the bits it gets from k_gemv_split.  Loads are ordinary (cached): the other chunks
// of a group read the same rows on the same XCD close in time.  166-180 VGPRs (3 waves per SIMD in
// FP32, 2 in FP64).
constexpr int kTwinRows = 128;
template <class T, bool ROWS>
__global__ void __launch_bounds__(kBlock) k_gemv_split_twins(DevBatch<T> B, const int4* items, const int* envs,
                                                             const int* skip, T* partial, const int64_t* poff) {
  constexpr int VW = (int)(16 / sizeof(T));
  constexpr int TILE = 64 * VW;
  constexpr int UNROLL = 4;
  constexpr int WS = kBlock / 64;
  constexpr int EB = kTwinChunk;
  constexpr int SR = kTwinRows;
  static_assert(kSplitRows % SR == 0 && SR % (WS * UNROLL) == 0, "staging must keep every row on its wave");
  static_assert(UNROLL == 4, "a wave reads its rows' shared indices as one int4");
  static_assert(EB % 4 == 0, "right-hand sides are read 4 envs at a time");
  // s_one holds row r at perm_row(r): a wave's UNROLL rows rb + WS * u (rb = wave + WS * UNROLL * k)
  // lie side by side from perm_row(rb) on
  auto perm_row = [](int r) { return r / (WS * UNROLL) * (WS * UNROLL) + r % WS * UNROLL + r / WS % UNROLL; };
  typedef T vec_t __attribute__((ext_vector_type(VW)));
  typedef T f4_t __attribute__((ext_vector_type(4)));
  __shared__ f4_t s_vec[SR * EB];   // [row][env] the env's right-hand side at this position, 0 if none
  __shared__ int s_row[SR * EB];    // [row][env] inverse row the env reads at this position, -1 if none
  __shared__ __align__(16) int s_one[SR];   // the row every reading env reads (rows permuted, below)
  __shared__ int s_mixed;           // some position has envs reading different rows
  __shared__ T s_red[(WS - 1) * 3 * TILE];
  __shared__ int s_e[EB], s_r1[EB];
  const int4 item = items[blockIdx.x];
  if (item.w <= 0) return;   // padding item
  const int tile0 = item.y, split = item.z, w = item.w;
  const int e0 = envs[item.x];
  const int n = B.voff[e0 + 1] - B.voff[e0];   // the same mesh, inverse and split size for the chunk
  const int ld = B.gld[e0];
  const int R = split_rows(split_cover(n, B.cap));
  const int r0 = split * R;
  if (threadIdx.x < EB) {
    int e = -1, r1 = r0;
    if ((int)threadIdx.x < w) {
      e = envs[item.x + threadIdx.x];
      const int nrows = ROWS ? B.ccount[e] : n;
      if (!(skip && skip[e]) && r0 < nrows) r1 = min(r0 + R, nrows);
    }
    s_e[threadIdx.x] = e;
    s_r1[threadIdx.x] = r1;
  }
  __syncthreads();
  int r1m = r0;
  for (int t = 0; t < EB; ++t) r1m = max(r1m, s_r1[t]);
  if (r1m == r0) return;   // no env of the chunk reads rows in this split (uniform over the block)
  const T* G = B.G + B.goff[e0];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col0 = tile0 + lane * VW;
  T acc[EB][VW][3];
#pragma unroll
  for (int t = 0; t < EB; ++t)
#pragma unroll
    for (int q = 0; q < VW; ++q) acc[t][q][0] = acc[t][q][1] = acc[t][q][2] = 0;
  for (int c0 = r0; c0 < r1m; c0 += SR) {
    const int nrm = min(SR, r1m - c0);
    __syncthreads();
    if (threadIdx.x == 0) s_mixed = 0;
    // all SR x EB slots are written: an env that reads no row at a position (past its rows, past
    // the chunk's envs) gets row -1 and a zero right-hand side
    for (int idx = threadIdx.x; idx < SR * EB; idx += kBlock) {
      const int r = idx / EB, t = idx - r * EB;
      const int e = s_e[t];
      int row = -1;
      f4_t f = {0, 0, 0, 0};
      if (e >= 0 && r < nrm && c0 + r < s_r1[t]) {
        if (ROWS) {
          const size_t j = (size_t)e * B.cap + c0 + r;
          row = B.cvert[j];
          f[0] = B.cforce[3 * j]; f[1] = B.cforce[3 * j + 1]; f[2] = B.cforce[3 * j + 2];
        } else {
          const int vb = B.voff[e] + c0 + r;
          row = c0 + r;
          f[0] = B.b[vb]; f[1] = B.b[B.NV + vb]; f[2] = B.b[2 * B.NV + vb];
        }
      }
      s_row[idx] = row;
      s_vec[idx] = f;
    }
    __syncthreads();
    // the row every env that reads at this position reads (row 0 where none does); s_mixed is set
    // where envs read different rows
    for (int r = threadIdx.x; r < SR; r += kBlock) {
      int one = -1;
      bool same = true;
      for (int t = 0; t < EB; ++t) {
        const int q = s_row[r * EB + t];
        if (q < 0) continue;
        if (one < 0) one = q;
        else if (q != one) same = false;
      }
      s_one[perm_row(r)] = one < 0 ? 0 : one;
      if (!same) s_mixed = 1;
    }
    __syncthreads();
    // One pass with one load per row for the whole chunk, or, where the envs read different rows
    // somewhere in these rows, one pass per env over its own rows (its row indices written to
    // s_one first, a scalar env mask selecting its sums).
    const bool mixed = __builtin_amdgcn_readfirstlane(s_mixed) != 0;   // the same over the block
    const int npass = mixed ? w : 1;
    const int wsc = __builtin_amdgcn_readfirstlane(wid);
    for (int p = 0; p < npass; ++p) {
      if (mixed) {
        __syncthreads();
        for (int r = threadIdx.x; r < SR; r += kBlock) {
          const int q = s_row[r * EB + p];
          s_one[perm_row(r)] = q < 0 ? 0 : q;
        }
        __syncthreads();
      }
      const unsigned mask = mixed ? (1u << p) : ((1u << w) - 1u);
      if (col0 < ld) {   // ld is a multiple of 32 columns: a lane's VW columns lie inside the row
        // Row indices are the same over the wave (scalar registers), so the UNROLL loads go out
        // together, and the next UNROLL rows' loads go out before this iteration's FMAs (double
        // buffer).  An env's sum takes g * b at every row of the wave; where it reads nothing b
        // is zero and g * 0 leaves the sum as it is (the sums start at +0 and the inverse is
        // finite), so each env adds exactly its own rows in k_gemv_split's order.  The rows
        // rb + WS * u stay below SR (SR is a multiple of WS * UNROLL).
        auto load_rows = [&](int rb, vec_t* g) {
          const int4 o4 = *reinterpret_cast<const int4*>(s_one + perm_row(rb));
          const int ones[4] = {o4.x, o4.y, o4.z, o4.w};
#pragma unroll
          for (int u = 0; u < UNROLL; ++u)
            g[u] = *reinterpret_cast<const vec_t*>(G + (size_t)__builtin_amdgcn_readfirstlane(ones[u]) * ld + col0);
        };
        vec_t gn[UNROLL];
        if (wsc < nrm) load_rows(wsc, gn);
        for (int rb = wsc; rb < nrm; rb += WS * UNROLL) {
          vec_t g[UNROLL];
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) g[u] = gn[u];
          if (rb + WS * UNROLL < nrm) load_rows(rb + WS * UNROLL, gn);
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            // right-hand sides read 4 envs at a time (one LDS wait per 4 envs); 4 x 4 values live
#pragma unroll
            for (int t0 = 0; t0 < EB; t0 += 4) {
              if (!((mask >> t0) & 0xFu)) continue;   // none of these 4 envs takes the row
              f4_t bb[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) bb[i] = s_vec[(rb + WS * u) * EB + t0 + i];
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                if (!((mask >> (t0 + i)) & 1u)) continue;
#pragma unroll
                for (int q = 0; q < VW; ++q) {
                  acc[t0 + i][q][0] += g[u][q] * bb[i][0];
                  acc[t0 + i][q][1] += g[u][q] * bb[i][1];
                  acc[t0 + i][q][2] += g[u][q] * bb[i][2];
                }
              }
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
      }
    }
  }
  // per env, k_gemv_split's fixed-order reduction over the waves
#pragma unroll
  for (int t = 0; t < EB; ++t) {
    const int e = s_e[t];
    if (e < 0 || s_r1[t] <= r0) continue;   // uniform over the block
    __syncthreads();
    if (wid > 0)
      for (int q = 0; q < VW; ++q)
        for (int k = 0; k < 3; ++k) s_red[((wid - 1) * 3 + k) * TILE + lane * VW + q] = acc[t][q][k];
    __syncthreads();
    if (wid == 0) {
      T* P = partial + poff[e];
      for (int q = 0; q < VW; ++q) {
        const int col = col0 + q;
        if (col >= n) continue;
        for (int k = 0; k < 3; ++k) {
          T s = acc[t][q][k];
          for (int w2 = 0; w2 < WS - 1; ++w2) s += s_red[(w2 * 3 + k) * TILE + lane * VW + q];
          P[((size_t)split * 3 + k) * n + col] = s;
        }
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
  if (S.n_items > 0)
    hipLaunchKernelGGL((k_gemv_split<T, false>), dim3((unsigned)S.n_items), dim3(kBlock), 0, s, B, S.items,
                       (const int*)nullptr, P, S.poff);
  if (S.n_twin_items > 0)
    hipLaunchKernelGGL((k_gemv_split_twins<T, false>), dim3((unsigned)S.n_twin_items), dim3(kBlock), 0, s, B,
                       S.twin_items, S.twin_envs, (const int*)nullptr, P, S.poff);
  hipLaunchKernelGGL((k_gemv_merge<T, false>), dim3((unsigned)((B.NV + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, B,
                     (const int*)nullptr, (const T*)P, S.poff);
}

template <class T>
void launch_split_correct(const DevBatch<T>& B, const SplitSchedule& S, const int* skip, hipStream_t s) {
  T* P = static_cast<T*>(S.partial);
  if (S.n_items > 0)
    hipLaunchKernelGGL((k_gemv_split<T, true>), dim3((unsigned)S.n_items), dim3(kBlock), 0, s, B, S.items, skip, P,
                       S.poff);
  if (S.n_twin_items > 0)
    hipLaunchKernelGGL((k_gemv_split_twins<T, true>), dim3((unsigned)S.n_twin_items), dim3(kBlock), 0, s, B,
                       S.twin_items, S.twin_envs, skip, P, S.poff);
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
