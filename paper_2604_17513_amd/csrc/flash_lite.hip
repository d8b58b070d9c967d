// Lightweight contact update in global memory (Alg. 1 with the inertia-only metric of Eq. 10)
// for contact counts beyond what one CU's LDS holds.
//
// Each update reads the current displacement u = z + h^2 Gbar H^T lambda (the position update
// of Alg. 1, formed by the explicit-inverse product over the contact rows), evaluates Phi and its
// generalized-Jacobian blocks at Y = F^T u per contact, and takes lambda <- lambda + delta with
// (K W~ + E) delta = -Phi per vertex, W~ = h^2 H M^-1 H^T.  The metric couples only the contacts
// of one vertex, so every vertex group is updated by one thread from global memory; one
// workgroup per env reduces the env's residual.  The contact displacement follows lambda through
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

// One workgroup per env.  it = -1 (once per step, after detection): world forces F lambda of
// the warm start, which the first position update reads.  it >= 0 counts the updates already
// taken in this local-global iteration: the update evaluates the FP64 residual at (u, lambda) and
// stops the env's iteration (done flag) when it is at inner_tol or `it` reached the budget;
// otherwise it updates every vertex group.  The done flag is cleared by the iteration's first
// call (it == 0).
template <class T, class CT>
__global__ void __launch_bounds__(kBlock) k_lite_update(DevBatch<T> B, const T* mu_env, int it, int first_lg) {
  __shared__ double sh_red[kBlock / 64];
  const int e = blockIdx.x;
  if (it > 0 && B.lite_done[e]) return;
  const int c = B.ccount[e];
  const int tid = threadIdx.x;
  const size_t cb = (size_t)e * B.cap;
  const int v0 = B.voff[e];
  const int NV = B.NV;
  const CT* Fr;
  if constexpr (std::is_same<CT, T>::value) Fr = B.cframe + 9 * cb;
  else Fr = B.cframe64 + 9 * cb;
  const int* cv = B.cvert + cb;
  const int* cobs = B.cobs + cb;
  const CT mu = (CT)mu_env[e];
  if (it < 0) {
    for (int j = tid; j < c; j += kBlock) {
      const CT* F = Fr + 9 * j;
      const double* lj = B.clam + 3 * (cb + j);
      const CT l0 = (CT)lj[0], l1 = (CT)lj[1], l2 = (CT)lj[2];
      for (int k = 0; k < 3; ++k) B.cforce[3 * (cb + j) + k] = (T)(F[k] * l0 + F[3 + k] * l1 + F[6 + k] * l2);
    }
    if (tid == 0) B.lite_done[e] = 0;
    return;
  }
  // residual at the residual scale s = h^2 / m_v (FP64)
  double rloc = 0.0;
  for (int j = tid; j < c; j += kBlock) {
    const CT* F = Fr + 9 * j;
    const int vi = v0 + cv[j];
    const double uw0 = (double)B.u[vi], uw1 = (double)B.u[NV + vi], uw2 = (double)B.u[2 * NV + vi];
    double Y[3];
    for (int a = 0; a < 3; ++a) Y[a] = (double)F[3 * a] * uw0 + (double)F[3 * a + 1] * uw1 + (double)F[3 * a + 2] * uw2;
    const double s = (double)B.cs[cb + j];
    const double* lj = B.clam + 3 * (cb + j);
    const double cnd = B.cd0d[cb + j] + Y[0];
    const double ut1 = Y[1] - (double)B.cdob[2 * (cb + j)], ut2 = Y[2] - (double)B.cdob[2 * (cb + j) + 1];
    const bool att = cobs[j] >= kMaxObs;
    const double pn = att ? cnd : fmin(cnd, s * lj[0]);
    const double z1 = lj[1] - ut1 / s, z2 = lj[2] - ut2 / s;
    const double nz = sqrt(z1 * z1 + z2 * z2);
    const double rh = (double)mu * fmax(lj[0], 0.0);
    double q1 = z1, q2 = z2;
    if (!att && nz > rh) { const double f = nz > 0 ? rh / nz : 0.0; q1 = f * z1; q2 = f * z2; }
    const double t1 = s * (lj[1] - q1), t2 = s * (lj[2] - q2);
    double rj = fmax(fabs(pn), sqrt(t1 * t1 + t2 * t2));
    if (!(rj == rj)) rj = INFINITY;
    rloc = fmax(rloc, rj);
  }
  const double r = wg_max(rloc, sh_red);
  if (r <= B.tol || it >= B.max_newton) {
    if (tid == 0) {
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
  if (it == 0 && tid == 0) B.lite_done[e] = 0;
  const double dmaxf = B.max_force;
  // one update per vertex group (contacts are listed by vertex: a group is contiguous)
  for (int j = tid; j < c; j += kBlock) {
    if (j > 0 && cv[j - 1] == cv[j]) continue;
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
}

}  // namespace

template <class T>
void launch_lite_update(const DevBatch<T>& B, const T* mu_env, int it, int first_lg, hipStream_t s) {
  const dim3 g(B.n_envs), blk(kBlock);
  if (B.csp64) hipLaunchKernelGGL((k_lite_update<T, double>), g, blk, 0, s, B, mu_env, it, first_lg);
  else hipLaunchKernelGGL((k_lite_update<T, T>), g, blk, 0, s, B, mu_env, it, first_lg);
}

template void launch_lite_update<float>(const DevBatch<float>&, const float*, int, int, hipStream_t);
template void launch_lite_update<double>(const DevBatch<double>&, const double*, int, int, hipStream_t);

}  // namespace flash
