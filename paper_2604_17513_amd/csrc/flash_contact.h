// Per-contact blocks of the contact solves, shared by the explicit-inverse kernels and the
// global-memory lightweight update: the generalized-Jacobian blocks of the NCP function (min-map
// normal part, Alart-Curnier friction part, attachment rows) and the lightweight update of one
// vertex's contacts (Alg. 1 with the inertia-only metric of Eq. 10).
#pragma once
#include <hip/hip_runtime.h>

#include "flash_device.h"

namespace flash {

// class bits: 1 normal active, 2 tangential stick, 4 tangential slip (neither: rho = 0)
template <class T>
__device__ __forceinline__ void contact_KE(int cls, T sp, T mu, T kap, T y0, T y1, T K[3][3], T E[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) { K[a][b] = 0; E[a][b] = 0; }
  if (cls & 1) K[0][0] = 1; else E[0][0] = sp;
  if (cls & 2) { K[1][1] = 1; K[2][2] = 1; }
  else if (cls & 4) {
    T P00 = 1 - y0 * y0, P01 = -y0 * y1, P11 = 1 - y1 * y1;
    K[1][1] = kap * P00; K[1][2] = kap * P01; K[2][1] = kap * P01; K[2][2] = kap * P11;
    E[1][1] = sp * (1 - kap * P00); E[1][2] = -sp * kap * P01;
    E[2][1] = -sp * kap * P01; E[2][2] = sp * (1 - kap * P11);
    E[1][0] = -sp * mu * y0; E[2][0] = -sp * mu * y1;
  } else {
    E[1][1] = sp; E[2][2] = sp;
  }
}

// ---------------------------------------------------------------------------
// Fixed-budget lightweight contact update (Alg. 1 with the inertia-only metric of Eq. 10).
// Per local-global iteration, up to max_newton updates lambda <- lambda + delta with
// (K W~ + E) delta = -Phi, W~ = h^2 H M^-1 H^T (blocks (h^2 / m_v) F_j^T F_k between contacts of
// one vertex), Phi and (K, E) at the exact contact displacement Y = y_free + W lambda, proximal
// scale s = h^2 / m_v, no line search; stops early at inner_tol.  For a vertex with one contact
// W~ = s I and the system is [s 0 0; -s mu y^ (slip only), s I], solved in closed form; vertices
// touching several obstacles solve their 3m x 3m block by Gaussian elimination.
// ---------------------------------------------------------------------------

// Phi and the generalized-Jacobian blocks of one contact (proximal scale sp): K = dPhi/dY,
// E = dPhi/dlambda.  Returns the slip direction in yh (zero unless slipping).
template <class CT>
__device__ __forceinline__ void lite_contact(CT sp, CT mu, CT d0, CT dob1, CT dob2, const CT* Yj, const double* lj,
                                             bool att, CT phi[3], CT K[3][3], CT E[3][3]) {
  const CT l0 = (CT)lj[0], l1 = (CT)lj[1], l2 = (CT)lj[2];
  const CT cn = d0 + Yj[0];
  const CT ut1 = Yj[1] - dob1, ut2 = Yj[2] - dob2;
  if (att) {   // attachment row: Phi = Y - d, K = I, E = 0
    phi[0] = cn; phi[1] = ut1; phi[2] = ut2;
    contact_KE(3, sp, mu, CT(0), CT(0), CT(0), K, E);
    return;
  }
  int cls = (cn <= sp * l0) ? 1 : 0;
  phi[0] = fmin(cn, sp * l0);
  const CT y1 = l1 - ut1 / sp, y2 = l2 - ut2 / sp;
  const CT rho = mu * fmax(l0, CT(0));
  const CT ny = sqrt(y1 * y1 + y2 * y2);
  CT kap = 0, yh0 = 0, yh1 = 0, p1 = 0, p2 = 0;
  if (rho > CT(0)) {
    if (ny <= rho) { cls |= 2; p1 = y1; p2 = y2; }
    else { cls |= 4; kap = rho / ny; yh0 = y1 / ny; yh1 = y2 / ny; p1 = rho * yh0; p2 = rho * yh1; }
  }
  phi[1] = sp * (l1 - p1);
  phi[2] = sp * (l2 - p2);
  contact_KE(cls, sp, mu, kap, yh0, yh1, K, E);
}

// delta for the m contacts (m >= 2) of one vertex starting at contact j
template <class CT>
__device__ __noinline__ void lite_group_solve(int m, CT sp, CT mu, const CT* Fr, const CT* d0, const CT* dob,
                                              const CT* Y, const double* lam, const int* cobs, CT* dl) {
  double Z[3 * kCacheSlots][3 * kCacheSlots + 1];
  CT Kq[kCacheSlots][3][3], Eq[kCacheSlots][3][3], ph[kCacheSlots][3];
  for (int q = 0; q < m; ++q)
    lite_contact(sp, mu, d0[q], dob[2 * q], dob[2 * q + 1], Y + 3 * q, lam + 3 * q, cobs[q] >= kMaxObs, ph[q], Kq[q],
                 Eq[q]);
  const int n = 3 * m;
  for (int q = 0; q < m; ++q)
    for (int a = 0; a < 3; ++a) {
      const int row = 3 * q + a;
      for (int r = 0; r < m; ++r)
        for (int b = 0; b < 3; ++b) {
          // (K_q W~_qr)[a][b] with W~_qr = sp F_q^T F_r
          double acc = 0.0;
          for (int cc = 0; cc < 3; ++cc) {
            double g = 0.0;
            for (int k = 0; k < 3; ++k) g += (double)Fr[9 * q + 3 * cc + k] * (double)Fr[9 * r + 3 * b + k];
            acc += (double)Kq[q][a][cc] * (double)sp * g;
          }
          if (q == r) acc += (double)Eq[q][a][b];
          Z[row][3 * r + b] = acc;
        }
      Z[row][n] = -(double)ph[q][a];
    }
  for (int k = 0; k < n; ++k) {
    int pv = k;
    for (int i = k + 1; i < n; ++i)
      if (fabs(Z[i][k]) > fabs(Z[pv][k])) pv = i;
    if (pv != k)
      for (int t = k; t <= n; ++t) { const double tmp = Z[k][t]; Z[k][t] = Z[pv][t]; Z[pv][t] = tmp; }
    const double piv = Z[k][k];
    for (int i = k + 1; i < n; ++i) {
      const double f = piv != 0.0 ? Z[i][k] / piv : 0.0;
      for (int t = k; t <= n; ++t) Z[i][t] -= f * Z[k][t];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double acc = Z[k][n];
    for (int t = k + 1; t < n; ++t) acc -= Z[k][t] * (double)dl[t];
    dl[k] = Z[k][k] != 0.0 ? (CT)(acc / Z[k][k]) : CT(0);
  }
}

}  // namespace flash
