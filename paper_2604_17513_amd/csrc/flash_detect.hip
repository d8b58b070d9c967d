// Contact detection, prediction and step finalisation.
//
// This translation unit is compiled with -ffp-contract=off: the contact
// predicate, the predicted position and the obstacle track are evaluated in
// FP64 with a fixed operation order so that the contact list is bit-exact
// against any other FP64 evaluation of the same formulas.
#include "flash_device.h"
#include "flash_launch.h"

namespace flash {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Exclusive block scan of one int per thread (blockDim.x == kBlock).
__device__ int block_excl_scan(int v, int* sh, int* total) {
  int lane = lane_id(), wid = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) sh[wid] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    int s = sh[w];
    if (w < wid) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

// Signed-distance predicate of one obstacle at point p (margin test without sqrt).
__device__ bool obstacle_pred(int kind, const double* c, const double* R, const double* sz,
                              const double* p, double margin) {
  double r0 = p[0] - c[0], r1 = p[1] - c[1], r2 = p[2] - c[2];
  if (kind == 0) {
    double d = (R[1] * r0 + R[4] * r1) + R[7] * r2;
    return d < margin;
  }
  if (kind == 1) {
    bool outside = false;
    double m[3];
    for (int i = 0; i < 3; ++i) {
      double pi = (R[i] * r0 + R[3 + i] * r1) + R[6 + i] * r2;
      double qi = fabs(pi) - sz[i];
      outside |= qi > 0.0;
      m[i] = fmax(qi, 0.0);
    }
    if (!outside) return true;
    double d2 = (m[0] * m[0] + m[1] * m[1]) + m[2] * m[2];
    return d2 < margin * margin;
  }
  double a0 = R[0], a1 = R[3], a2 = R[6];
  double t = (a0 * r0 + a1 * r1) + a2 * r2;
  double s = fmin(fmax(t, -sz[1]), sz[1]);
  double w0 = r0 - s * a0, w1 = r1 - s * a1, w2 = r2 - s * a2;
  double d2 = (w0 * w0 + w1 * w1) + w2 * w2;
  double lim = sz[0] + margin;
  return d2 < lim * lim;
}

// Signed distance and outward normal of one obstacle at point p.
__device__ void obstacle_geom(int kind, const double* c, const double* R, const double* sz,
                              const double* p, double* d, double* n) {
  double r0 = p[0] - c[0], r1 = p[1] - c[1], r2 = p[2] - c[2];
  if (kind == 0) {
    n[0] = R[1]; n[1] = R[4]; n[2] = R[7];
    *d = (R[1] * r0 + R[4] * r1) + R[7] * r2;
    return;
  }
  if (kind == 1) {
    double pp[3], q[3], m[3], sg[3];
    bool outside = false;
    for (int i = 0; i < 3; ++i) {
      pp[i] = (R[i] * r0 + R[3 + i] * r1) + R[6 + i] * r2;
      q[i] = fabs(pp[i]) - sz[i];
      outside |= q[i] > 0.0;
      m[i] = fmax(q[i], 0.0);
      sg[i] = pp[i] >= 0.0 ? 1.0 : -1.0;
    }
    if (outside) {
      double d2 = (m[0] * m[0] + m[1] * m[1]) + m[2] * m[2];
      *d = sqrt(d2);
      double gl0 = m[0] * sg[0], gl1 = m[1] * sg[1], gl2 = m[2] * sg[2];
      double gw[3];
      for (int i = 0; i < 3; ++i) gw[i] = (R[3 * i] * gl0 + R[3 * i + 1] * gl1) + R[3 * i + 2] * gl2;
      double gn = sqrt((gw[0] * gw[0] + gw[1] * gw[1]) + gw[2] * gw[2]);
      n[0] = gw[0] / gn; n[1] = gw[1] / gn; n[2] = gw[2] / gn;
    } else {
      int is = 0;
      if (q[1] > q[is]) is = 1;
      if (q[2] > q[is]) is = 2;
      *d = fmax(fmax(q[0], q[1]), q[2]);
      n[0] = R[is] * sg[is]; n[1] = R[3 + is] * sg[is]; n[2] = R[6 + is] * sg[is];
    }
    return;
  }
  double a0 = R[0], a1 = R[3], a2 = R[6];
  double t = (a0 * r0 + a1 * r1) + a2 * r2;
  double s = fmin(fmax(t, -sz[1]), sz[1]);
  double w0 = r0 - s * a0, w1 = r1 - s * a1, w2 = r2 - s * a2;
  double d2 = (w0 * w0 + w1 * w1) + w2 * w2;
  double dn = sqrt(d2);
  *d = dn - sz[0];
  if (dn > 0.0) { n[0] = w0 / dn; n[1] = w1 / dn; n[2] = w2 / dn; }
  else { n[0] = a0; n[1] = a1; n[2] = a2; }
}

// t1 = unit(e_k x n), k = argmin |n_i| (lowest on ties); t2 = n x t1.
__device__ void tangent_frame(const double* n, double* t1, double* t2) {
  double an[3] = {fabs(n[0]), fabs(n[1]), fabs(n[2])};
  int k = 0;
  if (an[1] < an[k]) k = 1;
  if (an[2] < an[k]) k = 2;
  double e[3] = {0.0, 0.0, 0.0};
  e[k] = 1.0;
  t1[0] = e[1] * n[2] - e[2] * n[1];
  t1[1] = e[2] * n[0] - e[0] * n[2];
  t1[2] = e[0] * n[1] - e[1] * n[0];
  double l = sqrt((t1[0] * t1[0] + t1[1] * t1[1]) + t1[2] * t1[2]);
  t1[0] /= l; t1[1] /= l; t1[2] /= l;
  t2[0] = n[1] * t1[2] - n[2] * t1[1];
  t2[1] = n[2] * t1[0] - n[0] * t1[2];
  t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

// One workgroup per environment.  Predicts u = h v + h^2 g, finds the contacts
// (ordered by vertex, then obstacle) and seeds their multipliers.
template <class T>
__global__ void __launch_bounds__(kBlock) k_detect(DevBatch<T> B, const T* mu_env) {
  __shared__ int sh_scan[kBlock / 64];
  __shared__ double sh_c[kMaxObs][3];
  __shared__ double sh_dob[kMaxObs][3];
  __shared__ double sh_gc[kMaxGrip][3];    // gripper center at the start of the step (capture)
  __shared__ double sh_gcn[kMaxGrip][3];   // and at its end (attachment targets)
  __shared__ int sh_gcap[kMaxGrip];        // 1: grasping and holding nothing: captures this step
  __shared__ int sh_gon[kMaxGrip];         // grasp on
  __shared__ int sh_gheld[kMaxGrip];
  const int e = blockIdx.x;
  const int v0 = B.voff[e], v1 = B.voff[e + 1];
  const int nob = B.nobs[e];
  const int ng = B.ngrip ? B.ngrip[e] : 0;
  const double h = B.h, hh = B.h * B.h;
  const int cap = B.cap;
  if (threadIdx.x < nob) {
    int o = e * kMaxObs + threadIdx.x;
    bool moving = B.obs_move[o] != 0;
    for (int k = 0; k < 3; ++k) {
      double dob = moving ? h * B.obs_vel[3 * o + k] : 0.0;
      sh_dob[threadIdx.x][k] = dob;
      sh_c[threadIdx.x][k] = B.obs_c[3 * o + k] + dob;
    }
  }
  if (threadIdx.x < kMaxGrip) {
    const int g = threadIdx.x, q = e * kMaxGrip + g;
    const bool on = g < ng && B.grip_grasp[q] != 0;
    sh_gon[g] = on ? 1 : 0;
    sh_gcap[g] = (on && B.grip_held[q] == 0) ? 1 : 0;
    sh_gheld[g] = 0;
    if (g < ng) {
      const bool moving = B.grip_move[q] != 0;
      for (int k = 0; k < 3; ++k) {
        sh_gc[g][k] = B.grip_c[3 * q + k];
        sh_gcn[g][k] = B.grip_c[3 * q + k] + (moving ? h * B.grip_vel[3 * q + k] : 0.0);
      }
    }
  }
  if (threadIdx.x == 0) {
    B.nbase[e] = 0;
    B.lust[4 * e] = 0;
  }
  __syncthreads();
  const int cur = *B.stamp;
  int count = 0;
  for (int base = v0; base < v1; base += kBlock) {
    const int i = base + threadIdx.x;
    unsigned mask = 0;
    double xd[3], xt[3];
    if (i < v1) {
      for (int k = 0; k < 3; ++k) {
        double xk = (double)B.x[k * B.NV + i];
        double vk = (double)B.v[k * B.NV + i];
        xd[k] = xk;
        xt[k] = (xk + h * vk) + hh * B.g[k];
        T uk = (T)(h * vk + hh * B.g[k]);
        B.ut[k * B.NV + i] = uk;
        B.u[k * B.NV + i] = uk;
      }
      for (int o = 0; o < nob; ++o) {
        int oo = e * kMaxObs + o;
        const double* R = B.obs_R + 9 * oo;
        const double* sz = B.obs_size + 3 * oo;
        int kind = B.obs_kind[oo];
        bool hit = obstacle_pred(kind, sh_c[o], R, sz, xd, B.margin) ||
                   obstacle_pred(kind, sh_c[o], R, sz, xt, B.margin);
        if (hit) mask |= 1u << o;
      }
      if (ng > 0) {
        // attachment sets: release when the grasp is off; a grasping gripper that holds nothing
        // takes the free vertices within its radius (lowest gripper first), with their offsets
        int ag = B.att_g[i];
        if (ag >= 0 && !sh_gon[ag]) ag = -1;
        for (int g = 0; g < ng && ag < 0; ++g) {
          if (!sh_gcap[g]) continue;
          const double d0 = xd[0] - sh_gc[g][0], d1 = xd[1] - sh_gc[g][1], d2 = xd[2] - sh_gc[g][2];
          const double r = B.grip_r[e * kMaxGrip + g];
          if ((d0 * d0 + d1 * d1) + d2 * d2 <= r * r) {
            ag = g;
            B.att_off[3 * (size_t)i] = d0;
            B.att_off[3 * (size_t)i + 1] = d1;
            B.att_off[3 * (size_t)i + 2] = d2;
          }
        }
        B.att_g[i] = ag;
        if (ag >= 0) {
          // a held vertex's position is prescribed by its attachment: no obstacle rows
          mask = 1u << (kMaxObs + ag);
          atomicAdd(&sh_gheld[ag], 1);
        }
      }
    }
    int total;
    int off = block_excl_scan(__popc(mask), sh_scan, &total);
    if (mask) {
      int slot = count + off;
      for (int o = 0; o < kCacheSlots; ++o) {
        if (!(mask & (1u << o))) continue;
        if (slot < cap && o >= kMaxObs) {
          // attachment row of gripper g: frame I, target = end-of-step center + offset, stored as
          // d0 = -(target - x)_0 and dob = (target - x)_{1,2} so that Phi = Y - (target - x)
          const int g = o - kMaxObs;
          const int j = e * cap + slot;
          double d[3];
          for (int k = 0; k < 3; ++k) d[k] = (sh_gcn[g][k] + B.att_off[3 * (size_t)i + k]) - xd[k];
          B.cvert[j] = i - v0;
          B.cobs[j] = o;
          T* F = B.cframe + 9 * (size_t)j;
          for (int k = 0; k < 9; ++k) F[k] = (k % 4 == 0) ? T(1) : T(0);
          if (sizeof(T) == 4 && B.cframe64) {
            double* F64 = B.cframe64 + 9 * (size_t)j;
            for (int k = 0; k < 9; ++k) F64[k] = (k % 4 == 0) ? 1.0 : 0.0;
          }
          B.cd0[j] = (T)(-d[0]);
          B.cd0d[j] = -d[0];
          B.cdob[2 * j] = (T)d[1];
          B.cdob[2 * j + 1] = (T)d[2];
          B.cs[j] = (T)(hh / (double)B.mass[i]);
          const int ci = i * kCacheSlots + o;
          int fresh = 1;
          double l[3] = {0.0, 0.0, 0.0};
          if (B.warm_start != 0 && B.cache_stamp[ci] == cur - 1) {
            for (int k = 0; k < 3; ++k) l[k] = (double)B.cache_f[3 * ci + k];
            fresh = 0;
          }
          for (int k = 0; k < 3; ++k) B.clam[3 * j + k] = l[k];
          B.cnew[j] = fresh;
          ++slot;
          continue;
        }
        if (slot < cap) {
          int oo = e * kMaxObs + o;
          const double* R = B.obs_R + 9 * oo;
          const double* sz = B.obs_size + 3 * oo;
          double d, n[3], t1[3], t2[3];
          obstacle_geom(B.obs_kind[oo], sh_c[o], R, sz, xd, &d, n);
          tangent_frame(n, t1, t2);
          const int j = e * cap + slot;
          B.cvert[j] = i - v0;
          B.cobs[j] = o;
          T* F = B.cframe + 9 * (size_t)j;
          for (int k = 0; k < 3; ++k) { F[k] = (T)n[k]; F[3 + k] = (T)t1[k]; F[6 + k] = (T)t2[k]; }
          if (sizeof(T) == 4 && B.cframe64) {
            double* F64 = B.cframe64 + 9 * (size_t)j;
            for (int k = 0; k < 3; ++k) { F64[k] = n[k]; F64[3 + k] = t1[k]; F64[6 + k] = t2[k]; }
          }
          B.cd0[j] = (T)d;
          B.cd0d[j] = d;
          const double* dob = sh_dob[o];
          B.cdob[2 * j] = (T)((t1[0] * dob[0] + t1[1] * dob[1]) + t1[2] * dob[2]);
          B.cdob[2 * j + 1] = (T)((t2[0] * dob[0] + t2[1] * dob[1]) + t2[2] * dob[2]);
          B.cs[j] = (T)(hh / (double)B.mass[i]);
          // warm start from the previous step's world-frame force at this (vertex, obstacle)
          const int ci = i * kCacheSlots + o;
          T l0 = 0, l1 = 0, l2 = 0;
          int fresh = 1;
          if (B.warm_start != 0 && B.cache_stamp[ci] == cur - 1) {
            T f0 = B.cache_f[3 * ci], f1 = B.cache_f[3 * ci + 1], f2 = B.cache_f[3 * ci + 2];
            l0 = F[0] * f0 + F[1] * f1 + F[2] * f2;
            l1 = F[3] * f0 + F[4] * f1 + F[5] * f2;
            l2 = F[6] * f0 + F[7] * f1 + F[8] * f2;
            // project onto the friction cone of the new frame
            l0 = l0 > T(0) ? l0 : T(0);
            T lt = sqrt(l1 * l1 + l2 * l2);
            T rho = mu_env[e] * l0;
            if (lt > rho) {
              T f = lt > T(0) ? rho / lt : T(0);
              l1 *= f;
              l2 *= f;
            }
            fresh = 0;
          }
          B.clam[3 * j] = (double)l0; B.clam[3 * j + 1] = (double)l1; B.clam[3 * j + 2] = (double)l2;
          B.cnew[j] = fresh;
        }
        ++slot;
      }
    }
    count += total;
  }
  __syncthreads();
  if (threadIdx.x < ng) B.grip_held[e * kMaxGrip + threadIdx.x] = sh_gheld[threadIdx.x];
  if (threadIdx.x == 0) {
    B.ccount[e] = count < cap ? count : cap;
    B.iters[e] = 0;
    B.refac[e] = 0;
    B.fp64_polar[e] = 0;
    B.flags[e] = count > cap ? 4 : 0;
  }
}

// One workgroup per environment: v = u / h, x += u, FP64 NCP residual at the
// end positions, warm-start cache, obstacle track.
template <class T>
__global__ void __launch_bounds__(kBlock) k_finalize(DevBatch<T> B, const T* mu_env) {
  __shared__ double sh_red[kBlock / 64];
  const int e = blockIdx.x;
  const int v0 = B.voff[e], v1 = B.voff[e + 1];
  const double h = B.h;
  const T inv_h = (T)(1.0 / h);
  int bad = 0;
  for (int i = v0 + threadIdx.x; i < v1; i += kBlock) {
    for (int k = 0; k < 3; ++k) {
      T uk = B.u[k * B.NV + i];
      T xn = B.x[k * B.NV + i] + uk;
      T vn = uk * inv_h;
      bad |= !(isfinite((double)xn) && isfinite((double)vn));
      B.x[k * B.NV + i] = xn;
      B.v[k * B.NV + i] = vn;
    }
  }
  // residual r = max_j max(|min(C_n, s l_n)|, |s (l_t - Pi(l_t - u_t / s))|)
  const int c = B.ccount[e];
  const int cur = *B.stamp;
  const double mu = (double)mu_env[e];
  double r = 0.0;
  for (int jj = threadIdx.x; jj < c; jj += kBlock) {
    const int j = e * B.cap + jj;
    const int vi = v0 + B.cvert[j];
    double F[9];
    for (int k = 0; k < 9; ++k) F[k] = B.cframe64 ? B.cframe64[9 * (size_t)j + k] : (double)B.cframe[9 * (size_t)j + k];
    double uw[3] = {(double)B.u[vi], (double)B.u[B.NV + vi], (double)B.u[2 * B.NV + vi]};
    double Y[3];
    for (int a = 0; a < 3; ++a)
      Y[a] = F[3 * a] * uw[0] + F[3 * a + 1] * uw[1] + F[3 * a + 2] * uw[2];
    double s = h * h / (double)B.mass[vi];
    double ln = B.clam[3 * j], l1 = B.clam[3 * j + 1], l2 = B.clam[3 * j + 2];
    double cn = B.cd0d[j] + Y[0];
    const bool att = B.cobs[j] >= kMaxObs;      // attachment: Phi = Y - d, no cone
    double pn = att ? cn : fmin(cn, s * ln);
    double ut1 = Y[1] - (double)B.cdob[2 * j], ut2 = Y[2] - (double)B.cdob[2 * j + 1];
    double y1 = l1 - ut1 / s, y2 = l2 - ut2 / s;
    double rho = mu * fmax(ln, 0.0);
    double ny = sqrt(y1 * y1 + y2 * y2);
    double p1 = y1, p2 = y2;
    if (!att && ny > rho) { double f = ny > 0.0 ? rho / ny : 0.0; p1 = f * y1; p2 = f * y2; }
    double t1 = s * (l1 - p1), t2 = s * (l2 - p2);
    double rj = fmax(fabs(pn), sqrt(t1 * t1 + t2 * t2));
    if (!(rj == rj)) rj = INFINITY;
    r = fmax(r, rj);
    // cache the world force for the next step's warm start
    const int ci = vi * kCacheSlots + B.cobs[j];
    T f0 = B.cforce[3 * j], f1 = B.cforce[3 * j + 1], f2 = B.cforce[3 * j + 2];
    B.cache_f[3 * ci] = f0; B.cache_f[3 * ci + 1] = f1; B.cache_f[3 * ci + 2] = f2;
    B.cache_stamp[ci] = cur;
  }
  // block max
  for (int d = 32; d > 0; d >>= 1) r = fmax(r, __shfl_xor(r, d, 64));
  if (lane_id() == 0) sh_red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) m = fmax(m, sh_red[w]);
    B.resid[e] = m;
    // worst residual and failed step count since the last statistics reset; a step that
    // dropped contacts beyond the capacity (flag bit 2, set by detection) counts as failed
    double* hist = B.resid_hist + 4 * e;
    hist[0] = (m == m) ? fmax(hist[0], m) : INFINITY;
    if (!(m <= B.ncp_tol) || (B.flags[e] & 4)) hist[1] += 1.0;
    hist[2] += (double)B.iters[e];
    hist[3] += 1.0;
    if (B.ws_hist) {
      const int w = B.ws_state[e];
      B.ws_hist[2 * e] += (unsigned long long)(w & 1);
      B.ws_hist[2 * e + 1] += (unsigned long long)((w >> 2) & 1);
    }
  }
  if (bad) atomicOr(&B.flags[e], 1);
  __syncthreads();
  // obstacle and gripper tracks: poses at the start of the next step
  const int nob = B.nobs[e];
  if (threadIdx.x < nob) {
    int o = e * kMaxObs + threadIdx.x;
    int mv = B.obs_move[o];
    if (mv != 0) {
      for (int k = 0; k < 3; ++k) B.obs_c[3 * o + k] = B.obs_c[3 * o + k] + h * B.obs_vel[3 * o + k];
      if (mv > 0) B.obs_move[o] = mv - 1;
    }
  }
  const int ng = B.ngrip ? B.ngrip[e] : 0;
  if (threadIdx.x >= 64 && threadIdx.x < 64 + ng) {
    const int q = e * kMaxGrip + threadIdx.x - 64;
    const int mv = B.grip_move[q];
    if (mv != 0) {
      for (int k = 0; k < 3; ++k) B.grip_c[3 * q + k] = B.grip_c[3 * q + k] + h * B.grip_vel[3 * q + k];
      if (mv > 0) B.grip_move[q] = mv - 1;
    }
  }
}

__global__ void k_tick(int* stamp) { *stamp += 1; }

template <class T>
void launch_detect(const DevBatch<T>& B, const T* mu_env, hipStream_t s) {
  hipLaunchKernelGGL(k_detect<T>, dim3(B.n_envs), dim3(kBlock), 0, s, B, mu_env);
}
template <class T>
void launch_finalize(const DevBatch<T>& B, const T* mu_env, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize<T>, dim3(B.n_envs), dim3(kBlock), 0, s, B, mu_env);
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(1), 0, s, B.stamp);
}

template void launch_detect<float>(const DevBatch<float>&, const float*, hipStream_t);
template void launch_detect<double>(const DevBatch<double>&, const double*, hipStream_t);
template void launch_finalize<float>(const DevBatch<float>&, const float*, hipStream_t);
template void launch_finalize<double>(const DevBatch<double>&, const double*, hipStream_t);

}  // namespace flash
