// Host-callable launchers for the step kernels.
#pragma once
#include "flash_device.h"

namespace flash {

template <class T> void launch_detect(const DevBatch<T>& B, const T* mu_env, hipStream_t s);
template <class T> void launch_finalize(const DevBatch<T>& B, const T* mu_env, hipStream_t s);
template <class T> void launch_gather(const DevBatch<T>& B, hipStream_t s);
template <class T> void launch_hinge(const DevBatch<T>& B, hipStream_t s);
// Orders the contact-solve workgroups longest-first from the previous step's solve times.
template <class T> void launch_order(const DevBatch<T>& B, hipStream_t s);
template <class T> void launch_project(const DevBatch<T>& B, hipStream_t s);
template <class T> void launch_assemble(const DevBatch<T>& B, hipStream_t s);
// Work list and tile parameters of the explicit-inverse products (apply and position update).
struct GemvSchedule {
  const int2* items;   // (env, first column) per workgroup, largest envs first
  int n_items;
  int vw;              // 0, 1, 2: 8, 16 or 32 bytes of columns per lane
  int unroll;          // 4 or 8 rows in flight per wave
};
template <class T> constexpr int gemv_tile(int vw) { return 64 * (int)((8 << vw) / sizeof(T)); }

template <class T> void launch_apply(const DevBatch<T>& B, const GemvSchedule& S, hipStream_t s);
template <class T> void launch_csp(const DevBatch<T>& B, const T* mu_env, int first_lg, hipStream_t s);
template <class T> void launch_correct(const DevBatch<T>& B, const GemvSchedule& S, hipStream_t s);
// The whole local-global loop of a step, one workgroup per env (bitwise equal to the
// kernel-per-phase sequence project, assemble, apply, csp, correct repeated K times).
template <class T> void launch_lg_fused(const DevBatch<T>& B, const T* mu_env, hipStream_t s);
// Raises the dynamic LDS limit of the contact-solve kernels for `cap` contacts per env.
template <class T> void prepare_csp(int cap, int rmax);

}  // namespace flash
