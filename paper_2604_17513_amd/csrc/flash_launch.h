// Host-callable launchers for the step kernels.
#pragma once
#include "flash_device.h"

namespace flash {

template <class T> void launch_detect(const DevBatch<T>& B, const T* mu_env, hipStream_t s);
template <class T> void launch_finalize(const DevBatch<T>& B, const T* mu_env, hipStream_t s);
template <class T> void launch_gather(const DevBatch<T>& B, hipStream_t s);
template <class T> void launch_hinge(const DevBatch<T>& B, hipStream_t s);
template <class T> void launch_project(const DevBatch<T>& B, hipStream_t s);
template <class T> void launch_assemble(const DevBatch<T>& B, hipStream_t s);
template <class T> void launch_apply(const DevBatch<T>& B, int max_ld, hipStream_t s);
template <class T> void launch_csp(const DevBatch<T>& B, const T* mu_env, int first_lg, hipStream_t s);
template <class T> void launch_correct(const DevBatch<T>& B, int max_ld, hipStream_t s);
// Raises the dynamic LDS limit of the contact-solve kernel for `cap` contacts per env.
template <class T> void prepare_csp(int cap, int rmax);

}  // namespace flash
