// Device-to-device state transfer between caller buffers and a batch's SoA state
// (positions q_h and velocities v_h of the implicit step, Eq. 1), with the
// precision conversion done on the device and the warm-start cache invalidation
// that every state change implies.
#include <hip/hip_runtime.h>

#include "flash_launch.h"

namespace flash {

namespace {

// dst[k * ldd + i] = src[k * lds + i] for the three components k, converted to D
template <class D, class S>
__global__ void k_copy_soa3(D* __restrict__ dst, long ldd, const S* __restrict__ src, long lds, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i < n) dst[(long)k * ldd + i] = (D)src[(long)k * lds + i];
}

// no previous-step multiplier for the n vertices (cache stamps -1), learned-start state cleared
__global__ void k_forget(int* __restrict__ stamp, int n_entries, int* __restrict__ ws_state, int n_envs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_entries) stamp[i] = -1;
  if (i < n_envs) ws_state[i] = 0;
}

template <class D, class S>
void copy3(D* dst, long ldd, const S* src, long lds, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_copy_soa3<D, S>), dim3((unsigned)((n + 255) / 256), 3), dim3(256), 0, s, dst, ldd, src, lds,
                     n);
}

}  // namespace

template <class T>
void launch_state_in(const DevBatch<T>& B, int vo, int n, int e0, int e1, const void* x, const void* v, int elem,
                     long lds, hipStream_t s) {
  if (elem == 4) {
    copy3(B.x + vo, B.NV, static_cast<const float*>(x), lds, n, s);
    if (v) copy3(B.v + vo, B.NV, static_cast<const float*>(v), lds, n, s);
  } else {
    copy3(B.x + vo, B.NV, static_cast<const double*>(x), lds, n, s);
    if (v) copy3(B.v + vo, B.NV, static_cast<const double*>(v), lds, n, s);
  }
  const int entries = n * kCacheSlots, ne = e1 - e0;
  const int m = entries > ne ? entries : ne;
  if (m > 0)
    hipLaunchKernelGGL(k_forget, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, B.cache_stamp + (long)vo * kCacheSlots,
                       entries, B.ws_state + e0, ne);
}

template <class T>
void launch_state_out(const DevBatch<T>& B, int vo, int n, void* x, void* v, int elem, long ldd, hipStream_t s) {
  if (elem == 4) {
    if (x) copy3(static_cast<float*>(x), ldd, B.x + vo, B.NV, n, s);
    if (v) copy3(static_cast<float*>(v), ldd, B.v + vo, B.NV, n, s);
  } else {
    if (x) copy3(static_cast<double*>(x), ldd, B.x + vo, B.NV, n, s);
    if (v) copy3(static_cast<double*>(v), ldd, B.v + vo, B.NV, n, s);
  }
}

template void launch_state_in<float>(const DevBatch<float>&, int, int, int, int, const void*, const void*, int, long,
                                     hipStream_t);
template void launch_state_in<double>(const DevBatch<double>&, int, int, int, int, const void*, const void*, int,
                                      long, hipStream_t);
template void launch_state_out<float>(const DevBatch<float>&, int, int, void*, void*, int, long, hipStream_t);
template void launch_state_out<double>(const DevBatch<double>&, int, int, void*, void*, int, long, hipStream_t);

}  // namespace flash
