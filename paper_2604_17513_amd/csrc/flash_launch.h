// Host-callable launchers for the step kernels.
#pragma once
#include "flash_device.h"

namespace flash {

// State of vertices [vo, vo + n) (envs [e0, e1)) from / to caller device arrays [3][lds] of
// float (elem 4) or double (elem 8); state_in also forgets the warm-start history of those
// vertices and envs.
template <class T> void launch_state_in(const DevBatch<T>& B, int vo, int n, int e0, int e1, const void* x,
                                        const void* v, int elem, long lds, hipStream_t s);
template <class T> void launch_state_out(const DevBatch<T>& B, int vo, int n, void* x, void* v, int elem, long ldd,
                                         hipStream_t s);
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

// Row-split explicit-inverse products of the global-memory lightweight route: each workgroup sums
// one split of an env's rows (split_rows) for one column tile of 64 x 16 bytes into a partial, and a
// merge pass adds an env's partials in split order.  The split depends only on the env's own sizes,
// so an env gives the same bits alone or in any batch.
constexpr int kSplitRows = 512;   // rows staged in LDS at a time; the least rows per split
constexpr int kMaxSplits = 16;    // splits per env beyond which the splits grow instead
template <class T> constexpr int split_tile() { return 64 * (int)(16 / sizeof(T)); }
// Rows per split of an env whose products read at most `rows` rows: kSplitRows, or larger (a
// multiple of kSplitRows) so that there are at most about kMaxSplits splits.  A function of the
// env's own sizes only.
__host__ __device__ inline int split_rows(int rows) {
  const int per = (rows + kMaxSplits - 1) / kMaxSplits;
  const int r = (per + kSplitRows - 1) / kSplitRows * kSplitRows;
  return r > kSplitRows ? r : kSplitRows;
}
// The most rows an env's products read: its vertices (the apply) or its contact rows (position
// update), at most kCacheSlots per vertex.
__host__ __device__ inline int split_cover(int n, int cap) {
  const int c = cap < kCacheSlots * n ? cap : kCacheSlots * n;
  return n > c ? n : c;
}
// Envs that share one inverse (identical mesh and material) run their split products in chunks of
// up to kTwinChunk envs per workgroup: each inverse row vector loaded serves the whole chunk.
constexpr int kTwinChunk = 8;
struct SplitSchedule {
  const int4* items;       // (env, first column, split, 0) per workgroup, envs without a twin
  int n_items;
  const int4* twin_items;  // (first env of the chunk in twin_envs, first column, split, envs in the
                           // chunk; 0 pads) per workgroup, envs that share their inverse
  int n_twin_items;
  const int* twin_envs;    // chunks of envs sharing one inverse, in batch order within a group
  void* partial;           // T [sum over envs of splits x 3 x n]
  const int64_t* poff;     // [n_envs] element offset of each env's partials
};
template <class T> void launch_split_apply(const DevBatch<T>& B, const SplitSchedule& S, hipStream_t s);
template <class T> void launch_split_correct(const DevBatch<T>& B, const SplitSchedule& S, const int* skip,
                                             hipStream_t s);

template <class T> void launch_apply(const DevBatch<T>& B, const GemvSchedule& S, hipStream_t s);
template <class T> void launch_csp(const DevBatch<T>& B, const T* mu_env, int first_lg, hipStream_t s);
// skip (optional): envs with skip[e] != 0 keep their u
template <class T> void launch_correct(const DevBatch<T>& B, const GemvSchedule& S, hipStream_t s,
                                       const int* skip = nullptr);
// lightweight update in global memory: it = -1 prepares the warm start's forces (once per step),
// it >= 0 is the (it + 1)-th residual evaluation of local-global iteration k (an update unless the
// iteration stops)
template <class T> void launch_lite_update(const DevBatch<T>& B, const T* mu_env, int k, int it, int first_lg,
                                           hipStream_t s);
// The whole local-global loop of a step, one workgroup per env (bitwise equal to the
// kernel-per-phase sequence project, assemble, apply, csp, correct repeated K times).
template <class T> void launch_lg_fused(const DevBatch<T>& B, const T* mu_env, hipStream_t s);
// Contact capacity per env (0 asks for the default), rows of the largest capacitance system
// one contact solve factors, and the rows of its LU panel staged in LDS.
inline int csp_capacity(int requested) { return requested > 0 ? requested : 320; }
inline int csp_rows(int cap) { return 3 * cap < 1536 ? 3 * cap : 1536; }
inline int csp_lds_rows(int rmax) { return rmax < 480 ? rmax : 480; }
// Dynamic LDS of one contact solve in its precision CT: FP64 multipliers (3 per contact), the
// per-contact frames, Jacobian and E blocks (28 values), the staged LU panel (rlds rows of
// kBK + 2), contact indices (3 per contact) and a 64-value reduction area.
template <class CT>
__host__ __device__ constexpr size_t csp_smem_bytes(int cap, int rlds) {
  return (size_t)cap * 3 * sizeof(double) + (size_t)cap * (24 + 4) * sizeof(CT) + (size_t)rlds * (kBK + 2) * sizeof(CT) +
         (size_t)cap * 3 * sizeof(int) + 64 * sizeof(double);
}
// LDS of one gfx950 CU: the most one workgroup can be given, static and dynamic together.
constexpr size_t kLdsBytes = 160 * 1024;
// Reserve for the static LDS of the contact-solve kernels (k_csp and the fused loop: 4160 bytes
// with the FP64 contact solve, 2112 with the FP32 one); create checks the kernels' real static
// LDS against it.
constexpr size_t kCspStaticLds = 8192;
// Raises the dynamic LDS limit of the contact-solve kernels (both contact-solve precisions, per
// kernel and process-wide) to what a CU leaves beside the static reserve, the bound that create
// checks every capacity against, so batches of different capacities never lower it for each
// other; *static_lds receives the largest static LDS of those kernels as the runtime reports it
// (create fails if it exceeds the reserve); returns the first error of the runtime calls.
template <class T> hipError_t prepare_csp(size_t* static_lds);

}  // namespace flash
