// Batched depth ray casting of the envs' deformed surfaces (supplementary: depth simulation --
// depth maps, instance segmentation masks and point clouds cast from the simulation state).
//
// Create: per distinct surface topology a bounding-volume hierarchy over its triangles, built once
// on the host from the given rest shape (median split of triangle centroids along the longest axis,
// at most kLeafTris triangles per leaf, depth-first node order, nodes also listed level by level).
// Every frame: refit of each env's node boxes to its current vertex positions (one workgroup per
// env, deepest level first), then one thread per pixel traverses its env's hierarchy nearest child
// first (FP32 slab tests, Moller-Trumbore with a closed barycentric band so that rays along shared
// edges are caught) and tests the env's obstacles analytically (plane, box slabs, capsule).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/flash.h"
#include "flash_common.h"

namespace {

using flash::FlashError;

constexpr int kLeafTris = 4;
constexpr int kStack = 48;            // traversal stack; create rejects deeper hierarchies
constexpr int kTile = 16;             // pixels per side of one workgroup's tile
constexpr int kRefitBlock = 256;
constexpr float kEdgeBand = 1e-6f;    // barycentric band: FP32 solves of a ray on a shared edge

struct DevCam {
  float o[3], R[9], fx, fy, cx, cy;
};
struct DevObs {
  float c[3], R[9], size[3];
  int kind, pad[3];
};

struct Topo {
  int n_vertices = 0;
  std::vector<int32_t> tris;          // 3 per triangle, local ids, as given
  std::vector<int4> nodes;            // (left, right, first, count): count > 0 = leaf of tris first..
  std::vector<int32_t> order;         // triangles in leaf order (index into the given list)
  std::vector<int32_t> levels;        // node ids, deepest level first
  std::vector<int32_t> level_off;     // [n_levels + 1]
  int depth = 0;
  // device
  int4* d_nodes = nullptr;
  int* d_tri = nullptr;               // 3 per triangle, leaf order, local vertex ids
  int* d_levels = nullptr;
  int* d_level_off = nullptr;
};

// one env's part of a render
struct EnvRef {
  int topo;             // index of its topology
  int voff;             // first vertex column in x
  long long boxoff;     // first float of its node boxes (6 per node)
  int n_nodes;
  int n_levels;
};

// The triangles a body shows: membrane triangles as given, or the faces of a tet mesh that
// belong to exactly one tet (its boundary), in the tets' own vertex order.
std::vector<int32_t> surface_of(const flash_env_desc& d) {
  std::vector<int32_t> out;
  if (d.elem == FLASH_TRI) {
    out.assign(d.elements, d.elements + 3 * (size_t)d.n_elements);
    return out;
  }
  static const int F[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
  std::map<std::array<int32_t, 3>, int> count;
  for (int t = 0; t < d.n_elements; ++t)
    for (const auto& f : F) {
      std::array<int32_t, 3> key = {d.elements[4 * t + f[0]], d.elements[4 * t + f[1]], d.elements[4 * t + f[2]]};
      std::sort(key.begin(), key.end());
      count[key] += 1;
    }
  for (int t = 0; t < d.n_elements; ++t)
    for (const auto& f : F) {
      std::array<int32_t, 3> key = {d.elements[4 * t + f[0]], d.elements[4 * t + f[1]], d.elements[4 * t + f[2]]};
      std::sort(key.begin(), key.end());
      if (count[key] == 1)
        for (int a = 0; a < 3; ++a) out.push_back(d.elements[4 * t + f[a]]);
    }
  return out;
}

// Subtree over triangles order[lo, hi) at depth `level`; returns its node id.  Children follow
// their parent in depth-first order.
int build_node(Topo& T, const std::vector<float>& cen, int lo, int hi, int level, std::vector<int>& node_level) {
  if (level + 1 >= kStack) throw FlashError(FLASH_ERR_INVALID_ARG, "surface hierarchy too deep");
  const int id = (int)T.nodes.size();
  T.nodes.push_back(make_int4(-1, -1, lo, hi - lo));
  node_level.push_back(level);
  T.depth = std::max(T.depth, level);
  if (hi - lo <= kLeafTris) return id;
  float bl[3] = {INFINITY, INFINITY, INFINITY}, bh[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = lo; i < hi; ++i)
    for (int k = 0; k < 3; ++k) {
      bl[k] = std::min(bl[k], cen[3 * (size_t)T.order[i] + k]);
      bh[k] = std::max(bh[k], cen[3 * (size_t)T.order[i] + k]);
    }
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (bh[k] - bl[k] > bh[ax] - bl[ax]) ax = k;
  const int mid = lo + (hi - lo) / 2;
  std::nth_element(T.order.begin() + lo, T.order.begin() + mid, T.order.begin() + hi, [&](int a, int b) {
    const float ca = cen[3 * (size_t)a + ax], cb = cen[3 * (size_t)b + ax];
    return ca < cb || (ca == cb && a < b);
  });
  const int left = build_node(T, cen, lo, mid, level + 1, node_level);
  const int right = build_node(T, cen, mid, hi, level + 1, node_level);
  T.nodes[id] = make_int4(left, right, 0, 0);
  return id;
}

void build_bvh(Topo& T, const double* rest) {
  const int m = (int)(T.tris.size() / 3);
  std::vector<float> cen(3 * (size_t)m);
  for (int t = 0; t < m; ++t)
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += rest[3 * (size_t)T.tris[3 * t + a] + k];
      cen[3 * (size_t)t + k] = (float)(s / 3.0);
    }
  T.order.resize(m);
  for (int t = 0; t < m; ++t) T.order[t] = t;
  T.nodes.clear();
  T.depth = 0;
  std::vector<int> node_level;
  build_node(T, cen, 0, m, 0, node_level);
  // node ids by level, deepest first
  const int nn = (int)T.nodes.size();
  T.level_off.assign(T.depth + 2, 0);
  for (int i = 0; i < nn; ++i) T.level_off[T.depth - node_level[i] + 1] += 1;
  for (int l = 0; l <= T.depth; ++l) T.level_off[l + 1] += T.level_off[l];
  T.levels.assign(nn, 0);
  std::vector<int> fill(T.level_off.begin(), T.level_off.end() - 1);
  for (int i = 0; i < nn; ++i) T.levels[fill[T.depth - node_level[i]]++] = i;
}

// ---------------------------------------------------------------------------------------------
// device

__device__ __forceinline__ float3 vtx(const float* x, long long ld, int col) {
  return make_float3(x[col], x[ld + col], x[2 * ld + col]);
}

// Node boxes of one env, one workgroup, deepest level first (a node's children are deeper).
__global__ void __launch_bounds__(kRefitBlock) k_refit(const float* __restrict__ x, long long ld,
                                                       const EnvRef* __restrict__ envs, const int4* const* nodes_of,
                                                       const int* const* tri_of, const int* const* levels_of,
                                                       const int* const* level_off_of, float* __restrict__ boxes) {
  const EnvRef E = envs[blockIdx.x];
  const int4* nodes = nodes_of[E.topo];
  const int* tri = tri_of[E.topo];
  const int* levels = levels_of[E.topo];
  const int* loff = level_off_of[E.topo];
  float* bx = boxes + E.boxoff;
  for (int l = 0; l < E.n_levels; ++l) {
    for (int q = loff[l] + threadIdx.x; q < loff[l + 1]; q += kRefitBlock) {
      const int i = levels[q];
      const int4 nd = nodes[i];
      float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY, hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
      if (nd.w > 0) {
        for (int t = nd.z; t < nd.z + nd.w; ++t)
          for (int a = 0; a < 3; ++a) {
            const float3 p = vtx(x, ld, E.voff + tri[3 * t + a]);
            lo0 = fminf(lo0, p.x); lo1 = fminf(lo1, p.y); lo2 = fminf(lo2, p.z);
            hi0 = fmaxf(hi0, p.x); hi1 = fmaxf(hi1, p.y); hi2 = fmaxf(hi2, p.z);
          }
      } else {
        const float* a = bx + 6 * (size_t)nd.x;
        const float* b = bx + 6 * (size_t)nd.y;
        lo0 = fminf(a[0], b[0]); lo1 = fminf(a[1], b[1]); lo2 = fminf(a[2], b[2]);
        hi0 = fmaxf(a[3], b[3]); hi1 = fmaxf(a[4], b[4]); hi2 = fmaxf(a[5], b[5]);
      }
      float* o = bx + 6 * (size_t)i;
      o[0] = lo0; o[1] = lo1; o[2] = lo2; o[3] = hi0; o[4] = hi1; o[5] = hi2;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ float slab_entry(const float* b, float3 o, float3 inv, float tmax) {
  float t0 = (b[0] - o.x) * inv.x, t1 = (b[3] - o.x) * inv.x;
  float tn = fminf(t0, t1), tf = fmaxf(t0, t1);
  t0 = (b[1] - o.y) * inv.y; t1 = (b[4] - o.y) * inv.y;
  tn = fmaxf(tn, fminf(t0, t1)); tf = fminf(tf, fmaxf(t0, t1));
  t0 = (b[2] - o.z) * inv.z; t1 = (b[5] - o.z) * inv.z;
  tn = fmaxf(tn, fminf(t0, t1)); tf = fminf(tf, fmaxf(t0, t1));
  tn = fmaxf(tn, 0.0f);
  return (tn <= tf && tn < tmax) ? tn : INFINITY;
}

__device__ __forceinline__ float tri_hit(float3 o, float3 d, float3 A, float3 B, float3 C) {
  const float3 e1 = make_float3(B.x - A.x, B.y - A.y, B.z - A.z);
  const float3 e2 = make_float3(C.x - A.x, C.y - A.y, C.z - A.z);
  const float3 P = make_float3(d.y * e2.z - d.z * e2.y, d.z * e2.x - d.x * e2.z, d.x * e2.y - d.y * e2.x);
  const float det = P.x * e1.x + P.y * e1.y + P.z * e1.z;
  if (det == 0.0f) return INFINITY;
  const float inv = 1.0f / det;
  const float3 s = make_float3(o.x - A.x, o.y - A.y, o.z - A.z);
  const float b1 = (P.x * s.x + P.y * s.y + P.z * s.z) * inv;
  const float3 Q = make_float3(s.y * e1.z - s.z * e1.y, s.z * e1.x - s.x * e1.z, s.x * e1.y - s.y * e1.x);
  const float b2 = (d.x * Q.x + d.y * Q.y + d.z * Q.z) * inv;
  const float t = (e2.x * Q.x + e2.y * Q.y + e2.z * Q.z) * inv;
  const bool hit = b1 >= -kEdgeBand && b2 >= -kEdgeBand && b1 + b2 <= 1.0f + kEdgeBand && t > 0.0f;
  return hit ? t : INFINITY;
}

// nearest t > 0 of the ray with one obstacle (INFINITY: none)
__device__ float obstacle_hit(const DevObs& ob, float3 o, float3 d) {
  const float* R = ob.R;
  if (ob.kind == FLASH_PLANE) {
    const float n0 = R[1], n1 = R[4], n2 = R[7];
    const float dn = d.x * n0 + d.y * n1 + d.z * n2;
    if (dn == 0.0f) return INFINITY;
    const float t = ((ob.c[0] - o.x) * n0 + (ob.c[1] - o.y) * n1 + (ob.c[2] - o.z) * n2) / dn;
    return t > 0.0f ? t : INFINITY;
  }
  // ray in the obstacle frame: ol = R^T (o - c), dl = R^T d
  const float r0 = o.x - ob.c[0], r1 = o.y - ob.c[1], r2 = o.z - ob.c[2];
  float ol[3], dl[3];
  for (int k = 0; k < 3; ++k) {
    ol[k] = R[k] * r0 + R[3 + k] * r1 + R[6 + k] * r2;
    dl[k] = R[k] * d.x + R[3 + k] * d.y + R[6 + k] * d.z;
  }
  if (ob.kind == FLASH_BOX) {
    float tn = -INFINITY, tf = INFINITY;
    for (int k = 0; k < 3; ++k) {
      const float e = ob.size[k];
      if (dl[k] == 0.0f) {
        if (fabsf(ol[k]) > e) return INFINITY;
        continue;
      }
      const float inv = 1.0f / dl[k];
      const float t0 = (-e - ol[k]) * inv, t1 = (e - ol[k]) * inv;
      tn = fmaxf(tn, fminf(t0, t1));
      tf = fminf(tf, fmaxf(t0, t1));
    }
    if (tn > tf) return INFINITY;
    const float t = tn > 0.0f ? tn : tf;
    return t > 0.0f ? t : INFINITY;
  }
  // capsule: radius size[0] around the local x axis, half-length size[1]
  const float rad = ob.size[0], half = ob.size[1];
  float best = INFINITY;
  const float a = dl[1] * dl[1] + dl[2] * dl[2];
  if (a > 0.0f) {
    const float b = 2.0f * (ol[1] * dl[1] + ol[2] * dl[2]);
    const float cc = ol[1] * ol[1] + ol[2] * ol[2] - rad * rad;
    const float disc = b * b - 4.0f * a * cc;
    if (disc >= 0.0f) {
      const float sq = sqrtf(disc);
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const float t = (-b + (float)sgn * sq) / (2.0f * a);
        const float x0 = ol[0] + t * dl[0];
        if (t > 0.0f && fabsf(x0) <= half && t < best) best = t;
      }
    }
  }
  const float dd = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
  for (int end = -1; end <= 1; end += 2) {
    const float oc0 = ol[0] - (float)end * half, oc1 = ol[1], oc2 = ol[2];
    const float bb = dl[0] * oc0 + dl[1] * oc1 + dl[2] * oc2;
    const float c2 = oc0 * oc0 + oc1 * oc1 + oc2 * oc2 - rad * rad;
    const float disc = bb * bb - dd * c2;
    if (disc < 0.0f) continue;
    const float sq = sqrtf(disc);
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      const float t = (-bb + (float)sgn * sq) / dd;
      if (t > 0.0f && t < best) best = t;
    }
  }
  return best;
}

// one workgroup renders one 16 x 16 tile of one env's image
__global__ void __launch_bounds__(kTile * kTile) k_render(const float* __restrict__ x, long long ld,
                                                          const EnvRef* __restrict__ envs,
                                                          const int4* const* nodes_of, const int* const* tri_of,
                                                          const float* __restrict__ boxes, const DevCam* __restrict__ cams,
                                                          const DevObs* __restrict__ obs, const int* __restrict__ nobs,
                                                          int width, int height, int tiles_x, float* depth,
                                                          int* inst, float* pts) {
  const int e = blockIdx.y;
  const int tile = blockIdx.x;
  const int u = (tile % tiles_x) * kTile + (threadIdx.x % kTile);
  const int v = (tile / tiles_x) * kTile + (threadIdx.x / kTile);
  if (u >= width || v >= height) return;
  const EnvRef E = envs[e];
  const DevCam cam = cams[e];
  const float xn = ((float)u + 0.5f - cam.cx) / cam.fx;
  const float yn = ((float)v + 0.5f - cam.cy) / cam.fy;
  const float3 o = make_float3(cam.o[0], cam.o[1], cam.o[2]);
  const float3 d = make_float3(cam.R[0] * xn + cam.R[1] * yn + cam.R[2], cam.R[3] * xn + cam.R[4] * yn + cam.R[5],
                               cam.R[6] * xn + cam.R[7] * yn + cam.R[8]);
  const float3 inv = make_float3(1.0f / d.x, 1.0f / d.y, 1.0f / d.z);
  float tbest = INFINITY;
  int ibest = -1;
  if (E.n_nodes > 0) {
    const int4* nodes = nodes_of[E.topo];
    const int* tri = tri_of[E.topo];
    const float* bx = boxes + E.boxoff;
    int stack[kStack];
    int sp = 0;
    if (slab_entry(bx, o, inv, tbest) < INFINITY) stack[sp++] = 0;
    while (sp > 0) {
      const int i = stack[--sp];
      const int4 nd = nodes[i];
      if (nd.w > 0) {
        for (int t = nd.z; t < nd.z + nd.w; ++t) {
          const float th = tri_hit(o, d, vtx(x, ld, E.voff + tri[3 * t]), vtx(x, ld, E.voff + tri[3 * t + 1]),
                                   vtx(x, ld, E.voff + tri[3 * t + 2]));
          if (th < tbest) { tbest = th; ibest = 0; }
        }
        continue;
      }
      const float ta = slab_entry(bx + 6 * (size_t)nd.x, o, inv, tbest);
      const float tb = slab_entry(bx + 6 * (size_t)nd.y, o, inv, tbest);
      // nearer child on top of the stack
      if (ta <= tb) {
        if (tb < INFINITY) stack[sp++] = nd.y;
        if (ta < INFINITY) stack[sp++] = nd.x;
      } else {
        if (ta < INFINITY) stack[sp++] = nd.x;
        if (tb < INFINITY) stack[sp++] = nd.y;
      }
    }
  }
  const int no = nobs[e];
  for (int q = 0; q < no; ++q) {
    const float th = obstacle_hit(obs[(size_t)e * FLASH_MAX_OBSTACLES + q], o, d);
    if (th < tbest) { tbest = th; ibest = 1 + q; }
  }
  const size_t px = ((size_t)e * height + v) * width + u;
  const bool hit = ibest >= 0;
  if (depth) depth[px] = hit ? tbest : 0.0f;
  if (inst) inst[px] = ibest;
  if (pts) {
    pts[3 * px] = hit ? o.x + tbest * d.x : 0.0f;
    pts[3 * px + 1] = hit ? o.y + tbest * d.y : 0.0f;
    pts[3 * px + 2] = hit ? o.z + tbest * d.z : 0.0f;
  }
}

}  // namespace

struct flash_renderer {
  int n_envs = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<Topo> topos;
  std::vector<EnvRef> envs;
  std::vector<int> voff;
  long long n_boxes_f = 0;
  std::vector<void*> owned;
  EnvRef* d_envs = nullptr;
  const int4** d_nodes_of = nullptr;
  const int** d_tri_of = nullptr;
  const int** d_levels_of = nullptr;
  const int** d_level_off_of = nullptr;
  float* d_boxes = nullptr;
  DevCam* d_cams = nullptr;
  DevObs* d_obs = nullptr;
  int* d_nobs = nullptr;
  std::vector<DevCam> h_cams;
  std::vector<DevObs> h_obs;
  std::vector<int> h_nobs;

  ~flash_renderer() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : owned) (void)hipFree(p);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
  template <class X>
  X* alloc(size_t n) {
    void* p = nullptr;
    HIPCHK(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(X)));
    owned.push_back(p);
    return static_cast<X*>(p);
  }
};

extern "C" {

flash_status flash_renderer_create(const flash_env_desc* descs, int32_t n_envs, void* hip_stream,
                                   flash_renderer** out) {
  if (!out || !descs || n_envs <= 0) return flash::record_error(FLASH_ERR_INVALID_ARG, "null argument or n_envs <= 0");
  *out = nullptr;
  std::vector<std::vector<int32_t>> surf(n_envs);
  std::vector<int> n_vertices(n_envs), n_tris(n_envs);
  for (int e = 0; e < n_envs; ++e) {
    const flash_env_desc& d = descs[e];
    const int k = d.elem == FLASH_TET ? 4 : 3;
    if ((d.elem != FLASH_TET && d.elem != FLASH_TRI) || d.n_vertices <= 0 || d.n_elements <= 0 || !d.rest_x ||
        !d.elements)
      return flash::record_error(FLASH_ERR_INVALID_ARG, "invalid surface of env " + std::to_string(e));
    for (int64_t q = 0; q < (int64_t)k * d.n_elements; ++q)
      if (d.elements[q] < 0 || d.elements[q] >= d.n_vertices)
        return flash::record_error(FLASH_ERR_INVALID_ARG, "element vertex out of range in env " + std::to_string(e));
    surf[e] = surface_of(d);
    n_vertices[e] = d.n_vertices;
    n_tris[e] = (int)(surf[e].size() / 3);
  }
  flash_renderer* r = new flash_renderer();
  try {
    r->n_envs = n_envs;
    if (hip_stream) r->stream = static_cast<hipStream_t>(hip_stream);
    else { HIPCHK(hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking)); r->own_stream = true; }
    r->voff.assign(n_envs + 1, 0);
    for (int e = 0; e < n_envs; ++e) r->voff[e + 1] = r->voff[e] + n_vertices[e];
    // topologies: equal triangle lists over equal vertex counts share one hierarchy
    std::map<std::pair<int, int>, std::vector<int>> seen;
    for (int e = 0; e < n_envs; ++e) {
      int id = -1;
      for (int t : seen[{n_vertices[e], n_tris[e]}]) {
        const Topo& T = r->topos[t];
        if (T.tris == surf[e]) { id = t; break; }
      }
      if (id < 0) {
        Topo T;
        T.n_vertices = n_vertices[e];
        T.tris = surf[e];
        if (n_tris[e] > 0) build_bvh(T, descs[e].rest_x);
        id = (int)r->topos.size();
        r->topos.push_back(std::move(T));
        seen[{n_vertices[e], n_tris[e]}].push_back(id);
      }
      EnvRef E{};
      E.topo = id;
      E.voff = r->voff[e];
      E.boxoff = r->n_boxes_f;
      E.n_nodes = (int)r->topos[id].nodes.size();
      E.n_levels = r->topos[id].nodes.empty() ? 0 : r->topos[id].depth + 1;
      r->n_boxes_f += 6 * (long long)E.n_nodes;
      r->envs.push_back(E);
    }
    std::vector<const int4*> nodes_of;
    std::vector<const int*> tri_of, levels_of, loff_of;
    for (Topo& T : r->topos) {
      const size_t m = T.tris.size() / 3;
      std::vector<int> tri_leaf(3 * m);
      for (size_t i = 0; i < T.order.size(); ++i)
        for (int a = 0; a < 3; ++a) tri_leaf[3 * i + a] = T.tris[3 * (size_t)T.order[i] + a];
      T.d_nodes = r->alloc<int4>(T.nodes.size());
      T.d_tri = r->alloc<int>(tri_leaf.size());
      T.d_levels = r->alloc<int>(T.levels.size());
      T.d_level_off = r->alloc<int>(T.level_off.size());
      if (!T.nodes.empty()) {
        HIPCHK(hipMemcpy(T.d_nodes, T.nodes.data(), T.nodes.size() * sizeof(int4), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(T.d_tri, tri_leaf.data(), tri_leaf.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(T.d_levels, T.levels.data(), T.levels.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(T.d_level_off, T.level_off.data(), T.level_off.size() * sizeof(int), hipMemcpyHostToDevice));
      }
      nodes_of.push_back(T.d_nodes);
      tri_of.push_back(T.d_tri);
      levels_of.push_back(T.d_levels);
      loff_of.push_back(T.d_level_off);
    }
    const size_t nt = r->topos.size();
    r->d_nodes_of = const_cast<const int4**>(r->alloc<const int4*>(nt));
    r->d_tri_of = const_cast<const int**>(r->alloc<const int*>(nt));
    r->d_levels_of = const_cast<const int**>(r->alloc<const int*>(nt));
    r->d_level_off_of = const_cast<const int**>(r->alloc<const int*>(nt));
    HIPCHK(hipMemcpy((void*)r->d_nodes_of, nodes_of.data(), nt * sizeof(void*), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy((void*)r->d_tri_of, tri_of.data(), nt * sizeof(void*), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy((void*)r->d_levels_of, levels_of.data(), nt * sizeof(void*), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy((void*)r->d_level_off_of, loff_of.data(), nt * sizeof(void*), hipMemcpyHostToDevice));
    r->d_envs = r->alloc<EnvRef>(n_envs);
    HIPCHK(hipMemcpy(r->d_envs, r->envs.data(), n_envs * sizeof(EnvRef), hipMemcpyHostToDevice));
    r->d_boxes = r->alloc<float>((size_t)r->n_boxes_f);
    r->d_cams = r->alloc<DevCam>(n_envs);
    r->d_obs = r->alloc<DevObs>((size_t)n_envs * FLASH_MAX_OBSTACLES);
    r->d_nobs = r->alloc<int>(n_envs);
    r->h_cams.resize(n_envs);
    r->h_obs.resize((size_t)n_envs * FLASH_MAX_OBSTACLES);
    r->h_nobs.resize(n_envs);
  } catch (const FlashError& ex) {
    delete r;
    return flash::record_error(ex.st, ex.what());
  }
  *out = r;
  return FLASH_OK;
}

flash_status flash_renderer_destroy(flash_renderer* r) {
  if (!r) return flash::record_error(FLASH_ERR_INVALID_ARG, "null renderer");
  delete r;
  return FLASH_OK;
}

flash_status flash_render(flash_renderer* r, const float* x_dev, int64_t ld, const flash_obstacle* obstacles,
                          const int32_t* n_obstacles, const flash_camera* cams, int32_t width, int32_t height,
                          float* depth_dev, int32_t* instance_dev, float* points_dev) {
  if (!r || !cams || width <= 0 || height <= 0 || (!x_dev && r->voff.back() > 0))
    return flash::record_error(FLASH_ERR_INVALID_ARG, "null renderer, cameras or positions, or empty image");
  if (ld < r->voff.back()) return flash::record_error(FLASH_ERR_INVALID_ARG, "ld below the total vertex count");
  const int ne = r->n_envs;
  for (int e = 0; e < ne; ++e) {
    const int no = n_obstacles ? n_obstacles[e] : 0;
    if (no < 0 || no > FLASH_MAX_OBSTACLES || (no > 0 && !obstacles))
      return flash::record_error(FLASH_ERR_INVALID_ARG, "invalid obstacle count of env " + std::to_string(e));
    if (!(cams[e].fx > 0) || !(cams[e].fy > 0))
      return flash::record_error(FLASH_ERR_INVALID_ARG, "camera focal lengths must be positive");
    DevCam& c = r->h_cams[e];
    for (int k = 0; k < 3; ++k) c.o[k] = (float)cams[e].position[k];
    for (int k = 0; k < 9; ++k) c.R[k] = (float)cams[e].rot[k];
    c.fx = (float)cams[e].fx; c.fy = (float)cams[e].fy; c.cx = (float)cams[e].cx; c.cy = (float)cams[e].cy;
    r->h_nobs[e] = no;
    for (int q = 0; q < no; ++q) {
      const flash_obstacle& ob = obstacles[(size_t)e * FLASH_MAX_OBSTACLES + q];
      if (ob.kind != FLASH_PLANE && ob.kind != FLASH_BOX && ob.kind != FLASH_CAPSULE)
        return flash::record_error(FLASH_ERR_INVALID_ARG, "unknown obstacle kind");
      DevObs& d = r->h_obs[(size_t)e * FLASH_MAX_OBSTACLES + q];
      for (int k = 0; k < 3; ++k) { d.c[k] = (float)ob.center[k]; d.size[k] = (float)ob.size[k]; }
      for (int k = 0; k < 9; ++k) d.R[k] = (float)ob.rot[k];
      d.kind = ob.kind;
    }
  }
  try {
    HIPCHK(hipMemcpyAsync(r->d_cams, r->h_cams.data(), ne * sizeof(DevCam), hipMemcpyHostToDevice, r->stream));
    HIPCHK(hipMemcpyAsync(r->d_obs, r->h_obs.data(), r->h_obs.size() * sizeof(DevObs), hipMemcpyHostToDevice,
                          r->stream));
    HIPCHK(hipMemcpyAsync(r->d_nobs, r->h_nobs.data(), ne * sizeof(int), hipMemcpyHostToDevice, r->stream));
    hipLaunchKernelGGL(k_refit, dim3(ne), dim3(kRefitBlock), 0, r->stream, x_dev, (long long)ld, r->d_envs,
                       r->d_nodes_of, r->d_tri_of, r->d_levels_of, r->d_level_off_of, r->d_boxes);
    const int tx = (width + kTile - 1) / kTile, ty = (height + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_render, dim3((unsigned)(tx * ty), (unsigned)ne), dim3(kTile * kTile), 0, r->stream, x_dev,
                       (long long)ld, r->d_envs, r->d_nodes_of, r->d_tri_of, (const float*)r->d_boxes, r->d_cams,
                       r->d_obs, r->d_nobs, width, height, tx, depth_dev, instance_dev, points_dev);
    HIPCHK(hipGetLastError());
    // the host staging arrays are reused by the next call: let the copies finish
    HIPCHK(hipStreamSynchronize(r->stream));
  } catch (const FlashError& ex) {
    return flash::record_error(ex.st, ex.what());
  }
  return FLASH_OK;
}

}  // extern "C"
