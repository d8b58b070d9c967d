// C ABI of the FLASH step library: create-time precompute, device buffers,
// step enqueue (plain one-launch-per-phase schedule or a captured HIP graph),
// state / contact / residual queries and per-kernel event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/flash.h"
#include "flash_common.h"
#include "flash_device.h"
#include "flash_launch.h"
#include "flash_mlp.h"

using namespace flash;

namespace {
thread_local std::string g_err;
}  // namespace

flash_status flash::record_error(flash_status s, const std::string& m) {
  g_err = m;
  return s;
}

namespace {

flash_status fail(flash_status s, const std::string& m) { return record_error(s, m); }

// ----------------------------------------------------------------------------
// Create-time precompute (FP64, host).  Per env: oriented elements, D_m^-1,
// weights, lumped masses, the scalar system matrix Abar (A = Abar (x) I3,
// Eq. 4), its skyline Cholesky factor and the explicit inverse Gbar = Abar^-1
// (the paper forms A^-1 = S^T S from the inverse Cholesky factor, Alg. 1;
// here the product is formed once so that each global solve is one symmetric
// sweep and the contact-space Delassus operator is a gather).
// ----------------------------------------------------------------------------
struct HostEnv {
  int n = 0, m = 0, k = 4;
  std::vector<int> elem;      // 4 per element: oriented tet, or triangle + (-1)
  std::vector<double> Bm;     // 9 per element: D_m^-1 (tets, 3x3) or the 2x2 D_m^-1 in entries 0..3 (triangles)
  std::vector<double> w;      // per element
  std::vector<double> mass;   // per vertex
  std::vector<int> hidx;      // 4 per bending hinge (edge x0 x1, opposite x2 x3)
  std::vector<double> halpha; // 4 per hinge
  std::vector<double> hw;     // per hinge
  std::vector<double> Ginv;   // n*n symmetric (empty when twin >= 0)
  int twin = -1;              // an earlier env of the batch with the same mesh and material, whose
                              // explicit inverse this env shares
};

// The system matrix depends on the mesh, the material and h only (not on mu): envs equal in these
// share one inverse.  FNV-1a over the defining values; same_model confirms a key match.
uint64_t model_key(const flash_env_desc& d) {
  uint64_t hsh = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) { hsh ^= c[i]; hsh *= 1099511628211ull; }
  };
  const int k = d.elem == FLASH_TET ? 4 : 3;
  mix(&d.elem, sizeof(d.elem));
  mix(&d.n_vertices, sizeof(d.n_vertices));
  mix(&d.n_elements, sizeof(d.n_elements));
  mix(d.rest_x, 3 * (size_t)d.n_vertices * sizeof(double));
  mix(d.elements, (size_t)k * d.n_elements * sizeof(int32_t));
  const double sc[5] = {d.density, d.elem == FLASH_TRI ? d.thickness : 0.0, d.young, d.poisson,
                        d.elem == FLASH_TRI ? d.bending : 0.0};
  mix(sc, sizeof(sc));
  return hsh;
}

bool same_model(const flash_env_desc& a, const flash_env_desc& b) {
  if (a.elem != b.elem || a.n_vertices != b.n_vertices || a.n_elements != b.n_elements) return false;
  const int k = a.elem == FLASH_TET ? 4 : 3;
  if (std::memcmp(a.rest_x, b.rest_x, 3 * (size_t)a.n_vertices * sizeof(double)) != 0) return false;
  if (std::memcmp(a.elements, b.elements, (size_t)k * a.n_elements * sizeof(int32_t)) != 0) return false;
  if (a.density != b.density || a.young != b.young || a.poisson != b.poisson) return false;
  if (a.elem == FLASH_TRI && (a.thickness != b.thickness || a.bending != b.bending)) return false;
  return true;
}

void tet_data(const flash_env_desc& d, HostEnv& H) {
  const int n = d.n_vertices, m = d.n_elements;
  H.n = n; H.m = m; H.k = 4;
  H.elem.assign(d.elements, d.elements + 4 * (size_t)m);
  H.Bm.resize(9 * (size_t)m);
  H.w.resize(m);
  H.mass.assign(n, 0.0);
  const double muL = d.young / (2.0 * (1.0 + d.poisson));
  for (int t = 0; t < m; ++t) {
    int* id = &H.elem[4 * (size_t)t];
    for (int a = 0; a < 4; ++a)
      if (id[a] < 0 || id[a] >= n) throw FlashError(FLASH_ERR_INVALID_ARG, "element index out of range");
    double D[9];
    auto fill = [&]() {
      for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r) D[3 * r + a] = d.rest_x[3 * id[a + 1] + r] - d.rest_x[3 * id[0] + r];
    };
    fill();
    double det = D[0] * (D[4] * D[8] - D[5] * D[7]) - D[1] * (D[3] * D[8] - D[5] * D[6]) +
                 D[2] * (D[3] * D[7] - D[4] * D[6]);
    if (det < 0) { std::swap(id[2], id[3]); fill(); det = -det; }
    if (!(det > 0)) throw FlashError(FLASH_ERR_INVALID_ARG, "degenerate rest tet");
    double* Bt = &H.Bm[9 * (size_t)t];
    Bt[0] = (D[4] * D[8] - D[5] * D[7]) / det;
    Bt[1] = (D[2] * D[7] - D[1] * D[8]) / det;
    Bt[2] = (D[1] * D[5] - D[2] * D[4]) / det;
    Bt[3] = (D[5] * D[6] - D[3] * D[8]) / det;
    Bt[4] = (D[0] * D[8] - D[2] * D[6]) / det;
    Bt[5] = (D[2] * D[3] - D[0] * D[5]) / det;
    Bt[6] = (D[3] * D[7] - D[4] * D[6]) / det;
    Bt[7] = (D[1] * D[6] - D[0] * D[7]) / det;
    Bt[8] = (D[0] * D[4] - D[1] * D[3]) / det;
    const double V = det / 6.0;
    H.w[t] = 2.0 * muL * V;
    for (int a = 0; a < 4; ++a) H.mass[id[a]] += d.density * V / 4.0;
  }
}

// Membrane triangles (Sec. III-B projective constraints with the closest matrix of
// orthonormal columns): rest frame e1 = unit(X1 - X0), n = unit((X1 - X0) x (X2 - X0)),
// e2 = n x e1; D_m = rest edge coordinates in (e1, e2), B = D_m^-1; F = [x1 - x0 | x2 - x0] B;
// w = 2 mu_L A t; lumped mass rho t A / 3 per vertex.  Bending hinges on interior edges,
// flat rest state, target p = 0: G_h q = sum alpha_a x_a with alpha_2 = 1/d_2,
// alpha_3 = 1/d_3 (rest distances of the opposite vertices to the edge line) and
// alpha_0, alpha_1 from sum alpha = 0, sum alpha X = 0; w_h = 3 k_b |e|^2 / (A_1 + A_2).
void tri_data(const flash_env_desc& d, HostEnv& H) {
  const int n = d.n_vertices, m = d.n_elements;
  H.n = n; H.m = m; H.k = 3;
  H.elem.assign(4 * (size_t)m, -1);
  H.Bm.assign(9 * (size_t)m, 0.0);
  H.w.resize(m);
  H.mass.assign(n, 0.0);
  const double muL = d.young / (2.0 * (1.0 + d.poisson));
  auto X = [&](int v, int c) { return d.rest_x[3 * (size_t)v + c]; };
  std::vector<double> area(m);
  for (int t = 0; t < m; ++t) {
    int id[3];
    for (int a = 0; a < 3; ++a) {
      id[a] = d.elements[3 * (size_t)t + a];
      if (id[a] < 0 || id[a] >= n) throw FlashError(FLASH_ERR_INVALID_ARG, "element index out of range");
      H.elem[4 * (size_t)t + a] = id[a];
    }
    double E1[3], E2[3], nn[3], e1[3], e2[3];
    for (int c = 0; c < 3; ++c) { E1[c] = X(id[1], c) - X(id[0], c); E2[c] = X(id[2], c) - X(id[0], c); }
    nn[0] = E1[1] * E2[2] - E1[2] * E2[1];
    nn[1] = E1[2] * E2[0] - E1[0] * E2[2];
    nn[2] = E1[0] * E2[1] - E1[1] * E2[0];
    const double l1 = std::sqrt(E1[0] * E1[0] + E1[1] * E1[1] + E1[2] * E1[2]);
    const double ln = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    if (!(l1 > 0) || !(ln > 0)) throw FlashError(FLASH_ERR_INVALID_ARG, "degenerate rest triangle");
    for (int c = 0; c < 3; ++c) { e1[c] = E1[c] / l1; nn[c] /= ln; }
    e2[0] = nn[1] * e1[2] - nn[2] * e1[1];
    e2[1] = nn[2] * e1[0] - nn[0] * e1[2];
    e2[2] = nn[0] * e1[1] - nn[1] * e1[0];
    const double D00 = E1[0] * e1[0] + E1[1] * e1[1] + E1[2] * e1[2];
    const double D01 = E2[0] * e1[0] + E2[1] * e1[1] + E2[2] * e1[2];
    const double D10 = E1[0] * e2[0] + E1[1] * e2[1] + E1[2] * e2[2];
    const double D11 = E2[0] * e2[0] + E2[1] * e2[1] + E2[2] * e2[2];
    const double det = D00 * D11 - D01 * D10;
    if (!(std::fabs(det) > 0)) throw FlashError(FLASH_ERR_INVALID_ARG, "degenerate rest triangle");
    double* Bt = &H.Bm[9 * (size_t)t];
    Bt[0] = D11 / det; Bt[1] = -D01 / det; Bt[2] = -D10 / det; Bt[3] = D00 / det;
    area[t] = std::fabs(det) / 2.0;
    H.w[t] = 2.0 * muL * area[t] * d.thickness;
    for (int a = 0; a < 3; ++a) H.mass[id[a]] += d.density * d.thickness * area[t] / 3.0;
  }
  if (!(d.bending > 0)) return;
  // interior edges: (min vertex, max vertex) -> (triangle, opposite vertex) x 2
  std::map<std::pair<int, int>, std::vector<std::pair<int, int>>> edges;
  for (int t = 0; t < m; ++t) {
    const int* id = &H.elem[4 * (size_t)t];
    for (int a = 0; a < 3; ++a) {
      const int u = id[a], v = id[(a + 1) % 3], o = id[(a + 2) % 3];
      edges[{std::min(u, v), std::max(u, v)}].push_back({t, o});
    }
  }
  for (const auto& kv : edges) {
    if (kv.second.size() != 2) continue;
    const int i0 = kv.first.first, i1 = kv.first.second;
    const int w2 = kv.second[0].second, w3 = kv.second[1].second;
    double e[3], L2 = 0.0;
    for (int c = 0; c < 3; ++c) { e[c] = X(i1, c) - X(i0, c); L2 += e[c] * e[c]; }
    const double L = std::sqrt(L2);
    double proj[2], dist[2];
    const int opp[2] = {w2, w3};
    for (int q = 0; q < 2; ++q) {
      double r[3], a = 0.0;
      for (int c = 0; c < 3; ++c) { r[c] = X(opp[q], c) - X(i0, c); a += r[c] * e[c] / L; }
      double d2 = 0.0;
      for (int c = 0; c < 3; ++c) { const double z = r[c] - a * e[c] / L; d2 += z * z; }
      proj[q] = a;
      dist[q] = std::sqrt(d2);
    }
    if (!(dist[0] > 0) || !(dist[1] > 0)) throw FlashError(FLASH_ERR_INVALID_ARG, "degenerate hinge");
    const double al2 = 1.0 / dist[0], al3 = 1.0 / dist[1];
    const double al1 = -(al2 * proj[0] + al3 * proj[1]) / L;
    const double al0 = -(al1 + al2 + al3);
    const double A1 = area[kv.second[0].first], A2 = area[kv.second[1].first];
    H.hidx.insert(H.hidx.end(), {i0, i1, w2, w3});
    H.halpha.insert(H.halpha.end(), {al0, al1, al2, al3});
    H.hw.push_back(3.0 * d.bending * L2 / (A1 + A2));
  }
}

// Skyline (profile) Cholesky of Abar followed by the explicit inverse.
void system_inverse(const flash_env_desc& d, HostEnv& H, double h, int nthreads) {
  (void)d;
  const int n = H.n, m = H.m;
  std::vector<int> first(n);
  for (int i = 0; i < n; ++i) first[i] = i;
  const int k = H.k;
  auto profile = [&](const int* id, int cnt) {
    int lo = id[0];
    for (int a = 1; a < cnt; ++a) lo = std::min(lo, id[a]);
    for (int a = 0; a < cnt; ++a) first[id[a]] = std::min(first[id[a]], lo);
  };
  for (int t = 0; t < m; ++t) profile(&H.elem[4 * (size_t)t], k);
  const int nh = (int)H.hw.size();
  for (int q = 0; q < nh; ++q) profile(&H.hidx[4 * (size_t)q], 4);
  std::vector<size_t> rp(n + 1, 0);
  for (int i = 0; i < n; ++i) rp[i + 1] = rp[i] + (size_t)(i - first[i] + 1);
  std::vector<double> L(rp[n], 0.0);
  auto at = [&](int i, int j) -> double& { return L[rp[i] + (j - first[i])]; };
  for (int i = 0; i < n; ++i) at(i, i) += H.mass[i];
  const double hh = h * h;
  for (int t = 0; t < m; ++t) {
    const int* id = &H.elem[4 * (size_t)t];
    const double* Bt = &H.Bm[9 * (size_t)t];
    double gN[4][3] = {};
    if (k == 4) {
      for (int c = 0; c < 3; ++c) {
        gN[1][c] = Bt[c]; gN[2][c] = Bt[3 + c]; gN[3][c] = Bt[6 + c];
        gN[0][c] = -(Bt[c] + Bt[3 + c] + Bt[6 + c]);
      }
    } else {
      for (int c = 0; c < 2; ++c) {
        gN[1][c] = Bt[c]; gN[2][c] = Bt[2 + c];
        gN[0][c] = -(Bt[c] + Bt[2 + c]);
      }
    }
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) {
        int i = id[a], j = id[b];
        if (j > i) continue;
        double v = hh * H.w[t] * (gN[a][0] * gN[b][0] + gN[a][1] * gN[b][1] + gN[a][2] * gN[b][2]);
        at(i, j) += v;
      }
  }
  for (int q = 0; q < nh; ++q) {
    const int* id = &H.hidx[4 * (size_t)q];
    const double* al = &H.halpha[4 * (size_t)q];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int i = id[a], j = id[b];
        if (j > i) continue;
        at(i, j) += hh * H.hw[q] * al[a] * al[b];
      }
  }
  // Crout factorisation in place
  const bool progress = n >= 20000 && std::getenv("FLASH_PROGRESS") != nullptr;
  const int step = std::max(1, n / 20);
  for (int i = 0; i < n; ++i) {
    if (progress && i % step == 0) {
      std::fprintf(stderr, "flash: Cholesky factor of a %d-vertex env: row %d (%d%%)\n", n, i, 100 * i / n);
      std::fflush(stderr);
    }
    for (int j = first[i]; j <= i; ++j) {
      double s = at(i, j);
      const int k0 = std::max(first[i], first[j]);
      for (int k = k0; k < j; ++k) s -= at(i, k) * at(j, k);
      if (j < i) at(i, j) = s / at(j, j);
      else {
        if (!(s > 0)) throw FlashError(FLASH_ERR_INVALID_ARG, "system matrix not positive definite");
        at(i, i) = std::sqrt(s);
      }
    }
  }
  H.Ginv.assign((size_t)n * n, 0.0);
  std::atomic<int> next(0);
  // FLASH_PROGRESS set: envs of 20,000 vertices or more report every 5% of their rows and columns
  // on stderr (their factor and inverse take minutes on the host)
  auto worker = [&]() {
    std::vector<double> y(n);
    for (;;) {
      const int c = next.fetch_add(1);
      if (c >= n) break;
      if (progress && c % step == 0) {
        std::fprintf(stderr, "flash: explicit inverse of a %d-vertex env: column %d (%d%%)\n", n, c, 100 * c / n);
        std::fflush(stderr);
      }
      // L y = e_c
      y[c] = 1.0 / at(c, c);
      for (int i = c + 1; i < n; ++i) {
        double s = 0.0;
        for (int k = std::max(first[i], c); k < i; ++k) s -= at(i, k) * y[k];
        y[i] = s / at(i, i);
      }
      // L^T x = y, rows >= c only
      for (int i = n - 1; i >= c; --i) {
        const double xi = y[i] / at(i, i);
        y[i] = xi;
        for (int k = std::max(first[i], c); k < i; ++k) y[k] -= at(i, k) * xi;
      }
      for (int i = c; i < n; ++i) {
        H.Ginv[(size_t)i * n + c] = y[i];
        H.Ginv[(size_t)c * n + i] = y[i];
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nthreads; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

template <class T>
T* dalloc(size_t count, std::vector<void*>& owned) {
  void* p = nullptr;
  if (count == 0) count = 1;
  HIPCHK(hipMalloc(&p, count * sizeof(T)));
  owned.push_back(p);
  return static_cast<T*>(p);
}

const char* kNames[K_COUNT] = {"detect", "gather", "project", "assemble", "apply", "csp", "correct",
                               "finalize", "mlp", "lg_fused"};

}  // namespace

struct flash_batch {
  flash_params p{};
  int n_envs = 0;
  bool fp64 = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int NV = 0, NT = 0, max_ld = 0;
  std::vector<int> voff, toff, nv;
  std::vector<double> mu;
  std::vector<void*> owned;
  DevBatch<float> bf{};
  DevBatch<double> bd{};
  void* mu_dev = nullptr;
  // obstacles (host mirror of what was last set)
  std::vector<int> nobs;
  // timing
  bool timing = false;
  uint32_t timing_mask = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  double tot_ms[K_COUNT] = {};
  int64_t cnt[K_COUNT] = {};
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int device = 0;
  // env groups: a batch created with stream_groups >= 2 holds one sub-batch per contiguous
  // group of envs, each on a stream of its own, so that one group's contact-solve tail
  // overlaps the other groups' work; the C ABI dispatches env indices to the groups
  std::vector<flash_batch*> groups;
  std::vector<int> gofs;      // first env of each group, then n_envs
  // explicit-inverse product schedule: work lists for the three tile widths, the chosen
  // variant, and the autotuner's measurements (ms per apply launch of each candidate)
  int2* gemv_items[3] = {nullptr, nullptr, nullptr};
  int gemv_n_items[3] = {0, 0, 0};
  GemvSchedule sched{};
  SplitSchedule split{};      // row-split products (global-memory lightweight route only)
  bool tuned = false;
  double cand_ms[6] = {0, 0, 0, 0, 0, 0};
  // learned warm start: network weights, per-slot inference buffers, training-pair recording
  bool ws_loaded = false, ws_record = false;
  MlpBuffers mlp{};
  float* ws_lab = nullptr;
  int* ws_coff = nullptr;

  ~flash_batch() {
    for (flash_batch* g : groups) delete g;
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto& pe : pending) { (void)hipEventDestroy(pe.second.first); (void)hipEventDestroy(pe.second.second); }
    for (auto ev : pool) (void)hipEventDestroy(ev);
    for (void* q : owned) (void)hipFree(q);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  hipEvent_t ev() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
  }

  template <class F>
  void launch(int kid, F&& f) {
    if (!timing || !((timing_mask >> kid) & 1u)) { f(); return; }
    hipEvent_t a = ev(), b = ev();
    HIPCHK(hipEventRecord(a, stream));
    f();
    HIPCHK(hipEventRecord(b, stream));
    pending.push_back({kid, {a, b}});
  }

  void collect_timing() {
    if (pending.empty()) return;
    HIPCHK(hipStreamSynchronize(stream));
    for (auto& pe : pending) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
      tot_ms[pe.first] += ms;
      cnt[pe.first] += 1;
      pool.push_back(pe.second.first);
      pool.push_back(pe.second.second);
    }
    pending.clear();
  }

  template <class T>
  void enqueue_step(const DevBatch<T>& B) {
    const T* mu_d = static_cast<const T*>(mu_dev);
    launch(K_DETECT, [&] {
      launch_detect<T>(B, mu_d, stream);
      launch_hinge<T>(B, stream);
      launch_order<T>(B, stream);
    });
    const bool infer = ws_loaded && p.warm_start == FLASH_WS_LEARNED;
    if (infer || ws_record) {
      launch(K_MLP, [&] {
        launch_ws_features<T>(B, mu_d, mlp.feat, mlp.need, stream);
        if (infer) launch_ws_infer<T>(B, mu_d, mlp, stream);
      });
    }
    if (B.lite_global) {
      // lightweight update from global memory: per local-global iteration the free displacement
      // z = Gbar b, then alternately u = z + h^2 Gbar H^T lambda (envs still iterating) and one
      // update of every vertex group; the last residual evaluation only decides
      launch(K_CSP, [&] { launch_lite_update<T>(B, mu_d, 0, -1, 0, stream); });
      const int N = B.max_newton;
      for (int k = 0; k < p.lg_iterations; ++k) {
        launch(K_PROJECT, [&] { launch_project<T>(B, stream); });
        launch(K_ASSEMBLE, [&] { launch_assemble<T>(B, stream); });
        launch(K_APPLY, [&] { launch_split_apply<T>(B, split, stream); });
        launch(K_CORRECT, [&] { launch_split_correct<T>(B, split, nullptr, stream); });
        for (int it = 0; it <= N; ++it) {
          launch(K_CSP, [&] { launch_lite_update<T>(B, mu_d, k, it, k == 0 ? 1 : 0, stream); });
          if (it < N) launch(K_CORRECT, [&] { launch_split_correct<T>(B, split, B.lite_done, stream); });
        }
        if (k == 0 && ws_record) launch(K_MLP, [&] { launch_ws_labels<T>(B, mlp.feat, ws_lab, stream); });
      }
      launch(K_FINALIZE, [&] { launch_finalize<T>(B, mu_d, stream); });
      HIPCHK(hipGetLastError());
      return;
    }
    launch(K_GATHER, [&] { launch_gather<T>(B, stream); });
    if (p.fused_lg && !ws_record) {
      // the whole local-global loop in one launch, one workgroup per env
      launch(K_FUSED, [&] { launch_lg_fused<T>(B, mu_d, stream); });
      launch(K_FINALIZE, [&] { launch_finalize<T>(B, mu_d, stream); });
      HIPCHK(hipGetLastError());
      return;
    }
    for (int k = 0; k < p.lg_iterations; ++k) {
      launch(K_PROJECT, [&] { launch_project<T>(B, stream); });
      launch(K_ASSEMBLE, [&] { launch_assemble<T>(B, stream); });
      launch(K_APPLY, [&] { launch_apply<T>(B, sched, stream); });
      launch(K_CSP, [&] { launch_csp<T>(B, mu_d, k == 0 ? 1 : 0, stream); });
      if (k == 0 && ws_record) launch(K_MLP, [&] { launch_ws_labels<T>(B, mlp.feat, ws_lab, stream); });
      launch(K_CORRECT, [&] { launch_correct<T>(B, sched, stream); });
    }
    launch(K_FINALIZE, [&] { launch_finalize<T>(B, mu_d, stream); });
    HIPCHK(hipGetLastError());
  }

  void drop_graph() {
    if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
    if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
  }

  // per-slot buffers of the learned warm start (allocated on first use)
  void ensure_ws_buffers() {
    if (mlp.feat) return;
    const size_t rows = (size_t)n_envs * (size_t)(fp64 ? bd.cap : bf.cap);
    mlp.W = dalloc<float>(MlpLayout::total, owned);
    mlp.norm = dalloc<float>(kNorm, owned);
    mlp.feat = dalloc<float>(rows * kFeat, owned);
    mlp.need = dalloc<int>(rows, owned);
    mlp.Y = dalloc<float>(rows * kOut, owned);
    mlp.lam_ml = dalloc<double>(rows * 3, owned);
    ws_lab = dalloc<float>(rows * kOut, owned);
    ws_coff = dalloc<int>((size_t)n_envs + 1, owned);
    HIPCHK(hipMemset(mlp.feat, 0, rows * kFeat * sizeof(float)));
    HIPCHK(hipMemset(mlp.Y, 0, rows * kOut * sizeof(float)));
    prepare_mlp();
  }

  GemvSchedule schedule(int vw, int unroll) const {
    GemvSchedule g;
    g.items = gemv_items[vw];
    g.n_items = gemv_n_items[vw];
    g.vw = vw;
    g.unroll = unroll;
    return g;
  }

  // Autotuner: times every (tile width, unroll) candidate of the global apply on this
  // batch (one warm-up launch, then 3 timed launches each) and keeps the fastest for the
  // apply and the position update.  The candidates give identical bits, so the choice
  // never changes results.  The apply only writes z, which every step recomputes.
  template <class T>
  void autotune(const DevBatch<T>& B) {
    hipEvent_t a, c;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&c));
    double best = 1e30;
    int bk = 3;
    for (int k = 0; k < 6; ++k) {
      const GemvSchedule g = schedule(k / 2, (k & 1) ? 8 : 4);
      launch_apply<T>(B, g, stream);
      HIPCHK(hipEventRecord(a, stream));
      for (int r = 0; r < 3; ++r) launch_apply<T>(B, g, stream);
      HIPCHK(hipEventRecord(c, stream));
      HIPCHK(hipEventSynchronize(c));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, a, c));
      cand_ms[k] = ms / 3.0;
      if (cand_ms[k] < best) { best = cand_ms[k]; bk = k; }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(c);
    HIPCHK(hipGetLastError());
    sched = schedule(bk / 2, (bk & 1) ? 8 : 4);
  }

  void step(int n) {
    if (!tuned) {
      // the global-memory lightweight route runs the row-split products, not the tuned ones
      const bool split_route = fp64 ? bd.lite_global : bf.lite_global;
      if (!p.fixed_schedule && !split_route) { if (fp64) autotune(bd); else autotune(bf); }
      tuned = true;
    }
    if (p.use_graph && !timing) {
      if (!gexec) {
        HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        try {
          if (fp64) enqueue_step(bd); else enqueue_step(bf);
        } catch (...) {
          hipGraph_t g;
          (void)hipStreamEndCapture(stream, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        HIPCHK(hipStreamEndCapture(stream, &graph));
        HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
      }
      for (int i = 0; i < n; ++i) HIPCHK(hipGraphLaunch(gexec, stream));
      return;
    }
    for (int i = 0; i < n; ++i) {
      if (fp64) enqueue_step(bd); else enqueue_step(bf);
    }
  }
};

namespace {

// LDS one workgroup needs to hold an env's contact data at this capacity (contact solve in LDS)
size_t csp_lds_need(const flash_params& p) {
  const int cap = csp_capacity(p.max_contacts_per_env);
  const int rlds = csp_lds_rows(csp_rows(cap));
  const bool ct64 = p.precision == FLASH_FP64 || !p.contact_fp32;
  return (ct64 ? csp_smem_bytes<double>(cap, rlds) : csp_smem_bytes<float>(cap, rlds)) + kCspStaticLds;
}

// the lightweight metric's update runs from global memory (on request, or beyond one CU's LDS)
bool lite_in_global_memory(const flash_params& p) {
  return p.contact_metric == FLASH_METRIC_LIGHTWEIGHT && (p.global_contact_solve == 1 || csp_lds_need(p) > kLdsBytes);
}

template <class T>
void build_device(flash_batch* b, std::vector<HostEnv>& H, const flash_env_desc* envs) {
  auto& own = b->owned;
  const int ne = b->n_envs;
  DevBatch<T> B{};
  B.n_envs = ne;
  B.NV = b->NV;
  B.NT = b->NT;
  B.cap = csp_capacity(b->p.max_contacts_per_env);
  B.rmax = csp_rows(B.cap);
  B.rlds = csp_lds_rows(B.rmax);
  B.max_newton = b->p.max_inner_iterations > 0 ? b->p.max_inner_iterations : 50;
  B.lg_iterations = b->p.lg_iterations;
  B.h = b->p.h;
  for (int k = 0; k < 3; ++k) B.g[k] = b->p.gravity[k];
  B.margin = b->p.contact_margin;
  B.tol = b->p.inner_tol > 0 ? b->p.inner_tol : (sizeof(T) == 4 ? 0.25 * b->p.ncp_tol : 1e-12);
  B.max_force = b->p.max_force;
  B.warm_start = b->p.warm_start;
  B.reuse = 1;   // reuse of a capacitance factorisation while the contact classes hold
  B.lite = b->p.contact_metric == FLASH_METRIC_LIGHTWEIGHT ? 1 : 0;
  B.lite_global = lite_in_global_memory(b->p) ? 1 : 0;
  const int NV = b->NV, NT = b->NT;
  const size_t cap = (size_t)B.cap;

  std::vector<int> vert_env(NV), tet_env(NT);
  for (int e = 0; e < ne; ++e) {
    for (int i = b->voff[e]; i < b->voff[e + 1]; ++i) vert_env[i] = e;
    for (int t = b->toff[e]; t < b->toff[e + 1]; ++t) tet_env[t] = e;
  }
  std::vector<T> x(3 * (size_t)NV), mass(NV), tB(9 * (size_t)NT), tw(NT);
  std::vector<int> tidx(4 * (size_t)NT);
  std::vector<int> inc_off(NV + 1, 0), slot(4 * (size_t)NT);
  for (int e = 0; e < ne; ++e) {
    const HostEnv& h = H[e];
    const int vo = b->voff[e], to = b->toff[e];
    for (int i = 0; i < h.n; ++i) {
      mass[vo + i] = (T)h.mass[i];
      for (int k = 0; k < 3; ++k) x[(size_t)k * NV + vo + i] = (T)envs[e].rest_x[3 * i + k];
    }
    for (int t = 0; t < h.m; ++t) {
      for (int a = 0; a < 4; ++a) {
        const int v = h.elem[4 * (size_t)t + a];
        tidx[(size_t)a * NT + to + t] = v < 0 ? -1 : vo + v;   // -1: triangle
        if (v >= 0) inc_off[vo + v + 1] += 1;
      }
      for (int q = 0; q < 9; ++q) tB[(size_t)q * NT + to + t] = (T)h.Bm[9 * (size_t)t + q];
      tw[to + t] = (T)h.w[t];
    }
  }
  // bending hinges (4 incidences each), after the elements
  int NH = 0;
  for (int e = 0; e < ne; ++e) NH += (int)H[e].hw.size();
  std::vector<int> hidx(4 * (size_t)NH), hslot(4 * (size_t)NH);
  std::vector<T> halpha(4 * (size_t)NH), hw(NH);
  {
    int q0 = 0;
    for (int e = 0; e < ne; ++e) {
      const HostEnv& h = H[e];
      const int vo = b->voff[e], nh = (int)h.hw.size();
      for (int q = 0; q < nh; ++q) {
        for (int a = 0; a < 4; ++a) {
          const int v = vo + h.hidx[4 * (size_t)q + a];
          hidx[(size_t)a * NH + q0 + q] = v;
          halpha[(size_t)a * NH + q0 + q] = (T)h.halpha[4 * (size_t)q + a];
          inc_off[v + 1] += 1;
        }
        hw[q0 + q] = (T)h.hw[q];
      }
      q0 += nh;
    }
  }
  for (int i = 0; i < NV; ++i) inc_off[i + 1] += inc_off[i];
  {
    std::vector<int> fillp(inc_off.begin(), inc_off.end() - 1);
    for (int t = 0; t < NT; ++t)
      for (int a = 0; a < 4; ++a) {
        const int v = tidx[(size_t)a * NT + t];
        slot[(size_t)t * 4 + a] = v < 0 ? -1 : fillp[v]++;
      }
    for (int q = 0; q < NH; ++q)
      for (int a = 0; a < 4; ++a) hslot[(size_t)a * NH + q] = fillp[hidx[(size_t)a * NH + q]]++;
  }
  // dense inverses
  std::vector<int64_t> goff(ne);
  std::vector<int> gld(ne);
  int64_t gtot = 0;
  int max_ld = 0;
  for (int e = 0; e < ne; ++e) {
    const int n = H[e].n;
    const int ld = (n + 31) / 32 * 32;   // 128-byte aligned rows
    gld[e] = ld;
    max_ld = std::max(max_ld, ld);
    if (H[e].twin >= 0) { goff[e] = goff[H[e].twin]; continue; }
    goff[e] = gtot;
    gtot += (int64_t)n * ld;
  }
  b->max_ld = max_ld;
  // work lists of the explicit-inverse products: every existing column tile, largest envs first
  {
    std::vector<int> order(ne);
    for (int e = 0; e < ne; ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return H[a].n > H[c].n; });
    for (int vw = 0; vw < 3; ++vw) {
      const int tile = gemv_tile<T>(vw);
      std::vector<int2> items;
      for (int e : order)
        for (int t0 = 0; t0 < H[e].n; t0 += tile) items.push_back(make_int2(e, t0));
      int2* d = dalloc<int2>(items.size(), own);
      HIPCHK(hipMemcpy(d, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
      b->gemv_items[vw] = d;
      b->gemv_n_items[vw] = (int)items.size();
    }
    b->sched = b->schedule(1, 4);   // 16 bytes per lane, 4 rows in flight: the untuned default
  }
  if (B.lite_global) {
    // row-split work list of the global-memory lightweight route: every block (split of split_rows
    // rows, column tile) of every env; an env's splits cover the most rows either product
    // reads (its vertices, or its contact capacity).  Workgroups are dealt to the 8 XCDs round-robin,
    // so the list runs over groups of 8 consecutive blocks and gives every env the group's 8 blocks
    // in a row: block b always lands on XCD b mod 8, and all envs read it close together in time
    // (envs sharing an inverse then share that XCD's L2 lines).  Slots of blocks an env lacks are
    // padded with empty items (env -1).  The item order never changes the bits.
    const int tile = split_tile<T>();
    std::vector<int64_t> poff(ne);
    std::vector<int> nsplit(ne);
    int64_t ptot = 0;
    for (int e = 0; e < ne; ++e) {
      const int n = H[e].n;
      const int rows = split_cover(n, B.cap);
      const int R = split_rows(rows);
      nsplit[e] = (rows + R - 1) / R;
      poff[e] = ptot;
      ptot += (int64_t)nsplit[e] * 3 * n;
    }
    // envs that share an inverse (twin >= 0 names the group's first env) run in chunks of up to
    // kTwinChunk envs (k_gemv_split_twins); the others one env per workgroup (k_gemv_split)
    std::vector<std::vector<int>> groups;
    std::vector<int> group_of(ne, -1);
    for (int e = 0; e < ne; ++e) {
      if (H[e].twin < 0) { group_of[e] = (int)groups.size(); groups.push_back({e}); }
      else groups[group_of[H[e].twin]].push_back(e);
    }
    // A group's chunk size is twin_chunk, or by default 8, else 4, whichever still leaves
    // kMinTwinItems workgroups per product (fewer, longer workgroups leave CUs idle), else one env
    // per workgroup.  Measured with the first version of the chunk kernel on the 64 x 64 folding
    // sheet (5 x 10 budget, ms per step at chunk 1 / 4 / 8): 8 envs 3.8 / 5.4 / 7.4, 16 envs
    // 6.2 / 5.7 / 7.5, 32 envs 10.0 / 9.5 / 7.8, 256 envs 60.2 / 52.4 / 43.2; chunks of 2 were
    // slower than 1 at every size.
    constexpr int kMinTwinItems = 512;
    std::vector<int> order;       // envs run one per workgroup, largest first
    std::vector<int> gorder;      // twin groups run in chunks, largest envs first
    std::vector<int> gchunk(groups.size(), 1);
    for (int g = 0; g < (int)groups.size(); ++g) {
      const int e = groups[g][0], m = (int)groups[g].size();
      const int per_env = (H[e].n + tile - 1) / tile * nsplit[e];
      int c = 1;
      if (b->p.twin_chunk > 0) {
        c = std::min(b->p.twin_chunk, m);
      } else {
        for (const int cand : {kTwinChunk, 4})
          if (m >= cand && (int64_t)((m + cand - 1) / cand) * per_env >= kMinTwinItems) { c = cand; break; }
      }
      gchunk[g] = c;
      if (c == 1) order.insert(order.end(), groups[g].begin(), groups[g].end());
      else gorder.push_back(g);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return H[a].n > H[c].n; });
    std::stable_sort(gorder.begin(), gorder.end(),
                     [&](int a, int c) { return H[groups[a][0]].n > H[groups[c][0]].n; });
    constexpr int kXcds = 8;
    // blocks run split-major (all column tiles of split 0, then of split 1, ...): the position
    // update reads only the splits that hold contact rows, and in that order every group of 8
    // consecutive blocks still spreads over the 8 XCDs (tile-major order left the XCDs of the
    // empty splits idle: 3 of 8 busy on the 100k-vertex slab's 19.5k contact rows)
    int max_n = 0, max_split = 0;
    for (int e = 0; e < ne; ++e) { max_n = std::max(max_n, H[e].n); max_split = std::max(max_split, nsplit[e]); }
    const int max_tiles = (max_n + tile - 1) / tile;
    const int nblk = max_tiles * max_split;
    std::vector<int4> items, titems;
    std::vector<int> tenvs;
    std::vector<int4> chunks;     // (first in tenvs, count, env, 0)
    for (int g : gorder)
      for (size_t c0 = 0; c0 < groups[g].size(); c0 += gchunk[g]) {
        const int cnt = (int)std::min<size_t>(gchunk[g], groups[g].size() - c0);
        chunks.push_back(make_int4((int)tenvs.size(), cnt, groups[g][0], 0));
        tenvs.insert(tenvs.end(), groups[g].begin() + c0, groups[g].begin() + c0 + cnt);
      }
    for (int bg = 0; bg < nblk; bg += kXcds) {
      for (int e : order) {
        bool any = false;
        int4 grp[kXcds];
        for (int j = 0; j < kXcds; ++j) {
          const int blk = bg + j, t0 = blk % max_tiles * tile, sp = blk / max_tiles;
          const bool has = blk < nblk && t0 < H[e].n && sp < nsplit[e];
          grp[j] = has ? make_int4(e, t0, sp, 0) : make_int4(-1, 0, 0, 0);
          any = any || has;
        }
        if (any) items.insert(items.end(), grp, grp + kXcds);
      }
      for (const int4& ch : chunks) {
        const int e = ch.z;
        bool any = false;
        int4 grp[kXcds];
        for (int j = 0; j < kXcds; ++j) {
          const int blk = bg + j, t0 = blk % max_tiles * tile, sp = blk / max_tiles;
          const bool has = blk < nblk && t0 < H[e].n && sp < nsplit[e];
          grp[j] = has ? make_int4(ch.x, t0, sp, ch.y) : make_int4(0, 0, 0, 0);
          any = any || has;
        }
        if (any) titems.insert(titems.end(), grp, grp + kXcds);
      }
    }
    int4* d_items = items.empty() ? nullptr : dalloc<int4>(items.size(), own);
    if (!items.empty())
      HIPCHK(hipMemcpy(d_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice));
    int4* d_titems = titems.empty() ? nullptr : dalloc<int4>(titems.size(), own);
    int* d_tenvs = tenvs.empty() ? nullptr : dalloc<int>(tenvs.size(), own);
    if (!titems.empty()) {
      HIPCHK(hipMemcpy(d_titems, titems.data(), titems.size() * sizeof(int4), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(d_tenvs, tenvs.data(), tenvs.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    int64_t* d_poff = dalloc<int64_t>(ne, own);
    HIPCHK(hipMemcpy(d_poff, poff.data(), ne * sizeof(int64_t), hipMemcpyHostToDevice));
    b->split.items = d_items;
    b->split.n_items = (int)items.size();
    b->split.twin_items = d_titems;
    b->split.n_twin_items = (int)titems.size();
    b->split.twin_envs = d_tenvs;
    b->split.partial = dalloc<T>((size_t)ptot, own);
    b->split.poff = d_poff;
  }
  T* G = dalloc<T>((size_t)gtot, own);
  {
    // one env at a time: its inverse (FP64, host), converted and uploaded, then freed, so that the
    // host holds one inverse at a time whatever the batch
    const int nth = std::max(1, std::min(64, (int)std::thread::hardware_concurrency()));
    std::vector<T> blk;
    for (int e = 0; e < ne; ++e) {
      if (H[e].twin >= 0) continue;
      HostEnv& he = H[e];
      system_inverse(envs[e], he, b->p.h, nth);
      const int n = he.n, ld = gld[e];
      blk.assign((size_t)n * ld, T(0));
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) blk[(size_t)i * ld + j] = (T)he.Ginv[(size_t)i * n + j];
      HIPCHK(hipMemcpy(G + goff[e], blk.data(), blk.size() * sizeof(T), hipMemcpyHostToDevice));
      std::vector<double>().swap(he.Ginv);
    }
  }
  auto up = [&](auto* dst, const auto& src) {
    HIPCHK(hipMemcpy(dst, src.data(), src.size() * sizeof(src[0]), hipMemcpyHostToDevice));
  };
  int* d_voff = dalloc<int>(ne + 1, own); up(d_voff, b->voff);
  int* d_toff = dalloc<int>(ne + 1, own); up(d_toff, b->toff);
  int* d_ve = dalloc<int>(NV, own); up(d_ve, vert_env);
  int* d_te = dalloc<int>(NT, own); up(d_te, tet_env);
  B.voff = d_voff; B.toff = d_toff; B.vert_env = d_ve; B.tet_env = d_te;
  B.x = dalloc<T>(3 * (size_t)NV, own); up(B.x, x);
  B.v = dalloc<T>(3 * (size_t)NV, own);
  HIPCHK(hipMemset(B.v, 0, 3 * (size_t)NV * sizeof(T)));
  B.u = dalloc<T>(3 * (size_t)NV, own);
  B.ut = dalloc<T>(3 * (size_t)NV, own);
  B.z = dalloc<T>(3 * (size_t)NV, own);
  B.b = dalloc<T>(3 * (size_t)NV, own);
  HIPCHK(hipMemset(B.u, 0, 3 * (size_t)NV * sizeof(T)));
  T* d_mass = dalloc<T>(NV, own); up(d_mass, mass); B.mass = d_mass;
  int* d_tidx = dalloc<int>(4 * (size_t)NT, own); up(d_tidx, tidx); B.tet_idx = d_tidx;
  T* d_tB = dalloc<T>(9 * (size_t)NT, own); up(d_tB, tB); B.tet_B = d_tB;
  T* d_tw = dalloc<T>(NT, own); up(d_tw, tw); B.tet_w = d_tw;
  B.fel = dalloc<T>(3 * (size_t)inc_off[NV], own);
  HIPCHK(hipMemset(B.fel, 0, 3 * (size_t)inc_off[NV] * sizeof(T)));
  int* d_io = dalloc<int>(NV + 1, own); up(d_io, inc_off); B.inc_off = d_io;
  int* d_slot = dalloc<int>(4 * (size_t)NT, own); up(d_slot, slot); B.slot = d_slot;
  B.NH = NH;
  int* d_hidx = dalloc<int>(4 * (size_t)NH, own); if (NH) up(d_hidx, hidx); B.hinge_idx = d_hidx;
  T* d_hal = dalloc<T>(4 * (size_t)NH, own); if (NH) up(d_hal, halpha); B.hinge_alpha = d_hal;
  T* d_hw = dalloc<T>(NH, own); if (NH) up(d_hw, hw); B.hinge_w = d_hw;
  int* d_hsl = dalloc<int>(4 * (size_t)NH, own); if (NH) up(d_hsl, hslot); B.hinge_slot = d_hsl;
  B.G = G;
  int64_t* d_goff = dalloc<int64_t>(ne, own); up(d_goff, goff); B.goff = d_goff;
  int* d_gld = dalloc<int>(ne, own); up(d_gld, gld); B.gld = d_gld;
  // obstacles
  const size_t no = (size_t)ne * kMaxObs;
  B.nobs = dalloc<int>(ne, own);
  HIPCHK(hipMemset(B.nobs, 0, ne * sizeof(int)));
  B.obs_kind = dalloc<int>(no, own);
  B.obs_move = dalloc<int>(no, own);
  B.obs_c = dalloc<double>(3 * no, own);
  B.obs_R = dalloc<double>(9 * no, own);
  B.obs_size = dalloc<double>(3 * no, own);
  B.obs_vel = dalloc<double>(3 * no, own);
  // grippers and attachment sets (none until flash_set_grippers)
  const size_t ngs = (size_t)ne * kMaxGrip;
  B.ngrip = dalloc<int>(ne, own);
  HIPCHK(hipMemset(B.ngrip, 0, ne * sizeof(int)));
  B.grip_grasp = dalloc<int>(ngs, own);
  B.grip_move = dalloc<int>(ngs, own);
  B.grip_held = dalloc<int>(ngs, own);
  HIPCHK(hipMemset(B.grip_grasp, 0, ngs * sizeof(int)));
  HIPCHK(hipMemset(B.grip_move, 0, ngs * sizeof(int)));
  HIPCHK(hipMemset(B.grip_held, 0, ngs * sizeof(int)));
  B.grip_c = dalloc<double>(3 * ngs, own);
  B.grip_vel = dalloc<double>(3 * ngs, own);
  B.grip_r = dalloc<double>(ngs, own);
  B.att_g = dalloc<int>(NV, own);
  HIPCHK(hipMemset(B.att_g, 0xFF, (size_t)NV * sizeof(int)));
  B.att_off = dalloc<double>(3 * (size_t)NV, own);
  // contacts
  B.ccount = dalloc<int>(ne, own);
  HIPCHK(hipMemset(B.ccount, 0, ne * sizeof(int)));
  B.cvert = dalloc<int>(ne * cap, own);
  B.cobs = dalloc<int>(ne * cap, own);
  B.cframe = dalloc<T>(9 * ne * cap, own);
  B.cd0 = dalloc<T>(ne * cap, own);
  B.cdob = dalloc<T>(2 * ne * cap, own);
  B.cs = dalloc<T>(ne * cap, own);
  B.clam = dalloc<double>(3 * ne * cap, own);
  B.cforce = dalloc<T>(3 * ne * cap, own);
  B.cnew = dalloc<int>(ne * cap, own);
  B.cd0d = dalloc<double>(ne * cap, own);
  B.csp64 = (sizeof(T) == 8 || !b->p.contact_fp32) ? 1 : 0;
  if constexpr (sizeof(T) == 8) B.cframe64 = reinterpret_cast<double*>(B.cframe);
  else B.cframe64 = B.csp64 ? dalloc<double>(9 * ne * cap, own) : nullptr;
  const size_t cts = B.csp64 ? sizeof(double) : sizeof(T);
  // contact-space matrices of the solves in LDS (none for the global-memory lightweight update)
  const size_t csq = B.lite_global ? 1 : ne * cap * cap * cts;
  B.Gc = dalloc<unsigned char>(csq, own);
  B.Ginv = dalloc<unsigned char>(csq, own);
  {
    const size_t rm = (size_t)B.rmax;
    B.Cm = dalloc<unsigned char>(B.lite_global ? 1 : ne * (rm * rm + 16 * rm) * cts + 4 * ne * rm * sizeof(int), own);
    B.lupan = dalloc<unsigned char>(B.lite_global ? 1 : ne * rm * (kBK + 2) * cts, own);
  }
  B.base = dalloc<int>(B.lite_global ? 1 : ne * cap, own);
  B.scr = dalloc<unsigned char>(B.lite_global ? 1 : ne * cap * 16 * cts, own);
  B.lite_done = dalloc<int>(ne, own);
  HIPCHK(hipMemset(B.lite_done, 0, ne * sizeof(int)));
  B.lite_r = dalloc<unsigned long long>(B.lite_global ? (size_t)ne * B.lg_iterations * (B.max_newton + 1) : 1, own);
  B.cyf = dalloc<unsigned char>(3 * ne * cap * cts, own);
  B.lust = dalloc<int>(4 * ne, own);
  HIPCHK(hipMemset(B.lust, 0, 4 * ne * sizeof(int)));
  B.nbase = dalloc<int>(ne, own);
  HIPCHK(hipMemset(B.nbase, 0, ne * sizeof(int)));
  B.cache_f = dalloc<T>(3 * (size_t)NV * kCacheSlots, own);
  B.cache_stamp = dalloc<int>((size_t)NV * kCacheSlots, own);
  HIPCHK(hipMemset(B.cache_stamp, 0xFF, (size_t)NV * kCacheSlots * sizeof(int)));
  B.stamp = dalloc<int>(1, own);
  {
    int one = 1;
    HIPCHK(hipMemcpy(B.stamp, &one, sizeof(int), hipMemcpyHostToDevice));
  }
  B.resid = dalloc<double>(ne, own);
  HIPCHK(hipMemset(B.resid, 0, ne * sizeof(double)));
  B.resid_hist = dalloc<double>(4 * (size_t)ne, own);
  HIPCHK(hipMemset(B.resid_hist, 0, 4 * (size_t)ne * sizeof(double)));
  B.ws_hist = dalloc<unsigned long long>(2 * (size_t)ne, own);
  HIPCHK(hipMemset(B.ws_hist, 0, 2 * (size_t)ne * sizeof(unsigned long long)));
  B.ncp_tol = b->p.ncp_tol;
  B.iters = dalloc<int>(ne, own);
  B.refac = dalloc<int>(ne, own);
  B.flags = dalloc<int>(ne, own);
  B.fp64_polar = dalloc<int>(ne, own);
  HIPCHK(hipMemset(B.iters, 0, ne * sizeof(int)));
  HIPCHK(hipMemset(B.refac, 0, ne * sizeof(int)));
  HIPCHK(hipMemset(B.flags, 0, ne * sizeof(int)));
  HIPCHK(hipMemset(B.fp64_polar, 0, ne * sizeof(int)));
  B.phase = dalloc<unsigned long long>((size_t)ne * 16, own);
  HIPCHK(hipMemset(B.phase, 0, (size_t)ne * 16 * sizeof(unsigned long long)));
  B.order = nullptr;
  B.cost = nullptr;
  if (ne <= 4096 && !b->p.fixed_schedule) {
    std::vector<int> ident(ne);
    for (int e = 0; e < ne; ++e) ident[e] = e;
    int* d_order = dalloc<int>(ne, own); up(d_order, ident); B.order = d_order;
    B.cost = dalloc<unsigned long long>(ne, own);
    HIPCHK(hipMemset(B.cost, 0, ne * sizeof(unsigned long long)));
  }
  B.lam_ml = nullptr;
  B.ws_state = dalloc<int>(ne, own);
  HIPCHK(hipMemset(B.ws_state, 0, ne * sizeof(int)));
  std::vector<T> mu(ne);
  for (int e = 0; e < ne; ++e) mu[e] = (T)b->mu[e];
  T* d_mu = dalloc<T>(ne, own); up(d_mu, mu);
  b->mu_dev = d_mu;
  if constexpr (sizeof(T) == 4) b->bf = B; else b->bd = B;
}

template <class T>
DevBatch<T>& dev(flash_batch* b);
template <> DevBatch<float>& dev<float>(flash_batch* b) { return b->bf; }
template <> DevBatch<double>& dev<double>(flash_batch* b) { return b->bd; }

template <class T>
void set_state_t(flash_batch* b, int env, const double* x, const double* v) {
  DevBatch<T>& B = dev<T>(b);
  const int e0 = env < 0 ? 0 : env, e1 = env < 0 ? b->n_envs : env + 1;
  const int vo = b->voff[e0], n = b->voff[e1] - vo;
  std::vector<T> buf(n);
  for (int k = 0; k < 3; ++k) {
    for (int i = 0; i < n; ++i) buf[i] = (T)x[3 * (size_t)i + k];
    HIPCHK(hipMemcpyAsync(B.x + (size_t)k * b->NV + vo, buf.data(), n * sizeof(T), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    if (v) {
      for (int i = 0; i < n; ++i) buf[i] = (T)v[3 * (size_t)i + k];
      HIPCHK(hipMemcpyAsync(B.v + (size_t)k * b->NV + vo, buf.data(), n * sizeof(T), hipMemcpyHostToDevice, b->stream));
      HIPCHK(hipStreamSynchronize(b->stream));
    }
  }
  HIPCHK(hipMemsetAsync(B.cache_stamp + (size_t)vo * kCacheSlots, 0xFF, (size_t)n * kCacheSlots * sizeof(int),
                        b->stream));
  HIPCHK(hipMemsetAsync(B.ws_state + e0, 0, (size_t)(e1 - e0) * sizeof(int), b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
}

template <class T>
void get_state_t(flash_batch* b, int env, double* x, double* v) {
  DevBatch<T>& B = dev<T>(b);
  HIPCHK(hipStreamSynchronize(b->stream));
  const int e0 = env < 0 ? 0 : env, e1 = env < 0 ? b->n_envs : env + 1;
  const int vo = b->voff[e0], n = b->voff[e1] - vo;
  std::vector<T> buf(n);
  for (int k = 0; k < 3; ++k) {
    if (x) {
      HIPCHK(hipMemcpy(buf.data(), B.x + (size_t)k * b->NV + vo, n * sizeof(T), hipMemcpyDeviceToHost));
      for (int i = 0; i < n; ++i) x[3 * (size_t)i + k] = (double)buf[i];
    }
    if (v) {
      HIPCHK(hipMemcpy(buf.data(), B.v + (size_t)k * b->NV + vo, n * sizeof(T), hipMemcpyDeviceToHost));
      for (int i = 0; i < n; ++i) v[3 * (size_t)i + k] = (double)buf[i];
    }
  }
}

template <class T>
int contacts_t(flash_batch* b, int env, flash_contact* out, int capacity, int* n_out) {
  DevBatch<T>& B = dev<T>(b);
  HIPCHK(hipStreamSynchronize(b->stream));
  const int ne = b->n_envs, cap = B.cap;
  std::vector<int> cnt(ne);
  HIPCHK(hipMemcpy(cnt.data(), B.ccount, ne * sizeof(int), hipMemcpyDeviceToHost));
  const int e0 = env < 0 ? 0 : env, e1 = env < 0 ? ne : env + 1;
  int total = 0;
  for (int e = e0; e < e1; ++e) total += cnt[e];
  *n_out = total;
  if (total > capacity || !out) return total > capacity ? 1 : 0;
  int o = 0;
  std::vector<int> cv(cap), co(cap);
  std::vector<T> fr(9 * (size_t)cap), frc(3 * (size_t)cap);
  std::vector<double> lam(3 * (size_t)cap);
  std::vector<double> d0(cap);
  for (int e = e0; e < e1; ++e) {
    const int c = cnt[e];
    if (!c) continue;
    const size_t base = (size_t)e * cap;
    HIPCHK(hipMemcpy(cv.data(), B.cvert + base, c * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(co.data(), B.cobs + base, c * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(fr.data(), B.cframe + 9 * base, 9 * (size_t)c * sizeof(T), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(lam.data(), B.clam + 3 * base, 3 * (size_t)c * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(frc.data(), B.cforce + 3 * base, 3 * (size_t)c * sizeof(T), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(d0.data(), B.cd0d + base, c * sizeof(double), hipMemcpyDeviceToHost));
    for (int j = 0; j < c; ++j) {
      flash_contact& r = out[o++];
      r.env = e;
      r.vertex = cv[j];
      r.obstacle = co[j];
      for (int k = 0; k < 3; ++k) {
        r.normal[k] = (double)fr[9 * j + k];
        r.tangent1[k] = (double)fr[9 * j + 3 + k];
        r.lambda[k] = lam[3 * j + k];
        r.impulse[k] = b->p.h * (double)frc[3 * j + k];
      }
      r.gap = d0[j];
      const double ln = r.lambda[0], lt = std::sqrt(r.lambda[1] * r.lambda[1] + r.lambda[2] * r.lambda[2]);
      if (co[j] >= kMaxObs) r.mode = 3;   // attachment row (bilateral)
      else r.mode = ln <= 0 ? 0 : (lt < b->mu[e] * ln * (1.0 - 1e-6) ? 1 : 2);
    }
  }
  return 0;
}

template <class T>
void stats_t(flash_batch* b, flash_env_stats* st) {
  DevBatch<T>& B = dev<T>(b);
  HIPCHK(hipStreamSynchronize(b->stream));
  const int ne = b->n_envs;
  std::vector<double> r(ne);
  std::vector<int> it(ne), rf(ne), fl(ne), fp(ne), cc(ne);
  HIPCHK(hipMemcpy(r.data(), B.resid, ne * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(it.data(), B.iters, ne * sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(rf.data(), B.refac, ne * sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(fl.data(), B.flags, ne * sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(fp.data(), B.fp64_polar, ne * sizeof(int), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(cc.data(), B.ccount, ne * sizeof(int), hipMemcpyDeviceToHost));
  std::vector<int> ws(ne);
  HIPCHK(hipMemcpy(ws.data(), B.ws_state, ne * sizeof(int), hipMemcpyDeviceToHost));
  for (int e = 0; e < ne; ++e) {
    st[e].inner_iterations = it[e];
    st[e].refactorizations = rf[e];
    st[e].contacts = cc[e];
    st[e].fp64_polar = fp[e];
    st[e].flags = fl[e] | (r[e] > b->p.ncp_tol ? 2 : 0);
    st[e].ws_state = ws[e];
    st[e].residual = r[e];
  }
}

template <class T>
void set_obstacles_t(flash_batch* b, int env, const flash_obstacle* o, int n) {
  DevBatch<T>& B = dev<T>(b);
  const int e0 = env < 0 ? 0 : env, e1 = env < 0 ? b->n_envs : env + 1;
  const int ne = e1 - e0;
  std::vector<int> kind((size_t)ne * kMaxObs, 0), mv((size_t)ne * kMaxObs, 0), cnt(ne, n);
  std::vector<double> c(3 * (size_t)ne * kMaxObs, 0), R(9 * (size_t)ne * kMaxObs, 0), sz(3 * (size_t)ne * kMaxObs, 0),
      vel(3 * (size_t)ne * kMaxObs, 0);
  for (int e = 0; e < ne; ++e)
    for (int q = 0; q < n; ++q) {
      const flash_obstacle& ob = o[(size_t)e * n + q];
      const size_t s = (size_t)e * kMaxObs + q;
      kind[s] = ob.kind;
      mv[s] = ob.move_steps;
      for (int k = 0; k < 3; ++k) { c[3 * s + k] = ob.center[k]; sz[3 * s + k] = ob.size[k]; vel[3 * s + k] = ob.lin_vel[k]; }
      for (int k = 0; k < 9; ++k) R[9 * s + k] = ob.rot[k];
    }
  const size_t so = (size_t)e0 * kMaxObs;
  HIPCHK(hipStreamSynchronize(b->stream));
  HIPCHK(hipMemcpy(B.obs_kind + so, kind.data(), kind.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(B.obs_move + so, mv.data(), mv.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(B.obs_c + 3 * so, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(const_cast<double*>(B.obs_R) + 9 * so, R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(const_cast<double*>(B.obs_size) + 3 * so, sz.data(), sz.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(const_cast<double*>(B.obs_vel) + 3 * so, vel.data(), vel.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(B.nobs + e0, cnt.data(), ne * sizeof(int), hipMemcpyHostToDevice));
  for (int e = e0; e < e1; ++e) b->nobs[e] = n;
}

template <class T>
void set_grippers_t(flash_batch* b, int env, const flash_gripper* gp, int n) {
  DevBatch<T>& B = dev<T>(b);
  HIPCHK(hipStreamSynchronize(b->stream));
  const int e0 = env < 0 ? 0 : env, e1 = env < 0 ? b->n_envs : env + 1;
  const int ne = e1 - e0;
  const size_t q0 = (size_t)e0 * kMaxGrip, nq = (size_t)ne * kMaxGrip;
  std::vector<int> grasp(nq, 0), mv(nq, 0), held(nq, 0), cnt(ne, n);
  std::vector<double> c(3 * nq, 0.0), vel(3 * nq, 0.0), r(nq, 0.0);
  HIPCHK(hipMemcpy(held.data(), B.grip_held + q0, nq * sizeof(int), hipMemcpyDeviceToHost));
  for (int e = 0; e < ne; ++e)
    for (int g = 0; g < n; ++g) {
      const flash_gripper& G = gp[(size_t)e * n + g];
      const size_t q = (size_t)e * kMaxGrip + g;
      grasp[q] = G.grasp ? 1 : 0;
      mv[q] = G.move_steps;
      r[q] = G.radius;
      for (int k = 0; k < 3; ++k) { c[3 * q + k] = G.center[k]; vel[3 * q + k] = G.lin_vel[k]; }
    }
  // grippers beyond n hold nothing: their vertices are released at the next step
  for (int e = 0; e < ne; ++e)
    for (int g = n; g < kMaxGrip; ++g) held[(size_t)e * kMaxGrip + g] = 0;
  HIPCHK(hipMemcpy(B.ngrip + e0, cnt.data(), ne * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(B.grip_grasp + q0, grasp.data(), nq * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(B.grip_move + q0, mv.data(), nq * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(B.grip_held + q0, held.data(), nq * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(B.grip_c + 3 * q0, c.data(), 3 * nq * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(const_cast<double*>(B.grip_vel) + 3 * q0, vel.data(), 3 * nq * sizeof(double),
                   hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(const_cast<double*>(B.grip_r) + q0, r.data(), nq * sizeof(double), hipMemcpyHostToDevice));
}

template <class T>
void get_obstacles_t(flash_batch* b, int env, flash_obstacle* o, int n) {
  DevBatch<T>& B = dev<T>(b);
  HIPCHK(hipStreamSynchronize(b->stream));
  for (int q = 0; q < n; ++q) {
    const size_t s = (size_t)env * kMaxObs + q;
    flash_obstacle& ob = o[q];
    HIPCHK(hipMemcpy(&ob.kind, B.obs_kind + s, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&ob.move_steps, B.obs_move + s, sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ob.center, B.obs_c + 3 * s, 3 * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ob.rot, B.obs_R + 9 * s, 9 * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ob.size, B.obs_size + 3 * s, 3 * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ob.lin_vel, B.obs_vel + 3 * s, 3 * sizeof(double), hipMemcpyDeviceToHost));
  }
}

bool bad_env(flash_batch* b, int env) { return env < -1 || env >= b->n_envs; }

// ----------------------------------------------------------------------------
// Checkpoint: everything the next step reads besides the constant model and
// the network weights, per env, so that a batch created from the same envs
// and parameters resumes bitwise whatever its stream grouping.  Warm-start
// cache entries are stored as a valid bit and rebased on load onto the
// loading batch's step counter.
// ----------------------------------------------------------------------------
constexpr char kCkptMagic[8] = {'F', 'L', 'A', 'S', 'H', 'C', 'K', '1'};
struct CkptHeader {
  char magic[8];
  int32_t n_envs, elem, max_obs, max_grip, slots, reserved;
  int64_t nv_total;
};

template <class T>
size_t env_ckpt_bytes(int nv) {
  return sizeof(int32_t)                                            // vertex count
         + 6 * (size_t)nv * sizeof(T)                                 // x, v
         + sizeof(int32_t) + kMaxObs * (2 * sizeof(int32_t) + 18 * sizeof(double))
         + sizeof(int32_t) + kMaxGrip * (3 * sizeof(int32_t) + 7 * sizeof(double))
         + (size_t)nv * (sizeof(int32_t) + 3 * sizeof(double))       // holding gripper, offset
         + (size_t)nv * kCacheSlots * (3 * sizeof(T) + 1)            // cache force, valid
         + sizeof(int32_t);                                          // learned-start state
}

struct Cursor {
  unsigned char* w = nullptr;
  const unsigned char* r = nullptr;
  template <class X>
  void put(const X* src, size_t n) { std::memcpy(w, src, n * sizeof(X)); w += n * sizeof(X); }
  template <class X>
  void get(X* dst, size_t n) { std::memcpy(dst, r, n * sizeof(X)); r += n * sizeof(X); }
};

template <class X>
void d2h(X* dst, const X* src, size_t n) { if (n) HIPCHK(hipMemcpy(dst, src, n * sizeof(X), hipMemcpyDeviceToHost)); }
template <class X>
void h2d(X* dst, const X* src, size_t n) { if (n) HIPCHK(hipMemcpy(dst, src, n * sizeof(X), hipMemcpyHostToDevice)); }

// b is a leaf batch (no groups), e its local env index
template <class T>
void save_env_t(flash_batch* b, int e, Cursor& c) {
  DevBatch<T>& B = dev<T>(b);
  const int vo = b->voff[e], nv = b->voff[e + 1] - vo;
  const int32_t nv32 = nv;
  c.put(&nv32, 1);
  std::vector<T> t((size_t)nv * kCacheSlots * 3);
  for (int k = 0; k < 3; ++k) { d2h(t.data(), B.x + (size_t)k * b->NV + vo, nv); c.put(t.data(), nv); }
  for (int k = 0; k < 3; ++k) { d2h(t.data(), B.v + (size_t)k * b->NV + vo, nv); c.put(t.data(), nv); }
  const size_t so = (size_t)e * kMaxObs, sg = (size_t)e * kMaxGrip;
  int32_t i4[3 * kMaxGrip + 2 * kMaxObs];
  double d8[18 * kMaxObs + 7 * kMaxGrip];
  d2h(i4, B.nobs + e, 1); c.put(i4, 1);
  d2h(i4, B.obs_kind + so, kMaxObs); d2h(i4 + kMaxObs, B.obs_move + so, kMaxObs); c.put(i4, 2 * kMaxObs);
  d2h(d8, B.obs_c + 3 * so, 3 * kMaxObs); d2h(d8 + 3 * kMaxObs, B.obs_R + 9 * so, 9 * kMaxObs);
  d2h(d8 + 12 * kMaxObs, B.obs_size + 3 * so, 3 * kMaxObs); d2h(d8 + 15 * kMaxObs, B.obs_vel + 3 * so, 3 * kMaxObs);
  c.put(d8, 18 * kMaxObs);
  d2h(i4, B.ngrip + e, 1); c.put(i4, 1);
  d2h(i4, B.grip_grasp + sg, kMaxGrip); d2h(i4 + kMaxGrip, B.grip_move + sg, kMaxGrip);
  d2h(i4 + 2 * kMaxGrip, B.grip_held + sg, kMaxGrip); c.put(i4, 3 * kMaxGrip);
  d2h(d8, B.grip_c + 3 * sg, 3 * kMaxGrip); d2h(d8 + 3 * kMaxGrip, B.grip_vel + 3 * sg, 3 * kMaxGrip);
  d2h(d8 + 6 * kMaxGrip, B.grip_r + sg, kMaxGrip); c.put(d8, 7 * kMaxGrip);
  std::vector<int32_t> ag(nv);
  std::vector<double> off(3 * (size_t)nv);
  d2h(ag.data(), B.att_g + vo, nv); c.put(ag.data(), nv);
  d2h(off.data(), B.att_off + 3 * (size_t)vo, 3 * (size_t)nv); c.put(off.data(), 3 * (size_t)nv);
  const size_t ne = (size_t)nv * kCacheSlots;
  d2h(t.data(), B.cache_f + 3 * (size_t)vo * kCacheSlots, 3 * ne); c.put(t.data(), 3 * ne);
  std::vector<int32_t> st(ne);
  int32_t cur = 0;
  d2h(st.data(), B.cache_stamp + (size_t)vo * kCacheSlots, ne);
  d2h(&cur, B.stamp, 1);
  std::vector<unsigned char> valid(ne);
  for (size_t i = 0; i < ne; ++i) valid[i] = st[i] == cur - 1 ? 1 : 0;
  c.put(valid.data(), ne);
  d2h(i4, B.ws_state + e, 1); c.put(i4, 1);
}

template <class T>
void load_env_t(flash_batch* b, int e, Cursor& c) {
  DevBatch<T>& B = dev<T>(b);
  const int vo = b->voff[e], nv = b->voff[e + 1] - vo;
  int32_t nv32 = 0;
  c.get(&nv32, 1);   // checked against nv before any load
  std::vector<T> t((size_t)nv * kCacheSlots * 3);
  for (int k = 0; k < 3; ++k) { c.get(t.data(), nv); h2d(B.x + (size_t)k * b->NV + vo, t.data(), nv); }
  for (int k = 0; k < 3; ++k) { c.get(t.data(), nv); h2d(B.v + (size_t)k * b->NV + vo, t.data(), nv); }
  const size_t so = (size_t)e * kMaxObs, sg = (size_t)e * kMaxGrip;
  int32_t i4[3 * kMaxGrip + 2 * kMaxObs];
  double d8[18 * kMaxObs + 7 * kMaxGrip];
  c.get(i4, 1); h2d(B.nobs + e, i4, 1); b->nobs[e] = i4[0];
  c.get(i4, 2 * kMaxObs); h2d(B.obs_kind + so, i4, kMaxObs); h2d(B.obs_move + so, i4 + kMaxObs, kMaxObs);
  c.get(d8, 18 * kMaxObs);
  h2d(B.obs_c + 3 * so, d8, 3 * kMaxObs); h2d(const_cast<double*>(B.obs_R) + 9 * so, d8 + 3 * kMaxObs, 9 * kMaxObs);
  h2d(const_cast<double*>(B.obs_size) + 3 * so, d8 + 12 * kMaxObs, 3 * kMaxObs);
  h2d(const_cast<double*>(B.obs_vel) + 3 * so, d8 + 15 * kMaxObs, 3 * kMaxObs);
  c.get(i4, 1); h2d(B.ngrip + e, i4, 1);
  c.get(i4, 3 * kMaxGrip);
  h2d(B.grip_grasp + sg, i4, kMaxGrip); h2d(B.grip_move + sg, i4 + kMaxGrip, kMaxGrip);
  h2d(B.grip_held + sg, i4 + 2 * kMaxGrip, kMaxGrip);
  c.get(d8, 7 * kMaxGrip);
  h2d(B.grip_c + 3 * sg, d8, 3 * kMaxGrip); h2d(const_cast<double*>(B.grip_vel) + 3 * sg, d8 + 3 * kMaxGrip, 3 * kMaxGrip);
  h2d(const_cast<double*>(B.grip_r) + sg, d8 + 6 * kMaxGrip, kMaxGrip);
  std::vector<int32_t> ag(nv);
  std::vector<double> off(3 * (size_t)nv);
  c.get(ag.data(), nv); h2d(B.att_g + vo, ag.data(), nv);
  c.get(off.data(), 3 * (size_t)nv); h2d(B.att_off + 3 * (size_t)vo, off.data(), 3 * (size_t)nv);
  const size_t ne = (size_t)nv * kCacheSlots;
  c.get(t.data(), 3 * ne); h2d(B.cache_f + 3 * (size_t)vo * kCacheSlots, t.data(), 3 * ne);
  std::vector<unsigned char> valid(ne);
  c.get(valid.data(), ne);
  int32_t cur = 0;
  d2h(&cur, B.stamp, 1);
  std::vector<int32_t> st(ne);
  for (size_t i = 0; i < ne; ++i) st[i] = valid[i] ? cur - 1 : -1;
  h2d(B.cache_stamp + (size_t)vo * kCacheSlots, st.data(), ne);
  c.get(i4, 1); h2d(B.ws_state + e, i4, 1);
}


}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* flash_last_error(void) { return g_err.c_str(); }
const char* flash_version(void) { return "flash-mi355x 0.1 (gfx950)"; }
const char* flash_kernel_name(int32_t i) { return (i >= 0 && i < K_COUNT) ? kNames[i] : ""; }

flash_status flash_create_batch(const flash_env_desc* envs, int32_t n_envs, const flash_params* p,
                                void* hip_stream, flash_batch** out) {
  if (!envs || !p || !out || n_envs <= 0) return fail(FLASH_ERR_INVALID_ARG, "null argument or n_envs <= 0");
  *out = nullptr;
  const bool lite = p->contact_metric == FLASH_METRIC_LIGHTWEIGHT;
  if (!(p->h > 0) || p->lg_iterations <= 0 || !(p->ncp_tol > 0) || !(p->contact_margin >= 0) ||
      !(p->inner_tol >= 0) || p->max_contacts_per_env < 0 || p->max_contacts_per_env > (lite ? 65536 : 4096))
    return fail(FLASH_ERR_INVALID_ARG, "invalid solver parameters");
  if (p->precision != FLASH_FP32 && p->precision != FLASH_FP64)
    return fail(FLASH_ERR_INVALID_ARG, "precision must be FLASH_FP32 or FLASH_FP64");
  if (p->contact_metric != FLASH_METRIC_EXACT && p->contact_metric != FLASH_METRIC_LIGHTWEIGHT)
    return fail(FLASH_ERR_INVALID_ARG, "contact_metric must be FLASH_METRIC_EXACT or FLASH_METRIC_LIGHTWEIGHT");
  if (p->global_contact_solve != 0 && p->global_contact_solve != 1)
    return fail(FLASH_ERR_INVALID_ARG, "global_contact_solve must be 0 or 1");
  if (p->global_contact_solve == 1 && !lite)
    return fail(FLASH_ERR_INVALID_ARG, "global_contact_solve = 1 needs the lightweight contact metric");
  if (p->twin_chunk < 0 || p->twin_chunk > kTwinChunk)
    return fail(FLASH_ERR_INVALID_ARG, "twin_chunk must be 0..8");
  if (!lite) {
    // one workgroup holds an env's contact data in LDS: the capacity must fit one CU's LDS
    // (the lightweight metric falls back to its global-memory update instead)
    const size_t need = csp_lds_need(*p);
    if (need > kLdsBytes)
      return fail(FLASH_ERR_INVALID_ARG, "max_contacts_per_env " + std::to_string(csp_capacity(p->max_contacts_per_env)) +
                                             " needs " + std::to_string(need) +
                                             " bytes of LDS per contact solve; a CU has " + std::to_string(kLdsBytes));
  }
  for (int e = 0; e < n_envs; ++e) {
    const flash_env_desc& d = envs[e];
    if (d.elem != FLASH_TET && d.elem != FLASH_TRI) return fail(FLASH_ERR_INVALID_ARG, "unknown element kind");
    if (d.elem == FLASH_TRI && (!(d.thickness > 0) || !(d.bending >= 0)))
      return fail(FLASH_ERR_INVALID_ARG, "triangle environments need thickness > 0 and bending >= 0");
    if (d.n_vertices <= 0 || d.n_elements <= 0 || !d.rest_x || !d.elements)
      return fail(FLASH_ERR_INVALID_ARG, "empty environment");
    if (!(d.density > 0) || !(d.young > 0) || !(d.poisson > -1 && d.poisson < 0.5) || !(d.mu >= 0))
      return fail(FLASH_ERR_INVALID_ARG, "invalid material");
  }
  if (p->stream_groups < 0) return fail(FLASH_ERR_INVALID_ARG, "stream_groups < 0");
  if (p->stream_groups > 1 && n_envs > 1) {
    if (hip_stream) return fail(FLASH_ERR_INVALID_ARG, "stream_groups >= 2 runs on streams owned by the batch");
    const int G = std::min<int>(p->stream_groups, n_envs);
    flash_batch* b = new flash_batch();
    b->p = *p;
    b->n_envs = n_envs;
    b->fp64 = p->precision == FLASH_FP64;
    b->voff.assign(n_envs + 1, 0);
    for (int e = 0; e < n_envs; ++e) b->voff[e + 1] = b->voff[e] + envs[e].n_vertices;
    b->NV = b->voff[n_envs];
    b->gofs.assign(G + 1, 0);
    for (int g = 0; g <= G; ++g) b->gofs[g] = (int)((int64_t)n_envs * g / G);
    flash_params q = *p;
    q.stream_groups = 0;
    for (int g = 0; g < G; ++g) {
      flash_batch* c = nullptr;
      const flash_status st = flash_create_batch(envs + b->gofs[g], b->gofs[g + 1] - b->gofs[g], &q, nullptr, &c);
      if (st != FLASH_OK) { delete b; return st; }
      b->groups.push_back(c);
    }
    b->tuned = true;
    *out = b;
    return FLASH_OK;
  }
  flash_batch* b = nullptr;
  try {
    b = new flash_batch();
    b->p = *p;
    b->n_envs = n_envs;
    b->fp64 = p->precision == FLASH_FP64;
    HIPCHK(hipGetDevice(&b->device));
    if (hip_stream) b->stream = static_cast<hipStream_t>(hip_stream);
    else { HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking)); b->own_stream = true; }
    b->voff.assign(n_envs + 1, 0);
    b->toff.assign(n_envs + 1, 0);
    b->mu.resize(n_envs);
    b->nobs.assign(n_envs, 0);
    for (int e = 0; e < n_envs; ++e) {
      b->voff[e + 1] = b->voff[e] + envs[e].n_vertices;
      b->toff[e + 1] = b->toff[e] + envs[e].n_elements;
      b->mu[e] = envs[e].mu;
    }
    b->NV = b->voff[n_envs];
    b->NT = b->toff[n_envs];
    std::vector<HostEnv> H(n_envs);
    // envs with the same mesh and material share one explicit inverse (host and device); the
    // inverses themselves are formed in build_device, one env at a time
    std::map<uint64_t, std::vector<int>> seen;
    for (int e = 0; e < n_envs; ++e) {
      if (envs[e].elem == FLASH_TET) tet_data(envs[e], H[e]); else tri_data(envs[e], H[e]);
      const uint64_t key = model_key(envs[e]);
      for (int f : seen[key])
        if (same_model(envs[e], envs[f])) { H[e].twin = f; break; }
      if (H[e].twin < 0) seen[key].push_back(e);
    }
    if (b->fp64) build_device<double>(b, H, envs); else build_device<float>(b, H, envs);
    // dynamic LDS limit of the contact-solve kernels
    size_t static_lds = 0;
    if (b->fp64) HIPCHK(prepare_csp<double>(&static_lds));
    else HIPCHK(prepare_csp<float>(&static_lds));
    if (static_lds > kCspStaticLds)
      throw FlashError(FLASH_ERR_DEVICE, "contact-solve kernels use " + std::to_string(static_lds) +
                                             " bytes of static LDS, above the " + std::to_string(kCspStaticLds) +
                                             " reserved beside the contact data");
    *out = b;
    return FLASH_OK;
  } catch (const FlashError& ex) {
    delete b;
    return fail(ex.st, ex.what());
  } catch (const std::exception& ex) {
    delete b;
    return fail(FLASH_ERR_OUT_OF_MEMORY, ex.what());
  }
}

flash_status flash_destroy_batch(flash_batch* b) {
  if (!b) return fail(FLASH_ERR_INVALID_ARG, "null batch");
  for (flash_batch* g : b->groups) (void)hipStreamSynchronize(g->stream);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  delete b;
  return FLASH_OK;
}

}  // extern "C"

// ---- env groups: dispatch to the sub-batches --------------------------------------
#define HIPCHK_STATUS(x)                                                               \
  do {                                                                                 \
    hipError_t _e = (x);                                                               \
    if (_e != hipSuccess) return fail(FLASH_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(_e)); \
  } while (0)
namespace {
int group_of(const flash_batch* b, int env) {
  int g = 0;
  while (env >= b->gofs[g + 1]) ++g;
  return g;
}
template <class F>
flash_status each_group(flash_batch* b, F&& f) {
  for (size_t g = 0; g < b->groups.size(); ++g) {
    const flash_status st = f((int)g, b->groups[g]);
    if (st != FLASH_OK) return st;
  }
  return FLASH_OK;
}
}  // namespace

extern "C" {

#define GUARD(body)                                            \
  try {                                                        \
    body;                                                      \
  } catch (const FlashError& ex) {                             \
    return fail(ex.st, ex.what());                             \
  } catch (const std::exception& ex) {                         \
    return fail(FLASH_ERR_DEVICE, ex.what());                  \
  }

flash_status flash_set_state(flash_batch* b, int32_t env, const double* x, const double* v) {
  if (!b || !x || bad_env(b, env)) return fail(FLASH_ERR_INVALID_ARG, "invalid batch, env or null x");
  if (!b->groups.empty()) {
    if (env >= 0) { const int g = group_of(b, env); return flash_set_state(b->groups[g], env - b->gofs[g], x, v); }
    return each_group(b, [&](int g, flash_batch* c) {
      const size_t o = 3 * (size_t)b->voff[b->gofs[g]];
      return flash_set_state(c, -1, x + o, v ? v + o : nullptr);
    });
  }
  GUARD(if (b->fp64) set_state_t<double>(b, env, x, v); else set_state_t<float>(b, env, x, v));
  return FLASH_OK;
}

flash_status flash_get_state(flash_batch* b, int32_t env, double* x, double* v) {
  if (!b || bad_env(b, env)) return fail(FLASH_ERR_INVALID_ARG, "invalid batch or env");
  if (!b->groups.empty()) {
    if (env >= 0) { const int g = group_of(b, env); return flash_get_state(b->groups[g], env - b->gofs[g], x, v); }
    return each_group(b, [&](int g, flash_batch* c) {
      const size_t o = 3 * (size_t)b->voff[b->gofs[g]];
      return flash_get_state(c, -1, x ? x + o : nullptr, v ? v + o : nullptr);
    });
  }
  GUARD(if (b->fp64) get_state_t<double>(b, env, x, v); else get_state_t<float>(b, env, x, v));
  return FLASH_OK;
}

}  // extern "C"

namespace {
// Device-pointer state transfer of env (or of every env for -1) of one ungrouped batch; the
// caller's arrays are [3][lds] with the first selected vertex at column src0.
flash_status state_device(flash_batch* b, int env, const void* x, const void* v, void* xo, void* vo_, int elem,
                          long lds, long src0) {
  const int e0 = env < 0 ? 0 : env, e1 = env < 0 ? b->n_envs : env + 1;
  const int vo = b->voff[e0], n = b->voff[e1] - vo;
  const size_t es = (size_t)elem;
  GUARD({
    if (x || v) {
      const char* xs = static_cast<const char*>(x) + src0 * es;
      const char* vs = v ? static_cast<const char*>(v) + src0 * es : nullptr;
      if (b->fp64) launch_state_in<double>(b->bd, vo, n, e0, e1, xs, vs, elem, lds, b->stream);
      else launch_state_in<float>(b->bf, vo, n, e0, e1, xs, vs, elem, lds, b->stream);
    } else {
      char* xd = xo ? static_cast<char*>(xo) + src0 * es : nullptr;
      char* vd = vo_ ? static_cast<char*>(vo_) + src0 * es : nullptr;
      if (b->fp64) launch_state_out<double>(b->bd, vo, n, xd, vd, elem, lds, b->stream);
      else launch_state_out<float>(b->bf, vo, n, xd, vd, elem, lds, b->stream);
    }
    HIPCHK(hipGetLastError());
  });
  return FLASH_OK;
}

flash_status state_device_all(flash_batch* b, int env, const void* x, const void* v, void* xo, void* vo, int elem) {
  if (!b->groups.empty()) {
    if (env >= 0) {
      const int g = group_of(b, env);
      flash_batch* c = b->groups[g];
      const int le = env - b->gofs[g];
      return state_device(c, le, x, v, xo, vo, elem, c->voff[le + 1] - c->voff[le], 0);
    }
    return each_group(b, [&](int g, flash_batch* c) {
      return state_device(c, -1, x, v, xo, vo, elem, b->NV, b->voff[b->gofs[g]]);
    });
  }
  const long n = env < 0 ? b->NV : b->voff[env + 1] - b->voff[env];
  return state_device(b, env, x, v, xo, vo, elem, n, 0);
}
}  // namespace

extern "C" {

flash_status flash_set_state_device(flash_batch* b, int32_t env, const void* x_dev, const void* v_dev,
                                    int32_t elem_size) {
  if (!b || !x_dev || bad_env(b, env) || (elem_size != 4 && elem_size != 8))
    return fail(FLASH_ERR_INVALID_ARG, "invalid batch, env, element size or null x");
  return state_device_all(b, env, x_dev, v_dev, nullptr, nullptr, elem_size);
}

flash_status flash_get_state_device(flash_batch* b, int32_t env, void* x_dev, void* v_dev, int32_t elem_size) {
  if (!b || (!x_dev && !v_dev) || bad_env(b, env) || (elem_size != 4 && elem_size != 8))
    return fail(FLASH_ERR_INVALID_ARG, "invalid batch, env, element size or no output");
  return state_device_all(b, env, nullptr, nullptr, x_dev, v_dev, elem_size);
}

flash_status flash_set_obstacles(flash_batch* b, int32_t env, const flash_obstacle* o, int32_t n) {
  if (!b || bad_env(b, env) || n < 0 || n > FLASH_MAX_OBSTACLES || (n > 0 && !o))
    return fail(FLASH_ERR_INVALID_ARG, "invalid batch, env or obstacle count");
  const int ne = env < 0 ? b->n_envs : 1;
  for (int q = 0; q < ne * n; ++q)
    if (o[q].kind < FLASH_PLANE || o[q].kind > FLASH_CAPSULE) return fail(FLASH_ERR_INVALID_ARG, "bad obstacle kind");
  if (!b->groups.empty()) {
    if (env >= 0) { const int g = group_of(b, env); return flash_set_obstacles(b->groups[g], env - b->gofs[g], o, n); }
    return each_group(b, [&](int g, flash_batch* c) {
      return flash_set_obstacles(c, -1, o ? o + (size_t)b->gofs[g] * n : nullptr, n);
    });
  }
  GUARD(if (b->fp64) set_obstacles_t<double>(b, env, o, n); else set_obstacles_t<float>(b, env, o, n));
  return FLASH_OK;
}

flash_status flash_set_grippers(flash_batch* b, int32_t env, const flash_gripper* g, int32_t n) {
  if (!b || bad_env(b, env) || n < 0 || n > FLASH_MAX_GRIPPERS || (n > 0 && !g))
    return fail(FLASH_ERR_INVALID_ARG, "invalid batch, env or gripper count");
  const int ne = env < 0 ? b->n_envs : 1;
  for (int q = 0; q < ne * n; ++q)
    if (!(g[q].radius >= 0) || !std::isfinite(g[q].center[0] + g[q].center[1] + g[q].center[2]))
      return fail(FLASH_ERR_INVALID_ARG, "bad gripper radius or center");
  if (!b->groups.empty()) {
    if (env >= 0) { const int gi = group_of(b, env); return flash_set_grippers(b->groups[gi], env - b->gofs[gi], g, n); }
    return each_group(b, [&](int gi, flash_batch* c) {
      return flash_set_grippers(c, -1, g ? g + (size_t)b->gofs[gi] * n : nullptr, n);
    });
  }
  GUARD(if (b->fp64) set_grippers_t<double>(b, env, g, n); else set_grippers_t<float>(b, env, g, n));
  return FLASH_OK;
}

flash_status flash_get_obstacles(flash_batch* b, int32_t env, flash_obstacle* o, int32_t capacity, int32_t* n_out) {
  if (!b || env < 0 || env >= b->n_envs || !n_out) return fail(FLASH_ERR_INVALID_ARG, "invalid batch or env");
  if (!b->groups.empty()) {
    const int g = group_of(b, env);
    return flash_get_obstacles(b->groups[g], env - b->gofs[g], o, capacity, n_out);
  }
  const int n = b->nobs[env];
  *n_out = n;
  if (capacity < n || !o) return fail(FLASH_ERR_CAPACITY, "obstacle capacity too small");
  GUARD(if (b->fp64) get_obstacles_t<double>(b, env, o, n); else get_obstacles_t<float>(b, env, o, n));
  return FLASH_OK;
}

flash_status flash_step(flash_batch* b, int32_t n_steps) {
  if (!b || n_steps < 0) return fail(FLASH_ERR_INVALID_ARG, "invalid batch or step count");
  if (!b->groups.empty()) {
    // step by step across the groups, so that every group's queue is fed in turn
    for (int i = 0; i < n_steps; ++i) {
      const flash_status st = each_group(b, [&](int, flash_batch* c) { return flash_step(c, 1); });
      if (st != FLASH_OK) return st;
    }
    return FLASH_OK;
  }
  GUARD(b->step(n_steps));
  return FLASH_OK;
}

flash_status flash_synchronize(flash_batch* b) {
  if (b && !b->groups.empty()) return each_group(b, [&](int, flash_batch* c) { return flash_synchronize(c); });
  if (!b) return fail(FLASH_ERR_INVALID_ARG, "null batch");
  GUARD(HIPCHK(hipStreamSynchronize(b->stream)));
  return FLASH_OK;
}

flash_status flash_contacts(flash_batch* b, int32_t env, flash_contact* out, int32_t capacity, int32_t* n_out) {
  if (!b || bad_env(b, env) || !n_out || capacity < 0) return fail(FLASH_ERR_INVALID_ARG, "invalid arguments");
  if (!b->groups.empty()) {
    if (env >= 0) {
      const int g = group_of(b, env);
      const flash_status st = flash_contacts(b->groups[g], env - b->gofs[g], out, capacity, n_out);
      if (st == FLASH_OK)
        for (int k = 0; k < *n_out; ++k) out[k].env += b->gofs[g];
      return st;
    }
    int total = 0;
    bool short_cap = false;
    for (size_t g = 0; g < b->groups.size(); ++g) {
      int32_t ng = 0;
      const int room = std::max(capacity - total, 0);
      const flash_status st = flash_contacts(b->groups[g], -1, (out && room > 0) ? out + total : nullptr, room, &ng);
      if (st == FLASH_ERR_CAPACITY || (st == FLASH_ERR_INVALID_ARG && room == 0)) short_cap = true;
      else if (st != FLASH_OK) return st;
      if (!short_cap)
        for (int k = 0; k < ng; ++k) out[total + k].env += b->gofs[g];
      total += ng;
    }
    *n_out = total;
    if (short_cap || total > capacity) return fail(FLASH_ERR_CAPACITY, "contact capacity too small");
    return FLASH_OK;
  }
  int over = 0;
  GUARD(over = b->fp64 ? contacts_t<double>(b, env, out, capacity, n_out) : contacts_t<float>(b, env, out, capacity, n_out));
  if (over) return fail(FLASH_ERR_CAPACITY, "contact capacity too small");
  return FLASH_OK;
}

flash_status flash_stats(flash_batch* b, flash_env_stats* per_env) {
  if (!b || !per_env) return fail(FLASH_ERR_INVALID_ARG, "invalid arguments");
  if (!b->groups.empty())
    return each_group(b, [&](int g, flash_batch* c) { return flash_stats(c, per_env + b->gofs[g]); });
  GUARD(if (b->fp64) stats_t<double>(b, per_env); else stats_t<float>(b, per_env));
  return FLASH_OK;
}

flash_status flash_residual(flash_batch* b, double* per_env, double* max_out, int32_t* inner_iters) {
  if (!b) return fail(FLASH_ERR_INVALID_ARG, "null batch");
  std::vector<flash_env_stats> st(b->n_envs);
  flash_status s = flash_stats(b, st.data());
  if (s != FLASH_OK) return s;
  double m = 0.0;
  bool nonfinite = false, over = false, dropped = false;
  for (int e = 0; e < b->n_envs; ++e) {
    if (per_env) per_env[e] = st[e].residual;
    if (inner_iters) inner_iters[e] = st[e].inner_iterations;
    if (!(st[e].residual == st[e].residual) || (st[e].flags & 1)) nonfinite = true;
    else m = std::max(m, st[e].residual);
    if (st[e].residual > b->p.ncp_tol) over = true;
    if (st[e].flags & 4) dropped = true;
  }
  if (max_out) *max_out = nonfinite ? NAN : m;
  if (nonfinite) return fail(FLASH_ERR_NONFINITE, "an environment holds a non-finite state");
  if (dropped)
    return fail(FLASH_ERR_CAPACITY, "an environment detected more contacts than max_contacts_per_env; its step "
                                    "ignored the excess contacts");
  if (over) return fail(FLASH_ERR_NOT_CONVERGED, "an environment ended above ncp_tol");
  return FLASH_OK;
}

flash_status flash_set_kernel_timing(flash_batch* b, int32_t enable) {
  if (!b) return fail(FLASH_ERR_INVALID_ARG, "null batch");
  if (!b->groups.empty()) return each_group(b, [&](int, flash_batch* c) { return flash_set_kernel_timing(c, enable); });
  GUARD(b->collect_timing());
  b->timing = enable != 0;
  b->timing_mask = (uint32_t)enable;
  for (int k = 0; k < K_COUNT; ++k) { b->tot_ms[k] = 0; b->cnt[k] = 0; }
  return FLASH_OK;
}

flash_status flash_kernel_times(flash_batch* b, double* total_ms, int64_t* launches, int32_t cap, int32_t* n_out) {
  if (!b || !n_out) return fail(FLASH_ERR_INVALID_ARG, "invalid arguments");
  if (!b->groups.empty()) {
    // totals summed over the groups (their launches overlap in time)
    std::vector<double> t(K_COUNT, 0.0), tg(K_COUNT);
    std::vector<int64_t> n(K_COUNT, 0), ng(K_COUNT);
    const flash_status st = each_group(b, [&](int, flash_batch* c) {
      int32_t k = 0;
      const flash_status s2 = flash_kernel_times(c, tg.data(), ng.data(), K_COUNT, &k);
      for (int q = 0; q < K_COUNT; ++q) { t[q] += tg[q]; n[q] += ng[q]; }
      return s2;
    });
    if (st != FLASH_OK) return st;
    *n_out = K_COUNT;
    for (int k = 0; k < K_COUNT && k < cap; ++k) {
      if (total_ms) total_ms[k] = t[k];
      if (launches) launches[k] = n[k];
    }
    return FLASH_OK;
  }
  GUARD(b->collect_timing());
  *n_out = K_COUNT;
  for (int k = 0; k < K_COUNT && k < cap; ++k) {
    if (total_ms) total_ms[k] = b->tot_ms[k];
    if (launches) launches[k] = b->cnt[k];
  }
  return FLASH_OK;
}

flash_status flash_residual_history(flash_batch* b, double* max_out, int64_t* over_out, int64_t* newton_out,
                                    int64_t* env_steps_out, int32_t reset) {
  if (!b) return fail(FLASH_ERR_INVALID_ARG, "null batch");
  if (!b->groups.empty()) {
    double m = 0.0;
    int64_t over = 0, newton = 0, steps = 0;
    const flash_status st = each_group(b, [&](int, flash_batch* c) {
      double mg = 0.0;
      int64_t og = 0, ng = 0, sg = 0;
      const flash_status s2 = flash_residual_history(c, &mg, &og, &ng, &sg, reset);
      m = (mg > m || !(mg == mg)) ? mg : m;
      over += og; newton += ng; steps += sg;
      return s2;
    });
    if (max_out) *max_out = m;
    if (over_out) *over_out = over;
    if (newton_out) *newton_out = newton;
    if (env_steps_out) *env_steps_out = steps;
    return st;
  }
  try {
    HIPCHK(hipStreamSynchronize(b->stream));
    const int ne = b->n_envs;
    double* dp = b->fp64 ? b->bd.resid_hist : b->bf.resid_hist;
    std::vector<double> h(4 * (size_t)ne);
    HIPCHK(hipMemcpy(h.data(), dp, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    double m = 0.0;
    int64_t over = 0, newton = 0, steps = 0;
    for (int e = 0; e < ne; ++e) {
      const double* q = h.data() + 4 * (size_t)e;
      m = (q[0] > m || !(q[0] == q[0])) ? q[0] : m;
      over += (int64_t)q[1];
      newton += (int64_t)q[2];
      steps += (int64_t)q[3];
    }
    if (max_out) *max_out = m;
    if (over_out) *over_out = over;
    if (newton_out) *newton_out = newton;
    if (env_steps_out) *env_steps_out = steps;
    if (reset) HIPCHK(hipMemset(dp, 0, h.size() * sizeof(double)));
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_ws_history(flash_batch* b, int64_t* started_out, int64_t* restarted_out, int32_t reset) {
  if (!b) return fail(FLASH_ERR_INVALID_ARG, "null batch");
  if (!b->groups.empty()) {
    int64_t st = 0, rs = 0;
    const flash_status s = each_group(b, [&](int, flash_batch* c) {
      int64_t a = 0, r = 0;
      const flash_status s2 = flash_ws_history(c, &a, &r, reset);
      st += a; rs += r;
      return s2;
    });
    if (started_out) *started_out = st;
    if (restarted_out) *restarted_out = rs;
    return s;
  }
  try {
    HIPCHK(hipStreamSynchronize(b->stream));
    const int ne = b->n_envs;
    unsigned long long* dp = b->fp64 ? b->bd.ws_hist : b->bf.ws_hist;
    std::vector<unsigned long long> h(2 * (size_t)ne);
    HIPCHK(hipMemcpy(h.data(), dp, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    int64_t st = 0, rs = 0;
    for (int e = 0; e < ne; ++e) { st += (int64_t)h[2 * e]; rs += (int64_t)h[2 * e + 1]; }
    if (started_out) *started_out = st;
    if (restarted_out) *restarted_out = rs;
    if (reset) HIPCHK(hipMemset(dp, 0, h.size() * sizeof(unsigned long long)));
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_checkpoint_size(flash_batch* b, size_t* n_bytes) {
  if (!b || !n_bytes) return fail(FLASH_ERR_INVALID_ARG, "null argument");
  size_t n = sizeof(CkptHeader);
  for (int e = 0; e < b->n_envs; ++e) {
    const int nv = b->voff[e + 1] - b->voff[e];
    n += b->fp64 ? env_ckpt_bytes<double>(nv) : env_ckpt_bytes<float>(nv);
  }
  *n_bytes = n;
  return FLASH_OK;
}

flash_status flash_save_checkpoint(flash_batch* b, void* buf, size_t capacity, size_t* n_bytes) {
  size_t need = 0;
  const flash_status s0 = flash_checkpoint_size(b, &need);
  if (s0 != FLASH_OK) return s0;
  if (n_bytes) *n_bytes = need;
  if (!buf || capacity < need) return fail(FLASH_ERR_CAPACITY, "checkpoint buffer too small");
  try {
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, sizeof(h.magic));
    h.n_envs = b->n_envs; h.elem = b->fp64 ? 8 : 4; h.max_obs = kMaxObs; h.max_grip = kMaxGrip;
    h.slots = kCacheSlots; h.nv_total = b->voff[b->n_envs];
    Cursor c;
    c.w = static_cast<unsigned char*>(buf);
    c.put(&h, 1);
    for (int e = 0; e < b->n_envs; ++e) {
      flash_batch* leaf = b;
      int le = e;
      if (!b->groups.empty()) { const int g = group_of(b, e); leaf = b->groups[g]; le = e - b->gofs[g]; }
      HIPCHK(hipStreamSynchronize(leaf->stream));
      if (leaf->fp64) save_env_t<double>(leaf, le, c); else save_env_t<float>(leaf, le, c);
    }
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_load_checkpoint(flash_batch* b, const void* buf, size_t n_bytes) {
  size_t need = 0;
  const flash_status s0 = flash_checkpoint_size(b, &need);
  if (s0 != FLASH_OK) return s0;
  if (!buf || n_bytes != need) return fail(FLASH_ERR_INVALID_ARG, "checkpoint size does not match this batch");
  CkptHeader h{};
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, kCkptMagic, sizeof(h.magic)) != 0 || h.n_envs != b->n_envs ||
      h.elem != (b->fp64 ? 8 : 4) || h.max_obs != kMaxObs || h.max_grip != kMaxGrip || h.slots != kCacheSlots ||
      h.nv_total != b->voff[b->n_envs])
    return fail(FLASH_ERR_INVALID_ARG, "checkpoint does not belong to a batch of this shape and precision");
  // every env's vertex count before anything is written
  const unsigned char* rec = static_cast<const unsigned char*>(buf) + sizeof(CkptHeader);
  for (int e = 0; e < b->n_envs; ++e) {
    const int nv = b->voff[e + 1] - b->voff[e];
    int32_t nv32 = 0;
    std::memcpy(&nv32, rec, sizeof(nv32));
    if (nv32 != nv) return fail(FLASH_ERR_INVALID_ARG, "checkpoint vertex count differs at env " + std::to_string(e));
    rec += b->fp64 ? env_ckpt_bytes<double>(nv) : env_ckpt_bytes<float>(nv);
  }
  try {
    Cursor c;
    c.r = static_cast<const unsigned char*>(buf) + sizeof(CkptHeader);
    for (int e = 0; e < b->n_envs; ++e) {
      flash_batch* leaf = b;
      int le = e;
      if (!b->groups.empty()) { const int g = group_of(b, e); leaf = b->groups[g]; le = e - b->gofs[g]; }
      HIPCHK(hipStreamSynchronize(leaf->stream));
      if (leaf->fp64) load_env_t<double>(leaf, le, c); else load_env_t<float>(leaf, le, c);
      HIPCHK(hipDeviceSynchronize());
    }
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_schedule_info(flash_batch* b, int32_t* info, double* cand_ms) {
  if (!b || !info) return fail(FLASH_ERR_INVALID_ARG, "null argument");
  if (!b->groups.empty()) {
    // group 0's choice; work items summed over the groups; info[4] = groups
    int32_t items = 0, gi[5];
    for (size_t g = 0; g < b->groups.size(); ++g) {
      const flash_status st = flash_schedule_info(b->groups[g], gi, g == 0 ? cand_ms : nullptr);
      if (st != FLASH_OK) return st;
      if (g == 0) { info[0] = gi[0]; info[1] = gi[1]; info[3] = gi[3]; }
      items += gi[2];
    }
    info[2] = items;
    info[4] = (int32_t)b->groups.size();
    return FLASH_OK;
  }
  const int es = b->fp64 ? 8 : 4;
  info[0] = 64 * ((8 << b->sched.vw) / es);
  info[1] = b->sched.unroll;
  info[2] = b->sched.n_items;
  info[3] = (b->tuned && !b->p.fixed_schedule) ? 1 : 0;
  info[4] = 1;
  if (cand_ms)
    for (int k = 0; k < 6; ++k) cand_ms[k] = b->cand_ms[k];
  return FLASH_OK;
}

flash_status flash_phase_times(flash_batch* b, double* ms_out) {
  if (!b || !ms_out) return fail(FLASH_ERR_INVALID_ARG, "invalid arguments");
  if (!b->groups.empty()) {
    // per-env means weighted by the groups' env counts; the largest system is a maximum
    double acc[16] = {0}, g16[16];
    double rows = 0.0, facts = 0.0;
    const flash_status st = each_group(b, [&](int g, flash_batch* c) {
      const flash_status s2 = flash_phase_times(c, g16);
      const double w = (double)(b->gofs[g + 1] - b->gofs[g]) / b->n_envs;
      for (int k = 0; k < 16; ++k)
        if (k != 12 && k != 13) acc[k] += w * g16[k];
      rows += g16[12] * g16[8] * w;
      facts += g16[8] * w;
      acc[13] = std::max(acc[13], g16[13]);
      return s2;
    });
    for (int k = 0; k < 16; ++k) ms_out[k] = acc[k];
    ms_out[12] = facts > 0 ? rows / facts : 0.0;
    return st;
  }
  try {
    HIPCHK(hipStreamSynchronize(b->stream));
    const int ne = b->n_envs;
    unsigned long long* dp = b->fp64 ? b->bd.phase : b->bf.phase;
    std::vector<unsigned long long> h((size_t)ne * 16);
    HIPCHK(hipMemcpy(h.data(), dp, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    int khz = 0;
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device));
    for (int k = 0; k < 8; ++k) {
      double t = 0;
      for (int e = 0; e < ne; ++e) t += (double)h[(size_t)e * 8 + k];
      ms_out[k] = khz > 0 ? t / (double)khz / ne : 0.0;
    }
    const unsigned long long* cnt = h.data() + (size_t)ne * 8;
    double sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long mx = 0;
    for (int e = 0; e < ne; ++e) {
      for (int k = 0; k < 8; ++k) sum[k] += (double)cnt[8 * (size_t)e + k];
      mx = std::max(mx, cnt[8 * (size_t)e + 5]);
    }
    for (int k = 0; k < 4; ++k) ms_out[8 + k] = sum[k] / ne;
    ms_out[12] = sum[0] > 0 ? sum[4] / sum[0] : 0.0;   // mean capacitance rows per factorisation
    ms_out[13] = (double)mx;                           // largest capacitance system
    ms_out[14] = sum[6] / ne;                          // Newton iterations per env
    ms_out[15] = sum[7] / ne;                          // contact solves with contacts per env
    HIPCHK(hipMemset(dp, 0, h.size() * sizeof(unsigned long long)));
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_ws_load(flash_batch* b, const uint16_t* w, size_t n_params, const float* norm) {
  if (!b || !w || !norm) return fail(FLASH_ERR_INVALID_ARG, "null argument");
  if (!b->groups.empty()) return each_group(b, [&](int, flash_batch* c) { return flash_ws_load(c, w, n_params, norm); });
  if (n_params != (size_t)MlpLayout::total) return fail(FLASH_ERR_INVALID_ARG, "n_params must be 35587");
  for (int k = 0; k < kNorm; ++k)
    if (!std::isfinite(norm[k])) return fail(FLASH_ERR_INVALID_ARG, "non-finite normalisation");
  try {
    b->ensure_ws_buffers();
    // bf16 -> FP32 is exact; the GEMM rounds its operands back to the same bf16 values
    std::vector<float> wf(n_params);
    for (size_t i = 0; i < n_params; ++i) {
      uint32_t u = (uint32_t)w[i] << 16;
      std::memcpy(&wf[i], &u, 4);
    }
    HIPCHK(hipMemcpyAsync((void*)b->mlp.W, wf.data(), n_params * sizeof(float), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync((void*)b->mlp.norm, norm, kNorm * sizeof(float), hipMemcpyHostToDevice, b->stream));
    int* ws = b->fp64 ? b->bd.ws_state : b->bf.ws_state;
    HIPCHK(hipMemsetAsync(ws, 0, b->n_envs * sizeof(int), b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->ws_loaded = true;
    if (b->fp64) b->bd.lam_ml = b->mlp.lam_ml; else b->bf.lam_ml = b->mlp.lam_ml;
    if (b->p.warm_start != FLASH_WS_LEARNED) { b->bd.lam_ml = nullptr; b->bf.lam_ml = nullptr; }
    b->drop_graph();
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_ws_record(flash_batch* b, int32_t on) {
  if (!b) return fail(FLASH_ERR_INVALID_ARG, "null batch");
  if (!b->groups.empty()) {
    const flash_status st = each_group(b, [&](int, flash_batch* c) { return flash_ws_record(c, on); });
    b->ws_record = on != 0;
    return st;
  }
  try {
    if (on) b->ensure_ws_buffers();
    b->ws_record = on != 0;
    b->drop_graph();
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_ws_collect(flash_batch* b, float* feat_dev, float* lab_dev, int64_t capacity, int64_t* n_inout) {
  if (!b || !feat_dev || !lab_dev || !n_inout || *n_inout < 0 || capacity < 0)
    return fail(FLASH_ERR_INVALID_ARG, "null or negative argument");
  if (!b->ws_record) return fail(FLASH_ERR_INVALID_ARG, "recording is off (flash_ws_record)");
  if (!b->groups.empty()) {
    // rows of the groups in env order; nothing is written unless all of them fit
    int64_t rows = 0;
    for (flash_batch* c : b->groups) {
      HIPCHK_STATUS(hipStreamSynchronize(c->stream));
      std::vector<int> cc(c->n_envs);
      const int cap = c->fp64 ? c->bd.cap : c->bf.cap;
      HIPCHK_STATUS(hipMemcpy(cc.data(), c->fp64 ? c->bd.ccount : c->bf.ccount, c->n_envs * sizeof(int),
                              hipMemcpyDeviceToHost));
      for (int q : cc) rows += std::min(q, cap);
    }
    if (*n_inout + rows > capacity)
      return fail(FLASH_ERR_CAPACITY, "collect needs " + std::to_string(*n_inout + rows) + " rows");
    return each_group(b, [&](int, flash_batch* c) { return flash_ws_collect(c, feat_dev, lab_dev, capacity, n_inout); });
  }
  try {
    std::vector<int> cc(b->n_envs);
    const int cap = b->fp64 ? b->bd.cap : b->bf.cap;
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipMemcpy(cc.data(), b->fp64 ? b->bd.ccount : b->bf.ccount, b->n_envs * sizeof(int),
                     hipMemcpyDeviceToHost));
    int64_t rows = 0;
    for (int c : cc) rows += std::min(c, cap);
    if (*n_inout + rows > capacity) {
      return fail(FLASH_ERR_CAPACITY, "collect needs " + std::to_string(*n_inout + rows) + " rows");
    }
    if (b->fp64) {
      launch_ws_compact<double>(b->bd, b->mlp.feat, b->ws_lab, feat_dev, lab_dev, (long)*n_inout, b->ws_coff, b->stream);
    } else {
      launch_ws_compact<float>(b->bf, b->mlp.feat, b->ws_lab, feat_dev, lab_dev, (long)*n_inout, b->ws_coff, b->stream);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(b->stream));
    *n_inout += rows;
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

}  // extern "C"
