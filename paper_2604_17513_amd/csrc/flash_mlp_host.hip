// C ABI of the warm-start network trainer: device-resident FP32 master weights,
// Adam moments and minibatch scratch; every forward and backward GEMM runs in
// the bf16 MFMA kernel of flash_mlp.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/flash.h"
#include "flash_common.h"
#include "flash_mlp.h"

using namespace flash;

namespace {

// splitmix64 (Steele, Lea and Flood 2014): the seeded stream behind the
// parameter initialisation and the minibatch shuffles.
struct SplitMix64 {
  uint64_t s;
  explicit SplitMix64(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  uint64_t below(uint64_t n) { return n ? next() % n : 0; }
};

template <class T>
T* dmalloc(size_t n, std::vector<void*>& own) {
  void* p = nullptr;
  HIPCHK(hipMalloc(&p, (n ? n : 1) * sizeof(T)));
  own.push_back(p);
  return static_cast<T*>(p);
}

uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Scratch of flash_mlp_grad_noalloc, one copy per GPU for the life of the process: the
// hidden activations H1..H3 and the backward buffers dA, dB (rows x 128 floats each), the
// network output and its loss gradient (rows x 3 each), the split-K partial sums of the weight
// gradients (the trainer's size, so that both entry points split every product the same way)
// and the per-block loss partials.
constexpr long kNaRows = 2048;
constexpr long kNaWork = 64L * kHidden * kHidden;
constexpr long kNaPartials = (3 * kNaRows + 255) / 256 + 1;
constexpr size_t kNaHid = (size_t)kNaRows * kHidden * sizeof(float);
constexpr size_t kNaOut = (size_t)kNaRows * kOut * sizeof(float);
constexpr size_t kNaOffPartial = 0;
constexpr size_t kNaOffH = 256;
constexpr size_t kNaOffY = kNaOffH + 5 * kNaHid;
constexpr size_t kNaOffWork = kNaOffY + 2 * kNaOut + 256;
constexpr size_t kNaBytes = kNaOffWork + (size_t)kNaWork * sizeof(float);
static_assert(kNaPartials * sizeof(double) <= kNaOffH, "loss partials fit their slot");
static_assert(kNaOffWork % 256 == 0 && kNaOffY % 256 == 0, "aligned scratch regions");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

// Device address of this GPU's scratch, looked up once per device with that device current.
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mutex;
unsigned char* g_na_ptr[kNaMaxDevices] = {};

unsigned char* noalloc_scratch() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNaMaxDevices) throw FlashError(FLASH_ERR_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_na_mutex);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_na_ptr[dev] = static_cast<unsigned char*>(p);
  }
  return g_na_ptr[dev];
}

}  // namespace

struct flash_mlp {
  long max_rows = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<void*> own;
  float *W = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr, *norm = nullptr;
  float *X = nullptr, *L = nullptr, *H1 = nullptr, *H2 = nullptr, *H3 = nullptr, *Y = nullptr, *dY = nullptr;
  float *dA = nullptr, *dB = nullptr, *loss = nullptr;
  double* partial = nullptr;
  double* moments = nullptr;
  float* work = nullptr;                       // split-K partial sums of the weight gradients
  static constexpr long kWork = 64L * kHidden * kHidden;
  int adam_t = 0;
  std::vector<float> host_norm;

  ~flash_mlp() {
    for (void* p : own) (void)hipFree(p);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  void reset_adam() {
    HIPCHK(hipMemsetAsync(Mo, 0, MlpLayout::total * sizeof(float), stream));
    HIPCHK(hipMemsetAsync(Vo, 0, MlpLayout::total * sizeof(float), stream));
    adam_t = 0;
  }

  // loss and gradient of one minibatch already in X (normalised) and L (scaled labels)
  void grad(long n, float* loss_dst) {
    launch_mlp_fused(W, nullptr, X, n, nullptr, Y, H1, H2, H3, stream);
    mlp_loss(Y, L, n, dY, partial, loss_dst, stream);
    mlp_backward(W, X, n, H1, H2, H3, dY, dA, dB, G, work, kWork, stream);
  }
};

static_assert(kNaWork == flash_mlp::kWork, "the no-allocation gradient splits products like the trainer");

namespace {
flash_status fail(flash_status s, const std::string& m) { return record_error(s, m); }

bool finite_all(const float* p, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}
}  // namespace

extern "C" {

flash_status flash_mlp_create(int64_t max_rows, uint64_t seed, void* hip_stream, flash_mlp** out) {
  if (!out || max_rows <= 0 || max_rows > (int64_t)1 << 26) return fail(FLASH_ERR_INVALID_ARG, "bad max_rows or out");
  *out = nullptr;
  flash_mlp* m = new flash_mlp();
  try {
    m->max_rows = (long)max_rows;
    prepare_mlp();
    if (hip_stream) {
      m->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      HIPCHK(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
      m->own_stream = true;
    }
    const long P = MlpLayout::total, R = m->max_rows;
    m->W = dmalloc<float>(P, m->own);
    m->G = dmalloc<float>(P, m->own);
    m->Mo = dmalloc<float>(P, m->own);
    m->Vo = dmalloc<float>(P, m->own);
    m->norm = dmalloc<float>(kNorm, m->own);
    m->X = dmalloc<float>(R * kFeat, m->own);
    m->L = dmalloc<float>(R * kOut, m->own);
    m->H1 = dmalloc<float>(R * kHidden, m->own);
    m->H2 = dmalloc<float>(R * kHidden, m->own);
    m->H3 = dmalloc<float>(R * kHidden, m->own);
    m->dA = dmalloc<float>(R * kHidden, m->own);
    m->dB = dmalloc<float>(R * kHidden, m->own);
    m->Y = dmalloc<float>(R * kOut, m->own);
    m->dY = dmalloc<float>(R * kOut, m->own);
    m->loss = dmalloc<float>(1 << 16, m->own);
    m->partial = dmalloc<double>((3 * R + 255) / 256 + 1, m->own);
    m->moments = dmalloc<double>(2 * (kFeat + kOut), m->own);
    m->work = dmalloc<float>(flash_mlp::kWork, m->own);
    // He-uniform weights (bound sqrt(6 / fan_in)), zero biases
    std::vector<float> w(P, 0.f);
    SplitMix64 rng(seed);
    const MlpLayout Lo;
    auto fill = [&](long off, int fan_out, int fan_in) {
      const double a = std::sqrt(6.0 / fan_in);
      for (long i = 0; i < (long)fan_out * fan_in; ++i) w[off + i] = (float)((2.0 * rng.uniform() - 1.0) * a);
    };
    fill(Lo.w1, kHidden, kFeat);
    fill(Lo.w2, kHidden, kHidden);
    fill(Lo.w3, kHidden, kHidden);
    fill(Lo.w4, kOut, kHidden);
    HIPCHK(hipMemcpyAsync(m->W, w.data(), P * sizeof(float), hipMemcpyHostToDevice, m->stream));
    m->host_norm.assign(kNorm, 0.f);
    for (int k = kFeat; k < kNorm; ++k) m->host_norm[k] = 1.f;
    HIPCHK(hipMemcpyAsync(m->norm, m->host_norm.data(), kNorm * sizeof(float), hipMemcpyHostToDevice, m->stream));
    m->reset_adam();
    HIPCHK(hipStreamSynchronize(m->stream));
  } catch (const FlashError& ex) {
    delete m;
    return fail(ex.st, ex.what());
  }
  *out = m;
  return FLASH_OK;
}

flash_status flash_mlp_destroy(flash_mlp* m) {
  if (!m) return fail(FLASH_ERR_INVALID_ARG, "null network");
  (void)hipStreamSynchronize(m->stream);
  delete m;
  return FLASH_OK;
}

flash_status flash_mlp_set_params(flash_mlp* m, const float* w, int64_t n) {
  if (!m || !w || n != MlpLayout::total) return fail(FLASH_ERR_INVALID_ARG, "need 35587 parameters");
  if (!finite_all(w, (long)n)) return fail(FLASH_ERR_INVALID_ARG, "non-finite parameter");
  try {
    HIPCHK(hipMemcpyAsync(m->W, w, n * sizeof(float), hipMemcpyHostToDevice, m->stream));
    m->reset_adam();
    HIPCHK(hipStreamSynchronize(m->stream));
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_mlp_get_params(flash_mlp* m, float* w, int64_t n) {
  if (!m || !w || n != MlpLayout::total) return fail(FLASH_ERR_INVALID_ARG, "need 35587 parameters");
  try {
    HIPCHK(hipStreamSynchronize(m->stream));
    HIPCHK(hipMemcpy(w, m->W, n * sizeof(float), hipMemcpyDeviceToHost));
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_mlp_get_params_bf16(flash_mlp* m, uint16_t* w, int64_t n) {
  if (!m || !w || n != MlpLayout::total) return fail(FLASH_ERR_INVALID_ARG, "need 35587 parameters");
  std::vector<float> f((size_t)n);
  flash_status st = flash_mlp_get_params(m, f.data(), n);
  if (st != FLASH_OK) return st;
  for (int64_t i = 0; i < n; ++i) w[i] = to_bf16(f[(size_t)i]);
  return FLASH_OK;
}

flash_status flash_mlp_set_norm(flash_mlp* m, const float* norm) {
  if (!m || !norm) return fail(FLASH_ERR_INVALID_ARG, "null argument");
  if (!finite_all(norm, kNorm)) return fail(FLASH_ERR_INVALID_ARG, "non-finite normalisation");
  try {
    m->host_norm.assign(norm, norm + kNorm);
    HIPCHK(hipMemcpyAsync(m->norm, norm, kNorm * sizeof(float), hipMemcpyHostToDevice, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_mlp_get_norm(flash_mlp* m, float* norm) {
  if (!m || !norm) return fail(FLASH_ERR_INVALID_ARG, "null argument");
  std::memcpy(norm, m->host_norm.data(), kNorm * sizeof(float));
  return FLASH_OK;
}

flash_status flash_mlp_fit_norm(flash_mlp* m, const float* feat, const float* lab, int64_t n) {
  if (!m || !feat || !lab || n < 2) return fail(FLASH_ERR_INVALID_ARG, "need at least two rows");
  try {
    launch_col_moments(feat, (long)n, kFeat, m->moments, m->stream);
    launch_col_moments(lab, (long)n, kOut, m->moments + 2 * kFeat, m->stream);
    HIPCHK(hipGetLastError());
    double mo[2 * (kFeat + kOut)];
    HIPCHK(hipStreamSynchronize(m->stream));
    HIPCHK(hipMemcpy(mo, m->moments, sizeof(mo), hipMemcpyDeviceToHost));
    std::vector<float> nm(kNorm);
    for (int k = 0; k < kFeat; ++k) {
      const double mean = mo[2 * k] / n, var = std::max(mo[2 * k + 1] / n - mean * mean, 0.0);
      const double sd = std::sqrt(var);
      nm[k] = (float)mean;
      nm[kFeat + k] = sd > 1e-6 ? (float)(1.0 / sd) : 1.f;   // constant columns (the bias input) pass through
    }
    for (int k = 0; k < kOut; ++k) {
      const double* q = mo + 2 * kFeat + 2 * k;
      const double rms = std::sqrt(q[1] / n);
      nm[2 * kFeat + k] = rms > 1e-12 ? (float)(1.0 / rms) : 1.f;
    }
    // the bias feature stays 1 after normalisation
    nm[kFeat - 1] = 0.f;
    nm[2 * kFeat - 1] = 1.f;
    return flash_mlp_set_norm(m, nm.data());
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
}

flash_status flash_mlp_forward(flash_mlp* m, const float* x, int64_t n, float* y) {
  if (!m || !x || !y || n < 0) return fail(FLASH_ERR_INVALID_ARG, "null or negative argument");
  try {
    launch_mlp_fused(m->W, nullptr, x, (long)n, nullptr, y, nullptr, nullptr, nullptr, m->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(m->stream));
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_mlp_grad(flash_mlp* m, const float* x, const float* target, int64_t n, float* grad, float* loss) {
  if (!m || !x || !target || !grad || n <= 0) return fail(FLASH_ERR_INVALID_ARG, "null or empty argument");
  if (n > m->max_rows) return fail(FLASH_ERR_CAPACITY, "n exceeds the network's max_rows");
  try {
    HIPCHK(hipMemcpyAsync(m->X, x, n * kFeat * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
    HIPCHK(hipMemcpyAsync(m->L, target, n * kOut * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
    m->grad((long)n, m->loss);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(m->stream));
    HIPCHK(hipMemcpy(grad, m->G, MlpLayout::total * sizeof(float), hipMemcpyDeviceToHost));
    if (loss) HIPCHK(hipMemcpy(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost));
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_mlp_grad_noalloc(const float* params, const float* x, const float* target, int64_t n,
                                    float* grad, float* loss, void* hip_stream) {
  if (!params || !x || !target || !grad || n <= 0) return fail(FLASH_ERR_INVALID_ARG, "null or empty argument");
  if (n > kNaRows)
    return fail(FLASH_ERR_CAPACITY, "flash_mlp_grad_noalloc takes at most " + std::to_string(kNaRows) + " rows, got " +
                                        std::to_string((long long)n));
  try {
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    unsigned char* base = noalloc_scratch();
    prepare_mlp();
    double* partial = reinterpret_cast<double*>(base + kNaOffPartial);
    float* H1 = reinterpret_cast<float*>(base + kNaOffH);
    float* H2 = reinterpret_cast<float*>(base + kNaOffH + kNaHid);
    float* H3 = reinterpret_cast<float*>(base + kNaOffH + 2 * kNaHid);
    float* dA = reinterpret_cast<float*>(base + kNaOffH + 3 * kNaHid);
    float* dB = reinterpret_cast<float*>(base + kNaOffH + 4 * kNaHid);
    float* Y = reinterpret_cast<float*>(base + kNaOffY);
    float* dY = reinterpret_cast<float*>(base + kNaOffY + kNaOut);
    float* work = reinterpret_cast<float*>(base + kNaOffWork);
    // the loss goes to the caller's buffer, or to a slot after the network output when none is given
    float* loss_dst = loss ? loss : reinterpret_cast<float*>(base + kNaOffY + 2 * kNaOut);
    launch_mlp_fused(params, nullptr, x, (long)n, nullptr, Y, H1, H2, H3, s);
    mlp_loss(Y, target, (long)n, dY, partial, loss_dst, s);
    mlp_backward(params, x, (long)n, H1, H2, H3, dY, dA, dB, grad, work, kNaWork, s);
    HIPCHK(hipGetLastError());
  } catch (const FlashError& ex) {
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_mlp_train(flash_mlp* m, const float* feat, const float* lab, int64_t n, int32_t epochs,
                             int32_t batch, float lr, uint64_t seed, float* epoch_loss) {
  if (!m || !feat || !lab || n <= 0 || epochs <= 0 || batch <= 0 || !(lr > 0.f))
    return fail(FLASH_ERR_INVALID_ARG, "bad training arguments");
  if (batch > m->max_rows) return fail(FLASH_ERR_CAPACITY, "batch exceeds the network's max_rows");
  if (n > INT32_MAX) return fail(FLASH_ERR_INVALID_ARG, "too many rows");
  const long nb = (long)(n / batch);
  if (nb < 1) return fail(FLASH_ERR_INVALID_ARG, "fewer rows than one minibatch");
  if (nb > (1 << 16)) return fail(FLASH_ERR_INVALID_ARG, "more than 65536 minibatches per epoch");
  int* idx = nullptr;
  try {
    HIPCHK(hipMalloc(&idx, (size_t)n * sizeof(int)));
    std::vector<int> perm((size_t)n);
    std::vector<float> lh((size_t)nb);
    SplitMix64 rng(seed);
    for (int ep = 0; ep < epochs; ++ep) {
      for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = (int)i;
      for (int64_t i = n - 1; i > 0; --i) std::swap(perm[(size_t)i], perm[(size_t)rng.below((uint64_t)i + 1)]);
      HIPCHK(hipMemcpyAsync(idx, perm.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, m->stream));
      for (long q = 0; q < nb; ++q) {
        launch_gather_batch(feat, lab, idx + q * batch, batch, m->norm, m->X, m->L, m->stream);
        m->grad(batch, m->loss + q);
        launch_adam(m->W, m->G, m->Mo, m->Vo, (int)MlpLayout::total, lr, ++m->adam_t, m->stream);
      }
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(m->stream));
      HIPCHK(hipMemcpy(lh.data(), m->loss, nb * sizeof(float), hipMemcpyDeviceToHost));
      double s = 0.0;
      for (float v : lh) s += v;
      if (epoch_loss) epoch_loss[ep] = (float)(s / nb);
      if (!std::isfinite(s)) throw FlashError(FLASH_ERR_NONFINITE, "training loss became non-finite");
    }
    HIPCHK(hipFree(idx));
  } catch (const FlashError& ex) {
    if (idx) (void)hipFree(idx);
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

flash_status flash_mlp_eval(flash_mlp* m, const float* feat, const float* lab, int64_t n, float* loss) {
  if (!m || !feat || !lab || !loss || n <= 0) return fail(FLASH_ERR_INVALID_ARG, "null or empty argument");
  int* idx = nullptr;
  try {
    HIPCHK(hipMalloc(&idx, (size_t)std::min<int64_t>(n, m->max_rows) * sizeof(int)));
    double s = 0.0;
    for (int64_t r0 = 0; r0 < n; r0 += m->max_rows) {
      const long rows = (long)std::min<int64_t>(m->max_rows, n - r0);
      std::vector<int> id((size_t)rows);
      for (long i = 0; i < rows; ++i) id[(size_t)i] = (int)(r0 + i);
      HIPCHK(hipMemcpyAsync(idx, id.data(), rows * sizeof(int), hipMemcpyHostToDevice, m->stream));
      launch_gather_batch(feat, lab, idx, (int)rows, m->norm, m->X, m->L, m->stream);
      launch_mlp_fused(m->W, nullptr, m->X, rows, nullptr, m->Y, nullptr, nullptr, nullptr, m->stream);
      mlp_loss(m->Y, m->L, rows, m->dY, m->partial, m->loss, m->stream);
      float l = 0.f;
      HIPCHK(hipStreamSynchronize(m->stream));
      HIPCHK(hipMemcpy(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost));
      s += (double)l * rows;
    }
    *loss = (float)(s / n);
    HIPCHK(hipFree(idx));
  } catch (const FlashError& ex) {
    if (idx) (void)hipFree(idx);
    return fail(ex.st, ex.what());
  }
  return FLASH_OK;
}

}  // extern "C"
