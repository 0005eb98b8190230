// Host side of the join-cardinality MLP: gradient, training and BF16
// inference entry points, all running on the GPU kernels of kern_learn.hip.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fv.h"
#include "fv_types.h"

namespace fv {
std::string& global_error();
}

namespace {

using fv::u32;
using fv::u64;

struct Dev {
  std::vector<void*> bufs;
  bool ok = true;
  float* get(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(float)) != hipSuccess) { ok = false; (void)hipGetLastError(); return nullptr; }
    bufs.push_back(p);
    return static_cast<float*>(p);
  }
  ~Dev() { for (void* p : bufs) (void)hipFree(p); }
};

struct Net {   // views into a parameter (or gradient) vector
  float *W1, *b1, *W2, *b2, *W3, *b3;
  explicit Net(float* p) {
    W1 = p;
    b1 = W1 + fv::kMlpHidden * fv::kMlpIn;
    W2 = b1 + fv::kMlpHidden;
    b2 = W2 + fv::kMlpHidden * fv::kMlpHidden;
    W3 = b2 + fv::kMlpHidden;
    b3 = W3 + fv::kMlpHidden;
  }
};

struct Work {
  float *X, *y, *z1, *h1, *z2, *h2, *yhat, *dy, *dh2, *dh1, *loss;
  bool alloc(Dev& d, u32 n) {
    X = d.get(size_t(n) * fv::kMlpIn);
    y = d.get(n);
    z1 = d.get(size_t(n) * fv::kMlpHidden);
    h1 = d.get(size_t(n) * fv::kMlpHidden);
    z2 = d.get(size_t(n) * fv::kMlpHidden);
    h2 = d.get(size_t(n) * fv::kMlpHidden);
    yhat = d.get(n);
    dy = d.get(n);
    dh2 = d.get(size_t(n) * fv::kMlpHidden);
    dh1 = d.get(size_t(n) * fv::kMlpHidden);
    loss = d.get(1);
    return d.ok;
  }
};

#define g_err (fv::global_error())

#define CK(x) do { if ((x) != 0) { g_err = "HIP launch failed: " #x; return FV_EHIP; } } while (0)

constexpr float kInScale = 1.f / 16.f;

// forward + backward for the whole batch: grads (same layout as params), loss
fv_status fwd_bwd(const Work& w, u32 n, float* P, float* G, void* s) {
  Net p(P), g(G);
  const u32 H = fv::kMlpHidden, I = fv::kMlpIn;
  CK(fv::launch_dense_fwd(w.X, n, I, p.W1, p.b1, H, kInScale, w.z1, w.h1, 1, s));
  CK(fv::launch_dense_fwd(w.h1, n, H, p.W2, p.b2, H, 1.f, w.z2, w.h2, 1, s));
  CK(fv::launch_dense_fwd(w.h2, n, H, p.W3, p.b3, 1, 1.f, nullptr, w.yhat, 0, s));
  CK(fv::launch_mse(w.yhat, w.y, n, w.dy, w.loss, s));
  CK(fv::launch_dense_wgrad(w.dy, w.h2, n, H, 1, 1.f, g.W3, g.b3, s));
  CK(fv::launch_dense_dgrad(w.dy, p.W3, n, H, 1, w.dh2, s));
  CK(fv::launch_relu_bwd(w.dh2, w.z2, u64(n) * H, s));
  CK(fv::launch_dense_wgrad(w.dh2, w.h1, n, H, H, 1.f, g.W2, g.b2, s));
  CK(fv::launch_dense_dgrad(w.dh2, p.W2, n, H, H, w.dh1, s));
  CK(fv::launch_relu_bwd(w.dh1, w.z1, u64(n) * H, s));
  CK(fv::launch_dense_wgrad(w.dh1, w.X, n, I, H, kInScale, g.W1, g.b1, s));
  return FV_OK;
}

u64 splitmix(u64& st) {
  u64 z = (st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

fv_status fv_mlp_grad(const float* X, const float* y, uint32_t n, const float* params, float* grads, float* loss) {
  if (!X || !y || !params || !grads || n == 0) return FV_EINVAL;
  Dev d;
  Work w;
  float* P = d.get(fv::kMlpParams);
  float* G = d.get(fv::kMlpParams);
  if (!w.alloc(d, n) || !P || !G) { g_err = "device allocation failed"; return FV_ENOMEM; }
  if (hipMemcpy(w.X, X, size_t(n) * fv::kMlpIn * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w.y, y, size_t(n) * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P, params, fv::kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess) { g_err = "copy failed"; return FV_EHIP; }
  const fv_status rc = fwd_bwd(w, n, P, G, nullptr);
  if (rc != FV_OK) return rc;
  if (hipMemcpy(grads, G, fv::kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess) { g_err = "copy failed"; return FV_EHIP; }
  if (loss && hipMemcpy(loss, w.loss, 4, hipMemcpyDeviceToHost) != hipSuccess) { g_err = "copy failed"; return FV_EHIP; }
  return FV_OK;
}

fv_status fv_mlp_train(const float* X, const float* y, uint32_t n, uint32_t steps, float lr, uint64_t seed,
                       int init, float* params, float* loss) {
  if (!X || !y || !params || n == 0) return FV_EINVAL;
  std::vector<float> h(fv::kMlpParams, 0.f);
  if (init) {   // He-uniform weights from SplitMix64, zero biases
    u64 st = seed;
    Net p(h.data());
    auto fill = [&](float* w, u32 count, u32 fan_in) {
      const double a = std::sqrt(6.0 / fan_in);
      for (u32 i = 0; i < count; ++i) w[i] = float((double(splitmix(st) >> 11) * (1.0 / 9007199254740992.0) * 2 - 1) * a);
    };
    fill(p.W1, fv::kMlpHidden * fv::kMlpIn, fv::kMlpIn);
    fill(p.W2, fv::kMlpHidden * fv::kMlpHidden, fv::kMlpHidden);
    fill(p.W3, fv::kMlpHidden, fv::kMlpHidden);
  } else {
    std::memcpy(h.data(), params, fv::kMlpParams * 4);
  }
  Dev d;
  Work w;
  float* P = d.get(fv::kMlpParams);
  float* G = d.get(fv::kMlpParams);
  float* M = d.get(fv::kMlpParams);
  float* V = d.get(fv::kMlpParams);
  if (!w.alloc(d, n) || !P || !G || !M || !V) { g_err = "device allocation failed"; return FV_ENOMEM; }
  if (hipMemcpy(w.X, X, size_t(n) * fv::kMlpIn * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w.y, y, size_t(n) * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P, h.data(), fv::kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(M, 0, fv::kMlpParams * 4) != hipSuccess || hipMemset(V, 0, fv::kMlpParams * 4) != hipSuccess) {
    g_err = "copy failed";
    return FV_EHIP;
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  double p1 = 1, p2 = 1;
  for (uint32_t t = 0; t < steps; ++t) {
    const fv_status rc = fwd_bwd(w, n, P, G, nullptr);
    if (rc != FV_OK) return rc;
    p1 *= b1;
    p2 *= b2;
    CK(fv::launch_adam(P, G, M, V, fv::kMlpParams, lr, b1, b2, eps, float(1 - p1), float(1 - p2), nullptr));
  }
  // final loss at the trained parameters
  const fv_status rc = fwd_bwd(w, n, P, G, nullptr);
  if (rc != FV_OK) return rc;
  if (hipMemcpy(params, P, fv::kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess) { g_err = "copy failed"; return FV_EHIP; }
  if (loss && hipMemcpy(loss, w.loss, 4, hipMemcpyDeviceToHost) != hipSuccess) { g_err = "copy failed"; return FV_EHIP; }
  return FV_OK;
}

fv_status fv_mlp_predict(const float* X, uint32_t n, const float* params, float* yhat) {
  if (!X || !params || !yhat) return FV_EINVAL;
  if (n == 0) return FV_OK;
  Dev d;
  float* dX = d.get(size_t(n) * fv::kMlpIn);
  float* P = d.get(fv::kMlpParams);
  float* out = d.get(n);
  if (!d.ok) { g_err = "device allocation failed"; return FV_ENOMEM; }
  if (hipMemcpy(dX, X, size_t(n) * fv::kMlpIn * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P, params, fv::kMlpParams * 4, hipMemcpyHostToDevice) != hipSuccess) { g_err = "copy failed"; return FV_EHIP; }
  CK(fv::launch_mlp_infer_bf16(dX, n, P, out, nullptr));
  if (hipMemcpy(yhat, out, size_t(n) * 4, hipMemcpyDeviceToHost) != hipSuccess) { g_err = "copy failed"; return FV_EHIP; }
  return FV_OK;
}

}  // extern "C"
