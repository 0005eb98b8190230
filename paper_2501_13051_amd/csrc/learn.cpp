// Host side of the join-cardinality MLP: gradient, training and BF16
// inference entry points, all running on the GPU kernels of kern_learn.hip.
#include <hip/hip_runtime_api.h>

#include <algorithm>
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

// Device buffers of one call, from the caller's allocator hooks (fv_options)
// when given, else hipMalloc; freed when the call returns.  Copies and
// kernels run on the options' stream.
struct Dev {
  const fv_options* opt;
  hipStream_t stream;
  std::vector<void*> bufs;
  bool ok = true;
  explicit Dev(const fv_options* o) : opt(o && o->dev_alloc && o->dev_free ? o : nullptr),
                                      stream(o ? static_cast<hipStream_t>(o->stream) : nullptr) {}
  void* raw(size_t bytes) {
    void* p = nullptr;
    bytes = std::max<size_t>(bytes, 4);
    if (opt) {
      p = opt->dev_alloc(bytes, opt->stream, opt->user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    if (!p) { ok = false; return nullptr; }
    bufs.push_back(p);
    return p;
  }
  float* get(size_t n) { return static_cast<float*>(raw(n * sizeof(float))); }
  bool to_dev(void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream) == hipSuccess;
  }
  bool to_host(void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream) == hipSuccess &&
           hipStreamSynchronize(stream) == hipSuccess;
  }
  ~Dev() {
    if (!bufs.empty()) (void)hipStreamSynchronize(stream);
    for (void* p : bufs) {
      if (opt) opt->dev_free(p, opt->stream, opt->user);
      else (void)hipFree(p);
    }
  }
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

fv_status fv_mlp_grad(const fv_options* opt, const float* X, const float* y, uint32_t n, const float* params,
                      float* grads, float* loss) {
  if (!X || !y || !params || !grads || n == 0) return FV_EINVAL;
  Dev d(opt);
  Work w;
  float* P = d.get(fv::kMlpParams);
  float* G = d.get(fv::kMlpParams);
  if (!w.alloc(d, n) || !P || !G) { g_err = "device allocation failed"; return FV_ENOMEM; }
  if (!d.to_dev(w.X, X, size_t(n) * fv::kMlpIn * 4) || !d.to_dev(w.y, y, size_t(n) * 4) ||
      !d.to_dev(P, params, fv::kMlpParams * 4)) { g_err = "copy failed"; return FV_EHIP; }
  const fv_status rc = fwd_bwd(w, n, P, G, d.stream);
  if (rc != FV_OK) return rc;
  if (!d.to_host(grads, G, fv::kMlpParams * 4)) { g_err = "copy failed"; return FV_EHIP; }
  if (loss && !d.to_host(loss, w.loss, 4)) { g_err = "copy failed"; return FV_EHIP; }
  return FV_OK;
}

fv_status fv_mlp_train(const fv_options* opt, const float* X, const float* y, uint32_t n, uint32_t steps, float lr,
                       uint64_t seed, int init, float* params, float* loss) {
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
  Dev d(opt);
  Work w;
  float* P = d.get(fv::kMlpParams);
  float* G = d.get(fv::kMlpParams);
  float* M = d.get(fv::kMlpParams);
  float* V = d.get(fv::kMlpParams);
  if (!w.alloc(d, n) || !P || !G || !M || !V) { g_err = "device allocation failed"; return FV_ENOMEM; }
  if (!d.to_dev(w.X, X, size_t(n) * fv::kMlpIn * 4) || !d.to_dev(w.y, y, size_t(n) * 4) ||
      !d.to_dev(P, h.data(), fv::kMlpParams * 4) ||
      hipMemsetAsync(M, 0, fv::kMlpParams * 4, d.stream) != hipSuccess ||
      hipMemsetAsync(V, 0, fv::kMlpParams * 4, d.stream) != hipSuccess) {
    g_err = "copy failed";
    return FV_EHIP;
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  double p1 = 1, p2 = 1;
  for (uint32_t t = 0; t < steps; ++t) {
    const fv_status rc = fwd_bwd(w, n, P, G, d.stream);
    if (rc != FV_OK) return rc;
    p1 *= b1;
    p2 *= b2;
    CK(fv::launch_adam(P, G, M, V, fv::kMlpParams, lr, b1, b2, eps, float(1 - p1), float(1 - p2), d.stream));
  }
  // final loss at the trained parameters
  const fv_status rc = fwd_bwd(w, n, P, G, d.stream);
  if (rc != FV_OK) return rc;
  if (!d.to_host(params, P, fv::kMlpParams * 4)) { g_err = "copy failed"; return FV_EHIP; }
  if (loss && !d.to_host(loss, w.loss, 4)) { g_err = "copy failed"; return FV_EHIP; }
  return FV_OK;
}

fv_status fv_mlp_predict(const fv_options* opt, const float* X, uint32_t n, const float* params, float* yhat) {
  if (!X || !params || !yhat) return FV_EINVAL;
  if (n == 0) return FV_OK;
  Dev d(opt);
  float* dX = d.get(size_t(n) * fv::kMlpIn);
  float* P = d.get(fv::kMlpParams);
  float* out = d.get(n);
  if (!d.ok) { g_err = "device allocation failed"; return FV_ENOMEM; }
  if (!d.to_dev(dX, X, size_t(n) * fv::kMlpIn * 4) || !d.to_dev(P, params, fv::kMlpParams * 4)) {
    g_err = "copy failed";
    return FV_EHIP;
  }
  CK(fv::launch_mlp_infer_bf16(dX, n, P, out, d.stream));
  if (!d.to_host(yhat, out, size_t(n) * 4)) { g_err = "copy failed"; return FV_EHIP; }
  return FV_OK;
}

fv_status fv_hll_ndv(const fv_options* opt, const uint32_t* const* cols, uint32_t n_cols, uint64_t n_rows,
                     int on_device, double* estimates) {
  if (!cols || !estimates) { g_err = "null argument"; return FV_EINVAL; }
  for (uint32_t c = 0; c < n_cols; ++c)
    if (!cols[c] && n_rows) { g_err = "null column"; return FV_EINVAL; }
  if (n_cols == 0) return FV_OK;
  Dev d(opt);
  // per batch of up to kHllBatch columns: registers, and (estimate, rows) words
  const uint32_t nb = std::min<uint32_t>(n_cols, fv::kHllBatch);
  u32* regs = static_cast<u32*>(d.raw(size_t(nb) * fv::kHllRegs * 4));
  u64* words = static_cast<u64*>(d.raw(size_t(nb) * 16));
  std::vector<u32*> staged;
  if (!on_device && n_rows)
    for (uint32_t c = 0; c < nb; ++c) staged.push_back(static_cast<u32*>(d.raw(n_rows * 4)));
  if (!d.ok) { g_err = "device allocation failed"; return FV_ENOMEM; }
  CK(fv::launch_fill_u32(regs, u64(nb) * fv::kHllRegs, 0u, d.stream));
  std::vector<u64> out(size_t(nb) * 2);
  for (uint32_t c0 = 0; c0 < n_cols; c0 += nb) {
    const uint32_t k = std::min(nb, n_cols - c0);
    CK(fv::launch_fill_u64(words, u64(k) * 2, 0, d.stream));
    fv::HllBatch b{};
    b.n = k;
    for (uint32_t i = 0; i < k; ++i) {
      const u32* col = cols[c0 + i];
      if (!on_device && n_rows) {
        if (!d.to_dev(staged[i], col, n_rows * 4)) { g_err = "copy failed"; return FV_EHIP; }
        col = staged[i];
      }
      fv::HllParams& h = b.s[i];
      h.col[0] = col;
      h.c0 = 0;
      h.c1 = -1;
      h.src.begin = 0;
      h.src.end = n_rows;
      h.src.cap = n_rows;
      h.regs = regs + size_t(i) * fv::kHllRegs;
      h.estimate = words + 2 * i;
      h.rows = words + 2 * i + 1;
    }
    // (the estimate pass clears the registers again for the next batch)
    CK(fv::launch_hll_batch(b, n_rows, d.stream));
    if (!d.to_host(out.data(), words, size_t(k) * 16)) { g_err = "copy failed"; return FV_EHIP; }
    for (uint32_t i = 0; i < k; ++i) std::memcpy(&estimates[c0 + i], &out[2 * i], 8);
  }
  return FV_OK;
}

}  // extern "C"
