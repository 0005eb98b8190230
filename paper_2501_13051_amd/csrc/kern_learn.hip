// Kernels of the learned join-cardinality predictor.
//
// * HyperLogLog (Flajolet, Fusy, Gandouet, Meunier, "HyperLogLog: the
//   analysis of a near-optimal cardinality estimation algorithm", 2007):
//   2^12 registers; a value's 64-bit hash picks a register with its top 12
//   bits and offers rho = 1 + the number of leading zeros of the remaining
//   52 bits; the register keeps the maximum.  The estimate is
//   alpha_m m^2 / sum 2^-M[j], with linear counting m ln(m / V) when it is
//   below 5m/2 and V registers are still zero.
// * A multilayer perceptron 8 -> 64 -> 64 -> 1 with ReLU, trained in FP32 by
//   these kernels (forward, mean-squared-error gradient, backward, Adam) and
//   run for inference with BF16 weights and activations and FP32 sums.
#include "fv_device.h"

namespace fv {

constexpr int kHllP = 12;
constexpr int kHllM = 1 << kHllP;

__device__ __forceinline__ u64 hll_hash(u64 v) { return mix64(v + 0x9E3779B97F4A7C15ull); }

// Sketch blockIdx.y of the batch: registers of the keys of the rows that pass
// the probe filters (kept as the maximum per register), and their count.
__global__ __launch_bounds__(kBlock) void k_hll(HllBatch b) {
  __shared__ u32 s_reg[kHllM];
  const HllParams& p = b.s[blockIdx.y];
  for (int i = threadIdx.x; i < kHllM; i += kBlock) s_reg[i] = 0;
  __syncthreads();
  u64 begin, n;
  source_range(p.src, begin, n);
  u64 kept = 0;
  for (u64 r = u64(blockIdx.x) * kBlock + threadIdx.x; r < n; r += u64(gridDim.x) * kBlock) {
    const u64 row = begin + r;
    bool ok = true;
    for (u32 f = 0; f < p.n_pf; ++f) {
      const u32 a = p.pf[f].a.kind == kSrcConst ? p.pf[f].a.v : p.col[p.pf[f].a.v][row];
      const u32 c = p.pf[f].b.kind == kSrcConst ? p.pf[f].b.v : p.col[p.pf[f].b.v][row];
      ok = ok && (p.pf[f].op == kEq ? a == c : a != c);
    }
    if (!ok) continue;
    ++kept;
    const u64 v = p.c1 >= 0 ? ((u64(p.col[p.c0][row]) << 32) | p.col[p.c1][row]) : u64(p.col[p.c0][row]);
    const u64 h = hll_hash(v);
    const u32 idx = u32(h >> (64 - kHllP));
    const u64 rest = h << kHllP;
    const u32 rho = rest ? u32(__clzll((long long)rest)) + 1 : u32(64 - kHllP + 1);
    atomicMax(&s_reg[idx], rho);
  }
  const u64 wk = wave_sum(kept);
  if (lane_id() == 0 && wk) atomicAdd(reinterpret_cast<unsigned long long*>(p.rows), (unsigned long long)wk);
  __syncthreads();
  // registers only grow, so a register already at least this block's value
  // (read plainly: a stale read is only lower) needs no atomic; after the
  // first blocks most registers hold their final value and the flush is a
  // coalesced read
  for (int i = threadIdx.x; i < kHllM; i += kBlock)
    if (s_reg[i] > p.regs[i]) atomicMax(&p.regs[i], s_reg[i]);
}

// One block per sketch: the estimate (as a double's bits in a u64 counter
// slot), then the registers are cleared for the sketch's next use.
__global__ __launch_bounds__(kBlock) void k_hll_estimate(HllBatch b) {
  __shared__ double s_sum[kBlock];
  __shared__ u32 s_zero[kBlock];
  const HllParams& p = b.s[blockIdx.x];
  double sum = 0;
  u32 zeros = 0;
  for (int i = threadIdx.x; i < kHllM; i += kBlock) {
    const u32 r = p.regs[i];
    sum += ldexp(1.0, -int(r));
    zeros += r == 0;
  }
  s_sum[threadIdx.x] = sum;
  s_zero[threadIdx.x] = zeros;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) { s_sum[threadIdx.x] += s_sum[threadIdx.x + s]; s_zero[threadIdx.x] += s_zero[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = kHllM;
    const double alpha = 0.7213 / (1.0 + 1.079 / m);
    double e = alpha * m * m / s_sum[0];
    if (e <= 2.5 * m && s_zero[0] > 0) e = m * log(m / double(s_zero[0]));
    *p.estimate = __double_as_longlong(e);
  }
  for (int i = threadIdx.x; i < kHllM; i += kBlock) p.regs[i] = 0;
}

int launch_hll_batch(const HllBatch& b, u64 rows_hint, void* stream) {
  if (b.n == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  const u64 blocks = (rows_hint + kBlock - 1) / kBlock;
  const u32 g = u32(blocks == 0 ? 1 : (blocks > 1024 ? 1024 : blocks));
  hipLaunchKernelGGL(k_hll, dim3(g, b.n), dim3(kBlock), 0, s, b);
  hipLaunchKernelGGL(k_hll_estimate, dim3(b.n), dim3(kBlock), 0, s, b);
  return int(hipGetLastError());
}

// ------------------------------------------------------------------ MLP
// Parameter layout (float): W1[64][8] b1[64] W2[64][64] b2[64] W3[1][64] b3[1].
// Inputs are scaled by 1/16 before the first layer (features are log2 sizes).

// out[r][o] = act(sum_i in[r][i] W[o][i] + b[o]); z keeps the pre-activation
__global__ void k_dense_fwd(const float* in, u32 n, u32 din, const float* W, const float* b, u32 dout, float in_scale,
                            float* z, float* out, int relu) {
  const u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= u64(n) * dout) return;
  const u32 r = u32(t / dout), o = u32(t % dout);
  float acc = b[o];
  for (u32 i = 0; i < din; ++i) acc = fmaf(in[u64(r) * din + i] * in_scale, W[u64(o) * din + i], acc);
  if (z) z[t] = acc;
  out[t] = relu ? fmaxf(acc, 0.f) : acc;
}

// d(mean squared error)/d(yhat) and the loss itself (one block)
__global__ void k_mse(const float* yhat, const float* y, u32 n, float* dy, float* loss) {
  __shared__ float s[kBlock];
  float acc = 0;
  for (u32 i = threadIdx.x; i < n; i += kBlock) {
    const float d = yhat[i] - y[i];
    dy[i] = 2.f * d / float(n);
    acc += d * d;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = s[0] / float(n);
}

// dz = dout * relu'(z)  (in place on dout when relu)
__global__ void k_relu_bwd(float* dout, const float* z, u64 n) {
  const u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n && z[t] <= 0.f) dout[t] = 0.f;
}

// dW[o][i] = sum_r dz[r][o] in[r][i] * in_scale;  db[o] = sum_r dz[r][o]
__global__ void k_dense_wgrad(const float* dz, const float* in, u32 n, u32 din, u32 dout, float in_scale, float* dW,
                              float* db) {
  const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < dout * din) {
    const u32 o = t / din, i = t % din;
    float acc = 0;
    for (u32 r = 0; r < n; ++r) acc = fmaf(dz[u64(r) * dout + o], in[u64(r) * din + i] * in_scale, acc);
    dW[t] = acc;
  } else if (t < dout * din + dout) {
    const u32 o = t - dout * din;
    float acc = 0;
    for (u32 r = 0; r < n; ++r) acc += dz[u64(r) * dout + o];
    db[o] = acc;
  }
}

// din[r][i] = sum_o dz[r][o] W[o][i]
__global__ void k_dense_dgrad(const float* dz, const float* W, u32 n, u32 din, u32 dout, float* dinp) {
  const u64 t = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= u64(n) * din) return;
  const u32 r = u32(t / din), i = u32(t % din);
  float acc = 0;
  for (u32 o = 0; o < dout; ++o) acc = fmaf(dz[u64(r) * dout + o], W[u64(o) * din + i], acc);
  dinp[t] = acc;
}

// Adam (Kingma and Ba 2015) with bias correction
__global__ void k_adam(float* p, const float* g, float* m, float* v, u32 n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const u32 t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.f - b1) * gt;
  const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

// FP32 -> BF16 by round-to-nearest-even on the top 16 bits, back to FP32
__device__ __forceinline__ float bf16_round(float x) {
  u32 u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

// Inference: weights and activations rounded to BF16, sums in FP32; one
// thread per row.  out[r] = predicted target.
__global__ void k_mlp_infer_bf16(const float* X, u32 n, const float* P, float* out) {
  const u32 r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const float* W1 = P;
  const float* b1 = W1 + 64 * 8;
  const float* W2 = b1 + 64;
  const float* b2 = W2 + 64 * 64;
  const float* W3 = b2 + 64;
  const float* b3 = W3 + 64;
  float x[8], h1[64];
  for (int i = 0; i < 8; ++i) x[i] = bf16_round(X[u64(r) * 8 + i] * (1.f / 16.f));
  for (int o = 0; o < 64; ++o) {
    float acc = b1[o];
    for (int i = 0; i < 8; ++i) acc = fmaf(x[i], bf16_round(W1[o * 8 + i]), acc);
    h1[o] = bf16_round(fmaxf(acc, 0.f));
  }
  float y = b3[0];
  for (int o = 0; o < 64; ++o) {
    float acc = b2[o];
    for (int i = 0; i < 64; ++i) acc = fmaf(h1[i], bf16_round(W2[o * 64 + i]), acc);
    y = fmaf(bf16_round(fmaxf(acc, 0.f)), bf16_round(W3[o]), y);
  }
  out[r] = y;
}

// ------------------------------------------------------------------ online prediction
// Features of a join (all log2(1 + x)): probe rows, build rows, distinct build
// keys, distinct probe keys (HLL, or the probe rows), mean build run length,
// then the key width, the filter count and the step in the join chain.
__host__ __device__ inline void features_of(double probe, double build, double ndv_b, double ndv_p, u32 nkey,
                                            u32 nfilt, u32 step, float* f) {
  f[0] = float(log2(1.0 + probe));
  f[1] = float(log2(1.0 + build));
  f[2] = float(log2(1.0 + ndv_b));
  f[3] = float(log2(1.0 + ndv_p));
  f[4] = float(log2(1.0 + build / (ndv_b > 1.0 ? ndv_b : 1.0)));
  f[5] = float(nkey);
  f[6] = float(nfilt);
  f[7] = float(step);
}

void join_features(double probe_rows, double build_rows, double ndv_build, double ndv_probe, u32 nkey, u32 nfilt,
                   u32 step, float* f) {
  features_of(probe_rows, build_rows, ndv_build, ndv_probe, nkey, nfilt, step, f);
}

// One block of 64 threads: thread o computes hidden unit o of each layer.
__global__ void k_predict(const PredSpec* specs, u32 n, u64* ctr, const float* P) {
  __shared__ float s_x[8];
  __shared__ float s_h1[64];
  __shared__ float s_part[64];
  const float* W1 = P;
  const float* b1 = W1 + 64 * 8;
  const float* W2 = b1 + 64;
  const float* b2 = W2 + 64 * 64;
  const float* W3 = b2 + 64;
  const float* b3 = W3 + 64;
  const int o = threadIdx.x;
  double prev = 0, prev_bound = 0;
  double bound = 0;   // worst-case output of the current spec (thread 0)
  for (u32 k = 0; k < n; ++k) {
    const PredSpec sp = specs[k];
    if (o == 0) {
      double probe, probe_bound;
      if (sp.step == 0) {
        if (sp.probe_rows >= 0) {
          probe = double(ctr[sp.probe_rows]);
        } else {
          const double full = double(ctr[sp.probe_full]);
          probe = sp.probe_dbeg >= 0 ? full - double(ctr[sp.probe_dbeg]) : full;
        }
        probe_bound = probe;
      } else {
        probe = prev;
        probe_bound = prev_bound;
      }
      const double build = double(ctr[sp.rows_build >= 0 ? sp.rows_build : sp.build_full]);
      bound = probe_bound * (sp.maxrun_build >= 0 ? double(ctr[sp.maxrun_build]) : build);
      const double ndv_b = sp.ndv_build >= 0 ? double(ctr[sp.ndv_build]) : 1.0;
      double ndv_p = probe;
      if (sp.hll >= 0) {
        const double e = __longlong_as_double((long long)ctr[sp.hll]);
        ndv_p = e < probe ? e : probe;
      }
      float f[8];
      features_of(probe, build, ndv_b, ndv_p, sp.nkey, sp.nfilt, sp.step, f);
      for (int i = 0; i < 8; ++i) s_x[i] = bf16_round(f[i] * (1.f / 16.f));
    }
    __syncthreads();
    float acc = b1[o];
    for (int i = 0; i < 8; ++i) acc = fmaf(s_x[i], bf16_round(W1[o * 8 + i]), acc);
    s_h1[o] = bf16_round(fmaxf(acc, 0.f));
    __syncthreads();
    acc = b2[o];
    for (int i = 0; i < 64; ++i) acc = fmaf(s_h1[i], bf16_round(W2[o * 64 + i]), acc);
    s_part[o] = bf16_round(fmaxf(acc, 0.f)) * bf16_round(W3[o]);
    __syncthreads();
    if (o == 0) {
      float y = b3[0];
      for (int i = 0; i < 64; ++i) y += s_part[i];
      // the network predicts log2(1 + m) / 16
      double m = exp2(double(y) * 16.0) - 1.0;
      if (!(m >= 0)) m = 0;
      if (m > bound) m = bound;
      if (m > 1e15) m = 1e15;
      if (bound > 1e15) bound = 1e15;
      ctr[sp.out] = u64(m);
      prev = m;
      prev_bound = bound;
    }
    __syncthreads();
  }
}

int launch_predict(const PredSpec* specs, u32 n, u64* ctr, const float* params, void* stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_predict, dim3(1), dim3(64), 0, (hipStream_t)stream, specs, n, ctr, params);
  return int(hipGetLastError());
}

// ------------------------------------------------------------------ launchers
static dim3 grid1(u64 n) { return dim3(u32((n + kBlock - 1) / kBlock ? (n + kBlock - 1) / kBlock : 1)); }

int launch_dense_fwd(const float* in, u32 n, u32 din, const float* W, const float* b, u32 dout, float in_scale,
                     float* z, float* out, int relu, void* stream) {
  hipLaunchKernelGGL(k_dense_fwd, grid1(u64(n) * dout), dim3(kBlock), 0, (hipStream_t)stream, in, n, din, W, b, dout,
                     in_scale, z, out, relu);
  return int(hipGetLastError());
}

int launch_mse(const float* yhat, const float* y, u32 n, float* dy, float* loss, void* stream) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(kBlock), 0, (hipStream_t)stream, yhat, y, n, dy, loss);
  return int(hipGetLastError());
}

int launch_relu_bwd(float* dout, const float* z, u64 n, void* stream) {
  hipLaunchKernelGGL(k_relu_bwd, grid1(n), dim3(kBlock), 0, (hipStream_t)stream, dout, z, n);
  return int(hipGetLastError());
}

int launch_dense_wgrad(const float* dz, const float* in, u32 n, u32 din, u32 dout, float in_scale, float* dW,
                       float* db, void* stream) {
  hipLaunchKernelGGL(k_dense_wgrad, grid1(u64(dout) * din + dout), dim3(kBlock), 0, (hipStream_t)stream, dz, in, n,
                     din, dout, in_scale, dW, db);
  return int(hipGetLastError());
}

int launch_dense_dgrad(const float* dz, const float* W, u32 n, u32 din, u32 dout, float* dinp, void* stream) {
  hipLaunchKernelGGL(k_dense_dgrad, grid1(u64(n) * din), dim3(kBlock), 0, (hipStream_t)stream, dz, W, n, din, dout,
                     dinp);
  return int(hipGetLastError());
}

int launch_adam(float* p, const float* g, float* m, float* v, u32 n, float lr, float b1, float b2, float eps,
                float c1, float c2, void* stream) {
  hipLaunchKernelGGL(k_adam, grid1(n), dim3(kBlock), 0, (hipStream_t)stream, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return int(hipGetLastError());
}

int launch_mlp_infer_bf16(const float* X, u32 n, const float* P, float* out, void* stream) {
  hipLaunchKernelGGL(k_mlp_infer_bf16, grid1(n), dim3(kBlock), 0, (hipStream_t)stream, X, n, P, out);
  return int(hipGetLastError());
}

}  // namespace fv
