// fv_hll_ndv_noalloc: the per-column HyperLogLog estimates of fv_hll_ndv for
// callers that cannot allocate device memory.  The sketch registers and
// row counters live in `scratch`, a file-scope device array (one copy per
// GPU, held until the process ends); the kernels are those of fv_hll_ndv.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "../../include/fv.h"
#include "fv_types.h"

namespace fv {
std::string& global_error();
}

namespace {

using fv::u32;
using fv::u64;

// kHllBatch sketches: their registers, then an (estimate, rows) word pair each.
constexpr u64 kRegWords = u64(fv::kHllBatch) * fv::kHllRegs / 2;   // u32 registers, two per u64
constexpr u64 kScratchWords = kRegWords + 2 * fv::kHllBatch;
static_assert(FV_HLL_NOALLOC_MAX_COLS == fv::kHllBatch, "one launch sketches at most kHllBatch columns");

__device__ __align__(256) u64 scratch[kScratchWords];

// The host-side name of `scratch` is not its device address: each device's
// copy is looked up once, with that device current, and only that address is
// handed to kernels.
constexpr int kMaxDevices = 64;
u64* g_scratch[kMaxDevices] = {};
std::mutex g_mu;

hipError_t scratch_of_current_device(u64** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<u64*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" fv_status fv_hll_ndv_noalloc(const uint32_t* const* cols, uint32_t n_cols, uint64_t n_rows,
                                        double* estimates, void* stream) {
  auto fail = [](fv_status rc, const char* msg) {
    fv::global_error() = msg;
    return rc;
  };
  if (!cols || !estimates) return fail(FV_EINVAL, "null argument");
  if (n_cols > FV_HLL_NOALLOC_MAX_COLS)
    return fail(FV_EINVAL, "fv_hll_ndv_noalloc sketches at most FV_HLL_NOALLOC_MAX_COLS (8) columns per call");
  for (uint32_t c = 0; c < n_cols; ++c)
    if (!cols[c] && n_rows) return fail(FV_EINVAL, "null column");
  if (n_cols == 0) return FV_OK;
  u64* base = nullptr;
  if (scratch_of_current_device(&base) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FV_EHIP, "cannot find the scratch array on the current device");
  }
  u32* regs = reinterpret_cast<u32*>(base);
  u64* words = base + kRegWords;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the array keeps the last call's contents: clear registers and counters
  // (fill kernels, no memset, so that the call may be captured in a graph)
  if (fv::launch_fill_u32(regs, u64(n_cols) * fv::kHllRegs, 0u, s) != 0 ||
      fv::launch_fill_u64(words, 2 * u64(n_cols), 0, s) != 0)
    return fail(FV_EHIP, "fill launch failed");
  fv::HllBatch b{};
  b.n = n_cols;
  for (uint32_t i = 0; i < n_cols; ++i) {
    fv::HllParams& h = b.s[i];
    h.col[0] = cols[i];
    h.c0 = 0;
    h.c1 = -1;
    h.src.begin = 0;
    h.src.end = n_rows;
    h.src.cap = n_rows;
    h.regs = regs + size_t(i) * fv::kHllRegs;
    // the estimate pass writes the double's bits straight into the caller's array
    h.estimate = reinterpret_cast<u64*>(estimates + i);
    h.rows = words + 2 * i + 1;
  }
  if (fv::launch_hll_batch(b, n_rows, s) != 0) return fail(FV_EHIP, "sketch launch failed");
  return FV_OK;
}
