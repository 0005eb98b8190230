// LSD radix sort of packed tuples (Section 5.3: per-column storage lets the
// engine sort tuples with a parallel radix sort rather than a merge sort).
//
// A tuple of a relation is packed into one 64-bit key with per-column bit
// widths taken from the value domain, so a sort touches only the bits that
// can be set.  One histogram pass counts the 8-bit digits of every pass at
// once; each pass is then a single read and write of the keys ("onesweep"):
// a tile of 2048 keys is ranked stably in LDS (wave64 match masks built from
// eight ballots, per-wave digit counters), the tile's per-digit counts are
// chained across tiles with a decoupled look-back, and the keys are staged in
// LDS in digit order so that the global scatter writes contiguous runs.
#include "fv_device.h"

namespace fv {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortItems = kSortTile / kBlock;   // 8 keys per thread
constexpr int kMaxPasses = 8;
static_assert(kBlock == kRadix, "one thread per digit");

__device__ __forceinline__ u64 sort_n(const u64* n_ctr, u64 n_const, u64 cap) {
  return n_ctr ? min_u64(*n_ctr, cap) : n_const;
}

__global__ __launch_bounds__(kBlock) void k_rs_hist(const u64* keys, const u64* n_ctr, u64 n_const, u64 cap,
                                                   u32 passes, u32* hist, const u32* abort) {
  __shared__ u32 s_h[kMaxPasses][kRadix];
  if (abort && *abort) return;
  const u64 n = sort_n(n_ctr, n_const, cap);
  for (u32 p = 0; p < passes; ++p) s_h[p][threadIdx.x] = 0;
  __syncthreads();
  for (u64 i = u64(blockIdx.x) * kBlock + threadIdx.x; i < n; i += u64(gridDim.x) * kBlock) {
    const u64 k = keys[i];
    for (u32 p = 0; p < passes; ++p) atomicAdd(&s_h[p][(k >> (p * kRadixBits)) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  for (u32 p = 0; p < passes; ++p) {
    const u32 c = s_h[p][threadIdx.x];
    if (c) atomicAdd(&hist[p * kRadix + threadIdx.x], c);
  }
}

__global__ __launch_bounds__(kBlock) void k_rs_pass(const u64* __restrict__ in, u64* __restrict__ out,
                                                   const u64* n_ctr, u64 n_const, u64 cap, u32 shift,
                                                   const u32* hist_p, u64* status, u32* ticket,
                                                   const u32* epoch_base, u32 epoch_off, const u32* abort) {
  constexpr int kWaves = kBlock / kWave;
  __shared__ u64 s_keys[kSortTile];
  __shared__ u32 s_wcnt[kWaves][kRadix];
  __shared__ u32 s_tstart[kRadix];
  __shared__ u64 s_gbase[kRadix];
  __shared__ u64 s_dbase[kRadix];
  __shared__ u32 s_scan32[kWaves + 1];
  __shared__ u32 s_ticket;
  if (abort && *abort) return;
  const u32 epoch = launch_epoch(epoch_base, epoch_off);
  const u64 n = sort_n(n_ctr, n_const, cap);
  const u32 ntiles = u32((n + kSortTile - 1) / kSortTile);
  const int d = threadIdx.x;            // the digit this thread owns in per-digit steps
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  const u64 lt_mask = (1ull << lane) - 1;
  {
    u32 tot;
    s_dbase[d] = block_exclusive_sum<kBlock>(hist_p[d], s_scan32, &tot);
  }
  if (blockIdx.x >= participants(ntiles)) return;
  for (;;) {
    const u32 tile = take_ticket(ticket, ntiles, &s_ticket);
    if (tile >= ntiles) break;
    for (int i = 0; i < kWaves; ++i) s_wcnt[i][d] = 0;
    __syncthreads();
    const u64 t0 = u64(tile) * kSortTile;
    u64 key[kSortItems];
    u32 dig[kSortItems];
    u32 rank[kSortItems];
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const u64 idx = t0 + u64(w) * (kWave * kSortItems) + u64(i) * kWave + lane;
      const bool valid = idx < n;
      key[i] = valid ? in[idx] : 0;
      dig[i] = valid ? u32((key[i] >> shift) & (kRadix - 1)) : 0u;
      u64 mask = __ballot(valid);
#pragma unroll
      for (int b = 0; b < kRadixBits; ++b) {
        const bool bit = (dig[i] >> b) & 1u;
        const u64 bb = __ballot(bit);
        mask &= bit ? bb : ~bb;
      }
      // lanes with equal digits read the old count, then the lowest of them
      // (the leader) adds the group size; LDS ops of one wave stay in order.
      const u32 old = valid ? s_wcnt[w][dig[i]] : 0u;
      rank[i] = old + u32(__popcll(mask & lt_mask));
      if (valid && (mask & lt_mask) == 0) s_wcnt[w][dig[i]] = old + u32(__popcll(mask));
    }
    __syncthreads();
    u32 run = 0;
    for (int i = 0; i < kWaves; ++i) {
      const u32 c = s_wcnt[i][d];
      s_wcnt[i][d] = run;
      run += c;
    }
    const u32 tcount = run;
    u64* st = status + u64(tile) * kRadix + d;
    if (tile == 0) atomic_store_u64(st, lb_word(epoch, kFlagPrefix, tcount));
    else atomic_store_u64(st, lb_word(epoch, kFlagAgg, tcount));
    u32 ttot;
    const u32 tstart = block_exclusive_sum<kBlock>(tcount, s_scan32, &ttot);
    s_tstart[d] = tstart;
    u64 excl = 0;
    if (tile > 0) {
      // walk this digit's chain back to the nearest inclusive prefix, reading
      // a window of kWin predecessor tiles per round trip (rows of the status
      // array are contiguous over digits, so the loads coalesce)
      constexpr int kWin = 16;
      long long t = (long long)tile - 1;
      for (;;) {
        u64 wd[kWin];
#pragma unroll
        for (int j = 0; j < kWin; ++j)
          wd[j] = (t - j >= 0) ? atomic_load_u64(status + u64(t - j) * kRadix + d) : lb_word(epoch, kFlagPrefix, 0);
        bool done = false;
        int j = 0;
        for (; j < kWin; ++j) {
          u64 f = lb_flag(wd[j], epoch);
          while (f == 0) {                       // not published yet: wait for this one
            __builtin_amdgcn_s_sleep(1);
            wd[j] = atomic_load_u64(status + u64(t - j) * kRadix + d);
            f = lb_flag(wd[j], epoch);
          }
          excl += wd[j] & kValueMask;
          if (f == kFlagPrefix) { done = true; break; }
        }
        if (done) break;
        t -= kWin;
      }
      atomic_store_u64(st, lb_word(epoch, kFlagPrefix, excl + tcount));
    }
    s_gbase[d] = s_dbase[d] + excl;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const u64 idx = t0 + u64(w) * (kWave * kSortItems) + u64(i) * kWave + lane;
      if (idx < n) s_keys[s_tstart[dig[i]] + s_wcnt[w][dig[i]] + rank[i]] = key[i];
    }
    __syncthreads();
    const u32 tn = u32(min_u64(kSortTile, n - t0));
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
      const u32 q = u32(i) * kBlock + threadIdx.x;
      if (q < tn) {
        const u64 k = s_keys[q];
        const u32 dq = u32((k >> shift) & (kRadix - 1));
        out[s_gbase[dq] + (q - s_tstart[dq])] = k;
      }
    }
    __syncthreads();
  }
}

__global__ void k_fill_u32(u32* p, u64 n, u32 v) {
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += u64(gridDim.x) * blockDim.x) p[i] = v;
}

__global__ void k_fill_u64(u64* p, u64 n, u64 v) {
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += u64(gridDim.x) * blockDim.x) p[i] = v;
}

static int fill_grid(u64 n) {
  const u64 b = (n + 1023) / 1024;
  return int(b == 0 ? 1 : (b > 4096 ? 4096 : b));
}

int launch_fill_u32(u32* p, u64 n, u32 v, void* stream) {
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, (hipStream_t)stream, p, n, v);
  return int(hipGetLastError());
}

int launch_fill_u64(u64* p, u64 n, u64 v, void* stream) {
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, (hipStream_t)stream, p, n, v);
  return int(hipGetLastError());
}

int launch_rs_hist(const SortParams& p, void* stream, bool clear_hist) {
  const u32 passes = (p.bits + kRadixBits - 1) / kRadixBits;
  if (passes == 0) return 0;
  if (clear_hist) launch_fill_u32(p.hist, u64(passes) * kRadix, 0u, stream);
  const u64 tiles = (p.cap + kSortTile - 1) / kSortTile;
  const int hgrid = int(tiles == 0 ? 1 : (tiles > 1024 ? 1024 : tiles));
  hipLaunchKernelGGL(k_rs_hist, dim3(hgrid), dim3(kBlock), 0, (hipStream_t)stream, p.a, p.n_ctr, p.n_const,
                     p.cap, passes, p.hist, p.abort);
  return int(hipGetLastError());
}

int launch_rs_pass(const SortParams& p, u32 pass, const u64* src, u64* dst, u32 epoch_off, void* stream) {
  const u64 tiles = (p.cap + kSortTile - 1) / kSortTile;
  const int pgrid = int(tiles == 0 ? 1 : (tiles > 2048 ? 2048 : tiles));
  hipLaunchKernelGGL(k_rs_pass, dim3(pgrid), dim3(kBlock), 0, (hipStream_t)stream, src, dst, p.n_ctr, p.n_const,
                     p.cap, pass * kRadixBits, p.hist + pass * kRadix, p.status, p.ticket, p.epoch_base, epoch_off,
                     p.abort);
  return int(hipGetLastError());
}

}  // namespace fv
