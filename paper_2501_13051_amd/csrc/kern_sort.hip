// LSD radix sort of packed tuples (Section 5.3: per-column storage lets the
// engine sort tuples with a parallel radix sort rather than a merge sort).
//
// A tuple of a relation is packed into one 64-bit key with per-column bit
// widths taken from the value domain, so a sort touches only the bits that
// can be set.  One histogram pass counts the digits of every pass at once;
// each pass is then a single read and write of the keys ("onesweep"): a tile
// of 2048 keys (4096 in plain 8-bit passes over large buffers) is ranked stably
// in LDS (wave64 match masks built from one ballot per digit bit, per-wave
// digit counters), the tile's per-digit counts
// are chained across tiles with a decoupled look-back, and the keys are staged
// in LDS in digit order so that the global scatter writes contiguous runs.
// Digits are 8 or 11 bits (a tuning knob).
//
// The last pass can also take the difference against full (Section 4, "Union
// and Deduplication") instead of writing the sorted keys: inside a tile, equal
// keys are adjacent in the LDS staging area (earlier passes ordered the low
// bits, this pass the top digit); equal keys in different tiles are settled by
// the tuple set's insert-if-absent, which admits exactly one of them.
// Survivors are appended to full with one atomic reservation per tile.
#include "fv_device.h"

namespace fv {


__device__ __forceinline__ u64 sort_n(const u64* n_ctr, u64 n_const, u64 cap) {
  return n_ctr ? min_u64(*n_ctr, cap) : n_const;
}

template <int kBits>
__global__ __launch_bounds__(kBlock) void k_rs_hist(const u64* keys, const u64* n_ctr, u64 n_const, u64 cap,
                                                   u32 passes, u32* hist, const u32* abort) {
  constexpr int kRadix = 1 << kBits;
  constexpr int kMaxPasses = (64 + kBits - 1) / kBits;
  __shared__ u32 s_h[kMaxPasses * kRadix];
  if (abort && *abort) return;
  const u64 n = sort_n(n_ctr, n_const, cap);
  for (u32 i = threadIdx.x; i < passes * kRadix; i += kBlock) s_h[i] = 0;
  __syncthreads();
  // kH keys per thread and step, loaded before any is counted
  constexpr int kH = 8;
  const u64 stride = u64(gridDim.x) * kBlock;
  const u64 lt_mask = (1ull << lane_id()) - 1;
  for (u64 i0 = u64(blockIdx.x) * kBlock + threadIdx.x; i0 < n; i0 += stride * kH) {
    u64 k[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) k[j] = i0 + j * stride < n ? keys[i0 + j * stride] : 0;
#pragma unroll
    for (int j = 0; j < kH; ++j) {
      // lanes past n are the wave's top lanes (indices rise with the lane),
      // so lane 0 is valid whenever any lane is
      const bool valid = i0 + j * stride < n;
      for (u32 p = 0; p < passes; ++p) {
        // packed keys often share their high digits across a whole wave: the
        // lanes holding lane 0's digit add once, through their lowest lane,
        // instead of queueing on one LDS word; the others add one by one
        const u32 d = u32(k[j] >> (p * kBits)) & (kRadix - 1);
        const u32 d0 = __builtin_amdgcn_readfirstlane(d);
        const bool same = valid && d == d0;
        const u64 m = __ballot(same);
        if (same) {
          if ((m & lt_mask) == 0) atomicAdd(&s_h[p * kRadix + d0], u32(__popcll(m)));
        } else if (valid) {
          atomicAdd(&s_h[p * kRadix + d], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (u32 i = threadIdx.x; i < passes * kRadix; i += kBlock) {
    const u32 c = s_h[i];
    if (c) atomicAdd(&hist[i], c);
  }
}

// Parameters of the fused difference + append (last pass only).
struct FuseArgs {
  u64* set;
  u32* set32;          // 32-bit set (instead of set), with its all-ones flag word
  u64* ones;
  u64 set_mask;
  u32* set_full;
  u32* cols[3];
  const u64* full_n;
  u64* out_delta;      // survivors, reserved atomically per tile
  u32 arity;
  u32 shift[3];
  u32 width[3];
  u64* ts;             // trace timing slot (nullable)
};

template <int kBits, bool kFuse, int kItems, int kB>
__global__ __launch_bounds__(kB) void k_rs_pass(const u64* __restrict__ in, u64* __restrict__ out,
                                                   const u64* n_ctr, u64 n_const, u64 cap, u32 shift,
                                                   const u32* hist_p, u64* status, u32* ticket,
                                                   const u32* epoch_base, u32 epoch_off, const u32* abort,
                                                   FuseArgs fz) {
  constexpr int kRadix = 1 << kBits;
  constexpr int kWaves = kB / kWave;
  // kItems keys per thread (see launch_rs_pass for the choice)
  constexpr u32 kTile = kB * kItems;
  constexpr int kDpt = kRadix > kB ? kRadix / kB : 1;   // digits owned per thread
  __shared__ u64 s_keys[kTile];
  __shared__ u32 s_wcnt[kWaves][kRadix];
  __shared__ u32 s_tstart[kRadix + 1];
  __shared__ u64 s_base[kRadix];
  __shared__ u32 s_scan32[kWaves + 1];
  __shared__ u32 s_ticket;
  __shared__ u64 s_out;
  ktime_start(fz.ts);
  if (abort && *abort) return;
  const u32 epoch = launch_epoch(epoch_base, epoch_off);
  const u64 n = sort_n(n_ctr, n_const, cap);
  const u32 ntiles = u32((n + kTile - 1) / kTile);
  const int w = threadIdx.x / kWave;
  const int lane = lane_id();
  const u64 lt_mask = (1ull << lane) - 1;
  if (blockIdx.x >= participants(ntiles)) return;
  u64 fbase = 0;
  if (kFuse) fbase = *fz.full_n;
  {
    // global digit bases: exclusive scan of this pass's histogram
    u32 run = 0;
    for (int j = 0; j < kDpt; ++j) {
      const int d = threadIdx.x * kDpt + j;
      run += d < kRadix ? hist_p[d] : 0u;
    }
    u32 tot;
    u32 ex = block_exclusive_sum<kB>(run, s_scan32, &tot);
    for (int j = 0; j < kDpt; ++j) {
      const int d = threadIdx.x * kDpt + j;
      if (d < kRadix) { s_base[d] = ex; ex += hist_p[d]; }
    }
  }
  __syncthreads();
  u64 dbase[kDpt];
  for (int j = 0; j < kDpt; ++j) {
    const int d = threadIdx.x * kDpt + j;
    dbase[j] = d < kRadix ? s_base[d] : 0;
  }
  for (;;) {
    const u32 tile = take_ticket(ticket, ntiles, &s_ticket);
    if (tile >= ntiles) break;
    for (int i = threadIdx.x; i < kWaves * kRadix; i += kB) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
    const u64 t0 = u64(tile) * kTile;
    u64 key[kItems];
    u32 rank[kItems];
    // all of the tile's loads go out before the ranking (whose ballots and
    // LDS counters would otherwise hold each load back until the last one
    // returned)
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const u64 idx = t0 + u64(w) * (kWave * kItems) + u64(i) * kWave + lane;
      key[i] = idx < n ? in[idx] : 0;
    }
    // (unrolled by 8, not fully: the ranking then fits in 128 registers, four
    // waves per SIMD, and the key and rank arrays are indexed with uniform
    // register offsets)
#pragma unroll 8
    for (int i = 0; i < kItems; ++i) {
      const u64 idx = t0 + u64(w) * (kWave * kItems) + u64(i) * kWave + lane;
      const bool valid = idx < n;
      const u32 dig = valid ? u32((key[i] >> shift) & (kRadix - 1)) : 0u;
      u64 mask = __ballot(valid);
#pragma unroll
      for (int b = 0; b < kBits; ++b) {
        const bool bit = (dig >> b) & 1u;
        const u64 bb = __ballot(bit);
        mask &= bit ? bb : ~bb;
      }
      // lanes with equal digits read the old count, then the lowest of them
      // (the leader) adds the group size; LDS ops of one wave stay in order.
      const u32 old = valid ? s_wcnt[w][dig] : 0u;
      rank[i] = old + u32(__popcll(mask & lt_mask));
      if (valid && (mask & lt_mask) == 0) s_wcnt[w][dig] = old + u32(__popcll(mask));
    }
    __syncthreads();
    u32 tcount[kDpt];
    u32 my_total = 0;
    for (int j = 0; j < kDpt; ++j) {
      const int d = threadIdx.x * kDpt + j;
      u32 run = 0;
      if (d < kRadix) {
        for (int i = 0; i < kWaves; ++i) {
          const u32 c = s_wcnt[i][d];
          s_wcnt[i][d] = run;
          run += c;
        }
        atomic_store_u64(status + u64(tile) * kRadix + d, lb_word(epoch, tile == 0 ? kFlagPrefix : kFlagAgg, run));
      }
      tcount[j] = run;
      my_total += run;
    }
    {
      u32 ttot;
      u32 ex = block_exclusive_sum<kB>(my_total, s_scan32, &ttot);
      for (int j = 0; j < kDpt; ++j) {
        const int d = threadIdx.x * kDpt + j;
        if (d < kRadix) s_tstart[d] = ex;
        ex += tcount[j];
      }
      if (threadIdx.x == 0) s_tstart[kRadix] = ttot;
    }
    __syncthreads();
    // stage the tile in LDS in digit order now (the local positions are
    // known), so that the keys and ranks are dead during the look-back
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const u64 idx = t0 + u64(w) * (kWave * kItems) + u64(i) * kWave + lane;
      if (idx < n) {
        const u32 dig = u32((key[i] >> shift) & (kRadix - 1));
        s_keys[s_tstart[dig] + s_wcnt[w][dig] + rank[i]] = key[i];
      }
    }
    for (int j = 0; j < kDpt; ++j) {
      const int d = threadIdx.x * kDpt + j;
      if (d >= kRadix) continue;
      u64 excl = 0;
      if (tile > 0) {
        // walk this digit's chain back to the nearest inclusive prefix, reading
        // a window of kWin predecessor tiles per round trip (a row of the
        // status array is contiguous over digits, so the loads coalesce).
        // The prefix is usually among the last few tiles: a window of 4 keeps
        // the status reads at a quarter of the tile's key bytes (these loads
        // bypass the L2, so each one costs HBM or Infinity Cache traffic).
        constexpr int kWin = 4;
        long long t = (long long)tile - 1;
        for (;;) {
          u64 wd[kWin];
#pragma unroll
          for (int q = 0; q < kWin; ++q)
            wd[q] = (t - q >= 0) ? atomic_load_u64(status + u64(t - q) * kRadix + d) : lb_word(epoch, kFlagPrefix, 0);
          bool done = false;
          for (int q = 0; q < kWin; ++q) {
            u64 f = lb_flag(wd[q], epoch);
            while (f == 0) {   // not published yet: its tile is owned by a running block
              __builtin_amdgcn_s_sleep(1);
              wd[q] = atomic_load_u64(status + u64(t - q) * kRadix + d);
              f = lb_flag(wd[q], epoch);
            }
            excl += wd[q] & kValueMask;
            if (f == kFlagPrefix) { done = true; break; }
          }
          if (done) break;
          t -= kWin;
        }
        atomic_store_u64(status + u64(tile) * kRadix + d, lb_word(epoch, kFlagPrefix, excl + tcount[j]));
      }
      s_base[d] = dbase[j] + excl;
    }
    __syncthreads();
    const u32 tn = u32(min_u64(kTile, n - t0));
    if (!kFuse) {
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        const u32 q = u32(i) * kB + threadIdx.x;
        if (q < tn) {
          const u64 k = s_keys[q];
          const u32 dq = u32((k >> shift) & (kRadix - 1));
          out[s_base[dq] + (q - s_tstart[dq])] = k;
        }
      }
    } else {
      // difference against full and append; consecutive LDS slots of one
      // digit hold consecutive keys of the sorted order
      bool surv[kItems], first[kItems];
      u64 kk[kItems];
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        const u32 q = threadIdx.x * kItems + u32(i);
        first[i] = false;
        kk[i] = 0;
        if (q < tn) {
          kk[i] = s_keys[q];
          const u32 dq = u32((kk[i] >> shift) & (kRadix - 1));
          first[i] = q == s_tstart[dq] || s_keys[q - 1] != kk[i];
        }
      }
      // the tile's set probes go out together (one round trip, not kItems)
      int ins[kItems];
      if (fz.set32) set32_insert_many<kItems>(fz.set32, fz.set_mask, kk, first, ins, fz.ones);
      else set_insert_many<kItems>(fz.set, fz.set_mask, kk, first, ins);
      u32 mine = 0;
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        if (ins[i] < 0) *fz.set_full = 1;
        surv[i] = first[i] && ins[i] > 0;
        mine += surv[i] ? 1u : 0u;
      }
      u32 tot;
      const u32 ex = block_exclusive_sum<kB>(mine, s_scan32, &tot);
      if (threadIdx.x == 0)
        s_out = tot ? atomicAdd(reinterpret_cast<unsigned long long*>(fz.out_delta), (unsigned long long)tot) : 0;
      __syncthreads();
      u64 pos = fbase + s_out + ex;
#pragma unroll
      for (int i = 0; i < kItems; ++i) {
        if (!surv[i]) continue;
        const u64 k = s_keys[threadIdx.x * kItems + u32(i)];
        for (u32 c = 0; c < fz.arity; ++c) {
          const u64 m = fz.width[c] >= 32 ? 0xFFFFFFFFull : ((1ull << fz.width[c]) - 1);
          fz.cols[c][pos] = u32((k >> fz.shift[c]) & m);
        }
        ++pos;
      }
    }
    __syncthreads();
  }
  ktime_end(fz.ts);
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
  const u32 db = p.digit_bits == 11 ? 11 : 8;
  const u32 passes = sort_passes(p.bits, db);
  if (passes == 0) return 0;
  if (clear_hist) launch_fill_u32(p.hist, u64(passes) << db, 0u, stream);
  const u64 tiles = (p.cap + kSortTile - 1) / kSortTile;
  const int hgrid = int(tiles == 0 ? 1 : (tiles > 4096 ? 4096 : tiles));
  if (db == 11)
    hipLaunchKernelGGL(k_rs_hist<11>, dim3(hgrid), dim3(kBlock), 0, (hipStream_t)stream, p.a, p.n_ctr, p.n_const,
                       p.cap, passes, p.hist, p.abort);
  else
    hipLaunchKernelGGL(k_rs_hist<8>, dim3(hgrid), dim3(kBlock), 0, (hipStream_t)stream, p.a, p.n_ctr, p.n_const,
                       p.cap, passes, p.hist, p.abort);
  return int(hipGetLastError());
}

int launch_rs_pass(const SortParams& p, u32 pass, const u64* src, u64* dst, u32 epoch_off, void* stream,
                   const SortFuse* fuse) {
  const u32 db = p.digit_bits == 11 ? 11 : 8;
  const u64 tiles = (p.cap + kSortTile - 1) / kSortTile;
  const u64 maxg = p.max_blocks ? p.max_blocks : 2048;
  const int pgrid = int(tiles == 0 ? 1 : (tiles > maxg ? maxg : tiles));
  FuseArgs fz{};
  fz.ts = p.ts;
  if (fuse) {
    fz.set = fuse->set;
    fz.set32 = fuse->set32;
    fz.ones = fuse->ones;
    fz.set_mask = fuse->set_mask;
    fz.set_full = fuse->set_full;
    for (int c = 0; c < 3; ++c) {
      fz.cols[c] = fuse->cols[c];
      fz.shift[c] = fuse->shift[c];
      fz.width[c] = fuse->width[c];
    }
    fz.full_n = fuse->full_n;
    fz.out_delta = fuse->out_delta;
    fz.arity = fuse->arity;
  }
  const u32 sh = pass * db;
  const u32* h = p.hist + (u64(pass) << db);
  hipStream_t s = (hipStream_t)stream;
  // Keys per thread: 16 (4096-key tiles, half the per-tile look-back and
  // scan work) for a plain 8-bit pass over at least 2^22 keys (expected, or
  // the buffer's capacity);
  // 8 otherwise, where more, smaller tiles keep the chip busy (small sorts),
  // 11-bit digit counters need the LDS, or the fused pass probes the set.
  const bool wide = db == 8 && !fuse && (p.n_hint ? p.n_hint : p.cap) >= (u64(1) << 22);
#define FV_PASS(B, F, I, T, G)                                                                               \
  hipLaunchKernelGGL((k_rs_pass<B, F, I, T>), dim3(G), dim3(T), 0, s, src, dst, p.n_ctr, p.n_const, p.cap, sh, h, \
                     p.status, p.ticket, p.epoch_base, epoch_off, p.abort, fz)
  if (db == 11) {
    if (fuse) FV_PASS(11, true, 8, kBlock, pgrid); else FV_PASS(11, false, 8, kBlock, pgrid);
  } else if (fuse) {
    FV_PASS(8, true, 8, kBlock, pgrid);
  } else if (wide) {
    // 512-thread blocks: 8,192-key tiles, half the tiles (and their
    // look-back chains) of 256-thread blocks, at the same four waves per SIMD
    const u64 wtiles = (p.cap + 8192 - 1) / 8192;
    const u64 wmax = maxg / 2 ? maxg / 2 : 1;
    const int wgrid = int(wtiles == 0 ? 1 : (wtiles > wmax ? wmax : wtiles));
    FV_PASS(8, false, 16, 512, wgrid);
  } else {
    FV_PASS(8, false, 8, kBlock, pgrid);
  }
#undef FV_PASS
  return int(hipGetLastError());
}

}  // namespace fv
