// Join, selection/projection, deduplication and merge kernels.
//
// Join follows the two phases of Algorithm 1 (Section 4, "Join"):
//  * k_probe -- every probe row looks its key up in the build side's unique
//    hashmap and gets a run (start, count) of build row ids; unmatched rows are
//    dropped and the run lengths are prefix-summed, so the output size is known
//    before anything is written (count-then-write, lock-free output).  The
//    filter, reduce and exclusive scan of Algorithm 1 are one pass here: a
//    wave-ballot/block scan per tile and a decoupled look-back across tiles.
//  * k_write -- output-balanced materialisation: output slot n finds the run j
//    with off[j] <= n < off[j+1] and takes build row perm[start[j] + n - off[j]].
//    Projection and selection are fused (late materialisation, Section 4):
//    only the columns the next step needs are gathered, and filters such as
//    x != y are applied before the write.
// k_dedup implements the difference operator (Section 4, "Union and
// Deduplication") on radix-sorted new tuples: adjacent repeats are dropped,
// tuples already in full are dropped, and the survivors -- the delta -- are
// appended to the contiguous full relation (Section 3, eager merge).
#include "fv_device.h"

namespace fv {

// Rows per thread of the join, selection and difference kernels; a tile is
// kB (the block size, a template parameter: 128, 256 or 512) times that.
constexpr int kProbeItems = 4;
constexpr int kWriteItems = 4;
constexpr int kDedupItems = 4;

__device__ __forceinline__ u32 probe_val(const Src& s, const u32* const* pcol, u64 row) {
  return s.kind == kSrcConst ? s.v : pcol[s.v][row];
}

__device__ __forceinline__ u32 src_val(const Src& s, const u32* const* pcol, u64 prow,
                                       const u32* const* bcol, u64 brow) {
  if (s.kind == kSrcConst) return s.v;
  if (s.kind == kSrcProbe) return pcol[s.v][prow];
  return bcol[s.v][brow];
}

__device__ __forceinline__ u64 make_key(u32 nkey, u32 a, u32 b) {
  return nkey == 2 ? ((u64(a) << 32) | u64(b)) : u64(a);
}

// Probe rows r0 + k * step (k < kN) of a source: want[k] when the row exists
// and passes the probe filters, key[k] its join key.
template <int kN>
__device__ __forceinline__ void probe_keys(const u32* const* pcol, u32 n_pf, const Filter* pf, u32 nkey,
                                           const Src* keysrc, u64 begin, u64 r0, u64 step, u64 n, bool* want,
                                           u64* key) {
#pragma unroll
  for (int k = 0; k < kN; ++k) {
    const u64 r = r0 + u64(k) * step;
    want[k] = false;
    key[k] = 0;
    if (r < n) {
      const u64 row = begin + r;
      bool ok = true;
      for (u32 f = 0; f < n_pf; ++f) {
        const u32 a = probe_val(pf[f].a, pcol, row);
        const u32 b = probe_val(pf[f].b, pcol, row);
        ok = ok && (pf[f].op == kEq ? a == b : a != b);
      }
      want[k] = ok;
      if (ok && nkey) {
        const u32 a = probe_val(keysrc[0], pcol, row);
        const u32 b = nkey == 2 ? probe_val(keysrc[1], pcol, row) : 0u;
        key[k] = make_key(nkey, a, b);
      }
    }
  }
}

// Runs (start, count) of kN keys: the home slots are read together (one
// round trip for the batch), and only a key whose home slot holds another
// key probes on.  A cross product (nkey 0) matches all nbuild build rows.
template <int kN>
__device__ __forceinline__ void lookup_many(const Slot* __restrict__ tab, u64 mask, u32 nkey, u32 nbuild,
                                            const bool* want, const u64* key, u32* st, u32* cnt) {
  Slot hs[kN];
#pragma unroll
  for (int k = 0; k < kN; ++k)
    if (want[k] && nkey) hs[k] = tab[mix64(key[k]) & mask];
#pragma unroll
  for (int k = 0; k < kN; ++k) {
    st[k] = 0;
    cnt[k] = 0;
    if (!want[k]) continue;
    if (nkey == 0) {
      cnt[k] = nbuild;
    } else if (hs[k].key == key[k]) {
      st[k] = hs[k].start;
      cnt[k] = hs[k].count;
    } else if (hs[k].key != kEmptyKey) {
      u32 s, c;
      if (index_find_after(tab, mask, key[k], mix64(key[k]) & mask, s, c)) { st[k] = s; cnt[k] = c; }
    }
  }
}

// ------------------------------------------------------------------ probe
template <int kB>
__global__ __launch_bounds__(kB) void k_probe(ProbeParams p) {
  constexpr u32 kProbeTile = kB * kProbeItems;
  __shared__ u32 s_ticket;
  __shared__ u32 s_m[kB / kWave + 1];
  __shared__ u64 s_t[kB / kWave + 1];
  __shared__ u64 s_excl[2];
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  u64 begin, n;
  source_range(p.src, begin, n);
  const u32 ntiles = u32((n + kProbeTile - 1) / kProbeTile);
  if (blockIdx.x == 0 && threadIdx.x == 0 && p.out_n) *p.out_n = n;
  if (ntiles == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) { *p.out_m = 0; *p.out_t = 0; }
  }
  if (blockIdx.x >= participants(ntiles)) return;
  const u32 epoch = launch_epoch(p.epoch_base, p.epoch_off);
  u64 nbuild = 0;
  if (p.nkey == 0) nbuild = p.build_rows_ctr ? min_u64(*p.build_rows_ctr, p.build_cap) : p.build_rows;

  for (;;) {
    const u32 tile = take_ticket(p.ticket, ntiles, &s_ticket);
    if (tile >= ntiles) break;
    const u64 r0 = u64(tile) * kProbeTile + u64(threadIdx.x) * kProbeItems;
    u32 st[kProbeItems], cnt[kProbeItems];
    u32 matched = 0;
    u64 tsum = 0;
    bool want[kProbeItems];
    u64 key[kProbeItems];
    probe_keys<kProbeItems>(p.pcol, p.n_pf, p.pf, p.nkey, p.key, begin, r0, 1, n, want, key);
    lookup_many<kProbeItems>(p.table, p.mask, p.nkey, u32(nbuild), want, key, st, cnt);
#pragma unroll
    for (int k = 0; k < kProbeItems; ++k)
      if (cnt[k]) { ++matched; tsum += cnt[k]; }
    u32 mtot;
    u64 ttot;
    const u32 mex = block_exclusive_sum<kB>(matched, s_m, &mtot);
    const u64 tex = block_exclusive_sum<kB>(tsum, s_t, &ttot);
    const int w = threadIdx.x / kWave;
    if (tile == 0) {
      if (threadIdx.x == 0) {
        atomic_store_u64(p.st_m + tile, lb_word(epoch, kFlagPrefix, mtot));
        atomic_store_u64(p.st_t + tile, lb_word(epoch, kFlagPrefix, ttot));
        s_excl[0] = 0;
        s_excl[1] = 0;
      }
    } else {
      if (threadIdx.x == 0) {
        atomic_store_u64(p.st_m + tile, lb_word(epoch, kFlagAgg, mtot));
        atomic_store_u64(p.st_t + tile, lb_word(epoch, kFlagAgg, ttot));
      }
      if (w < 2) {
        u64* st_arr = w == 0 ? p.st_m : p.st_t;
        const u64 ex = lookback_exclusive(st_arr, tile, epoch);
        if (lane_id() == 0) {
          atomic_store_u64(st_arr + tile, lb_word(epoch, kFlagPrefix, ex + (w == 0 ? u64(mtot) : ttot)));
          s_excl[w] = ex;
        }
      }
    }
    __syncthreads();
    const u64 ex_m = s_excl[0], ex_t = s_excl[1];
    u64 pos = ex_m + mex;
    u64 off = ex_t + tex;
#pragma unroll
    for (int k = 0; k < kProbeItems; ++k) {
      if (cnt[k]) {
        if (pos < p.m_cap) {
          p.m_row[pos] = u32(begin + r0 + k);
          p.m_start[pos] = st[k];
          p.m_off[pos] = off;
        } else {
          *p.fatal = 1;
        }
        ++pos;
        off += cnt[k];
      }
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) {
      *p.out_m = ex_m + mtot;
      *p.out_t = ex_t + ttot;
    }
    __syncthreads();
  }
  ktime_end(p.ts);
}

// ------------------------------------------------------------------ shared append
// Compact the kept outputs of a block-tile and append them at an atomically
// reserved position of the output (order inside a "new" buffer is free: it is
// sorted before deduplication).
struct OutVals {
  u32 v[kMaxCols];
};

// Digit counts of the keys a block writes (see OutSpec::hist): an LDS copy
// for all passes, cleared before the block's first tile and added to the
// relation's histogram after its last.
constexpr u32 kOutHistWords = 8 * 256;
template <int kB>
__device__ __forceinline__ void out_hist_clear(const OutSpec& o, u32* s_hist) {
  if (!o.hist) return;
  for (u32 i = threadIdx.x; i < o.hist_passes * 256; i += kB) s_hist[i] = 0;
  __syncthreads();
}
template <int kB>
__device__ __forceinline__ void out_hist_flush(const OutSpec& o, u32* s_hist) {
  if (!o.hist) return;
  __syncthreads();
  for (u32 i = threadIdx.x; i < o.hist_passes * 256; i += kB) {
    const u32 c = s_hist[i];
    if (c) atomicAdd(&o.hist[i], c);
  }
}

template <int kB, int kItems>
__device__ __forceinline__ void append_tile(const OutSpec& o, const bool* keep, const OutVals* vals,
                                            u32* s_cnt, u64* s_base, u32* overflow, u64* stat, u32* s_hist) {
  u32 mine = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) mine += keep[k] ? 1u : 0u;
  u32 tot;
  const u32 ex = block_exclusive_sum<kB>(mine, s_cnt, &tot);
  if (threadIdx.x == 0) {
    *s_base = tot ? atomicAdd(reinterpret_cast<unsigned long long*>(o.count), (unsigned long long)tot) : 0;
    if (stat && tot) atomicAdd(reinterpret_cast<unsigned long long*>(stat), (unsigned long long)tot);
  }
  __syncthreads();
  const u64 base = *s_base;
  if (base + tot > o.cap) {
    if (threadIdx.x == 0 && tot) *overflow = 1;
  } else {
    u64 pos = base + ex;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (!keep[k]) continue;
      if (o.packed) {
        u64 key = 0;
#pragma unroll
        for (u32 c = 0; c < kMaxCols; ++c)
          if (c < o.ncols) key |= u64(vals[k].v[c]) << o.shift[c];
        o.keys[pos] = key;
        if (o.hist)
          for (u32 q = 0; q < o.hist_passes; ++q) atomicAdd(&s_hist[q * 256 + u32((key >> (8 * q)) & 255)], 1u);
      } else {
#pragma unroll
        for (u32 c = 0; c < kMaxCols; ++c)
          if (c < o.ncols) o.cols[c][pos] = vals[k].v[c];
      }
      ++pos;
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ write
template <int kB>
__global__ __launch_bounds__(kB) void k_write(WriteParams p) {
  constexpr u32 kWriteTile = kB * kWriteItems;
  __shared__ u64 s_off[kWriteTile + 1];
  __shared__ u64 s_j0;
  __shared__ u32 s_cnt[kB / kWave + 1];
  __shared__ u64 s_base;
  __shared__ u32 s_hist[kOutHistWords];
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  out_hist_clear<kB>(p.out, s_hist);
  const u64 M = min_u64(*p.in_m, p.m_cap);
  const u64 T = *p.in_t;
  const u64 ntiles = (T + kWriteTile - 1) / kWriteTile;
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const u64 n0 = tile * kWriteTile;
    if (threadIdx.x == 0) {
      u64 lo = 0, hi = M;                      // first j with off[j] > n0
      while (lo < hi) {
        const u64 mid = (lo + hi) >> 1;
        if (p.m_off[mid] <= n0) lo = mid + 1; else hi = mid;
      }
      s_j0 = lo - 1;
    }
    __syncthreads();
    const u64 j0 = s_j0;
    for (u32 i = threadIdx.x; i <= kWriteTile; i += kB)
      s_off[i] = (j0 + i < M) ? p.m_off[j0 + i] : T;
    __syncthreads();

    // Each step below goes out for all of the thread's outputs before the
    // next one waits: the run search (LDS), then the run's probe row and
    // start, then the build row id, then the gathered columns -- a few
    // round trips per tile instead of a few per output.
    bool keep[kWriteItems], live[kWriteItems];
    OutVals vals[kWriteItems];
    u32 jl[kWriteItems];
    u64 prow[kWriteItems], idx[kWriteItems], brow[kWriteItems];
#pragma unroll
    for (int k = 0; k < kWriteItems; ++k) {
      const u64 nn = n0 + u64(threadIdx.x) * kWriteItems + k;
      live[k] = nn < T;
      u32 lo = 0, hi = kWriteTile + 1;         // last jl with s_off[jl] <= nn
      while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (s_off[mid] <= nn) lo = mid + 1; else hi = mid;
      }
      // an output past the end reads the tile's first run (which exists:
      // n0 < T), so every load below is in bounds and none is conditional
      jl[k] = live[k] ? lo - 1 : 0;
    }
#pragma unroll
    for (int k = 0; k < kWriteItems; ++k) {
      const u64 nn = n0 + u64(threadIdx.x) * kWriteItems + k;
      const u64 j = j0 + jl[k];
      prow[k] = u64(p.m_row[j]);
      idx[k] = u64(p.m_start[j]) + (live[k] ? nn - s_off[jl[k]] : 0);
    }
#pragma unroll
    for (int k = 0; k < kWriteItems; ++k) brow[k] = p.perm ? u64(p.perm[idx[k]]) : idx[k];
    // filters and columns term by term, each term for all outputs at once
    // (a term's source is uniform, so the outputs' loads go out together)
#pragma unroll
    for (int k = 0; k < kWriteItems; ++k) keep[k] = live[k];
    for (u32 f = 0; f < p.n_filter; ++f) {
      u32 a[kWriteItems], b[kWriteItems];
#pragma unroll
      for (int k = 0; k < kWriteItems; ++k) {
        a[k] = src_val(p.filt[f].a, p.pcol, prow[k], p.bcol, brow[k]);
        b[k] = src_val(p.filt[f].b, p.pcol, prow[k], p.bcol, brow[k]);
      }
#pragma unroll
      for (int k = 0; k < kWriteItems; ++k) keep[k] = keep[k] && (p.filt[f].op == kEq ? a[k] == b[k] : a[k] != b[k]);
    }
#pragma unroll
    for (u32 c = 0; c < kMaxCols; ++c) {
      if (c >= p.out.ncols) break;
#pragma unroll
      for (int k = 0; k < kWriteItems; ++k) vals[k].v[c] = src_val(p.out.src[c], p.pcol, prow[k], p.bcol, brow[k]);
    }
    append_tile<kB, kWriteItems>(p.out, keep, vals, s_cnt, &s_base, p.overflow, p.join_out_stat, s_hist);
  }
  out_hist_flush<kB>(p.out, s_hist);
  ktime_end(p.ts);
}

// Presized one-pass join: a block takes a tile of kFusedTile probe rows, looks
// their keys up, scans the match counts in LDS, reserves the tile's outputs
// with one atomic and writes them output-balanced (each thread finds the probe
// row of an output position by binary search over the tile's prefix).  With
// write filters the outputs are compacted per chunk of kB instead, one
// reservation per chunk.  Outputs past the buffer are counted, not written,
// and raise the overflow flag (the round then runs again with count-then-
// write joins).
constexpr u32 kFusedItems = 4;

// Output position <- the projected values of (probe row, build row).
__device__ __forceinline__ void fused_put(const OutSpec& out, const u32* const* pcol, const u32* const* bcol, u64 pos,
                                          u64 prow, u64 brow) {
  if (out.packed) {
    u64 key = 0;
#pragma unroll
    for (u32 c = 0; c < kMaxCols; ++c)
      if (c < out.ncols) key |= u64(src_val(out.src[c], pcol, prow, bcol, brow)) << out.shift[c];
    out.keys[pos] = key;
  } else {
#pragma unroll
    for (u32 c = 0; c < kMaxCols; ++c)
      if (c < out.ncols) out.cols[c][pos] = src_val(out.src[c], pcol, prow, bcol, brow);
  }
}

// Output position <- already gathered values.
__device__ __forceinline__ void put_vals(const OutSpec& out, u64 pos, const OutVals& v) {
  if (out.packed) {
    u64 key = 0;
#pragma unroll
    for (u32 c = 0; c < kMaxCols; ++c)
      if (c < out.ncols) key |= u64(v.v[c]) << out.shift[c];
    out.keys[pos] = key;
  } else {
#pragma unroll
    for (u32 c = 0; c < kMaxCols; ++c)
      if (c < out.ncols) out.cols[c][pos] = v.v[c];
  }
}

// Tile index of output o: the last j with off[j] <= o (its count is > 0).
template <int kB>
__device__ __forceinline__ u32 fused_owner(const u64* off, u64 o) {
  constexpr u32 kFusedTile = kB * kFusedItems;
  u32 lo = 0, hi = kFusedTile;
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if (off[mid] <= o) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int kB>
__global__ __launch_bounds__(kB) void k_join_fused(FusedJoinParams p) {
  constexpr u32 kFusedTile = kB * kFusedItems;
  __shared__ u64 s_off[kFusedTile + 1];
  __shared__ u32 s_start[kFusedTile];
  __shared__ u64 s_scan[kB / kWave + 1];
  __shared__ u32 s_keep[kB / kWave + 1];
  __shared__ u64 s_base;
  __shared__ u32 s_stop;
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  u64 begin, n;
  source_range(p.src, begin, n);
  u64 nbuild = 0;
  if (p.nkey == 0) nbuild = p.build_rows_ctr ? min_u64(*p.build_rows_ctr, p.build_cap) : p.build_rows;
  u64 pre_total = 0, kept_total = 0;   // thread 0's tallies
  const u64 ntiles = (n + kFusedTile - 1) / kFusedTile;
  if (blockIdx.x == 0 && threadIdx.x == 0 && p.out_n) *p.out_n = n;
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // once some output did not fit, the round runs again with exact joins:
    // the remaining tiles stop (their counts only size the rerun's buffers,
    // which grow geometrically if they still fall short)
    if (threadIdx.x == 0) s_stop = __hip_atomic_load(p.overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (s_stop) break;
    const u64 t0 = tile * kFusedTile;
    u32 st[kFusedItems], cnt[kFusedItems];
    u64 mine = 0;
    bool want[kFusedItems];
    u64 key[kFusedItems];
    probe_keys<kFusedItems>(p.pcol, p.n_pf, p.pf, p.nkey, p.key, begin, t0 + u64(threadIdx.x) * kFusedItems, 1, n,
                            want, key);
    lookup_many<kFusedItems>(p.table, p.mask, p.nkey, u32(nbuild), want, key, st, cnt);
#pragma unroll
    for (u32 k = 0; k < kFusedItems; ++k) mine += cnt[k];
    u64 tot;
    u64 ex = block_exclusive_sum<kB>(mine, s_scan, &tot);
#pragma unroll
    for (u32 k = 0; k < kFusedItems; ++k) {
      s_off[threadIdx.x * kFusedItems + k] = ex;
      s_start[threadIdx.x * kFusedItems + k] = st[k];
      ex += cnt[k];
    }
    if (threadIdx.x == 0) s_off[kFusedTile] = tot;
    __syncthreads();
    if (threadIdx.x == 0) pre_total += tot;
    if (tot == 0) continue;   // block-uniform; nothing reads the tile's LDS
    if (p.n_filter == 0) {
      if (threadIdx.x == 0) s_base = atomicAdd(reinterpret_cast<unsigned long long*>(p.out.count), (unsigned long long)tot);
      __syncthreads();
      const u64 base = s_base;
      if (threadIdx.x == 0) kept_total += tot;
      if (base + tot > p.out.cap) {
        if (threadIdx.x == 0) *p.overflow = 1;
      } else {
        // kFusedItems outputs per thread and step: their build row ids are
        // read together, then their columns
        for (u64 o0 = 0; o0 < tot; o0 += u64(kB) * kFusedItems) {
          u32 j[kFusedItems];
          u64 idx[kFusedItems], brow[kFusedItems];
#pragma unroll
          for (u32 k = 0; k < kFusedItems; ++k) {
            const u64 o = o0 + u64(k) * kB + threadIdx.x;
            j[k] = o < tot ? fused_owner<kB>(s_off, o) : 0u;
            idx[k] = o < tot ? u64(s_start[j[k]]) + (o - s_off[j[k]]) : 0;
          }
#pragma unroll
          for (u32 k = 0; k < kFusedItems; ++k) {
            const u64 o = o0 + u64(k) * kB + threadIdx.x;
            brow[k] = (o < tot && p.perm) ? u64(p.perm[idx[k]]) : idx[k];
          }
          OutVals v[kFusedItems];
#pragma unroll
          for (u32 c = 0; c < kMaxCols; ++c) {
            if (c >= p.out.ncols) break;
#pragma unroll
            for (u32 k = 0; k < kFusedItems; ++k) {
              const u64 o = o0 + u64(k) * kB + threadIdx.x;
              v[k].v[c] = o < tot ? src_val(p.out.src[c], p.pcol, begin + t0 + j[k], p.bcol, brow[k]) : 0u;
            }
          }
#pragma unroll
          for (u32 k = 0; k < kFusedItems; ++k) {
            const u64 o = o0 + u64(k) * kB + threadIdx.x;
            if (o < tot) put_vals(p.out, base + o, v[k]);
          }
        }
      }
    } else {
      for (u64 c0 = 0; c0 < tot; c0 += kB) {
        const u64 o = c0 + threadIdx.x;
        bool keep = false;
        u64 prow = 0, brow = 0;
        if (o < tot) {
          const u32 j = fused_owner<kB>(s_off, o);
          const u64 idx = u64(s_start[j]) + (o - s_off[j]);
          prow = begin + t0 + j;
          brow = p.perm ? u64(p.perm[idx]) : idx;
          bool ok = true;
          for (u32 f = 0; f < p.n_filter; ++f) {
            const u32 a = src_val(p.filt[f].a, p.pcol, prow, p.bcol, brow);
            const u32 b = src_val(p.filt[f].b, p.pcol, prow, p.bcol, brow);
            ok = ok && (p.filt[f].op == kEq ? a == b : a != b);
          }
          keep = ok;
        }
        u32 kc;
        const u32 kpos = block_exclusive_sum<kB>(keep ? 1u : 0u, s_keep, &kc);
        if (kc == 0) continue;   // block-uniform
        if (threadIdx.x == 0) s_base = atomicAdd(reinterpret_cast<unsigned long long*>(p.out.count), (unsigned long long)kc);
        __syncthreads();
        const u64 base = s_base;
        if (threadIdx.x == 0) kept_total += kc;
        if (base + kc > p.out.cap) {
          if (threadIdx.x == 0) *p.overflow = 1;
        } else if (keep) {
          fused_put(p.out, p.pcol, p.bcol, base + kpos, prow, brow);
        }
        __syncthreads();   // s_base and s_keep are reused by the next chunk
      }
    }
    __syncthreads();   // the next tile overwrites s_off / s_start
  }
  if (threadIdx.x == 0) {
    if (pre_total) atomicAdd(reinterpret_cast<unsigned long long*>(p.out_t), (unsigned long long)pre_total);
    if (kept_total && p.join_out_stat)
      atomicAdd(reinterpret_cast<unsigned long long*>(p.join_out_stat), (unsigned long long)kept_total);
  }
  ktime_end(p.ts);
}

// ------------------------------------------------------------------ select / project
template <int kB>
__global__ __launch_bounds__(kB) void k_select(SelectParams p) {
  constexpr u32 kWriteTile = kB * kWriteItems;
  __shared__ u32 s_cnt[kB / kWave + 1];
  __shared__ u64 s_base;
  __shared__ u32 s_hist[kOutHistWords];
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  out_hist_clear<kB>(p.out, s_hist);
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 ntiles = (n + kWriteTile - 1) / kWriteTile;
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    bool keep[kWriteItems];
    OutVals vals[kWriteItems];
#pragma unroll
    for (int k = 0; k < kWriteItems; ++k) {
      const u64 r = tile * kWriteTile + u64(k) * kB + threadIdx.x;
      keep[k] = false;
      if (r >= n) continue;
      const u64 row = begin + r;
      bool ok = true;
      for (u32 f = 0; f < p.n_filter; ++f) {
        const u32 a = probe_val(p.filt[f].a, p.pcol, row);
        const u32 b = probe_val(p.filt[f].b, p.pcol, row);
        ok = ok && (p.filt[f].op == kEq ? a == b : a != b);
      }
      keep[k] = ok;
      if (ok) {
#pragma unroll
        for (u32 c = 0; c < kMaxCols; ++c)
          if (c < p.out.ncols) vals[k].v[c] = probe_val(p.out.src[c], p.pcol, row);
      }
    }
    append_tile<kB, kWriteItems>(p.out, keep, vals, s_cnt, &s_base, p.overflow, p.join_out_stat, s_hist);
  }
  out_hist_flush<kB>(p.out, s_hist);
  ktime_end(p.ts);
}

// ------------------------------------------------------------------ dedup + append
// Algorithm 2's membership test for kN sorted new tuples (act[k]: the first
// of a run of equal keys): present[k] when some row of full holds the tuple.
// Every column's range lookup goes out together; then each tuple scans the
// row ids of its shortest range and compares the other columns.
template <int kN>
__device__ __forceinline__ void ranges_present(const RangeDedup& rd, const u32* shift, const u32* width,
                                               const u64* key, const bool* act, bool* present) {
  u32 v[3][kN], st[3][kN], cnt[3][kN];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const bool on = u32(c) < rd.ncol;
    const u64 m = width[c] >= 32 ? 0xFFFFFFFFull : ((1ull << width[c]) - 1);
    u64 ck[kN];
    bool want[kN];
#pragma unroll
    for (int k = 0; k < kN; ++k) {
      v[c][k] = on ? u32((key[k] >> shift[c]) & m) : 0u;
      ck[k] = u64(v[c][k]);
      want[k] = on && act[k];
    }
    if (on) {
      lookup_many<kN>(rd.table[c], rd.mask[c], 1, 0, want, ck, st[c], cnt[c]);
    } else {
#pragma unroll
      for (int k = 0; k < kN; ++k) { st[c][k] = 0; cnt[c][k] = 0xFFFFFFFFu; }
    }
  }
#pragma unroll
  for (int k = 0; k < kN; ++k) {
    present[k] = false;
    if (!act[k]) continue;
    // the shortest range (columns past ncol count as all ones: never chosen)
    const u32 c01 = cnt[1][k] < cnt[0][k] ? 1u : 0u;
    const u32 n01 = c01 ? cnt[1][k] : cnt[0][k];
    const u32 best = cnt[2][k] < n01 ? 2u : c01;
    if (cnt[0][k] == 0 || cnt[1][k] == 0 || cnt[2][k] == 0) continue;   // a value full never holds there
    const u32 s0 = best == 0 ? st[0][k] : best == 1 ? st[1][k] : st[2][k];
    const u32 n = best == 0 ? cnt[0][k] : best == 1 ? cnt[1][k] : cnt[2][k];
    const u32* perm = rd.perm[best];
    for (u32 i = 0; i < n; ++i) {
      const u32 r = perm[s0 + i];
      bool all = true;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (u32(c) < rd.ncol && u32(c) != best) all = all && rd.fcol[c][r] == v[c][k];
      if (all) { present[k] = true; break; }
    }
  }
}

template <int kB>
__global__ __launch_bounds__(kB) void k_dedup(DedupParams p) {
  constexpr u32 kDedupTile = kB * kDedupItems;
  __shared__ u32 s_ticket;
  __shared__ u32 s_c[kB / kWave + 1];
  __shared__ u64 s_excl;
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 fbase = *p.full_n;
  const u32 epoch = launch_epoch(p.epoch_base, p.epoch_off);
  const u32 ntiles = u32((n + kDedupTile - 1) / kDedupTile);
  if (ntiles == 0 && blockIdx.x == 0 && threadIdx.x == 0) *p.out_delta = 0;
  if (blockIdx.x >= participants(ntiles)) return;
  for (;;) {
    const u32 tile = take_ticket(p.ticket, ntiles, &s_ticket);
    if (tile >= ntiles) break;
    const u64 r0 = u64(tile) * kDedupTile + u64(threadIdx.x) * kDedupItems;
    u64 key[kDedupItems];
    bool surv[kDedupItems], first[kDedupItems];
#pragma unroll
    for (int k = 0; k < kDedupItems; ++k) {
      const u64 r = r0 + k;
      key[k] = 0;
      first[k] = false;
      if (r < n) {
        key[k] = p.keys[begin + r];
        first[k] = (r == 0) || (p.keys[begin + r - 1] != key[k]);
      }
    }
    u32 mine = 0;
    if (p.set || p.set32) {
      // the thread's set probes go out together (one round trip, not kDedupItems)
      int ins[kDedupItems];
      if (p.set32) set32_insert_many<kDedupItems>(p.set32, p.set_mask, key, first, ins, p.ones);
      else set_insert_many<kDedupItems>(p.set, p.set_mask, key, first, ins);
#pragma unroll
      for (int k = 0; k < kDedupItems; ++k) {
        if (ins[k] < 0) *p.set_full = 1;   // never the flag this kernel checks on entry
        surv[k] = first[k] && ins[k] > 0;
        mine += surv[k] ? 1u : 0u;
      }
    } else if (p.rd.ncol) {
      bool present[kDedupItems];
      ranges_present<kDedupItems>(p.rd, p.shift, p.width, key, first, present);
#pragma unroll
      for (int k = 0; k < kDedupItems; ++k) {
        surv[k] = first[k] && !present[k];
        mine += surv[k] ? 1u : 0u;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kDedupItems; ++k) {
        surv[k] = first[k];
        mine += surv[k] ? 1u : 0u;
      }
    }
    u32 tot;
    const u32 ex = block_exclusive_sum<kB>(mine, s_c, &tot);
    if (tile == 0) {
      if (threadIdx.x == 0) {
        atomic_store_u64(p.status + tile, lb_word(epoch, kFlagPrefix, tot));
        s_excl = 0;
      }
    } else {
      if (threadIdx.x == 0) atomic_store_u64(p.status + tile, lb_word(epoch, kFlagAgg, tot));
      if (threadIdx.x < kWave) {
        const u64 e = lookback_exclusive(p.status, tile, epoch);
        if (threadIdx.x == 0) {
          atomic_store_u64(p.status + tile, lb_word(epoch, kFlagPrefix, e + tot));
          s_excl = e;
        }
      }
    }
    __syncthreads();
    u64 pos = fbase + s_excl + ex;
#pragma unroll
    for (int k = 0; k < kDedupItems; ++k) {
      if (!surv[k]) continue;
      for (u32 c = 0; c < p.arity; ++c) {
        const u64 m = (p.width[c] >= 32) ? 0xFFFFFFFFull : ((1ull << p.width[c]) - 1);
        p.cols[c][pos] = u32((key[k] >> p.shift[c]) & m);
      }
      ++pos;
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) *p.out_delta = s_excl + tot;
    __syncthreads();
  }
  ktime_end(p.ts);
}

// ------------------------------------------------------------------ difference by merge
// The difference of the round's sorted new keys b (repeats adjacent) against
// full's sorted keys a, fused with the merge that keeps full's keys sorted
// for the next round.  In the merge of a and b in which a tie is taken from a
// first, a key of b is new iff it differs from the key before it: a key of
// full equal to it, or an earlier copy of it, would come just before.  The
// merged sequence is cut into tiles of kDiffTile outputs; tile t takes
// a[i0, i1) and b[j0, j1).
//   k_diff_split: one wave per tile boundary: i0 found on the boundary's
//                 diagonal by a 64-way search;
//   k_diff_count: per tile, the number of new keys;
//   k_diff_scan:  one block: each tile's first new-key and dropped-key ranks;
//   k_diff_write: per tile, the merge again: a's keys and the new keys go to
//                 the merged array (dropped repeats close up), the new keys'
//                 columns are appended to full.
// Every kernel is a grid-stride loop over independent tiles: no tile waits
// for another.
constexpr u32 kDiffItems = 16;

// Number of a's keys among the first d outputs of the merge of a[0, na) and
// b[0, nb) with ties taken from a, by a whole wave (every lane calls it with
// the same arguments): a's key i is among them iff a[i] <= b[d - i - 1],
// which holds for a prefix of the candidates, 64 of them probed per round trip.
__device__ __forceinline__ u64 wave_merge_split(const u64* a, u64 na, const u64* b, u64 nb, u64 d) {
  const u32 lane = u32(__lane_id());
  u64 lo = d > nb ? d - nb : 0, hi = d < na ? d : na;   // the answer lies in [lo, hi]
  while (hi - lo > u64(kWave)) {
    const u64 step = (hi - lo + kWave - 1) / kWave;
    const u64 i = lo + u64(lane) * step;
    const bool before = i < hi && a[i] <= b[d - i - 1];
    const u32 c = u32(__popcll(__ballot(before)));
    if (c == 0) return lo;
    const u64 nxt = lo + u64(c) * step;
    if (c < u32(kWave) && nxt < hi) hi = nxt;
    lo = lo + u64(c - 1) * step + 1;
  }
  const u64 i = lo + lane;
  const bool before = i < hi && a[i] <= b[d - i - 1];
  return lo + u64(__popcll(__ballot(before)));
}

// The same split by one thread (binary search), within a tile's staged keys
// (a's part at s[0, la), b's at s[la, la + lb)).
__device__ __forceinline__ u32 merge_split_le(const u64* s, u32 la, u32 lb, u32 d) {
  u32 lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  while (lo < hi) {
    const u32 i = (lo + hi) >> 1;
    if (s[i] <= s[la + d - i - 1]) lo = i + 1;
    else hi = i;
  }
  return lo;
}

// One thread's stretch of a tile's merge: outputs [e0, e1) (e1 - e0 <= kN)
// of the merge of the staged a[0, la) and b[0, lb) (at s[i] and s[la + j]),
// the key before output e0 being `prev` (has_prev false: none).  f(k, v, from_b, is_new) is called for output e0 + k, in order.
template <int kN, class F>
__device__ __forceinline__ void diff_walk(const u64* s, u32 la, u32 lb, u32 e0, u32 e1, bool has_prev, u64 prev,
                                          F&& f) {
  u32 i = merge_split_le(s, la, lb, e0);
  u32 j = e0 - i;
  if (e0 > 0) {   // the output before e0 is the larger of the last keys taken from each side
    has_prev = true;
    prev = i > 0 ? s[i - 1] : 0;
    if (j > 0 && (i == 0 || s[la + j - 1] > prev)) prev = s[la + j - 1];
  }
#pragma unroll
  for (u32 k = 0; k < u32(kN); ++k) {
    if (e0 + k >= e1) break;
    const bool take_a = j >= lb || (i < la && s[i] <= s[la + j]);
    const u64 v = take_a ? s[i++] : s[la + j++];
    f(k, v, !take_a, !take_a && !(has_prev && prev == v));
    prev = v;
    has_prev = true;
  }
}

// Stage a[i0, i1) and b[j0, j1) in s_in and find the key before the tile
// (the larger of a[i0 - 1] and b[j0 - 1]).  Block-uniform.
__device__ __forceinline__ void diff_stage(const u64* a, const u64* b, u64 i0, u32 la, u64 j0, u32 lb, u64* s_in,
                                           u32 nthreads, bool& has_prev, u64& prev) {
  for (u32 q = threadIdx.x; q < la + lb; q += nthreads) s_in[q] = q < la ? a[i0 + q] : b[j0 + (q - la)];
  has_prev = i0 > 0 || j0 > 0;
  prev = i0 > 0 ? a[i0 - 1] : 0;
  if (j0 > 0 && (i0 == 0 || b[j0 - 1] > prev)) prev = b[j0 - 1];
  __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_diff_split(DedupParams p, u32 tile_keys) {
  if (p.abort && *p.abort) return;
  u64 begin, nb;
  source_range(p.src, begin, nb);
  const u64 na = *p.full_n;
  const u64 total = na + nb;
  const u64 ntiles = (total + tile_keys - 1) / tile_keys;
  constexpr u32 kWaves = kBlock / kWave;
  for (u64 t = u64(blockIdx.x) * kWaves + threadIdx.x / kWave; t <= ntiles; t += u64(gridDim.x) * kWaves) {
    const u64 r = wave_merge_split(p.sorted_full, na, p.keys + begin, nb, min_u64(t * tile_keys, total));
    if (lane_id() == 0) p.mtile[t] = r;
  }
}

template <int kB>
__global__ __launch_bounds__(kB) void k_diff_count(DedupParams p) {
  constexpr u32 kDiffTile = kB * kDiffItems;
  __shared__ u64 s_in[kDiffTile];
  __shared__ u32 s_red[kB / kWave + 1];
  if (p.abort && *p.abort) return;
  u64 begin, nb;
  source_range(p.src, begin, nb);
  const u64* a = p.sorted_full;
  const u64* b = p.keys + begin;
  const u64 na = *p.full_n;
  const u64 total = na + nb;
  const u64 ntiles = (total + kDiffTile - 1) / kDiffTile;
  const u64* split = p.mtile;          // ntiles + 1 splits
  u64* cnt = p.mtile + (ntiles + 1);   // ntiles new-key counts
  for (u64 t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const u64 d0 = t * kDiffTile, d1 = min_u64(d0 + kDiffTile, total);
    const u64 i0 = split[t], i1 = split[t + 1];
    const u64 j0 = d0 - i0;
    const u32 la = u32(i1 - i0), lb = u32((d1 - i1) - j0);
    u32 mine = 0;
    if (lb) {   // block-uniform: a tile of a's keys alone has no new keys
      bool has_prev;
      u64 prev;
      diff_stage(a, b, i0, la, j0, lb, s_in, kB, has_prev, prev);
      const u32 e0 = threadIdx.x * kDiffItems;
      if (e0 < la + lb)
        diff_walk<kDiffItems>(s_in, la, lb, e0, min_u32(e0 + kDiffItems, la + lb), has_prev, prev,
                              [&](u32, u64, bool, bool is_new) { mine += is_new ? 1u : 0u; });
    }
    const u32 tot = block_sum<kB>(mine, s_red);
    if (threadIdx.x == 0) cnt[t] = tot;
    __syncthreads();   // s_in is reused by the next tile
  }
}

// One block of 1024 threads, kScanItems tiles per thread and step: each
// tile's rank of its first new key (soff) and of its first dropped key of b
// (doff), and the number of new keys.
constexpr u32 kDiffScanBlock = 1024;
constexpr u32 kScanItems = 8;
__global__ __launch_bounds__(kDiffScanBlock) void k_diff_scan(DedupParams p, u32 tile_keys) {
  __shared__ u64 s_scan[kDiffScanBlock / kWave + 1];
  if (p.abort && *p.abort) return;
  u64 begin, nb;
  source_range(p.src, begin, nb);
  const u64 na = *p.full_n;
  const u64 total = na + nb;
  const u64 ntiles = (total + tile_keys - 1) / tile_keys;
  const u64* split = p.mtile;
  const u64* cnt = p.mtile + (ntiles + 1);
  u64* soff = p.mtile + (ntiles + 1) + ntiles;
  u64* doff = soff + ntiles;
  u64 run_s = 0, run_d = 0;
  for (u64 t0 = 0; t0 < ntiles; t0 += u64(kDiffScanBlock) * kScanItems) {
    const u64 tb = t0 + u64(threadIdx.x) * kScanItems;
    u64 cs[kScanItems], cd[kScanItems], ms = 0, md = 0;
#pragma unroll
    for (u32 k = 0; k < kScanItems; ++k) {
      const u64 t = tb + k;
      cs[k] = cd[k] = 0;
      if (t < ntiles) {
        const u64 d0 = t * tile_keys, d1 = min_u64(d0 + tile_keys, total);
        const u64 lb = (d1 - split[t + 1]) - (d0 - split[t]);
        cs[k] = cnt[t];
        cd[k] = lb - cnt[t];
      }
      ms += cs[k];
      md += cd[k];
    }
    u64 ts, td;
    u64 es = block_exclusive_sum<kDiffScanBlock>(ms, s_scan, &ts);
    u64 ed = block_exclusive_sum<kDiffScanBlock>(md, s_scan, &td);
#pragma unroll
    for (u32 k = 0; k < kScanItems; ++k) {
      const u64 t = tb + k;
      if (t < ntiles) {
        soff[t] = run_s + es;
        doff[t] = run_d + ed;
      }
      es += cs[k];
      ed += cd[k];
    }
    run_s += ts;
    run_d += td;
  }
  if (threadIdx.x == 0) *p.out_delta = run_s;
}

template <int kB>
__global__ __launch_bounds__(kB) void k_diff_write(DedupParams p) {
  constexpr u32 kDiffTile = kB * kDiffItems;
  __shared__ u64 s_in[kDiffTile];
  __shared__ u64 s_scan[kB / kWave + 1];
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  u64 begin, nb;
  source_range(p.src, begin, nb);
  const u64* a = p.sorted_full;
  const u64* b = p.keys + begin;
  const u64 na = *p.full_n;
  const u64 total = na + nb;
  const u64 ntiles = (total + kDiffTile - 1) / kDiffTile;
  const u64* split = p.mtile;
  const u64* soff = p.mtile + (ntiles + 1) + ntiles;
  const u64* doff = soff + ntiles;
  for (u64 t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const u64 d0 = t * kDiffTile, d1 = min_u64(d0 + kDiffTile, total);
    const u64 i0 = split[t], i1 = split[t + 1];
    const u64 j0 = d0 - i0;
    const u32 la = u32(i1 - i0), lb = u32((d1 - i1) - j0);
    bool has_prev;
    u64 prev;
    diff_stage(a, b, i0, la, j0, lb, s_in, kB, has_prev, prev);
    const u32 e0 = threadIdx.x * kDiffItems;
    const u32 e1 = min_u32(e0 + kDiffItems, la + lb);
    // one walk: the thread's outputs and their kinds (0 kept from full, 1
    // new, 2 dropped) in registers; new keys counted in the high half,
    // dropped ones in the low half, then ranked in the block
    u64 v[kDiffItems];
    u32 kind[kDiffItems];
    u64 mine = 0;
#pragma unroll
    for (u32 k = 0; k < kDiffItems; ++k) {
      v[k] = 0;
      kind[k] = 2u;
    }
    if (e0 < e1)
      diff_walk<kDiffItems>(s_in, la, lb, e0, e1, has_prev, prev,
                            [&](u32 k, u64 x, bool from_b, bool is_new) {
                              v[k] = x;
                              kind[k] = is_new ? 1u : (from_b ? 2u : 0u);
                              mine += is_new ? (u64(1) << 32) : (from_b ? 1u : 0u);
                            });
    u64 tot;
    const u64 ex = block_exclusive_sum<kB>(mine, s_scan, &tot);
    u64 snew = soff[t] + (ex >> 32);                // rank of the thread's first new key
    u64 drop = doff[t] + (ex & 0xFFFFFFFFull);     // dropped keys before its first output
    const u64 m0 = d0 + e0;                         // merge position of its first output
#pragma unroll
    for (u32 k = 0; k < kDiffItems; ++k) {
      if (e0 + k >= e1) break;
      if (kind[k] == 2u) {
        ++drop;
        continue;
      }
      p.merged[m0 + k - drop] = v[k];
      if (kind[k] == 1u) {
        const u64 pos = na + snew++;
        for (u32 c = 0; c < p.arity; ++c) {
          const u64 mk = (p.width[c] >= 32) ? 0xFFFFFFFFull : ((1ull << p.width[c]) - 1);
          p.cols[c][pos] = u32((v[k] >> p.shift[c]) & mk);
        }
      }
    }
    __syncthreads();   // s_in is reused by the next tile
  }
  ktime_end(p.ts);
}

__global__ void k_commit(CommitParams p) {
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const u64 d = *p.delta;
    const u64 f = *p.full_n;
    *p.d_begin = f;
    *p.full_n = f + d;
    if (p.new_count) *p.new_count = 0;
    if (p.derived) *p.derived += d;
  }
}

// Start of a round: zero the round's counters, the overflow flag and the
// radix histograms in one launch.
__global__ void k_round_prologue(u64* ctr, u64 n_ctr, u32* flag, u32* hist, u64 n_hist, u32* epoch_base,
                                 int sticky) {
  const u64 i0 = u64(blockIdx.x) * blockDim.x + threadIdx.x;
  const u64 stride = u64(gridDim.x) * blockDim.x;
  // A round enqueued behind one that may still fail: if that one raised a
  // flag, this round must do nothing at all (its counters, histograms and
  // epoch stay as the failed round left them).  The void word makes every
  // join and selection of the round return at entry (their look-back would
  // otherwise meet the failed round's status words under the same epoch),
  // and the overflow flag stops the sorts, differences, commits and index
  // work.
  if (sticky && flag && (flag[kFlagOverflow] || flag[kFlagSetFull])) {
    if (i0 == 0) { flag[kFlagOverflow] = 1; flag[kFlagVoid] = 1; }
    return;
  }
  for (u64 i = i0; i < n_ctr; i += stride) ctr[i] = 0;
  for (u64 i = i0; i < n_hist; i += stride) hist[i] = 0;
  if (i0 == 0) {
    if (flag) { flag[kFlagOverflow] = 0; flag[kFlagSetFull] = 0; flag[kFlagVoid] = 0; }
    *epoch_base += kEpochStride;
  }
}

// ------------------------------------------------------------------ launchers
int launch_round_prologue(u64* ctr, u64 n_ctr, u32* flag, u32* hist, u64 n_hist, u32* epoch_base, void* stream,
                          bool sticky) {
  hipLaunchKernelGGL(k_round_prologue, dim3(8), dim3(256), 0, (hipStream_t)stream, ctr, n_ctr, flag, hist, n_hist,
                     epoch_base, int(sticky));
  return int(hipGetLastError());
}

static int grid_for(u64 tiles, int cap_blocks) {
  if (tiles == 0) return 1;
  return int(tiles < u64(cap_blocks) ? tiles : u64(cap_blocks));
}

// Launch kernel K<kB> with kB the block size given (128, 256 or 512; anything
// else runs 256-thread blocks).
#define FV_LAUNCH_BLOCK(K, block, grid, stream, arg)                                                              \
  do {                                                                                                        \
    if ((block) == 128)                                                                                       \
      hipLaunchKernelGGL(K<128>, dim3(grid), dim3(128), 0, (hipStream_t)(stream), arg);                       \
    else if ((block) == 512)                                                                                  \
      hipLaunchKernelGGL(K<512>, dim3(grid), dim3(512), 0, (hipStream_t)(stream), arg);                       \
    else                                                                                                      \
      hipLaunchKernelGGL(K<256>, dim3(grid), dim3(256), 0, (hipStream_t)(stream), arg);                       \
  } while (0)

static u64 block_of(u32 block) { return block == 128 || block == 512 ? block : 256; }

int launch_probe(const ProbeParams& p, u64 probe_cap, int grid, void* stream, u32 block) {
  const u64 tile = block_of(block) * kProbeItems;
  const u64 tiles = (probe_cap + tile - 1) / tile;
  const int g = grid > 0 ? grid : grid_for(tiles, 2048);
  FV_LAUNCH_BLOCK(k_probe, block, g, stream, p);
  return int(hipGetLastError());
}

int launch_write(const WriteParams& p, u64 out_tiles_hint, void* stream, u32 block) {
  const u64 tile = block_of(block) * kWriteItems;
  const u64 tiles = (out_tiles_hint + tile - 1) / tile;
  FV_LAUNCH_BLOCK(k_write, block, grid_for(tiles, 4096), stream, p);
  return int(hipGetLastError());
}

int launch_join_fused(const FusedJoinParams& p, u64 rows_hint, void* stream, u32 block) {
  const u64 tile = block_of(block) * kFusedItems;
  const u64 tiles = (rows_hint + tile - 1) / tile;
  FV_LAUNCH_BLOCK(k_join_fused, block, grid_for(tiles, 4096), stream, p);
  return int(hipGetLastError());
}

int launch_select(const SelectParams& p, u64 rows_hint, void* stream, u32 block) {
  const u64 tile = block_of(block) * kWriteItems;
  const u64 tiles = (rows_hint + tile - 1) / tile;
  FV_LAUNCH_BLOCK(k_select, block, grid_for(tiles, 4096), stream, p);
  return int(hipGetLastError());
}

int launch_dedup(const DedupParams& p, u64 rows_cap, void* stream, u32 block) {
  const u64 tile = block_of(block) * kDedupItems;
  const u64 tiles = (rows_cap + tile - 1) / tile;
  FV_LAUNCH_BLOCK(k_dedup, block, grid_for(tiles, 2048), stream, p);
  return int(hipGetLastError());
}

int launch_diff_sorted(const DedupParams& p, u64 total_cap, void* stream, u32 block) {
  const u64 tile = block_of(block) * kDiffItems;
  const u64 tiles = (total_cap + tile - 1) / tile;
  const int g = grid_for(tiles, 4096);
  hipLaunchKernelGGL(k_diff_split, dim3(grid_for((tiles + 1 + kBlock / kWave - 1) / (kBlock / kWave), 4096)),
                     dim3(kBlock), 0, (hipStream_t)stream, p, u32(tile));
  FV_LAUNCH_BLOCK(k_diff_count, block, g, stream, p);
  hipLaunchKernelGGL(k_diff_scan, dim3(1), dim3(kDiffScanBlock), 0, (hipStream_t)stream, p, u32(tile));
  FV_LAUNCH_BLOCK(k_diff_write, block, g, stream, p);
  return int(hipGetLastError());
}

u64 diff_sorted_scratch_words(u64 total_cap) {
  const u64 tiles = (total_cap + 128 * kDiffItems - 1) / (128 * kDiffItems);   // the smallest tiles
  return 4 * (tiles + 1);
}

int launch_commit(const CommitParams& p, void* stream) {
  hipLaunchKernelGGL(k_commit, dim3(1), dim3(64), 0, (hipStream_t)stream, p);
  return int(hipGetLastError());
}

}  // namespace fv
