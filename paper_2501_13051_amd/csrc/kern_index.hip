// Join-index construction and column utilities.
//
// The join index of a relation on a key (one or two columns) is the hybrid
// index of Section 3: an open-addressing table that holds each distinct key
// once (run-length encoding of the key column, which keeps repeated values
// from piling into long collision chains) with the value (start, count) into
// a row-id array in which the rows of one key are contiguous.  It is built
// without a sort: count rows per distinct key in the table, exclusive-scan the
// counts over the table to get each run's start, then scatter row ids into
// their runs.  Row order inside a run is unspecified, which joins do not
// observe.
#include "fv_device.h"

namespace fv {

constexpr u32 kScanTile = kBlock * 4;

__device__ __forceinline__ bool row_indexed(const IndexParams& p, u64 row) {
  bool ok = true;
#pragma unroll
  for (u32 i = 0; i < 2; ++i)
    if (i < p.nfilt) ok = ok && p.col[p.fcol[i]][row] == p.fval[i];
  return ok;
}

__device__ __forceinline__ u64 row_key(const IndexParams& p, u64 row) {
  const u32 a = p.col[p.keycol[0]][row];
  if (p.nkey == 2) return (u64(a) << 32) | u64(p.col[p.keycol[1]][row]);
  return u64(a);
}

__global__ void k_idx_clear(Slot* tab, u64 cap, const u32* abort, u64* ndv, u64* maxrun, u64* full, u64* rows) {
  if (abort && *abort) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (ndv) *ndv = 0;
    if (maxrun) *maxrun = 0;
    if (full) *full = 0;
    if (rows) *rows = 0;
  }
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < cap; i += u64(gridDim.x) * blockDim.x)
    tab[i] = Slot{kEmptyKey, 0u, 0u};
}

// Rows are taken a tile at a time and grouped by key in an LDS map first, so
// that the global table sees one probe and one atomic per distinct key per
// tile rather than per row: a key that covers millions of rows (a predicate
// column, say) would otherwise serialise every row on one counter.
constexpr u32 kIdxItems = 4;
constexpr u32 kIdxTile = kBlock * kIdxItems;   // rows per block step
constexpr u32 kLdsMap = 2 * kIdxTile;           // LDS map slots: load <= 1/2

struct IdxLds {
  u64 key[kLdsMap];
  u32 cnt[kLdsMap];
  u32 pos[kLdsMap];
};

__device__ __forceinline__ void lds_map_clear(IdxLds& m) {
  for (u32 i = threadIdx.x; i < kLdsMap; i += kBlock) {
    m.key[i] = kEmptyKey;
    m.cnt[i] = 0u;
  }
}

// Slot of `key` in the block's map (inserted if absent) and the row's rank
// among the tile's rows with that key.  At most kIdxTile keys go into
// kLdsMap slots, so an empty slot is always reached.
__device__ __forceinline__ u32 lds_map_add(IdxLds& m, u64 key, u32& rank) {
  u32 h = u32(mix64(key)) & (kLdsMap - 1);
  for (u32 i = 0; i < kLdsMap; ++i) {
    const u64 cur = __hip_atomic_load(&m.key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == key) break;
    if (cur == kEmptyKey) {
      const u64 prev = atomicCAS(reinterpret_cast<unsigned long long*>(&m.key[h]), kEmptyKey, key);
      if (prev == kEmptyKey || prev == key) break;
    }
    h = (h + 1) & (kLdsMap - 1);
  }
  rank = atomicAdd(&m.cnt[h], 1u);
  return h;
}

// kInc: an update over the appended rows, counting into dcnt; block 0 also
// saves the old row count and clears the statistics the scan recomputes.
template <bool kInc>
__global__ __launch_bounds__(kBlock) void k_idx_count(IndexParams p) {
  __shared__ IdxLds m;
  if (p.abort && *p.abort) return;
  if (kInc && p.abort2 && *p.abort2) return;
  if (kInc && blockIdx.x == 0 && threadIdx.x == 0) {
    *p.rows_prev = *p.rows;
    *p.rows = 0;
    *p.ndv = 0;
    *p.maxrun = 0;
  }
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 mask = p.cap - 1;
  const u64 ntiles = (n + kIdxTile - 1) / kIdxTile;
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    lds_map_clear(m);
    __syncthreads();
    const u64 r0 = tile * kIdxTile + threadIdx.x;
#pragma unroll
    for (u32 k = 0; k < kIdxItems; ++k) {
      const u64 r = r0 + u64(k) * kBlock;
      if (r < n && row_indexed(p, begin + r)) {
        u32 rank;
        (void)lds_map_add(m, row_key(p, begin + r), rank);
      }
    }
    __syncthreads();
    for (u32 e = threadIdx.x; e < kLdsMap; e += kBlock) {
      const u32 c = m.cnt[e];
      if (!c) continue;
      // once the table has overflowed the index is rebuilt larger anyway:
      // later keys skip the (long) probe sequence of a full table
      if (p.full && (__hip_atomic_load(p.full, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1)) continue;
      const u64 h = index_insert(p.table, mask, m.key[e]);
      if (h == kNoSlot) {
        if (p.full) atomicOr(reinterpret_cast<unsigned long long*>(p.full), 1ull);
        continue;
      }
      atomicAdd(kInc ? &p.dcnt[h] : &p.table[h].count, c);
    }
    __syncthreads();
  }
}

// Exclusive scan over the table in slot order (look-back across tiles).
// Build: start <- prefix of counts, count <- 0 (it becomes the fill cursor),
// or count kept (kKeep: the sorted build has already placed the rows).
// Update (kInc): dsh <- prefix of the appended counts, start += dsh, dcnt <- 0
// (kept with kKeep: the sorted update still needs it); count keeps the old
// rows, so the fill appends after them.  Both recompute the distinct keys,
// longest run and rows of the result.
template <bool kInc, bool kKeep = false>
__global__ __launch_bounds__(kBlock) void k_idx_scan(IndexParams p) {
  __shared__ u32 s_ticket;
  __shared__ u32 s_c[kBlock / kWave + 1];
  __shared__ u64 s_excl;
  if (p.abort && *p.abort) return;
  if (kInc && p.abort2 && *p.abort2) return;
  const u32 epoch = launch_epoch(p.epoch_base, p.epoch_off);
  const u32 ntiles = u32((p.cap + kScanTile - 1) / kScanTile);
  if (blockIdx.x >= participants(ntiles)) return;
  for (;;) {
    const u32 tile = take_ticket(p.ticket, ntiles, &s_ticket);
    if (tile >= ntiles) break;
    const u64 s0 = u64(tile) * kScanTile + u64(threadIdx.x) * 4;
    u32 c[4];
    u32 mine = 0, keys = 0, longest = 0, total = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool in = s0 + k < p.cap;
      const u32 old = in ? p.table[s0 + k].count : 0u;
      c[k] = kInc ? (in ? p.dcnt[s0 + k] : 0u) : old;
      const u32 all = kInc ? old + c[k] : old;
      mine += c[k];
      total += all;
      keys += all ? 1u : 0u;
      longest = all > longest ? all : longest;
    }
    if (p.ndv) {
      const u32 wk = wave_sum(keys);
      if (lane_id() == 0 && wk) atomicAdd(reinterpret_cast<unsigned long long*>(p.ndv), (unsigned long long)wk);
    }
    if (p.rows) {
      const u64 wr = wave_sum(u64(total));
      if (lane_id() == 0 && wr) atomicAdd(reinterpret_cast<unsigned long long*>(p.rows), (unsigned long long)wr);
    }
    if (p.maxrun) {
      for (int d = kWave / 2; d >= 1; d >>= 1) {
        const u32 o = __shfl_xor(longest, d, kWave);
        longest = o > longest ? o : longest;
      }
      if (lane_id() == 0 && longest)
        atomicMax(reinterpret_cast<unsigned long long*>(p.maxrun), (unsigned long long)longest);
    }
    u32 tot;
    const u32 ex = block_exclusive_sum<kBlock>(mine, s_c, &tot);
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
    u64 run = s_excl + ex;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (s0 + k < p.cap) {
        if (kInc) {
          p.dsh[s0 + k] = u32(run);
          if (!kKeep) p.dcnt[s0 + k] = 0u;
          p.table[s0 + k].start += u32(run);
        } else {
          p.table[s0 + k].start = u32(run);
          if (!kKeep) p.table[s0 + k].count = 0u;
        }
      }
      run += c[k];
    }
    __syncthreads();
  }
}

// Scatter row ids into their key's run: the tile's rows are grouped in the
// LDS map again, one global atomic per distinct key reserves the group's
// places in the run, and each row takes the place of its rank in the group.
template <bool kInc>
__global__ __launch_bounds__(kBlock) void k_idx_fill(IndexParams p) {
  __shared__ IdxLds m;
  if (p.abort && *p.abort) return;
  if (kInc && p.abort2 && *p.abort2) return;
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 mask = p.cap - 1;
  const u64 ntiles = (n + kIdxTile - 1) / kIdxTile;
  u32* perm = kInc ? p.perm_out : p.perm;
  u32* pslot = kInc ? p.pslot_out : p.pslot;
  if (p.full && (*p.full & 1)) return;   // keys are missing: the index is rebuilt larger
  if (*p.rows > p.perm_cap) {   // the runs would not fit: flag it, write nothing
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(reinterpret_cast<unsigned long long*>(p.full), 2ull);
    return;
  }
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    lds_map_clear(m);
    __syncthreads();
    const u64 r0 = tile * kIdxTile + threadIdx.x;
    u32 ent[kIdxItems], rank[kIdxItems];
#pragma unroll
    for (u32 k = 0; k < kIdxItems; ++k) {
      const u64 r = r0 + u64(k) * kBlock;
      ent[k] = ~0u;
      rank[k] = 0;
      if (r < n && row_indexed(p, begin + r)) ent[k] = lds_map_add(m, row_key(p, begin + r), rank[k]);
    }
    __syncthreads();
    for (u32 e = threadIdx.x; e < kLdsMap; e += kBlock) {
      const u32 c = m.cnt[e];
      if (!c) continue;
      const u64 h = index_slot_of(p.table, mask, m.key[e]);
      // a key whose insert failed has no run: the host rebuilds a larger table
      m.pos[e] = h == kNoSlot ? ~0u : p.table[h].start + atomicAdd(&p.table[h].count, c);
      m.key[e] = h;   // the slot, for pslot (the map is not probed again)
    }
    __syncthreads();
#pragma unroll
    for (u32 k = 0; k < kIdxItems; ++k) {
      if (ent[k] == ~0u) continue;
      const u32 base = m.pos[ent[k]];
      if (base == ~0u) continue;
      perm[base + rank[k]] = u32(begin + r0 + u64(k) * kBlock);
      pslot[base + rank[k]] = u32(m.key[ent[k]]);
    }
    __syncthreads();
  }
}

// Update: old position i of slot s moves to i + dsh[s] (runs keep their
// order and shift right by the rows appended to earlier slots).
__global__ __launch_bounds__(kBlock) void k_idx_move(IndexParams p) {
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  if (*p.rows > p.perm_cap) return;   // flagged by the fill
  if (p.full && (*p.full & 1)) return;   // keys are missing: the index is rebuilt larger
  const u64 n = *p.rows_prev;
  for (u64 i = u64(blockIdx.x) * kBlock + threadIdx.x; i < n; i += u64(gridDim.x) * kBlock) {
    const u32 s = p.pslot[i];
    const u64 j = i + p.dsh[s];
    p.perm_out[j] = p.perm[i];
    p.pslot_out[j] = s;
  }
}

// ------------------------------------------------------------------ sorted build
// The construction of Section 3 sorts the key column and run-length encodes
// it.  Here every indexed row finds (or inserts) its key's slot with a plain
// probe -- no per-row counter, so a hot key costs nothing extra -- and the
// word (row << row_shift | slot) goes through a stable LSD radix sort over
// the slot bits (launch_rs_hist / launch_rs_pass, run by the caller).  The
// sorted words list the rows grouped by slot, runs in slot order and row ids
// ascending inside a run: the layout the counting build produces, so the
// incremental update applies to it unchanged.  A run's count comes from its
// two boundaries (one atomic each, order-free modulo 2^32), and the table
// scan turns counts into starts.  Rows outside the index's filter take the
// slot value `cap`, which sorts after every real slot, and are dropped.

// Find-or-insert with a plain first read: slots only go from empty to a key
// during a build, so a stale read can only show "empty", which the CAS then
// corrects (the same argument as for the tuple set).
__device__ __forceinline__ u64 index_insert_probe(Slot* tab, u64 mask, u64 key) {
  u64 h = mix64(key) & mask;
  for (u32 i = 0; i < kMaxProbe && i <= mask; ++i) {
    const u64 cur = tab[h].key;
    if (cur == key) return h;
    if (cur == kEmptyKey) {
      const u64 prev = atomic_cas_u64(&tab[h].key, kEmptyKey, key);
      if (prev == kEmptyKey || prev == key) return h;
    }
    h = (h + 1) & mask;
  }
  return kNoSlot;
}

__global__ __launch_bounds__(kBlock) void k_idx_slotkeys(IndexParams p, u64* keys, u32 row_shift) {
  if (p.abort && *p.abort) return;
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 mask = p.cap - 1;
  // kS rows per thread and step: their keys, then their home slots, are
  // read together; only a key whose home slot is taken by another key (or
  // still empty) goes on to the find-or-insert
  constexpr int kS = 4;
  const u64 stride = u64(gridDim.x) * kBlock;
  for (u64 r0 = u64(blockIdx.x) * kBlock + threadIdx.x; r0 < n; r0 += stride * kS) {
    bool in[kS];
    u64 key[kS];
#pragma unroll
    for (int j = 0; j < kS; ++j) {
      const u64 r = min_u64(r0 + j * stride, n - 1);   // reads stay in bounds, unconditionally
      in[j] = r0 + j * stride < n && row_indexed(p, begin + r);
      key[j] = row_key(p, begin + r);
    }
    // once the table has overflowed the index is rebuilt larger: later rows
    // skip the long probe sequences of a full table
    const bool full = p.full && (__hip_atomic_load(p.full, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1);
    u64 home[kS];
#pragma unroll
    for (int j = 0; j < kS; ++j) home[j] = (in[j] && !full) ? p.table[mix64(key[j]) & mask].key : kEmptyKey;
#pragma unroll
    for (int j = 0; j < kS; ++j) {
      const u64 r = r0 + j * stride;
      if (r >= n) break;
      u64 slot = p.cap;   // rows outside the filter sort after every slot
      if (in[j]) {
        slot = full ? kNoSlot
                    : home[j] == key[j] ? (mix64(key[j]) & mask) : index_insert_probe(p.table, mask, key[j]);
        if (slot == kNoSlot) {
          if (p.full && !full) atomicOr(reinterpret_cast<unsigned long long*>(p.full), 1ull);
          slot = 0;
        }
      }
      keys[r] = (r << row_shift) | slot;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_idx_runs(IndexParams p, const u64* __restrict__ keys, u32 row_shift) {
  if (p.abort && *p.abort) return;
  if (p.full && (*p.full & 1)) return;   // keys are missing: the index is rebuilt larger
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 smask = (u64(1) << row_shift) - 1;
  bool over = false;
  for (u64 i = u64(blockIdx.x) * kBlock + threadIdx.x; i < n; i += u64(gridDim.x) * kBlock) {
    const u64 k = keys[i];
    const u64 s = k & smask;
    if (s >= p.cap) continue;   // outside the filter (sorted last)
    if (i < p.perm_cap) {
      p.perm[i] = u32(begin + (k >> row_shift));
      p.pslot[i] = u32(s);
    } else {
      over = true;
    }
    const bool head = i == 0 || (keys[i - 1] & smask) != s;
    const bool tail = i + 1 == n || (keys[i + 1] & smask) != s;
    if (head || tail) atomicAdd(&p.table[s].count, (tail ? u32(i + 1) : 0u) - (head ? u32(i) : 0u));
  }
  // the runs would not fit: flag it (the host regrows the positions)
  if (over && p.full) atomicOr(reinterpret_cast<unsigned long long*>(p.full), 2ull);
}

// ------------------------------------------------------------------ sorted update
// An update over many appended rows sorts them by slot as the sorted build
// does (k_idx_slotkeys over the appended range, then the radix sort), so
// that no appended row needs a per-row atomic: the boundaries of each slot's
// run give its appended count, the update scan shifts the old runs, and the
// appended rows are written after each key's old rows at their rank in the
// run.  After that pass each slot's count takes its appended rows and the
// per-slot counter is cleared for the next update.

__global__ __launch_bounds__(kBlock) void k_idx_druns(IndexParams p, const u64* __restrict__ keys, u32 row_shift) {
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  if (p.full && (*p.full & 1)) return;   // keys are missing: the index is rebuilt larger
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *p.rows_prev = *p.rows;
    *p.rows = 0;
    *p.ndv = 0;
    *p.maxrun = 0;
  }
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 smask = (u64(1) << row_shift) - 1;
  for (u64 j = u64(blockIdx.x) * kBlock + threadIdx.x; j < n; j += u64(gridDim.x) * kBlock) {
    const u64 s = keys[j] & smask;
    if (s >= p.cap) continue;   // outside the filter (sorted last)
    const bool head = j == 0 || (keys[j - 1] & smask) != s;
    const bool tail = j + 1 == n || (keys[j + 1] & smask) != s;
    if (head || tail) atomicAdd(&p.dcnt[s], (tail ? u32(j + 1) : 0u) - (head ? u32(j) : 0u));
  }
}

// Appended row j of slot s goes to start(s) + count(s) + (j - dsh(s)): its
// key's new run start, past the key's old rows, at its rank among the key's
// appended rows (dsh(s) is where that key's rows begin in the sorted words).
__global__ __launch_bounds__(kBlock) void k_idx_dfill(IndexParams p, const u64* __restrict__ keys, u32 row_shift) {
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  if (p.full && (*p.full & 1)) return;
  if (*p.rows > p.perm_cap) {   // the runs would not fit: flag it, write nothing
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(reinterpret_cast<unsigned long long*>(p.full), 2ull);
    return;
  }
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 smask = (u64(1) << row_shift) - 1;
  for (u64 j = u64(blockIdx.x) * kBlock + threadIdx.x; j < n; j += u64(gridDim.x) * kBlock) {
    const u64 k = keys[j];
    const u64 s = k & smask;
    if (s >= p.cap) continue;
    const u64 pos = u64(p.table[s].start) + p.table[s].count + (j - p.dsh[s]);
    p.perm_out[pos] = u32(begin + (k >> row_shift));
    p.pslot_out[pos] = u32(s);
  }
}

// count += appended rows, appended counter cleared: one thread per slot (the
// head of its run), after every read of both.
__global__ __launch_bounds__(kBlock) void k_idx_dfinish(IndexParams p, const u64* __restrict__ keys, u32 row_shift) {
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  if (p.full && (*p.full & 1)) return;   // nothing was counted
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 smask = (u64(1) << row_shift) - 1;
  for (u64 j = u64(blockIdx.x) * kBlock + threadIdx.x; j < n; j += u64(gridDim.x) * kBlock) {
    const u64 s = keys[j] & smask;
    if (s >= p.cap) continue;
    if (j != 0 && (keys[j - 1] & smask) == s) continue;
    p.table[s].count += p.dcnt[s];
    p.dcnt[s] = 0u;
  }
}

static int grid_rows(u64 n, int cap) {
  const u64 b = (n + kBlock - 1) / kBlock;
  return int(b == 0 ? 1 : (b > u64(cap) ? u64(cap) : b));
}

int launch_index_build(const IndexParams& p, u64 rows_cap, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_idx_clear, dim3(grid_rows(p.cap, 4096)), dim3(kBlock), 0, s, p.table, p.cap, p.abort, p.ndv,
                     p.maxrun, p.full, p.rows);
  const u64 row_tiles = (rows_cap + kIdxTile - 1) / kIdxTile;
  const int row_grid = int(row_tiles == 0 ? 1 : (row_tiles > 4096 ? 4096 : row_tiles));
  hipLaunchKernelGGL(k_idx_count<false>, dim3(row_grid), dim3(kBlock), 0, s, p);
  const u64 tiles = (p.cap + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_idx_scan<false>, dim3(int(tiles > 2048 ? 2048 : tiles)), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_idx_fill<false>, dim3(row_grid), dim3(kBlock), 0, s, p);
  return int(hipGetLastError());
}

int launch_index_slotkeys(const IndexParams& p, u64 rows_cap, u64* keys, u32 row_shift, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_idx_clear, dim3(grid_rows(p.cap, 4096)), dim3(kBlock), 0, s, p.table, p.cap, p.abort, p.ndv,
                     p.maxrun, p.full, p.rows);
  hipLaunchKernelGGL(k_idx_slotkeys, dim3(grid_rows(rows_cap, 8192)), dim3(kBlock), 0, s, p, keys, row_shift);
  return int(hipGetLastError());
}

int launch_index_update_keys(const IndexParams& p, u64 delta_rows_cap, u64* keys, u32 row_shift, void* stream) {
  hipLaunchKernelGGL(k_idx_slotkeys, dim3(grid_rows(delta_rows_cap, 8192)), dim3(kBlock), 0, (hipStream_t)stream, p,
                     keys, row_shift);
  return int(hipGetLastError());
}

int launch_index_update_runs(const IndexParams& p, u64 delta_rows_cap, u64 old_rows_cap, const u64* sorted,
                             u32 row_shift, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const int dgrid = grid_rows(delta_rows_cap, 8192);
  hipLaunchKernelGGL(k_idx_druns, dim3(dgrid), dim3(kBlock), 0, s, p, sorted, row_shift);
  const u64 tiles = (p.cap + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL((k_idx_scan<true, true>), dim3(int(tiles > 2048 ? 2048 : tiles)), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_idx_move, dim3(grid_rows(old_rows_cap, 8192)), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_idx_dfill, dim3(dgrid), dim3(kBlock), 0, s, p, sorted, row_shift);
  hipLaunchKernelGGL(k_idx_dfinish, dim3(dgrid), dim3(kBlock), 0, s, p, sorted, row_shift);
  return int(hipGetLastError());
}

int launch_index_runs(const IndexParams& p, u64 rows_cap, const u64* sorted, u32 row_shift, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_idx_runs, dim3(grid_rows(rows_cap, 8192)), dim3(kBlock), 0, s, p, sorted, row_shift);
  const u64 tiles = (p.cap + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL((k_idx_scan<false, true>), dim3(int(tiles > 2048 ? 2048 : tiles)), dim3(kBlock), 0, s, p);
  return int(hipGetLastError());
}

int launch_index_update(const IndexParams& p, u64 delta_rows_cap, u64 old_rows_cap, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const u64 row_tiles = (delta_rows_cap + kIdxTile - 1) / kIdxTile;
  const int row_grid = int(row_tiles == 0 ? 1 : (row_tiles > 4096 ? 4096 : row_tiles));
  hipLaunchKernelGGL(k_idx_count<true>, dim3(row_grid), dim3(kBlock), 0, s, p);
  const u64 tiles = (p.cap + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_idx_scan<true>, dim3(int(tiles > 2048 ? 2048 : tiles)), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_idx_move, dim3(grid_rows(old_rows_cap, 8192)), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_idx_fill<true>, dim3(row_grid), dim3(kBlock), 0, s, p);
  return int(hipGetLastError());
}

// ------------------------------------------------------------------ column utilities
__global__ void k_colmax(const u32* col, u64 n, u32* out) {
  u32 m = 0;
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += u64(gridDim.x) * blockDim.x)
    m = col[i] > m ? col[i] : m;
  // wave max, one atomic per wave
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const u32 o = __shfl_xor(m, d, kWave);
    m = o > m ? o : m;
  }
  if (lane_id() == 0) atomicMax(out, m);
}

int launch_colmax(const u32* col, u64 n, u32* out, void* stream) {
  hipLaunchKernelGGL(k_colmax, dim3(grid_rows(n, 2048)), dim3(kBlock), 0, (hipStream_t)stream, col, n, out);
  return int(hipGetLastError());
}

struct PackArgs {
  const u32* cols[3];
  u32 arity;
  u32 shift[3];
  u32 width[3];
};

__global__ void k_pack(PackArgs a, u64 n, u64* keys) {
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += u64(gridDim.x) * blockDim.x) {
    u64 k = 0;
    for (u32 c = 0; c < a.arity; ++c) k |= u64(a.cols[c][i]) << a.shift[c];
    keys[i] = k;
  }
}

__global__ void k_unpack(const u64* keys, u64 n, PackArgs a, u32* o0, u32* o1, u32* o2) {
  u32* outs[3] = {o0, o1, o2};
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += u64(gridDim.x) * blockDim.x) {
    const u64 k = keys[i];
    for (u32 c = 0; c < a.arity; ++c) {
      const u64 m = a.width[c] >= 32 ? 0xFFFFFFFFull : ((1ull << a.width[c]) - 1);
      outs[c][i] = u32((k >> a.shift[c]) & m);
    }
  }
}

__global__ void k_set_rows(PackArgs a, u64 n, u64* set, u64 mask) {
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += u64(gridDim.x) * blockDim.x) {
    u64 k = 0;
    for (u32 c = 0; c < a.arity; ++c) k |= u64(a.cols[c][i]) << a.shift[c];
    (void)set_insert(set, mask, k);
  }
}

__global__ void k_set_rows32(PackArgs a, u64 n, u32* set, u64 mask, u64* ones) {
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += u64(gridDim.x) * blockDim.x) {
    u64 k = 0;
    for (u32 c = 0; c < a.arity; ++c) k |= u64(a.cols[c][i]) << a.shift[c];
    (void)set32_insert(set, mask, u32(k), ones);
  }
}

static PackArgs pack_args(const u32* const* cols, u32 arity, const u32* shift, const u32* width) {
  PackArgs a{};
  a.arity = arity;
  for (u32 c = 0; c < arity && c < 3; ++c) {
    a.cols[c] = cols ? cols[c] : nullptr;
    a.shift[c] = shift[c];
    a.width[c] = width ? width[c] : 32;
  }
  return a;
}

int launch_pack(const u32* const* cols, u32 arity, const u32* shift, u64 n, u64* keys, void* stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_pack, dim3(grid_rows(n, 4096)), dim3(kBlock), 0, (hipStream_t)stream,
                     pack_args(cols, arity, shift, nullptr), n, keys);
  return int(hipGetLastError());
}

int launch_unpack(const u64* keys, u64 n, u32 arity, const u32* shift, const u32* width, u32* const* cols,
                  void* stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_unpack, dim3(grid_rows(n, 4096)), dim3(kBlock), 0, (hipStream_t)stream, keys, n,
                     pack_args(nullptr, arity, shift, width), cols[0], arity > 1 ? cols[1] : nullptr,
                     arity > 2 ? cols[2] : nullptr);
  return int(hipGetLastError());
}

__global__ void k_add_u32(u32* p, u64 n, u32 delta) {
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += u64(gridDim.x) * blockDim.x) p[i] += delta;
}

int launch_add_u32(u32* p, u64 n, u32 delta, void* stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_add_u32, dim3(grid_rows(n, 4096)), dim3(kBlock), 0, (hipStream_t)stream, p, n, delta);
  return int(hipGetLastError());
}

// out[k] = first position of a sorted column whose value is >= k * stride,
// for k = 0 .. n_inst (out[n_inst] = n when every value is below n_inst * stride).
__global__ void k_bounds(const u32* col, u64 n, u32 stride, u32 n_inst, u64* out) {
  for (u32 k = blockIdx.x * blockDim.x + threadIdx.x; k <= n_inst; k += gridDim.x * blockDim.x) {
    const u64 key = u64(k) * stride;
    u64 lo = 0, hi = n;
    while (lo < hi) {
      const u64 mid = (lo + hi) >> 1;
      if (u64(col[mid]) < key) lo = mid + 1; else hi = mid;
    }
    out[k] = lo;
  }
}

int launch_bounds(const u32* col, u64 n, u32 stride, u32 n_inst, u64* out, void* stream) {
  hipLaunchKernelGGL(k_bounds, dim3((n_inst + 1 + kBlock - 1) / kBlock), dim3(kBlock), 0, (hipStream_t)stream, col,
                     n, stride, n_inst, out);
  return int(hipGetLastError());
}

// Concatenate the rows of many sources into one set of columns, adding a
// per-source offset to every value (the batched form's id relabelling).
__global__ void k_gather_relabel(const GatherDesc* d, u32 arity, u32* o0, u32* o1, u32* o2) {
  const GatherDesc g = d[blockIdx.y];
  u32* outs[3] = {o0, o1, o2};
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < g.n; i += u64(gridDim.x) * blockDim.x)
    for (u32 c = 0; c < arity; ++c) outs[c][g.dst + i] = g.src[c][i] + g.add;
}

int launch_gather_relabel(const GatherDesc* d, u32 n_src, u32 arity, u32* const* out, void* stream) {
  if (n_src == 0) return 0;
  hipLaunchKernelGGL(k_gather_relabel, dim3(16, n_src), dim3(kBlock), 0, (hipStream_t)stream, d, arity, out[0],
                     arity > 1 ? out[1] : nullptr, arity > 2 ? out[2] : nullptr);
  return int(hipGetLastError());
}

int launch_set_insert_rows(const u32* const* cols, u32 arity, const u32* shift, u64 n, u64* set, u64 mask,
                           void* stream, u32* set32, u64* ones) {
  if (n == 0) return 0;
  if (set32)
    hipLaunchKernelGGL(k_set_rows32, dim3(grid_rows(n, 4096)), dim3(kBlock), 0, (hipStream_t)stream,
                       pack_args(cols, arity, shift, nullptr), n, set32, mask, ones);
  else
    hipLaunchKernelGGL(k_set_rows, dim3(grid_rows(n, 4096)), dim3(kBlock), 0, (hipStream_t)stream,
                       pack_args(cols, arity, shift, nullptr), n, set, mask);
  return int(hipGetLastError());
}

}  // namespace fv
