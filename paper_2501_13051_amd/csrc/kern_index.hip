// Join-index construction and maintenance, and column utilities.
//
// The join index of a relation on a key (one or two columns) is the hybrid
// index of Section 3: an open-addressing table that holds each distinct key
// once (run-length encoding of the key column, which keeps repeated values
// from piling into long collision chains) with the value (start, count) into
// a row-id array (perm) in which the rows of one key are contiguous.  A build
// either counts rows per distinct key in the table, exclusive-scans the counts
// over the table to get each run's start and scatters the row ids into their
// runs, or (large builds) sorts (row, slot) words by slot as Section 3 sorts
// its key column.  Row order inside a run is unspecified, which joins do not
// observe.  Indices of derived relations are then updated every round with
// the rows the round appended, touching only the keys that got rows.
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

__global__ void k_fill_u32_idx(u32* p, u64 n) {
  for (u64 i = u64(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += u64(gridDim.x) * blockDim.x) p[i] = 0u;
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

// Group the indexed rows of a tile by key in the block's map.
__device__ __forceinline__ void map_tile(const IndexParams& p, IdxLds& m, u64 begin, u64 n, u64 tile,
                                         u32* ent, u32* rank) {
  const u64 r0 = tile * kIdxTile + threadIdx.x;
#pragma unroll
  for (u32 k = 0; k < kIdxItems; ++k) {
    const u64 r = r0 + u64(k) * kBlock;
    ent[k] = ~0u;
    rank[k] = 0;
    if (r < n && row_indexed(p, begin + r)) ent[k] = lds_map_add(m, row_key(p, begin + r), rank[k]);
  }
}

// Build, step 1: rows per distinct key, counted into the table.
__global__ __launch_bounds__(kBlock) void k_idx_count(IndexParams p) {
  __shared__ IdxLds m;
  if (p.abort && *p.abort) return;
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 mask = p.cap - 1;
  const u64 ntiles = (n + kIdxTile - 1) / kIdxTile;
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    lds_map_clear(m);
    __syncthreads();
    u32 ent[kIdxItems], rank[kIdxItems];
    map_tile(p, m, begin, n, tile, ent, rank);
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
      atomicAdd(&p.table[h].count, c);
    }
    __syncthreads();
  }
}

// Build, step 2: exclusive scan over the table in slot order (look-back
// across tiles): start <- prefix of the regions, and count <- 0 (it becomes
// the fill cursor) or kept (kKeep: the sorted build places the rows after
// this scan, or has placed them).  A loaded relation's index packs its runs
// (region = count); a derived relation's index (pcap set) gives each run a
// region of twice its rows, so that the next updates mostly append in place,
// records the regions in pcap and starts the bump pointer past the last one.
// The distinct keys, longest run and rows are recomputed; regions past the
// positions available raise bit 1 of the full flag.
template <bool kKeep>
__global__ __launch_bounds__(kBlock) void k_idx_scan(IndexParams p) {
  __shared__ u32 s_ticket;
  __shared__ u32 s_c[kBlock / kWave + 1];
  __shared__ u64 s_excl;
  __shared__ u64 s_red[kBlock / kWave];
  if (p.abort && *p.abort) return;
  const u32 epoch = launch_epoch(p.epoch_base, p.epoch_off);
  const u32 ntiles = u32((p.cap + kScanTile - 1) / kScanTile);
  if (blockIdx.x >= participants(ntiles)) return;
  // the statistics go to their counters once per block, after the last tile
  u64 keys_acc = 0, rows_acc = 0, longest_acc = 0;
  for (;;) {
    const u32 tile = take_ticket(p.ticket, ntiles, &s_ticket);
    if (tile >= ntiles) break;
    const u64 s0 = u64(tile) * kScanTile + u64(threadIdx.x) * 4;
    u32 c[4];
    u32 mine = 0;
    const u32 slack = p.pcap ? 2u : 1u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[k] = s0 + k < p.cap ? p.table[s0 + k].count : 0u;
      mine += slack * c[k];
      rows_acc += c[k];
      keys_acc += c[k] ? 1u : 0u;
      longest_acc = c[k] > longest_acc ? c[k] : longest_acc;
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
        p.table[s0 + k].start = u32(run);
        if (!kKeep) p.table[s0 + k].count = 0u;
        if (p.pcap) p.pcap[s0 + k] = slack * c[k];
      }
      run += slack * c[k];
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) {
      const u64 total = s_excl + tot;
      if (p.top) *p.top = total;
      if (total > p.perm_cap && p.full) atomicOr(reinterpret_cast<unsigned long long*>(p.full), 2ull);
    }
    __syncthreads();
  }
  const u64 bk = block_sum<kBlock>(keys_acc, s_red);
  const u64 br = block_sum<kBlock>(rows_acc, s_red);
  const u64 bl = block_max<kBlock>(longest_acc, s_red);
  if (threadIdx.x == 0) {
    if (p.ndv && bk) atomicAdd(reinterpret_cast<unsigned long long*>(p.ndv), (unsigned long long)bk);
    if (p.rows && br) atomicAdd(reinterpret_cast<unsigned long long*>(p.rows), (unsigned long long)br);
    if (p.maxrun && bl) atomicMax(reinterpret_cast<unsigned long long*>(p.maxrun), (unsigned long long)bl);
  }
}

// Build, step 3: scatter row ids into their key's run: the tile's rows are
// grouped in the LDS map again, one global atomic per distinct key reserves
// the group's places in the run, and each row takes the place of its rank in
// the group.
__global__ __launch_bounds__(kBlock) void k_idx_fill(IndexParams p) {
  __shared__ IdxLds m;
  if (p.abort && *p.abort) return;
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 mask = p.cap - 1;
  const u64 ntiles = (n + kIdxTile - 1) / kIdxTile;
  // keys are missing (the index is rebuilt larger) or the regions do not
  // fit (flagged by the scan): write nothing
  if (p.full && (*p.full & 3)) return;
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    lds_map_clear(m);
    __syncthreads();
    u32 ent[kIdxItems], rank[kIdxItems];
    map_tile(p, m, begin, n, tile, ent, rank);
    __syncthreads();
    for (u32 e = threadIdx.x; e < kLdsMap; e += kBlock) {
      const u32 c = m.cnt[e];
      if (!c) continue;
      const u64 h = index_slot_of(p.table, mask, m.key[e]);
      // a key whose insert failed has no run: the host rebuilds a larger table
      m.pos[e] = h == kNoSlot ? ~0u : p.table[h].start + atomicAdd(&p.table[h].count, c);
    }
    __syncthreads();
#pragma unroll
    for (u32 k = 0; k < kIdxItems; ++k) {
      if (ent[k] == ~0u) continue;
      const u32 base = m.pos[ent[k]];
      if (base == ~0u) continue;
      p.perm[base + rank[k]] = u32(begin + tile * kIdxTile + threadIdx.x + u64(k) * kBlock);
    }
    __syncthreads();
  }
}

// A larger table for an intact index of a derived relation: every key of the
// old table is inserted again with its run and region (the runs stay where
// they are in perm), so the index need not be rebuilt.  A key that finds no
// slot raises bit 0 of the full flag (the index is then rebuilt).
__global__ __launch_bounds__(kBlock) void k_idx_rehash(const Slot* __restrict__ old_tab,
                                                        const u32* __restrict__ old_pcap, u64 old_cap, Slot* tab,
                                                        u32* pcap, u64 cap, u64* full) {
  const u64 mask = cap - 1;
  for (u64 i = u64(blockIdx.x) * kBlock + threadIdx.x; i < old_cap; i += u64(gridDim.x) * kBlock) {
    const Slot sl = old_tab[i];
    if (sl.key == kEmptyKey) continue;
    const u64 h = index_insert(tab, mask, sl.key);
    if (h == kNoSlot) {
      atomicOr(reinterpret_cast<unsigned long long*>(full), 1ull);
      continue;
    }
    tab[h].start = sl.start;
    tab[h].count = sl.count;
    pcap[h] = old_pcap[i];
  }
}

// ------------------------------------------------------------------ update
// Update, step 1: the appended rows per key, grouped per tile in LDS, added
// to dcnt (new keys are inserted into the table with an empty run); a slot
// whose dcnt was zero joins the work list (one atomic per tile).  The value
// dcnt had before a group's add is the group's first place among the key's
// appended rows, so every appended row leaves rword[r] = slot << 32 | place
// (all ones when the row is not indexed): the placement then needs neither
// the grouping nor the table probe nor a second atomic per group.
__global__ __launch_bounds__(kBlock) void k_upd_count(IndexParams p) {
  __shared__ IdxLds m;
  __shared__ u32 s_c[kBlock / kWave + 1];
  __shared__ u64 s_wbase;
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 mask = p.cap - 1;
  const u64 ntiles = (n + kIdxTile - 1) / kIdxTile;
  for (u64 tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    lds_map_clear(m);
    __syncthreads();
    u32 ent[kIdxItems], rank[kIdxItems];
    map_tile(p, m, begin, n, tile, ent, rank);
    __syncthreads();
    // the tile's newly touched slots (kept in m.pos) join the work list
    // with one atomic per tile
    u32 pushes = 0;
    for (u32 e = threadIdx.x; e < kLdsMap; e += kBlock) {
      const u32 c = m.cnt[e];
      u32 slot = ~0u, first = 0u;
      if (c && !(__hip_atomic_load(p.full, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1)) {
        const u64 h = index_insert(p.table, mask, m.key[e]);
        if (h == kNoSlot) {
          atomicOr(reinterpret_cast<unsigned long long*>(p.full), 1ull);
        } else {
          first = atomicAdd(&p.dcnt[h], c);
          slot = u32(h);
        }
      }
      // the group's count is no longer needed: cnt now holds its first place
      // (top bit: the slot joins the work list)
      const bool push = slot != ~0u && first == 0u;
      m.pos[e] = slot;
      m.cnt[e] = push ? (first | 0x80000000u) : first;
      pushes += push ? 1u : 0u;
    }
    u32 tot;
    const u32 ex = block_exclusive_sum<kBlock>(pushes, s_c, &tot);
    if (threadIdx.x == 0)
      s_wbase = tot ? atomicAdd(reinterpret_cast<unsigned long long*>(p.wl_n), (unsigned long long)tot) : 0;
    __syncthreads();
    u64 at = s_wbase + ex;
    for (u32 e = threadIdx.x; e < kLdsMap; e += kBlock) {
      const u32 slot = m.pos[e];
      if (slot == ~0u || !(m.cnt[e] & 0x80000000u)) continue;
      if (at < p.cap) p.wl[at] = slot;
      ++at;
    }
    // (only indexed rows get a word: the placement tests the filter again)
#pragma unroll
    for (u32 k = 0; k < kIdxItems; ++k) {
      if (ent[k] == ~0u) continue;
      const u32 slot = m.pos[ent[k]];
      p.rword[tile * kIdxTile + threadIdx.x + u64(k) * kBlock] =
          slot == ~0u ? ~0ull : (u64(slot) << 32) | u64((m.cnt[ent[k]] & 0x7FFFFFFFu) + rank[k]);
    }
    __syncthreads();
  }
  ktime_end(p.ts);
}

// Copy a lane's old run (at most kInlineCopy rows) to its new region by the
// lane itself, kLaneCopy rows at a time with all of their loads in flight
// before the stores: every lane of the wave copies at once, so a wave whose
// lanes all move short runs waits for a few round trips, not one per run.
constexpr u32 kInlineCopy = 64;
constexpr u32 kLaneCopy = 8;
__device__ __forceinline__ void lane_copy_run(u32* perm, bool want, u32 from, u64 to, u32 count) {
  if (!want) return;
  for (u32 b = 0; b < count; b += kLaneCopy) {
    u32 v[kLaneCopy];
#pragma unroll
    for (u32 i = 0; i < kLaneCopy; ++i) v[i] = b + i < count ? perm[u64(from) + b + i] : 0u;
#pragma unroll
    for (u32 i = 0; i < kLaneCopy; ++i)
      if (b + i < count) perm[to + b + i] = v[i];
  }
}

constexpr u32 kMoveChunk = 1u << 16;   // rows per listed chunk of an old run

// Room for the runs of kResItems slots per thread (act[i], slot s[i] with
// c_old[i] old rows at position from[i], need[i] rows after the update):
// a run whose rows exceed its region gets a region of twice that many
// positions from the bump pointer (one atomic per block step for all of the
// block's runs), its old rows copied there on the spot (at most kInlineCopy)
// or listed in chunks, and its start / region size set.  A block-uniform
// call: every thread of the block must make it.
constexpr int kResItems = 2;
__device__ __forceinline__ void reserve_runs(const IndexParams& p, const bool* act, const u32* s, const u32* c_old,
                                             const u32* from, const u64* need, u64* s_scan, u64* s_base) {
  u64 newcap[kResItems], mine = 0;
#pragma unroll
  for (int i = 0; i < kResItems; ++i) {
    newcap[i] = act[i] && need[i] > p.pcap[s[i]] ? (need[i] < 8 ? 16 : 2 * need[i]) : 0;
    mine += newcap[i];
  }
  u64 btot;
  const u64 excl = block_exclusive_sum<kBlock>(mine, s_scan, &btot);
  if (threadIdx.x == 0) *s_base = btot ? atomicAdd(reinterpret_cast<unsigned long long*>(p.top), (unsigned long long)btot) : 0;
  __syncthreads();
  u64 at = *s_base + excl;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kResItems; ++i) {
    const u64 start_new = at;
    at += newcap[i];
    const bool fits = newcap[i] && start_new + newcap[i] <= p.perm_cap;
    lane_copy_run(p.perm, fits && c_old[i] <= kInlineCopy, from[i], start_new, c_old[i]);
    if (!newcap[i]) continue;
    if (!fits) {
      atomicOr(reinterpret_cast<unsigned long long*>(p.full), 2ull);   // rebuilt with more positions
      continue;
    }
    if (c_old[i] > kInlineCopy) {
      const u32 chunks = (c_old[i] + kMoveChunk - 1) / kMoveChunk;
      const u64 m = atomicAdd(reinterpret_cast<unsigned long long*>(p.moves_n), (unsigned long long)chunks);
      if (m + chunks > p.moves_cap) {
        atomicOr(reinterpret_cast<unsigned long long*>(p.full), 2ull);
      } else {
        if (p.moved_rows) atomicAdd(reinterpret_cast<unsigned long long*>(p.moved_rows), (unsigned long long)c_old[i]);
        for (u32 q = 0; q < chunks; ++q) {
          const u32 off = q * kMoveChunk;
          p.moves[m + q] = RunMove{from[i] + off, u32(start_new) + off, min_u32(kMoveChunk, c_old[i] - off)};
        }
      }
    }
    p.table[s[i]].start = u32(start_new);
    p.pcap[s[i]] = u32(newcap[i]);
  }
}

// The index statistics grow by the round's rows and new keys: one atomic per
// counter and block (every thread of the block must call this).
__device__ __forceinline__ void flush_update_stats(const IndexParams& p, u64 rows, u64 keys, u64 longest, u64* s_red) {
  const u64 br = block_sum<kBlock>(rows, s_red);
  const u64 bk = block_sum<kBlock>(keys, s_red);
  const u64 bl = block_max<kBlock>(longest, s_red);
  if (threadIdx.x == 0) {
    if (br) atomicAdd(reinterpret_cast<unsigned long long*>(p.rows), (unsigned long long)br);
    if (bk) atomicAdd(reinterpret_cast<unsigned long long*>(p.ndv), (unsigned long long)bk);
    if (bl) atomicMax(reinterpret_cast<unsigned long long*>(p.maxrun), (unsigned long long)bl);
  }
}

// Update, step 2: per touched slot (the work list), room for its appended
// rows (reserve_run); the slot's count becomes old + appended rows (dcnt
// keeps the appended count for the placement; k_upd_clear then clears it,
// also when the update fails, so that the rebuild finds it zero), and the
// index statistics grow by the round's rows and keys.
__global__ __launch_bounds__(kBlock) void k_upd_reserve(IndexParams p) {
  __shared__ u64 s_scan[kBlock / kWave + 1];
  __shared__ u64 s_base;
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  const u64 n = min_u64(*p.wl_n, p.cap);   // the work list holds at most one entry per slot
  const bool failed = (*p.full & 1) != 0;   // keys missing: the index is rebuilt (k_upd_clear clears dcnt)
  u64 st_rows = 0, st_keys = 0, st_long = 0;
  // every thread of a block runs the same number of steps (the block and
  // wave operations below need all of them)
  constexpr u64 kStep = u64(kBlock) * kResItems;
  for (u64 b0 = u64(blockIdx.x) * kStep; b0 < n; b0 += u64(gridDim.x) * kStep) {
    bool act[kResItems];
    u32 s[kResItems], d[kResItems], c_old[kResItems], from[kResItems];
    u64 need[kResItems];
#pragma unroll
    for (int i = 0; i < kResItems; ++i) {
      const u64 k = b0 + u64(i) * kBlock + threadIdx.x;
      act[i] = k < n && !failed;
      s[i] = act[i] ? p.wl[k] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kResItems; ++i) {
      d[i] = act[i] ? p.dcnt[s[i]] : 0u;
      const Slot sl = act[i] ? p.table[s[i]] : Slot{0, 0u, 0u};
      c_old[i] = sl.count;
      from[i] = sl.start;
      need[i] = u64(c_old[i]) + d[i];
    }
    reserve_runs(p, act, s, c_old, from, need, s_scan, &s_base);
#pragma unroll
    for (int i = 0; i < kResItems; ++i) {
      if (!act[i]) continue;
      p.table[s[i]].count = u32(need[i]);
      st_rows += d[i];
      st_keys += c_old[i] == 0 ? 1u : 0u;
      st_long = need[i] > st_long ? need[i] : st_long;
    }
  }
  flush_update_stats(p, st_rows, st_keys, st_long, s_scan);
  ktime_end(p.ts);
}

// Update, step 3: the listed old runs into their new regions, one chunk per
// block step.
__global__ __launch_bounds__(kBlock) void k_upd_move(IndexParams p) {
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  if (*p.full & 3) return;   // the index is rebuilt
  const u64 n = min_u64(*p.moves_n, p.moves_cap);
  for (u64 k = blockIdx.x; k < n; k += gridDim.x) {
    const RunMove mv = p.moves[k];
    for (u32 j = threadIdx.x; j < mv.count; j += kBlock) p.perm[u64(mv.to) + j] = p.perm[u64(mv.from) + j];
  }
  ktime_end(p.ts);
}

// Update, step 4: each appended row goes after its key's old rows, at the
// place k_upd_count gave it (count - dcnt is the old row count).
__global__ __launch_bounds__(kBlock) void k_upd_fill(IndexParams p) {
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  if (*p.full & 3) return;   // keys or positions missing: the index is rebuilt
  u64 begin, n;
  source_range(p.src, begin, n);
  for (u64 r = u64(blockIdx.x) * kBlock + threadIdx.x; r < n; r += u64(gridDim.x) * kBlock) {
    if (p.nfilt && !row_indexed(p, begin + r)) continue;
    const u64 w = p.rword[r];
    if (w == ~0ull) continue;
    const u32 s = u32(w >> 32);
    const Slot sl = p.table[s];
    p.perm[u64(sl.start) + (sl.count - p.dcnt[s]) + u32(w)] = u32(begin + r);
  }
  ktime_end(p.ts);
}

// Update, step 5: the appended counts of the touched slots cleared for the
// next update.
__global__ __launch_bounds__(kBlock) void k_upd_clear(IndexParams p) {
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  const u64 n = min_u64(*p.wl_n, p.cap);
  for (u64 i = u64(blockIdx.x) * kBlock + threadIdx.x; i < n; i += u64(gridDim.x) * kBlock) p.dcnt[p.wl[i]] = 0u;
}

// ------------------------------------------------------------------ sorted update
// An update over many appended rows whose keys are mostly distinct (where the
// per-tile grouping above saves nothing and every row would cost random
// accesses to the table and the counters) first sorts the appended rows'
// (row, slot) words by slot, as the sorted build does (k_idx_slotkeys over the
// appended range, then the radix sort).  Every per-slot access below then
// walks the table in slot order: the first word of each slot's run (its head)
// finds where the run ends, reserves room as k_upd_reserve does and notes in
// wl[s] the head's position minus the old row count, so that appended word j
// of slot s goes to start(s) + (j - wl[s]).  dcnt is not used.

__device__ __forceinline__ bool run_head(const u64* keys, u64 j, u64 smask) {
  return j == 0 || (keys[j - 1] & smask) != (keys[j] & smask);
}

// One past the last word of the run of slot s that holds word j (sorted
// words): a galloping search, so that the usual run of one or two words
// costs a read or two and a run of m words about 2 log2(m).
__device__ __forceinline__ u64 run_end(const u64* keys, u64 j, u64 n, u64 smask, u64 s) {
  u64 lo = j, step = 1;   // keys[lo] is in the run; so is every word before it from j on
  while (lo + step < n && (keys[lo + step] & smask) == s) {
    lo += step;
    step <<= 1;
  }
  u64 hi = min_u64(lo + step, n);   // not in the run (or n)
  while (hi - lo > 1) {
    const u64 mid = lo + ((hi - lo) >> 1);
    if ((keys[mid] & smask) == s) lo = mid;
    else hi = mid;
  }
  return hi;
}

// Sorted update, step 1: per run head, room for the appended rows and the
// slot's count set to old + appended rows.
__global__ __launch_bounds__(kBlock) void k_upds_reserve(IndexParams p, const u64* __restrict__ keys, u32 row_shift) {
  __shared__ u64 s_scan[kBlock / kWave + 1];
  __shared__ u64 s_base;
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 smask = (u64(1) << row_shift) - 1;
  const bool failed = (*p.full & 1) != 0;   // keys missing: the index is rebuilt
  u64 st_rows = 0, st_keys = 0, st_long = 0;
  constexpr u64 kStep = u64(kBlock) * kResItems;
  for (u64 b0 = u64(blockIdx.x) * kStep; b0 < n; b0 += u64(gridDim.x) * kStep) {
    bool act[kResItems];
    u32 s[kResItems], c_old[kResItems], from[kResItems];
    u64 j[kResItems], need[kResItems];
#pragma unroll
    for (int i = 0; i < kResItems; ++i) {
      j[i] = b0 + u64(i) * kBlock + threadIdx.x;
      act[i] = false;
      s[i] = 0;
      if (j[i] < n && !failed) {
        const u64 sl = keys[j[i]] & smask;
        act[i] = sl < p.cap && run_head(keys, j[i], smask);
        s[i] = act[i] ? u32(sl) : 0u;
      }
    }
#pragma unroll
    for (int i = 0; i < kResItems; ++i) {
      const u64 d = act[i] ? run_end(keys, j[i], n, smask, s[i]) - j[i] : 0;
      const Slot sl = act[i] ? p.table[s[i]] : Slot{0, 0u, 0u};
      c_old[i] = sl.count;
      from[i] = sl.start;
      need[i] = u64(c_old[i]) + d;
    }
    reserve_runs(p, act, s, c_old, from, need, s_scan, &s_base);
#pragma unroll
    for (int i = 0; i < kResItems; ++i) {
      if (!act[i]) continue;
      p.table[s[i]].count = u32(need[i]);
      p.wl[s[i]] = u32(j[i]) - c_old[i];
      st_rows += need[i] - c_old[i];
      st_keys += c_old[i] == 0 ? 1u : 0u;
      st_long = need[i] > st_long ? need[i] : st_long;
    }
  }
  flush_update_stats(p, st_rows, st_keys, st_long, s_scan);
  ktime_end(p.ts);
}

// Sorted update, step 3 (after k_upd_move): appended word j of slot s to
// its place after the key's old rows.
__global__ __launch_bounds__(kBlock) void k_upds_fill(IndexParams p, const u64* __restrict__ keys, u32 row_shift) {
  ktime_start(p.ts);
  if (p.abort && *p.abort) return;
  if (p.abort2 && *p.abort2) return;
  if (*p.full & 3) return;   // keys or positions missing: the index is rebuilt
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 smask = (u64(1) << row_shift) - 1;
  for (u64 j = u64(blockIdx.x) * kBlock + threadIdx.x; j < n; j += u64(gridDim.x) * kBlock) {
    const u64 k = keys[j];
    const u64 s = k & smask;
    if (s >= p.cap) continue;
    p.perm[u64(p.table[s].start) + u32(u32(j) - p.wl[s])] = u32(begin + (k >> row_shift));
  }
  ktime_end(p.ts);
}

// ------------------------------------------------------------------ sorted build
// The construction of Section 3 sorts the key column and run-length encodes
// it.  Here every indexed row finds (or inserts) its key's slot with a plain
// probe -- no per-row counter, so a hot key costs nothing extra -- and the
// word (row << row_shift | slot) goes through a stable LSD radix sort over
// the slot bits (launch_rs_hist / launch_rs_pass, run by the caller).  The
// sorted words list the rows grouped by slot, runs in slot order and row ids
// ascending inside a run: the layout the counting build produces, so the
// incremental update applies to either.  A run's count comes from its
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

// With hist, the words' 8-bit digits of the first `passes` passes are also
// counted (an LDS copy per block, lanes that share a digit adding once), so
// that their radix sort needs no histogram pass.
constexpr u32 kSlotHistPasses = 8;

__global__ __launch_bounds__(kBlock) void k_idx_slotkeys(IndexParams p, u64* keys, u32 row_shift, u32* hist,
                                                         u32 passes) {
  __shared__ u32 s_h[kSlotHistPasses * 256];
  if (p.abort && *p.abort) return;
  if (hist) {
    for (u32 i = threadIdx.x; i < passes * 256; i += kBlock) s_h[i] = 0;
    __syncthreads();
  }
  const u64 lt_mask = (1ull << lane_id()) - 1;
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
    u64 word[kS];
#pragma unroll
    for (int j = 0; j < kS; ++j) {
      const u64 r = r0 + j * stride;
      word[j] = 0;
      if (r < n) {
        u64 slot = p.cap;   // rows outside the filter sort after every slot
        if (in[j]) {
          slot = full ? kNoSlot
                      : home[j] == key[j] ? (mix64(key[j]) & mask) : index_insert_probe(p.table, mask, key[j]);
          if (slot == kNoSlot) {
            if (p.full && !full) atomicOr(reinterpret_cast<unsigned long long*>(p.full), 1ull);
            slot = 0;
          }
        }
        word[j] = (r << row_shift) | slot;
        keys[r] = word[j];
      }
    }
    if (hist) {
#pragma unroll
      for (int j = 0; j < kS; ++j) {
        const bool valid = r0 + j * stride < n;
        for (u32 q = 0; q < passes; ++q) {
          const u32 dg = u32(word[j] >> (8 * q)) & 255u;
          const u32 d0 = __builtin_amdgcn_readfirstlane(dg);
          const bool same = valid && dg == d0;
          const u64 m = __ballot(same);
          if (same) {
            if ((m & lt_mask) == 0) atomicAdd(&s_h[q * 256 + d0], u32(__popcll(m)));
          } else if (valid) {
            atomicAdd(&s_h[q * 256 + dg], 1u);
          }
        }
      }
    }
  }
  if (hist) {
    __syncthreads();
    for (u32 i = threadIdx.x; i < passes * 256; i += kBlock) {
      const u32 c = s_h[i];
      if (c) atomicAdd(&hist[i], c);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_idx_runs(IndexParams p, const u64* __restrict__ keys, u32 row_shift) {
  if (p.abort && *p.abort) return;
  if (p.full && (*p.full & 1)) return;   // keys are missing: the index is rebuilt larger
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 smask = (u64(1) << row_shift) - 1;
  // a loaded relation's index takes the packed layout (word i at position i);
  // a derived one's runs get regions with room to grow, placed after the
  // scan (k_idx_place), so here only each run's first word is noted
  const bool packed = p.pcap == nullptr;
  bool over = false;
  for (u64 i = u64(blockIdx.x) * kBlock + threadIdx.x; i < n; i += u64(gridDim.x) * kBlock) {
    const u64 k = keys[i];
    const u64 s = k & smask;
    if (s >= p.cap) continue;   // outside the filter (sorted last)
    if (packed) {
      if (i < p.perm_cap) p.perm[i] = u32(begin + (k >> row_shift));
      else over = true;
    }
    const bool head = i == 0 || (keys[i - 1] & smask) != s;
    const bool tail = i + 1 == n || (keys[i + 1] & smask) != s;
    if (head && !packed) p.wl[s] = u32(i);
    if (head || tail) atomicAdd(&p.table[s].count, (tail ? u32(i + 1) : 0u) - (head ? u32(i) : 0u));
  }
  // the runs would not fit: flag it (the host regrows the positions)
  if (over && p.full) atomicOr(reinterpret_cast<unsigned long long*>(p.full), 2ull);
}

// Sorted build of a derived relation's index, after the scan: word i of
// slot s goes to start(s) + (i - first word of s).
__global__ __launch_bounds__(kBlock) void k_idx_place(IndexParams p, const u64* __restrict__ keys, u32 row_shift) {
  if (p.abort && *p.abort) return;
  if (p.full && (*p.full & 3)) return;   // keys missing or regions past the positions: rebuilt
  u64 begin, n;
  source_range(p.src, begin, n);
  const u64 smask = (u64(1) << row_shift) - 1;
  for (u64 i = u64(blockIdx.x) * kBlock + threadIdx.x; i < n; i += u64(gridDim.x) * kBlock) {
    const u64 k = keys[i];
    const u64 s = k & smask;
    if (s >= p.cap) continue;
    p.perm[u64(p.table[s].start) + (i - p.wl[s])] = u32(begin + (k >> row_shift));
  }
}

static int grid_rows(u64 n, int cap) {
  const u64 b = (n + kBlock - 1) / kBlock;
  return int(b == 0 ? 1 : (b > u64(cap) ? u64(cap) : b));
}

static int grid_tiles(u64 rows) {
  const u64 t = (rows + kIdxTile - 1) / kIdxTile;
  return int(t == 0 ? 1 : (t > 4096 ? 4096 : t));
}

static int grid_scan(u64 cap) {
  const u64 t = (cap + kScanTile - 1) / kScanTile;
  return int(t == 0 ? 1 : (t > 2048 ? 2048 : t));
}

int launch_index_build(const IndexParams& p, u64 rows_cap, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_idx_clear, dim3(grid_rows(p.cap, 4096)), dim3(kBlock), 0, s, p.table, p.cap, p.abort, p.ndv,
                     p.maxrun, p.full, p.rows);
  hipLaunchKernelGGL(k_idx_count, dim3(grid_tiles(rows_cap)), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_idx_scan<false>, dim3(grid_scan(p.cap)), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_idx_fill, dim3(grid_tiles(rows_cap)), dim3(kBlock), 0, s, p);
  return int(hipGetLastError());
}

int launch_index_slotkeys(const IndexParams& p, u64 rows_cap, u64* keys, u32 row_shift, u32* hist, u32 passes,
                          void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (passes > kSlotHistPasses) hist = nullptr;
  if (hist) launch_fill_u32(hist, u64(passes) * 256, 0u, stream);
  hipLaunchKernelGGL(k_idx_clear, dim3(grid_rows(p.cap, 4096)), dim3(kBlock), 0, s, p.table, p.cap, p.abort, p.ndv,
                     p.maxrun, p.full, p.rows);
  hipLaunchKernelGGL(k_idx_slotkeys, dim3(grid_rows(rows_cap, 8192)), dim3(kBlock), 0, s, p, keys, row_shift, hist,
                     passes);
  return int(hipGetLastError());
}

int launch_index_rehash(const Slot* old_tab, const u32* old_pcap, u64 old_cap, Slot* tab, u32* pcap, u64 cap,
                        u64* full, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_idx_clear, dim3(grid_rows(cap, 4096)), dim3(kBlock), 0, s, tab, cap, nullptr, nullptr, nullptr,
                     full, nullptr);
  hipLaunchKernelGGL(k_fill_u32_idx, dim3(grid_rows(cap, 4096)), dim3(kBlock), 0, s, pcap, cap);
  hipLaunchKernelGGL(k_idx_rehash, dim3(grid_rows(old_cap, 8192)), dim3(kBlock), 0, s, old_tab, old_pcap, old_cap, tab,
                     pcap, cap, full);
  return int(hipGetLastError());
}

int launch_index_update_keys(const IndexParams& p, u64 delta_rows_cap, u64* keys, u32 row_shift, u32* hist,
                             u32 passes, void* stream) {
  if (passes > kSlotHistPasses) hist = nullptr;
  if (hist) launch_fill_u32(hist, u64(passes) * 256, 0u, stream);
  hipLaunchKernelGGL(k_idx_slotkeys, dim3(grid_rows(delta_rows_cap, 8192)), dim3(kBlock), 0, (hipStream_t)stream, p,
                     keys, row_shift, hist, passes);
  return int(hipGetLastError());
}

int launch_index_update_sorted(const IndexParams& p, u64 delta_rows_cap, const u64* sorted, u32 row_shift,
                               u64* const* ts, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  IndexParams q = p;
  q.ts = ts ? ts[0] : nullptr;
  hipLaunchKernelGGL(k_upds_reserve, dim3(grid_rows((delta_rows_cap + kResItems - 1) / kResItems, 4096)), dim3(kBlock), 0, s, q, sorted, row_shift);
  q.ts = ts ? ts[1] : nullptr;
  hipLaunchKernelGGL(k_upd_move, dim3(2048), dim3(kBlock), 0, s, q);
  q.ts = ts ? ts[2] : nullptr;
  hipLaunchKernelGGL(k_upds_fill, dim3(grid_rows(delta_rows_cap, 8192)), dim3(kBlock), 0, s, q, sorted, row_shift);
  return int(hipGetLastError());
}

int launch_index_runs(const IndexParams& p, u64 rows_cap, const u64* sorted, u32 row_shift, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_idx_runs, dim3(grid_rows(rows_cap, 8192)), dim3(kBlock), 0, s, p, sorted, row_shift);
  hipLaunchKernelGGL(k_idx_scan<true>, dim3(grid_scan(p.cap)), dim3(kBlock), 0, s, p);
  if (p.pcap)
    hipLaunchKernelGGL(k_idx_place, dim3(grid_rows(rows_cap, 8192)), dim3(kBlock), 0, s, p, sorted, row_shift);
  return int(hipGetLastError());
}

int launch_index_update(const IndexParams& p, u64 delta_rows_cap, u64 wl_cap, u64* const* ts, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  IndexParams q = p;
  q.ts = ts ? ts[0] : nullptr;
  hipLaunchKernelGGL(k_upd_count, dim3(grid_tiles(delta_rows_cap)), dim3(kBlock), 0, s, q);
  q.ts = ts ? ts[1] : nullptr;
  hipLaunchKernelGGL(k_upd_reserve, dim3(grid_rows((wl_cap + kResItems - 1) / kResItems, 4096)), dim3(kBlock), 0, s, q);
  q.ts = ts ? ts[2] : nullptr;
  hipLaunchKernelGGL(k_upd_move, dim3(2048), dim3(kBlock), 0, s, q);
  q.ts = ts ? ts[3] : nullptr;
  hipLaunchKernelGGL(k_upd_fill, dim3(grid_rows(delta_rows_cap, 8192)), dim3(kBlock), 0, s, q);
  q.ts = nullptr;
  hipLaunchKernelGGL(k_upd_clear, dim3(grid_rows(wl_cap, 4096)), dim3(kBlock), 0, s, q);
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

// Conditional column bounds (see launch_cond_bounds): every thread keeps
// the minimum, maximum and "any" of each condition set in registers over its
// rows, then waves and the block combine them and one atomic per value and
// block goes to out.
__global__ __launch_bounds__(kBlock) void k_cond_bounds(CondBoundsArgs a) {
  __shared__ u32 s_red[kCondSets * 8];
  u32 lo[kCondSets][3], hi[kCondSets][3], any[kCondSets];
#pragma unroll
  for (u32 q = 0; q < kCondSets; ++q) {
    any[q] = 0;
#pragma unroll
    for (u32 c = 0; c < 3; ++c) {
      lo[q][c] = 0xFFFFFFFFu;
      hi[q][c] = 0;
    }
  }
  for (u32 i = threadIdx.x; i < kCondSets * 8; i += kBlock) s_red[i] = (i % 8) < 3 ? 0xFFFFFFFFu : 0u;
  __syncthreads();
  for (u64 r = u64(blockIdx.x) * kBlock + threadIdx.x; r < a.n_rows; r += u64(gridDim.x) * kBlock) {
    u32 v[3];
#pragma unroll
    for (u32 c = 0; c < 3; ++c) v[c] = c < a.arity ? a.col[c][r] : 0u;
#pragma unroll
    for (u32 q = 0; q < kCondSets; ++q) {
      bool ok = q < a.nq;
#pragma unroll
      for (u32 i = 0; i < 3; ++i) {
        const u32 k = a.q[q].col[i];
        const u32 x = k == 0 ? v[0] : (k == 1 ? v[1] : v[2]);
        ok = ok && (i >= a.q[q].n || x == a.q[q].val[i]);
      }
      any[q] |= ok ? 1u : 0u;
#pragma unroll
      for (u32 c = 0; c < 3; ++c) {
        lo[q][c] = ok && v[c] < lo[q][c] ? v[c] : lo[q][c];
        hi[q][c] = ok && v[c] > hi[q][c] ? v[c] : hi[q][c];
      }
    }
  }
#pragma unroll
  for (u32 q = 0; q < kCondSets; ++q) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
      any[q] |= __shfl_xor(any[q], d, kWave);
#pragma unroll
      for (u32 c = 0; c < 3; ++c) {
        const u32 ol = __shfl_xor(lo[q][c], d, kWave), oh = __shfl_xor(hi[q][c], d, kWave);
        lo[q][c] = ol < lo[q][c] ? ol : lo[q][c];
        hi[q][c] = oh > hi[q][c] ? oh : hi[q][c];
      }
    }
    if (lane_id() == 0 && any[q] && q < a.nq) {
      atomicOr(&s_red[q * 8 + 6], 1u);
#pragma unroll
      for (u32 c = 0; c < 3; ++c) {
        atomicMin(&s_red[q * 8 + c], lo[q][c]);
        atomicMax(&s_red[q * 8 + 3 + c], hi[q][c]);
      }
    }
  }
  __syncthreads();
  for (u32 q = 0; q < a.nq; ++q) {
    if (!s_red[q * 8 + 6]) continue;   // block-uniform
    if (threadIdx.x == 0) atomicOr(&a.out[q * 8 + 6], 1u);
    if (threadIdx.x < 3) atomicMin(&a.out[q * 8 + threadIdx.x], s_red[q * 8 + threadIdx.x]);
    else if (threadIdx.x < 6) atomicMax(&a.out[q * 8 + threadIdx.x], s_red[q * 8 + threadIdx.x]);
  }
}

__global__ void k_cond_bounds_init(u32* out, u32 nq) {
  for (u32 i = threadIdx.x; i < nq * 8; i += blockDim.x) out[i] = (i % 8) < 3 ? 0xFFFFFFFFu : 0u;
}

int launch_cond_bounds(const CondBoundsArgs& a, void* stream) {
  if (a.nq == 0 || a.nq > kCondSets) return int(hipErrorInvalidValue);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_cond_bounds_init, dim3(1), dim3(64), 0, s, a.out, a.nq);
  if (a.n_rows) hipLaunchKernelGGL(k_cond_bounds, dim3(grid_rows(a.n_rows, 1024)), dim3(kBlock), 0, s, a);
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
