// Device-side building blocks shared by the engine's HIP kernels (gfx950,
// wave64): hashing, open-addressing probes, wave/block scans and the
// decoupled look-back used for order-preserving stream compaction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_types.h"

namespace fv {

// Kernel timing for traces: with ts set, block 0 stamps the start (ts[0])
// and every block raises one of kStampEnds end words (ts[1 + block % 64]) to
// its end, read from the constant-rate wall clock; the host takes the latest
// end minus the start as the kernel's own duration, with no inter-kernel
// dispatch gap in it.  Spreading the ends keeps thousands of exiting blocks
// off a single word.  ktime_end is reached by all threads of a block.
constexpr u32 kStampEnds = 64;
static_assert(kStampEnds + 1 == kStampWords, "stamp slot layout");
__device__ __forceinline__ void ktime_start(u64* ts) {
  if (ts && blockIdx.x == 0 && threadIdx.x == 0) ts[0] = u64(wall_clock64());
}
__device__ __forceinline__ void ktime_end(u64* ts) {
  if (!ts) return;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(ts + 1 + (blockIdx.x % kStampEnds)),
              (unsigned long long)wall_clock64());
}

constexpr int kWave = 64;

// --------------------------------------------------------------- hashing
// 64-bit finalizer of MurmurHash3 (Austin Appleby, public domain): a bijective
// avalanche mix, so distinct keys never collide before the table mask.
__device__ __forceinline__ u64 mix64(u64 k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ u64 atomic_load_u64(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_u64(u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 atomic_cas_u64(u64* p, u64 expect, u64 desired) {
  return atomicCAS(reinterpret_cast<unsigned long long*>(p), expect, desired);
}

// Hash tables probe linearly and give up after kMaxProbe slots: an insert
// that finds no free slot in that window reports failure (the host grows the
// table), so a key that is present always lies within kMaxProbe slots of its
// home and a lookup can stop there too.  Every probe loop is thus bounded,
// whatever state a table is in.
constexpr u32 kMaxProbe = 1u << 12;

// Index lookup over {key, start, count} slots (Section 3, "unique hashmap":
// one slot per distinct key, value = its run in the grouped row ids).
__device__ __forceinline__ bool index_find(const Slot* __restrict__ tab, u64 mask, u64 key,
                                           u32& start, u32& count) {
  u64 h = mix64(key) & mask;
  for (u32 i = 0; i < kMaxProbe && i <= mask; ++i) {
    const Slot s = tab[h];
    if (s.key == key) { start = s.start; count = s.count; return true; }
    if (s.key == kEmptyKey) return false;
    h = (h + 1) & mask;
  }
  return false;
}

// Find-or-insert a key into an index table; returns its slot, or kNoSlot if
// the kMaxProbe slots from its home all hold other keys.
constexpr u64 kNoSlot = ~0ull;
__device__ __forceinline__ u64 index_insert(Slot* tab, u64 mask, u64 key) {
  u64 h = mix64(key) & mask;
  for (u32 i = 0; i < kMaxProbe && i <= mask; ++i) {
    u64 cur = atomic_load_u64(&tab[h].key);
    if (cur == key) return h;
    if (cur == kEmptyKey) {
      u64 prev = atomic_cas_u64(&tab[h].key, kEmptyKey, key);
      if (prev == kEmptyKey || prev == key) return h;
    }
    h = (h + 1) & mask;
  }
  return kNoSlot;
}

// Slot of a key already inserted (kNoSlot if its insert failed).
__device__ __forceinline__ u64 index_slot_of(const Slot* tab, u64 mask, u64 key) {
  u64 h = mix64(key) & mask;
  for (u32 i = 0; i < kMaxProbe && i <= mask; ++i) {
    const u64 cur = tab[h].key;
    if (cur == key) return h;
    if (cur == kEmptyKey) return kNoSlot;
    h = (h + 1) & mask;
  }
  return kNoSlot;
}

// Continuations for callers that read the home slots of several keys at once
// (independent loads in flight, then one resolution per key): probing goes on
// after home slot h, which the caller found holding another key, within the
// same kMaxProbe window.
__device__ __forceinline__ bool index_find_after(const Slot* __restrict__ tab, u64 mask, u64 key, u64 h,
                                                 u32& start, u32& count) {
  for (u32 i = 1; i < kMaxProbe && i <= mask; ++i) {
    h = (h + 1) & mask;
    const Slot s = tab[h];
    if (s.key == key) { start = s.start; count = s.count; return true; }
    if (s.key == kEmptyKey) return false;
  }
  return false;
}

// Tuple set insert-if-absent over 8-byte slots.  Returns 1 if the key was
// new, 0 if present, -1 if kMaxProbe slots were all taken (the table is too
// full; the caller flags it and the host grows the set).  Slots only ever go
// from empty to a key, so a plain (possibly stale) load can only mislead
// towards "empty", which the CAS then corrects.
__device__ __forceinline__ int set_insert(u64* tab, u64 mask, u64 key) {
  u64 h = mix64(key) & mask;
  for (u32 i = 0; i < kMaxProbe; ++i) {
    const u64 cur = tab[h];
    if (cur == key) return 0;
    if (cur == kEmptyKey) {
      const u64 prev = atomic_cas_u64(&tab[h], kEmptyKey, key);
      if (prev == kEmptyKey) return 1;
      if (prev == key) return 0;
    }
    h = (h + 1) & mask;
  }
  return -1;
}

// set_insert after home slot h, which the caller found (or made, by a failed
// CAS) holding another key.
__device__ __forceinline__ int set_insert_after(u64* tab, u64 mask, u64 key, u64 h) {
  for (u32 i = 1; i < kMaxProbe; ++i) {
    h = (h + 1) & mask;
    const u64 cur = tab[h];
    if (cur == key) return 0;
    if (cur == kEmptyKey) {
      const u64 prev = atomic_cas_u64(&tab[h], kEmptyKey, key);
      if (prev == kEmptyKey) return 1;
      if (prev == key) return 0;
    }
  }
  return -1;
}

// Insert-if-absent of up to kN keys per thread with their home-slot reads and
// CASes issued together: res[i] receives set_insert's result for the keys
// with act[i] set.
template <int kN>
__device__ __forceinline__ void set_insert_many(u64* tab, u64 mask, const u64* key, const bool* act, int* res) {
  u64 h[kN], cur[kN], prev[kN];
  bool cas[kN];
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    h[i] = mix64(key[i]) & mask;
    cur[i] = act[i] ? tab[h[i]] : key[i];
  }
  // every test reads the loads first, then the CASes are issued back to
  // back (their results are read only below)
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    cas[i] = act[i] && cur[i] == kEmptyKey;
    prev[i] = cur[i];
  }
#pragma unroll
  for (int i = 0; i < kN; ++i)
    if (cas[i]) prev[i] = atomic_cas_u64(&tab[h[i]], kEmptyKey, key[i]);
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    res[i] = 0;
    if (!act[i]) continue;
    if (cas[i] && prev[i] == kEmptyKey) res[i] = 1;   // inserted it
    else if (prev[i] != key[i]) res[i] = set_insert_after(tab, mask, key[i], h[i]);
  }
}

// Tuple sets of relations whose packed tuples fit in 32 bits use 4-byte slots
// (half the footprint, so more of the set stays in cache), empty = all ones.
// The one key equal to that marker (kEmptyKey32) is kept out of the table: a
// flag word records whether it is in the set.

__device__ __forceinline__ int set32_insert_after(u32* tab, u64 mask, u32 key, u64 h) {
  for (u32 i = 1; i < kMaxProbe; ++i) {
    h = (h + 1) & mask;
    const u32 cur = tab[h];
    if (cur == key) return 0;
    if (cur == kEmptyKey32) {
      const u32 prev = atomicCAS(&tab[h], kEmptyKey32, key);
      if (prev == kEmptyKey32) return 1;
      if (prev == key) return 0;
    }
  }
  return -1;
}

__device__ __forceinline__ int set32_insert(u32* tab, u64 mask, u32 key, u64* ones) {
  if (key == kEmptyKey32) return atomicExch(reinterpret_cast<unsigned long long*>(ones), 1ull) == 0 ? 1 : 0;
  const u64 h = mix64(key) & mask;
  const u32 cur = tab[h];
  if (cur == key) return 0;
  if (cur == kEmptyKey32) {
    const u32 prev = atomicCAS(&tab[h], kEmptyKey32, key);
    if (prev == kEmptyKey32) return 1;
    if (prev == key) return 0;
  }
  return set32_insert_after(tab, mask, key, h);
}

// set_insert_many over a 32-bit set (keys given as u64, all below 2^32).
template <int kN>
__device__ __forceinline__ void set32_insert_many(u32* tab, u64 mask, const u64* key64, const bool* act, int* res,
                                                  u64* ones) {
  u64 h[kN];
  u32 key[kN], cur[kN], prev[kN];
  bool tabled[kN], cas[kN];
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    key[i] = u32(key64[i]);
    tabled[i] = act[i] && key[i] != kEmptyKey32;
    h[i] = mix64(key[i]) & mask;
    cur[i] = tabled[i] ? tab[h[i]] : key[i];
  }
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    cas[i] = tabled[i] && cur[i] == kEmptyKey32;
    prev[i] = cur[i];
  }
#pragma unroll
  for (int i = 0; i < kN; ++i)
    if (cas[i]) prev[i] = atomicCAS(&tab[h[i]], kEmptyKey32, key[i]);
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    res[i] = 0;
    if (!act[i]) continue;
    if (!tabled[i]) res[i] = atomicExch(reinterpret_cast<unsigned long long*>(ones), 1ull) == 0 ? 1 : 0;
    else if (cas[i] && prev[i] == kEmptyKey32) res[i] = 1;
    else if (prev[i] != key[i]) res[i] = set32_insert_after(tab, mask, key[i], h[i]);
  }
}

// --------------------------------------------------------------- wave / block scans
__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Block-wide sum and maximum (every thread gets the result); `lds` must hold
// kBlock / kWave entries.  Used to give a whole block one atomic on a shared
// counter instead of one per wave: counters that every wave of a large launch
// adds to serialise on their address otherwise.
template <int kBlock, typename T>
__device__ __forceinline__ T block_sum(T v, T* lds) {
  constexpr int kWaves = kBlock / kWave;
  T w = wave_sum(v);
  if (lane_id() == 0) lds[threadIdx.x / kWave] = w;
  __syncthreads();
  T t = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) t += lds[i];
  __syncthreads();
  return t;
}

template <int kBlock, typename T>
__device__ __forceinline__ T block_max(T v, T* lds) {
  constexpr int kWaves = kBlock / kWave;
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const T o = __shfl_xor(v, d, kWave);
    v = o > v ? o : v;
  }
  if (lane_id() == 0) lds[threadIdx.x / kWave] = v;
  __syncthreads();
  T t = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) t = lds[i] > t ? lds[i] : t;
  __syncthreads();
  return t;
}

// Block-wide exclusive scan; `lds` must hold kBlock / kWave + 1 entries.
// Returns the exclusive prefix of v; *total receives the block sum.
template <int kBlock, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* lds, T* total) {
  constexpr int kWaves = kBlock / kWave;
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  T inc = wave_inclusive_sum(v);
  if (lane == kWave - 1) lds[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int i = 0; i < kWaves; ++i) { T c = lds[i]; lds[i] = run; run += c; }
    lds[kWaves] = run;
  }
  __syncthreads();
  T r = lds[w] + inc - v;
  *total = lds[kWaves];
  __syncthreads();
  return r;
}

// --------------------------------------------------------------- decoupled look-back
// A status word per tile: [63:42] launch epoch (22 bits) | [41:40] flag |
// [39:0] value.  Words from another launch (different epoch) read as "not
// ready", so status arrays never need clearing between launches.
constexpr u64 kFlagAgg = 1, kFlagPrefix = 2;
constexpr u64 kValueMask = (1ull << 40) - 1;

__device__ __forceinline__ u64 lb_word(u32 epoch, u64 flag, u64 value) {
  return (u64(epoch & kEpochMask) << 42) | (flag << 40) | (value & kValueMask);
}
__device__ __forceinline__ u64 lb_flag(u64 w, u32 epoch) {
  return (u32(w >> 42) == (epoch & kEpochMask)) ? ((w >> 40) & 3) : 0;
}

// Wave-cooperative look-back over status[0 .. tile-1]: each lane inspects one
// predecessor, the nearest inclusive prefix stops the walk.  All 64 lanes of
// the calling wave must participate.  Predecessor tiles were handed out
// earlier by the ticket counter, so their blocks are resident and publish an
// aggregate without waiting on anyone: the spin always ends.
__device__ __forceinline__ u64 lookback_exclusive(const u64* status, u32 tile, u32 epoch) {
  u64 excl = 0;
  long long base = (long long)tile - 1;
  const int lane = lane_id();
  while (base >= 0) {
    long long idx = base - lane;
    u64 w = 0, f = kFlagPrefix;
    if (idx >= 0) {
      for (;;) {
        w = atomic_load_u64(status + idx);
        f = lb_flag(w, epoch);
        if (f != 0) break;
        __builtin_amdgcn_s_sleep(1);
      }
    }
    const u64 pm = __ballot(f == kFlagPrefix);
    const int stop = pm ? __ffsll((long long)pm) - 1 : kWave;   // nearest prefix lane
    u64 v = (lane <= stop && idx >= 0) ? (w & kValueMask) : 0;
    excl += wave_sum(v);
    if (pm) break;
    base -= kWave;
  }
  return excl;
}

// Ticket-ordered tile loop: blocks take tiles in increasing order so that a
// tile's predecessors are always owned by running blocks.  Only the first
// min(gridDim.x, ntiles) blocks participate (the others leave at once, so a
// grid sized for the buffer capacity costs nothing when the input is small);
// each participant makes exactly one failing increment, and the last of those
// resets the counter for the next launch.
__device__ __forceinline__ u32 participants(u32 ntiles) {
  const u32 p = ntiles < gridDim.x ? ntiles : gridDim.x;
  return p ? p : 1u;
}

__device__ __forceinline__ u32 take_ticket(u32* ticket, u32 ntiles, u32* lds_slot) {
  if (threadIdx.x == 0) {
    u32 t = atomicAdd(ticket, 1u);
    if (t >= ntiles && t == ntiles + participants(ntiles) - 1) atomicExch(ticket, 0u);
    *lds_slot = t;
  }
  __syncthreads();
  u32 t = *lds_slot;
  __syncthreads();
  return t;
}

__device__ __forceinline__ u64 min_u64(u64 a, u64 b) { return a < b ? a : b; }

// lower_bound_u64 by a whole wave (every lane calls it with the same
// arguments and gets the same result): each round probes 64 evenly spaced
// keys at once and keeps the gap between the last one below k and the next,
// so a search over n keys takes about log64(n) round trips instead of log2(n).
__device__ __forceinline__ u64 wave_lower_bound_u64(const u64* v, u64 lo, u64 hi, u64 k) {
  const u32 lane = u32(__lane_id());
  while (hi - lo > u64(kWave)) {
    const u64 step = (hi - lo + kWave - 1) / kWave;
    const u64 pos = lo + u64(lane) * step;
    const bool below = pos < hi && v[pos] < k;
    const u32 c = u32(__popcll(__ballot(below)));   // the lanes below k are a prefix
    if (c == 0) return lo;
    const u64 nlo = lo + u64(c - 1) * step + 1;
    const u64 nxt = lo + u64(c) * step;
    if (c < u32(kWave) && nxt < hi) hi = nxt;
    lo = nlo;
  }
  const bool below = lo + lane < hi && v[lo + lane] < k;
  return lo + u64(__popcll(__ballot(below)));
}

// First index in [lo, hi) of ascending v whose key is >= k (hi if none).
__device__ __forceinline__ u64 lower_bound_u64(const u64* v, u64 lo, u64 hi, u64 k) {
  while (lo < hi) {
    const u64 mid = (lo + hi) >> 1;
    if (v[mid] < k) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ u32 min_u32(u32 a, u32 b) { return a < b ? a : b; }

__device__ __forceinline__ u32 launch_epoch(const u32* base, u32 off) { return (*base + off) & kEpochMask; }

// Number of rows of a source: min(counter, capacity) minus its begin offset.
__device__ __forceinline__ void source_range(const RowRange& r, u64& begin, u64& n) {
  u64 b = r.begin_ctr ? *r.begin_ctr : r.begin;
  u64 e = r.end_ctr ? min_u64(*r.end_ctr, r.cap) : r.end;
  begin = b;
  n = e > b ? e - b : 0;
}

}  // namespace fv
