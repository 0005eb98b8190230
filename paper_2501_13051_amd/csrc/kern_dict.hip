// Value compaction for relations whose packed tuples would need more than
// 64 bits.  Datalog without function symbols only compares values for
// equality and never creates new ones, so every value of the loaded facts
// and of the rules' constants can be replaced by its rank among the distinct
// values: the fixpoint is the same up to that renaming, and ranks are dense,
// so each column needs only ceil(log2(distinct values)) bits.  Ranks keep the
// order of the values, so exported rows sorted by rank are sorted by value
// once mapped back.
//
//   k_dict_count / k_dict_scan / k_dict_write: the distinct values of a
//     sorted key array, in order (heads of runs, counted per tile, scanned,
//     then written at their ranks)
//   k_dict_remap: value -> rank (binary search in the sorted distinct values)
//   k_dict_gather: rank -> value
#include "fv_device.h"

namespace fv {

namespace {

// keys per thread and per tile of the ordered compaction: each thread owns
// kDictItems consecutive keys, so the heads it finds are written in order
constexpr u32 kDictItems = 16;
constexpr u32 kDictTile = kBlock * kDictItems;

__device__ __forceinline__ u32 count_heads(const u64* keys, u64 n, u64 i0) {
  u32 c = 0;
  for (u32 j = 0; j < kDictItems; ++j) {
    const u64 i = i0 + j;
    if (i < n && (i == 0 || keys[i] != keys[i - 1])) ++c;
  }
  return c;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_dict_count(const u64* keys, u64 n, u64* tile_cnt) {
  __shared__ u32 s_scan[kBlock / kWave + 1];
  const u64 i0 = u64(blockIdx.x) * kDictTile + u64(threadIdx.x) * kDictItems;
  u32 tot;
  block_exclusive_sum<kBlock>(count_heads(keys, n, i0), s_scan, &tot);
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = tot;
}

// One block: exclusive scan of the tile counts in place; the total goes to *count.
__global__ __launch_bounds__(kBlock) void k_dict_scan(u64* tile_cnt, u64 ntiles, u64* count) {
  __shared__ u64 s_scan[kBlock / kWave + 1];
  u64 run = 0;
  for (u64 b0 = 0; b0 < ntiles; b0 += kBlock) {
    const u64 b = b0 + threadIdx.x;
    const u64 v = b < ntiles ? tile_cnt[b] : 0;
    u64 tot;
    const u64 ex = block_exclusive_sum<kBlock>(v, s_scan, &tot);
    if (b < ntiles) tile_cnt[b] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) *count = run;
}

__global__ __launch_bounds__(kBlock) void k_dict_write(const u64* keys, u64 n, const u64* tile_base, u32* dict) {
  __shared__ u32 s_scan[kBlock / kWave + 1];
  const u64 i0 = u64(blockIdx.x) * kDictTile + u64(threadIdx.x) * kDictItems;
  u32 tot;
  u64 pos = tile_base[blockIdx.x] + block_exclusive_sum<kBlock>(count_heads(keys, n, i0), s_scan, &tot);
  for (u32 j = 0; j < kDictItems; ++j) {
    const u64 i = i0 + j;
    if (i < n && (i == 0 || keys[i] != keys[i - 1])) dict[pos++] = u32(keys[i]);
  }
}

// col[i] := the index of col[i] in dict (sorted, distinct, holding every value)
__global__ __launch_bounds__(kBlock) void k_dict_remap(u32* col, u64 n, const u32* dict, u64 nd) {
  for (u64 i = u64(blockIdx.x) * kBlock + threadIdx.x; i < n; i += u64(gridDim.x) * kBlock) {
    const u32 v = col[i];
    u64 lo = 0, hi = nd;
    while (lo < hi) {
      const u64 mid = (lo + hi) >> 1;
      if (dict[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    col[i] = u32(lo);
  }
}

__global__ __launch_bounds__(kBlock) void k_dict_gather(u32* col, u64 n, const u32* dict) {
  for (u64 i = u64(blockIdx.x) * kBlock + threadIdx.x; i < n; i += u64(gridDim.x) * kBlock) col[i] = dict[col[i]];
}

u64 dict_tiles(u64 n) { return (n + kDictTile - 1) / kDictTile; }

int launch_dict_unique(const u64* sorted, u64 n, u64* tile_cnt, u32* dict, u64* count, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const u64 tiles = dict_tiles(n);
  if (tiles == 0) return launch_fill_u64(count, 1, 0, stream);
  hipLaunchKernelGGL(k_dict_count, dim3(u32(tiles)), dim3(kBlock), 0, s, sorted, n, tile_cnt);
  hipLaunchKernelGGL(k_dict_scan, dim3(1), dim3(kBlock), 0, s, tile_cnt, tiles, count);
  hipLaunchKernelGGL(k_dict_write, dim3(u32(tiles)), dim3(kBlock), 0, s, sorted, n, tile_cnt, dict);
  return int(hipGetLastError());
}

static u32 dict_grid(u64 n) {
  const u64 b = (n + kBlock - 1) / kBlock;
  return u32(b == 0 ? 1 : (b > 8192 ? 8192 : b));
}

int launch_dict_remap(u32* col, u64 n, const u32* dict, u64 nd, void* stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_dict_remap, dim3(dict_grid(n)), dim3(kBlock), 0, (hipStream_t)stream, col, n, dict, nd);
  return int(hipGetLastError());
}

int launch_dict_gather(u32* col, u64 n, const u32* dict, void* stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_dict_gather, dim3(dict_grid(n)), dim3(kBlock), 0, (hipStream_t)stream, col, n, dict);
  return int(hipGetLastError());
}

}  // namespace fv
