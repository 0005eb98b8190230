// Plain types shared by the host runtime and the HIP kernels: kernel
// parameter blocks, hash slots and launch-wrapper declarations.  No HIP
// device code here, so host-only translation units can include it.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace fv {

using u32 = uint32_t;
using u64 = uint64_t;

constexpr u64 kEmptyKey = ~0ull;         // empty hash slot (0xFFFFFFFF is a reserved value)
constexpr u32 kEmptyKey32 = 0xFFFFFFFFu; // empty slot of a 32-bit tuple set
constexpr u32 kEpochMask = (1u << 22) - 1;
// Each phase of work (a round, an ingest, an index build) first advances a
// device-resident epoch base by kEpochStride; a look-back launch inside the
// phase uses base + its own offset (1 .. kEpochStride-1), so replaying a
// captured graph never meets status words of an earlier replay.
constexpr u32 kEpochStride = 1024;
// Flag words after the counter block: [0] overflow (a round must run again),
// [1] fatal (join scratch too small), [2] a tuple set ran out of slots,
// [3] the epoch base, [4] void (a look-ahead round queued behind a failed
// one: every kernel of that round returns at entry).  Words 5..7 are spare.
constexpr u32 kFlagOverflow = 0, kFlagFatal = 1, kFlagSetFull = 2, kFlagEpoch = 3, kFlagVoid = 4;
constexpr size_t kFlagBytes = 32;
constexpr u32 kStampWords = 65;   // per timed launch (traces): start, then 64 end words
constexpr int kMaxCols = 6;              // columns of an intermediate result
constexpr int kMaxFilters = 8;

// One slot of a join index: a distinct key and its run [start, start+count)
// in the index's row permutation (the RLE "unique hashmap" of Section 3).
struct alignas(16) Slot {
  u64 key;
  u32 start;
  u32 count;
};

// Rows [begin, end) of a set of columns.  begin/end come from device
// counters when the pointers are set (sizes only known on the device), and
// end is clamped to cap so an overflowed producer is never over-read.
struct RowRange {
  const u64* begin_ctr;
  const u64* end_ctr;
  u64 begin;
  u64 end;
  u64 cap;
};

enum SrcKind : u32 { kSrcProbe = 0, kSrcBuild = 1, kSrcConst = 2 };
struct Src {
  u32 kind;
  u32 v;   // column index, or the constant
};

enum FilterOp : u32 { kEq = 0, kNe = 1 };
struct Filter {
  Src a, b;
  u32 op;
};

// Output of a join/select: either intermediate columns or packed tuple keys
// appended to a relation's "new" buffer.
struct OutSpec {
  u32 ncols;
  Src src[kMaxCols];
  u32 packed;            // 1: write key = sum(v_c << shift[c]) into keys
  u32 shift[kMaxCols];
  u32* cols[kMaxCols];
  u64* keys;
  u64* count;            // device counter: tuples written (may exceed cap)
  u64 cap;
  // packed outputs into a relation's new keys may also count the 8-bit
  // digits of every radix pass of those keys ([pass][256] words, added to),
  // so that the sort needs no histogram pass of its own
  u32* hist;
  u32 hist_passes;
};

struct ProbeParams {
  const u32* pcol[kMaxCols];
  RowRange src;
  u32 n_pf;              // filters on the probe row (constants, repeated variables)
  Filter pf[kMaxFilters];
  u32 nkey;              // 0, 1 or 2 key terms
  Src key[2];
  const Slot* table;
  u64 mask;
  const u64* build_rows_ctr;   // nkey == 0: every probe row matches all build rows
  u64 build_rows;
  u64 build_cap;
  u32* m_row;
  u32* m_start;
  u64* m_off;
  u64 m_cap;
  u64* out_m;            // matched probe rows
  u64* out_t;            // join output size before filters
  u64* out_n;            // probe rows in the source range (nullable; traces)
  u64* st_m;             // look-back status arrays
  u64* st_t;
  u32* ticket;
  const u32* epoch_base;
  u32 epoch_off;
  const u32* abort;
  u32* fatal;
  u64* ts;               // trace timing slot (see ktime_start), nullable
};

struct WriteParams {
  const u32* pcol[kMaxCols];
  const u32* bcol[3];
  const u32* perm;       // null: identity (cross product)
  const u32* m_row;
  const u32* m_start;
  const u64* m_off;
  u64 m_cap;
  const u64* in_m;
  const u64* in_t;
  u32 n_filter;
  Filter filt[kMaxFilters];
  OutSpec out;
  u64* join_out_stat;    // running total of tuples written by joins
  const u32* abort;
  const u32* abort2;     // second cancel word (a voided round), nullable
  u32* overflow;
  u64* ts;               // trace timing slot (see ktime_start), nullable
};

// Probe + write in one pass into a presized output (see k_join_fused).
struct FusedJoinParams {
  const u32* pcol[kMaxCols];
  RowRange src;
  u32 n_pf;
  Filter pf[kMaxFilters];
  u32 nkey;
  Src key[2];
  const Slot* table;
  u64 mask;
  const u64* build_rows_ctr;
  u64 build_rows;
  u64 build_cap;
  const u32* bcol[3];
  const u32* perm;
  u32 n_filter;
  Filter filt[kMaxFilters];
  OutSpec out;
  u64* out_t;            // join output size before filters (added per wave)
  u64* out_n;            // probe rows in the source range (nullable; traces)
  u64* join_out_stat;
  const u32* abort;      // nonzero: return at entry (a voided round), nullable
  u32* overflow;
  u64* ts;               // trace timing slot (see ktime_start), nullable
};

struct SelectParams {
  const u32* pcol[kMaxCols];
  RowRange src;
  u32 n_filter;
  Filter filt[kMaxFilters];
  OutSpec out;
  u64* join_out_stat;
  const u32* abort;
  u32* overflow;
  u64* ts;               // trace timing slot (see ktime_start), nullable
};

// The difference by Algorithm 2 (Section 4, "Union and Deduplication"): a new
// tuple is already in full iff the ranges of its values in the per-column
// indices of full (Section 3's hybrid index: one slot per distinct value, its
// run of row ids) share a row id.  An empty range proves the tuple new; else
// the row ids of the shortest range are checked against the other columns'
// values (an id lies in the range of value v in column c iff full's column c
// holds v at that row), which is the intersection of the ranges.
struct RangeDedup {
  u32 ncol;              // 0: off
  const Slot* table[3];  // per column of full: the index table, its mask, its row ids
  u64 mask[3];
  const u32* perm[3];
  const u32* fcol[3];    // full's columns
};

struct DedupParams {
  const u64* keys;       // sorted packed tuples
  RowRange src;          // [0, n)
  u64* set;              // tuple set of full (null with set32 null: only drop adjacent repeats)
  u32* set32;            // 32-bit tuple set instead of set (keys below 2^32), and its all-ones flag
  u64* ones;
  u64 set_mask;
  u32* set_full;         // raised (with the overflow flag) when an insert finds no slot
  u32* cols[3];          // full columns to append to
  const u64* full_n;     // append position
  u32 arity;
  u32 shift[3];
  u32 width[3];
  u64* out_delta;        // survivors
  u64* status;
  u32* ticket;
  const u32* epoch_base;
  u32 epoch_off;
  const u32* abort;
  u64* ts;               // trace timing slot (see ktime_start), nullable
  RangeDedup rd;         // with rd.ncol > 0 (and no set): the difference by per-column ranges
  // with sorted_full (launch_diff_sorted): the difference against full's
  // packed tuples in ascending order, *full_n of them, merged with the new
  // ones into `merged`; mtile is the launches' per-tile scratch
  const u64* sorted_full;
  u64* merged;
  u64* mtile;
};

struct CommitParams {
  u64* full_n;
  u64* d_begin;
  const u64* delta;
  u64* new_count;
  u64* derived;          // running total of appended tuples
  const u32* abort;
  const u32* abort2;
};

// ------------------------------------------------------------------ launchers
// Each wrapper enqueues kernels on `stream` (a hipStream_t) and returns the
// hipError_t of the launch as int.
// `block`: threads per block of the launch, 128, 256 or 512 (others: 256).
// A look-back launch of n rows uses ceil(n / (block x 4)) status words.
int launch_probe(const ProbeParams& p, u64 probe_cap, int grid, void* stream, u32 block = 256);
int launch_write(const WriteParams& p, u64 out_tiles_hint, void* stream, u32 block = 256);
int launch_select(const SelectParams& p, u64 rows_hint, void* stream, u32 block = 256);
int launch_join_fused(const FusedJoinParams& p, u64 rows_hint, void* stream, u32 block = 256);
int launch_dedup(const DedupParams& p, u64 rows_cap, void* stream, u32 block = 256);
// The difference against full's sorted keys fused with their merge
// (p.sorted_full, p.merged and p.mtile set; set, set32 and ranges unused):
// three launches (count, scan, write) over the merge of full's keys and the
// new keys; the new keys are appended to full's columns, *out_delta receives
// their number and merged[0, *full_n + *out_delta) full's keys after the
// round, in order.  total_cap bounds full's keys plus the new keys;
// p.mtile holds diff_sorted_scratch_words(total_cap) words.
int launch_diff_sorted(const DedupParams& p, u64 total_cap, void* stream, u32 block = 256);
u64 diff_sorted_scratch_words(u64 total_cap);
int launch_commit(const CommitParams& p, void* stream);
// Zero n_ctr counters, n_hist histogram words and (if flag) the overflow and
// set-full flags (flag[0], flag[2]), and advance the epoch base by kEpochStride.
// sticky: a look-ahead round, which does nothing if a flag is already raised
int launch_round_prologue(u64* ctr, u64 n_ctr, u32* flag, u32* hist, u64 n_hist, u32* epoch_base, void* stream,
                          bool sticky = false);

// LSD radix sort of n packed u64 keys (n from *n_ctr clamped to cap, or
// n_const) on the low `bits` bits, digit_bits (8 or 11) per pass:
// launch_rs_hist counts the digits of all passes, then one launch_rs_pass per
// pass moves keys src->dst.  With `fuse`, the last pass instead takes the
// difference against a tuple set and appends the survivors to full.
struct SortParams {
  u64* a;
  u64* b;
  const u64* n_ctr;
  u64 n_const;
  u64 cap;
  u64 n_hint;            // expected keys (0: cap), for the choice of tile size
  u32 bits;
  u32 digit_bits;        // 8 or 11
  u32 max_blocks;        // grid cap of a pass (0: 2048)
  u32* hist;             // [passes][2^digit_bits] scratch (see kHistWords)
  u64* status;           // [tiles][2^digit_bits] look-back words
  u32* ticket;
  const u32* epoch_base;
  const u32* abort;
  u64* ts;               // trace timing slot (see ktime_start), nullable
};
struct SortFuse {
  u64* set;
  u32* set32;            // 32-bit set instead of set (keys below 2^32), and its all-ones flag
  u64* ones;
  u64 set_mask;
  u32* set_full;
  u32* cols[3];
  const u64* full_n;
  u64* out_delta;
  u32 arity;
  u32 shift[3];
  u32 width[3];
};
int launch_rs_hist(const SortParams& p, void* stream, bool clear_hist = true);
int launch_rs_pass(const SortParams& p, u32 pass, const u64* src, u64* dst, u32 epoch_off, void* stream,
                   const SortFuse* fuse = nullptr);
inline u32 sort_passes(u32 bits, u32 digit_bits = 8) { return (bits + digit_bits - 1) / digit_bits; }
constexpr u32 kHistWords = 6 * 2048;   // per relation: enough for 8 passes of 8 bits or 6 of 11
constexpr u32 kMaxRadix = 2048;
constexpr u32 kSortTile = 2048;

// A run of perm positions moving to a fresh region (see launch_index_update).
struct RunMove {
  u32 from, to, count;
};

// Index build over rows [0, n) of a relation's columns: table of distinct
// keys with runs into perm (the sorted-id array of Section 3, grouped by key).
struct IndexParams {
  const u32* col[3];
  RowRange src;
  u32 nkey;
  u32 keycol[2];
  Slot* table;
  u64 cap;               // slots, power of two
  u32* perm;
  u64* status;
  u32* ticket;
  const u32* epoch_base;
  u32 epoch_off;
  const u32* abort;
  u64* ndv;              // receives the number of distinct keys (nullable)
  u64* maxrun;           // receives the largest number of rows of one key (nullable)
  u64* full;             // bit 0: a key found no slot; bit 1: rows exceed perm_cap (index incomplete)
  u64* rows;             // receives the number of rows indexed (nullable)
  u32 nfilt;             // rows indexed: only those with col[fcol[i]] == fval[i], i < nfilt
  u32 fcol[2];
  u32 fval[2];
  u64 perm_cap;          // positions available in perm
  // Incremental updates (launch_index_update; derived relations): `src` is
  // the range of rows appended by the round.  Each slot's run lives in a
  // region of pcap[s] positions; the appended rows go after the run's old
  // rows, and a run that outgrows its region moves to a fresh region at the
  // bump pointer *top (the old region is left unused until the next build).
  u32* pcap;             // per slot: positions of its region (a build sets the run's count)
  u64* top;              // first position of perm no region uses (set by a build)
  u32* dcnt;             // per slot: rows appended this round (zero between updates)
  u32* wl;               // slots that got rows this round (the update's work list)
  u64* wl_n;             // its length (zero before the update)
  RunMove* moves;        // old runs to copy into their new regions, in chunks
  u64* moves_n;          // chunks listed (zero before the update)
  u64 moves_cap;
  u64* moved_rows;       // rows in the listed chunks (nullable; traces)
  u64* rword;            // counting update: per appended row, slot << 32 | place (scratch, delta_rows_cap words)
  const u32* abort2;     // a second flag that cancels an update (set-full round)
  u64* ts;               // trace timing slot of the launch (see ktime_start), nullable
};
int launch_index_build(const IndexParams& p, u64 rows_cap, void* stream);
// Incremental update over the appended rows, five launches on one stream:
// count the appended rows per key (inserting new keys), list the touched
// slots and note each row's slot and place among its key's appended rows in
// rword; give every touched run room for its appended rows (a run that
// outgrows its region gets one of twice its new size at the bump pointer,
// short runs copied on the spot, long ones listed in chunks); copy the listed
// chunks; place the appended rows after each key's old rows; clear the
// touched slots' appended counts.  No slot or row that the round did not
// touch is read or written.  ts[0..3] time the first four launches
// (nullable).
int launch_index_update(const IndexParams& p, u64 delta_rows_cap, u64 wl_cap, u64* const* ts, void* stream);
// The same update for many appended rows with mostly distinct keys, after
// sorting them by slot: launch_index_update_keys writes the appended rows'
// words (row - begin) << row_shift | slot (inserting new keys); the caller
// radix-sorts them over the slot bits; launch_index_update_sorted reserves
// room per run head (a run's length from its boundaries), copies listed old
// runs and places the appended rows, walking the table in slot order.
// ts[0..2] time the reserve, move and fill launches (nullable).
// With hist (passes <= 8), the words' 8-bit digits of the first `passes`
// radix passes are counted into hist (cleared here), so that the caller's
// sort needs no histogram pass; hist may be null.
int launch_index_update_keys(const IndexParams& p, u64 delta_rows_cap, u64* keys, u32 row_shift, u32* hist,
                             u32 passes, void* stream);
// Move an index into a larger table (tab, pcap of cap slots, cleared here):
// keys, runs and regions carried over, perm untouched; bit 0 of *full (also
// cleared here) reports a key that found no slot.
int launch_index_rehash(const Slot* old_tab, const u32* old_pcap, u64 old_cap, Slot* tab, u32* pcap, u64 cap,
                        u64* full, void* stream);
int launch_index_update_sorted(const IndexParams& p, u64 delta_rows_cap, const u64* sorted, u32 row_shift,
                               u64* const* ts, void* stream);
// Sorted build, in three steps on one stream: launch_index_slotkeys clears
// the table and writes keys[r] = r << row_shift | slot for rows r < n of the
// source (slot = cap for rows outside the filter); the caller radix-sorts
// keys over bits [0, row_shift) (row_shift a multiple of the digit width;
// hist as for launch_index_update_keys);
// launch_index_runs turns the sorted words into perm, counts and starts.
// keys holds rows_cap words.
int launch_index_slotkeys(const IndexParams& p, u64 rows_cap, u64* keys, u32 row_shift, u32* hist, u32 passes,
                          void* stream);
int launch_index_runs(const IndexParams& p, u64 rows_cap, const u64* sorted, u32 row_shift, void* stream);

int launch_fill_u64(u64* p, u64 n, u64 value, void* stream);
int launch_fill_u32(u32* p, u64 n, u32 value, void* stream);
int launch_colmax(const u32* col, u64 n, u32* out_max, void* stream);
// Column bounds under conditions: for each condition set q < nq (rows whose
// column col[i] equals val[i], i < n, n <= 3; n = 0: every row), the minimum
// and maximum of each column over the qualifying rows of the first n_rows
// rows: out[q * 8 + c] = minimum, out[q * 8 + 3 + c] = maximum (c < arity),
// out[q * 8 + 6] = 1 if any row qualified.  out holds nq * 8 words and is
// initialised here.
constexpr u32 kCondSets = 8;
struct CondSet {
  u32 n;
  u32 col[3];
  u32 val[3];
};
struct CondBoundsArgs {
  const u32* col[3];
  u32 arity;
  u64 n_rows;
  u32 nq;
  CondSet q[kCondSets];
  u32* out;
};
int launch_cond_bounds(const CondBoundsArgs& a, void* stream);
// Pack columns into keys (rows [0,n)), shift per column.
int launch_pack(const u32* const* cols, u32 arity, const u32* shift, u64 n, u64* keys, void* stream);
int launch_unpack(const u64* keys, u64 n, u32 arity, const u32* shift, const u32* width,
                  u32* const* cols, void* stream);
// Re-insert rows [0, n) of full into a tuple set (the 64-bit set, or with
// set32 non-null the 32-bit one and its all-ones flag word).
int launch_set_insert_rows(const u32* const* cols, u32 arity, const u32* shift, u64 n,
                           u64* set, u64 mask, void* stream, u32* set32 = nullptr, u64* ones = nullptr);

struct GatherDesc {
  const u32* src[3];
  u64 n;
  u64 dst;
  u32 add;
  u32 pad;
};
// out[c][d.dst + i] = d.src[c][i] + d.add for every descriptor d (n_src of
// them, in device memory) and i < d.n.
int launch_gather_relabel(const GatherDesc* d, u32 n_src, u32 arity, u32* const* out, void* stream);
// p[i] += delta (mod 2^32) for i < n.
int launch_add_u32(u32* p, u64 n, u32 delta, void* stream);

// Value compaction (kern_dict.hip).  launch_dict_unique writes the distinct
// keys of a sorted array (low 32 bits) to dict in order and their number to
// *count; tile_cnt holds dict_tiles(n) words of scratch.
u64 dict_tiles(u64 n);
int launch_dict_unique(const u64* sorted, u64 n, u64* tile_cnt, u32* dict, u64* count, void* stream);
int launch_dict_remap(u32* col, u64 n, const u32* dict, u64 nd, void* stream);
int launch_dict_gather(u32* col, u64 n, const u32* dict, void* stream);
// Instance boundaries of a sorted column (see k_bounds).
int launch_bounds(const u32* col, u64 n, u32 stride, u32 n_inst, u64* out, void* stream);

// Learned predictor (see kern_learn.hip)
constexpr u32 kHllRegs = 4096;
constexpr u32 kMlpIn = 8, kMlpHidden = 64;
constexpr u32 kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;
// Sketch of a join's probe side: the rows of `src` that pass the probe
// filters are counted into *rows and their key (col[c0], or col[c0] << 32 |
// col[c1]) goes into the HyperLogLog registers; *estimate gets the distinct
// count estimate (a double's bits).
struct HllParams {
  const u32* col[3];
  u32 c0;
  int c1;                 // -1: one-column key
  RowRange src;
  u32 n_pf;
  Filter pf[kMaxFilters];
  u32* regs;
  u64* estimate;
  u64* rows;
};
// Up to kHllBatch sketches in one launch (descriptors travel as the kernel
// argument).  The estimate pass also clears each sketch's registers for its
// next use; the row counts must be zero before the launch.
constexpr u32 kHllBatch = 8;
struct HllBatch {
  u32 n;
  HllParams s[kHllBatch];
};
static_assert(sizeof(HllBatch) <= 4096, "a sketch batch must fit in the kernel argument block");
int launch_hll_batch(const HllBatch& b, u64 rows_hint, void* stream);
int launch_dense_fwd(const float* in, u32 n, u32 din, const float* W, const float* b, u32 dout, float in_scale,
                     float* z, float* out, int relu, void* stream);
int launch_mse(const float* yhat, const float* y, u32 n, float* dy, float* loss, void* stream);
int launch_relu_bwd(float* dout, const float* z, u64 n, void* stream);
int launch_dense_wgrad(const float* dz, const float* in, u32 n, u32 din, u32 dout, float in_scale, float* dW,
                       float* db, void* stream);
int launch_dense_dgrad(const float* dz, const float* W, u32 n, u32 din, u32 dout, float* dinp, void* stream);
int launch_adam(float* p, const float* g, float* m, float* v, u32 n, float lr, float b1, float b2, float eps,
                float c1, float c2, void* stream);
int launch_mlp_infer_bf16(const float* X, u32 n, const float* P, float* out, void* stream);

// One join step whose output size the predictor estimates at the end of a
// round for the next one.  Counter indices refer to the engine's counter
// block; -1 means "not available".
struct PredSpec {
  int probe_full;        // counter: n_full of the probe-side relation (step 0)
  int probe_dbeg;        // counter: d_begin of it (delta plans; -1: read full)
  int build_full;        // counter: n_full of the build relation
  int ndv_build;         // counter: distinct keys of the build index (-1: cross product)
  int maxrun_build;      // counter: largest run of one key in the build index (-1: cross product)
  int rows_build;        // counter: rows held by the build index (-1: cross product, use build_full)
  int probe_rows;        // counter: probe rows passing the probe filters (-1: use the delta or full size)
  int hll;               // counter: HLL estimate (double bits) of the probe key (-1: none)
  u32 nkey, nfilt, step;
  int out;               // counter receiving the predicted output size
};
// Features of each spec from the counters, BF16 MLP inference, predictions
// written back to the counters.  Specs are ordered plan by plan; a step > 0
// takes the previous spec's prediction as its probe size.  A prediction never
// exceeds the join's worst case, probe rows x the longest run of one build key
// (probe rows x build rows for a cross product), carried along the chain.
int launch_predict(const PredSpec* specs, u32 n, u64* ctr, const float* params, void* stream);
void join_features(double probe_rows, double build_rows, double ndv_build, double ndv_probe, u32 nkey, u32 nfilt,
                   u32 step, float* f);

constexpr int kBlock = 256;

}  // namespace fv
