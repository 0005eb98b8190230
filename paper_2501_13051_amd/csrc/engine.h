// Host runtime of the engine: device memory, relations, rule plans and the
// semi-naive round loop.  The C ABI in api.cpp is a thin shell over this.
#pragma once

#include <hip/hip_runtime_api.h>

#include <chrono>
#include <map>
#include <memory>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fv.h"
#include "fv_types.h"

namespace fv {

struct Error : std::runtime_error {
  fv_status code;
  Error(fv_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

constexpr u32 kMaxVars = 16;
constexpr u32 kMaxBody = 8;
constexpr u32 kMaxNeq = 8;
constexpr u32 kMaxJoinOrders = 3;   // join orders planned per rule variant (FV_LEARNED)
constexpr u32 kNoIndex = ~0u;

struct Term { u32 value; bool is_const; };
struct AtomR { u32 rel; std::vector<Term> t; };
struct RuleR {
  AtomR head;
  std::vector<AtomR> body;
  std::vector<std::pair<u32, u32>> neq;
};

struct Relation {
  std::string name;
  u32 arity = 0;
  bool idb = false;          // appears in a rule head
  // staged loads (before the fixpoint), device columns
  Buf stage[3];
  u64 staged = 0, stage_cap = 0;
  u32 maxv[3] = {0, 0, 0};   // per-column value bound (domain analysis)
  u32 lmax[3] = {0, 0, 0};   // per-column maximum of the loaded facts
  bool has_rows = false;
  // full relation: contiguous columns; delta = rows [d_begin, n_full)
  Buf col[3];
  u64 cap = 0;
  // new tuples of a round as packed keys, plus the sort's second buffer
  Buf newk, newk2;
  u64 new_cap = 0;
  u64 last_new = 0;          // new tuples of the last finished round
  u64 prev_new = 0;          //   and of the round before it
  // tuple set of full, for the difference operator
  Buf set;
  // difference by merge (dedup_ranges = 2): full's packed tuples in ascending
  // order, and the buffer the round's merge writes (swapped in when the round
  // succeeds)
  Buf sfull, sfull2;
  u64 sfull_cap = 0;
  bool merged_this_round = false;
  u64 set_cap = 0;
  u64 set_min = 0;           // lower bound on the next set size (after a set-full round)
  bool set_stale = false;    // holds keys of an aborted round: rebuild before the next one
  bool set32 = false;        // packed tuples fit in 32 bits: 4-byte set slots
  bool hist_by_writers = false;  // this round's writers of new keys count their sort digits
  int c_ones = -1;           // device counter: the 32-bit set holds the all-ones key
  u32 dix[3] = {kNoIndex, kNoIndex, kNoIndex};   // per-column indices of full (Algorithm 2 difference)
  u32 width[3] = {0, 0, 0}, shift[3] = {0, 0, 0}, bits = 0;
  u32 exp_shift[3] = {0, 0, 0};   // lexicographic packing for export
  // host mirrors of device counters (valid after each sync)
  u64 n_full = 0, d_begin = 0, n_delta = 0, seeds = 0;
  bool used_as_head = false;
};

struct Index {
  u32 rel;
  u32 nkey;
  u32 keycol[2];
  u32 nfilt = 0;              // only rows with col[fcol[i]] == fval[i] are indexed
  u32 fcol[2] = {0, 0};
  u32 fval[2] = {0, 0};
  int c_ndv = -1;             // device counter: distinct keys after the last build
  int c_maxrun = -1;          // device counter: rows of the most frequent key
  int c_full = -1;            // device counter: 1 if the last build ran out of slots
  int c_rows = -1;            // device counter: rows the last build indexed
  int c_top = -1;             // device counter: first position of perm no run region uses
  int c_wl = -1;              // device counter: slots an update touched (cleared every round)
  int c_moves = -1;           // device counter: old-run chunks an update listed (cleared every round)
  int c_mrows = -1;           // device counter: rows in those chunks (cleared every round)
  u64 keys_seen = 0;          // distinct keys found by the last complete build
  u64 rows_seen = 0;          // rows indexed by the last complete build or update
  u64 keys_hint = 0;          // before the first build: estimated distinct keys (sketch)
  u64 rows_hint = 0;          //   and the exact rows it will hold
  bool hinted = false;
  bool grow = false;          // the last build ran out of slots: rebuild larger
  bool perm_grow = false;     // the last build ran out of positions: rebuild with more
  Buf table, perm;            // slots; row ids grouped by key (runs in regions of perm)
  Buf pcap, dcnt, wl;         // per slot: region size, rows appended this round; touched slots
  u64 cap = 0, perm_cap = 0;
  u64 top_seen = 0;           // host mirror of the bump pointer after the last round
  bool dirty = true;          // storage (re)allocated since the last build
  u32 sort_shift = 0;         // nonzero: built by sorting (row << sort_shift | slot) words
  u32 sort_bits = 0;          //   over this many slot bits
  u32 upd_shift = 0;          // nonzero: updated by sorting the appended rows' (row << upd_shift | slot) words
};

// One join (or, with index == kNoIndex and brel == kNone, one selection):
// probe source -> build relation -> output.
struct Step {
  bool select_only = false;
  u32 brel = 0;
  u32 index = kNoIndex;       // kNoIndex with !select_only: cross product
  u32 nkey = 0;
  Src key[2];
  std::vector<Filter> pf;     // probe-row filters (first step only)
  std::vector<Filter> wf;     // filters after the build row is known
  std::vector<Src> out;       // output columns (or head columns)
  int out_buf = -1;           // intermediate id, or -1: head relation's new keys
  u32 head_rel = 0;
  int c_m = -1, c_t = -1;     // device counters for this join's sizes
  int c_n = -1;               // device counter: probe rows the join read (traces)
  int c_pred = -1;            // device counter: predicted output size (learned mode)
  int hll = -1;               // HLL sketch of the probe key (step 0, learned/logging modes)
  bool fused = false;         // this round runs it as a presized one-pass join
};

struct Plan {
  u32 rule;
  int delta_pos;              // body position read from delta; -1 = all full
  u32 src_rel;
  bool src_delta;
  u32 second = 0;             // body position the first join reads (build side)
  int alt = -1;               // plans of one rule and delta position in other join orders share an id
  bool alt_default = false;   // the group's most-bound-first order
  bool active = true;         // this round runs it (one plan of each alternative group)
  std::vector<Step> steps;
};

struct HllSketch {
  u32 rel;
  u32 c0;
  int c1;                     // second key column or -1
  bool delta;                 // sketch of the delta rows (else of full)
  std::vector<Filter> pf;     // probe filters: only rows passing them are sketched
  Buf regs;
  int ctr = -1;               // estimate (double bits)
  int ctr_rows = -1;          // rows passing the filters
};

struct Inter {
  u32 ncols;
  Buf col[kMaxCols];
  u64 cap = 0;
  int ctr = -1;
  u64 last_used = 0;   // rows of the last finished round
  u64 prev_used = 0;   //   and of the round before it
};

struct KClass {
  std::string name;
  u64 launches = 0;
  double ms = 0, bytes = 0;
  u64 items = 0;
};

struct PendingEvent {
  int cls;
  hipEvent_t a, b;
  double bytes;   // < 0: computed later from counters (see bytes_fn)
  int kind;       // which counter-derived formula
  int ref0, ref1; // counter references
  u64 aux;
  int stamp = -1;  // >= 0: timed by the kernel's own stamps in this slot
  u64 seq = 0;     // the round it belongs to (emit_seq_ when enqueued)
};

class Engine;
struct HostState;   // host evaluator state (host_engine.cpp)

// Result of a batched fixpoint, shared by the instance contexts: every
// relation sorted lexicographically in the merged id space, plus where each
// instance's rows start.
struct BatchResult {
  std::shared_ptr<Engine> merged;
  u64 stride = 0;
  std::vector<std::vector<Buf>> cols;       // [relation][column], from `merged`'s allocator
  std::vector<std::vector<u64>> bounds;     // [relation][instance + 1]
  std::vector<u64> deltas;
  ~BatchResult();                           // hands cols back through `merged`
};

class Engine {
  friend struct BatchResult;

 public:
  explicit Engine(const fv_options* opt);
  ~Engine();

  u32 relation_create(const char* name, u32 arity);
  u32 relation_find(const char* name) const;
  void load_columns(u32 rel, const u32* const* cols, u64 n, bool on_device);
  void add_rule(const fv_rule& r);
  void run(fv_stats* stats);
  u64 relation_size(u32 rel) const;
  void export_rel(u32 rel, u32* const* cols, u64 capacity, u64* n_out, bool on_device);
  const std::vector<u64>& delta_sizes() const { return batch_ ? batch_->deltas : deltas_; }
  // Evaluate n contexts holding the same program over their own facts in one
  // fixpoint (see fv_run_batch).
  static void run_batch(Engine* const* es, u32 n, fv_stats* stats);
  const std::vector<KClass>& profile() const { return kprof_; }
  // one row per executed join step: 8 features, log2(1+output)/16, predicted size (-1: none)
  const std::vector<float>& join_trace() const { return trace_rows_; }
  static constexpr u32 kTraceCols = 10;

  std::string last_error;
  bool terminal = false;

 private:
  // memory
  Buf alloc(size_t bytes);
  void release(Buf& b);
  void grow(Buf& b, size_t bytes, size_t keep_bytes);
  void hip(hipError_t e, const char* what);
  void launched(int rc, const char* what);
  void sync();

  // setup
  void alloc_control();
  bool domain_analysis();    // false: some relation's packed tuple needs more than 64 bits
  void refine_bounds();      // tighter column bounds from the rules' constant conditions
  // bounds of the loaded facts of `rel` under condition sets (launch_cond_bounds' layout)
  void fact_bounds(u32 rel, const CondSet* q, u32 nq, u32* out);
  void host_fact_bounds(u32 rel, const CondSet* q, u32 nq, u32* out);
  void fit_packing();
  void compact_values();
  void host_compact_values();
  void map_back(u32* const* cols, u32 arity, u64 n, bool on_device);
  void plan_all();
  Plan plan_rule(u32 rule, int delta_pos, int second = -1);
  void choose_join_orders();
  void take_merged_full();
  bool merge_diff() const { return tune_.dedup_ranges == 2; }
  u32 block_for(int cls, u64 rows) const;
  u32 get_index(u32 rel, u32 nkey, const u32* keycol, u32 nfilt, const u32* fcol, const u32* fval);
  void ingest();
  // true if any buffer was (dry: would be) reallocated; with look-ahead every
  // derived relation is sized for two rounds of new tuples
  bool ensure_capacity(bool dry = false);
  // look-back words per tile of the shared sort status array: one per digit
  // value of the widest digits any sort of this context uses (index sorts
  // always take 8-bit digits)
  u64 sort_status_words() const { return tune_.radix_bits == 11 ? kMaxRadix : 256; }
  void build_indices(bool idb_only);
  void build_index(Index& ix);

  // rounds
  void run_round(bool initial);
  void setup_learning();
  void emit_sketches_and_prediction(bool initial);
  void size_from_predictions(bool initial);
  void note_index_builds();
  void presize_indices();
  void verify_builds(std::vector<u32> built);
  void update_index(Index& ix);
  void log_joins(bool initial);
  void exec_plan(Plan& p);
  void finish_relation(Relation& R, bool in_round);
  void commit_relation(Relation& R);
  void read_counters();
  u32 next_epoch();
  void begin_phase();
  void emit_round(bool initial, bool all_plans, bool sticky = false);
  void grow_after_failure(bool initial);
  void finish_round(bool initial, std::chrono::steady_clock::time_point th);
  bool can_look_ahead() const;
  void run_with_look_ahead();
  void wait_event(hipEvent_t e);
  bool capture_round();
  void drop_graph();

  // profiling
  int kclass(const char* name);
  // traces: host time of one round phase, as a class of its own
  void host_time(const char* name, std::chrono::steady_clock::time_point since);
  u64* ev_begin(int cls, bool single = false);
  hipEvent_t pooled_event();
  void ev_end(int cls, double bytes, int kind = 0, int ref0 = -1, int ref1 = -1, u64 aux = 0);
  void ev_cancel();
  void collect_events(u64 upto, bool discard);   // launches of rounds up to `upto`

  u64* ctr(int i) { return ctr_dev_.as<u64>() + i; }
  u32* epoch_base() { return flags_dev_.as<u32>() + kFlagEpoch; }

  fv_options opt_{};
  fv_tuning tune_{};
  hipStream_t stream_ = nullptr;
  bool ran_ = false;
  std::vector<Relation> rels_;
  std::map<std::string, u32> by_name_;
  std::vector<RuleR> rules_;
  std::vector<Index> indices_;
  std::vector<Plan> init_plans_, delta_plans_;
  std::vector<Inter> inters_;

  // device control block
  Buf ctr_dev_, flags_dev_, ticket_dev_, hist_dev_, maxv_dev_;
  u64* ctr_host_ = nullptr;   // pinned mirror
  u32* flags_host_ = nullptr;
  int n_ctr_ = 0;
  int c_derived_ = 0, c_joinout_ = 1;
  int c_full0_ = 0, c_dbeg0_ = 0, c_delta0_ = 0, c_new0_ = 0, c_reset_begin_ = 0;
  // scratch
  Buf m_row_, m_start_, m_off_;
  u64 m_cap_ = 0;
  Buf st_a_, st_b_, st_sort_;
  Buf ixk_a_, ixk_b_;     // sorted index builds: (row, slot) words and the sort's second buffer
  std::vector<u32> rehashed_;   // indices moved to larger tables, to be checked before a round reads them
  Buf moves_;             // index updates: old-run chunks to copy (shared, updates run one by one)
  Buf mdiff_;             // the difference by merge: per-tile splits, counts and ranks (shared)
  u64 mdiff_cap_ = 0;     // its words
  u64 moves_cap_ = 0;
  u64 ixk_cap_ = 0;
  u64 st_cap_ = 0, st_sort_tiles_ = 0;
  u32 epoch_off_ = 1;     // next look-back offset within the current phase
  u64 phases_ = 0;        // epoch-base advances since the status arrays were cleared
  // captured recursive round
  bool use_graph_ = true;
  bool graph_dirty_ = true;
  bool graph_events_ok_ = true;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t graph_exec_ = nullptr;
  bool capturing_ = false;
  bool graph_replayed_ = false;
  u32 graph_captures_ = 0, graph_replays_ = 0;
  u64 n_allocs_ = 0;
  std::vector<PendingEvent> graph_events_;

  std::vector<u64> deltas_;
  u32 redo_ = 0;
  // FV_HOST: the same plans evaluated on host threads (host_engine.cpp)
  bool host_mode_ = false;
  u32 host_threads_ = 1;
  std::shared_ptr<HostState> host_;
  static u32 host_threads();
  void host_load(u32 rel, const u32* const* cols, u64 n, bool on_device);
  void host_build_index(u32 i);
  void host_exec_plan(Plan& p);
  u64 host_finish_relation(u32 ri);
  void run_host(fv_stats* stats);
  void host_export(u32 rel, u32* const* cols, u64 n, bool on_device);
  // test hooks (see the constructor)
  std::set<u64> fail_rounds_;   // enqueued rounds (1-based) made to fail once
  u64 emitted_ = 0;             // rounds enqueued so far (captures excluded)
  bool small_caps_ = false;
  // learned predictor
  bool learned_ = false, log_joins_ = false, use_fused_ = false;
  u64 base_cap_ = 0;   // new-tuple capacity set at ingest (2x the loaded facts, at least 2^16)
  std::vector<bool> fused_steps_, graph_fused_steps_;   // per-step one-pass choice (now / when captured)
  void choose_join_algorithms(bool initial);
  std::vector<float> predictor_;          // MLP parameters (host copy)
  Buf predictor_dev_;
  std::vector<HllSketch> sketches_;
  std::vector<PredSpec> pspec_init_, pspec_delta_;
  Buf pspec_init_dev_, pspec_delta_dev_;
  std::vector<u64> start_ctr_;            // counters as they were when the round started
  std::vector<float> trace_rows_;
  // value compaction (packed tuples wider than 64 bits): the sorted distinct
  // values of the loaded facts and rule constants; a value's rank replaces it
  bool compacted_ = false;
  bool allow_compaction_ = true;
  Buf dict_;
  std::vector<u32> dict_host_;
  std::vector<double> qerrors_;
  u32 reordered_rounds_ = 0;
  std::vector<char> alt_distrusted_;   // per join-order group: its predicted order overflowed once
  u32 overflows_ = 0;
  int c_ndv0_ = 0, c_hll0_ = 0, c_pred0_ = 0;
  u64 join_out_ = 0;

  bool trace_ = false;
  std::string trace_only_;     // non-empty: only this kernel class gets events
  bool touched_device_ = false;
  std::shared_ptr<BatchResult> batch_;   // set on instance contexts of a batch
  u32 inst_ = 0;
  std::vector<KClass> kprof_;
  std::vector<PendingEvent> pending_;
  std::vector<hipEvent_t> ev_pool_;
  u64* rb_host_[2] = {nullptr, nullptr};    // pinned counter read-backs (two with look-ahead)
  hipEvent_t rb_ev_[2] = {nullptr, nullptr};
  u64 emit_seq_ = 0;                        // rounds enqueued so far
  bool ahead_active_ = false;               // rounds run with look-ahead (run_with_look_ahead)
  hipEvent_t ev_open_ = nullptr;
  bool ev_is_open_ = false;
  int ev_stamp_ = -1;
  static constexpr u32 kMaxStamps = 8192;   // stamped launches per round
  Buf stamps_dev_;                          // [kMaxStamps][start, 64 ends] device clock
  u32 stamps_used_ = 0;
  std::vector<std::pair<int, u32>> stamped_;   // (kernel class, slot) awaiting flush_stamps
  void flush_stamps();
  double wall_khz_ = 100000.0;              // device wall clock rate
};

}  // namespace fv
