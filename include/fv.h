/*
 * fv.h -- C ABI of libfv.so, a semi-naive Datalog engine over column-stored
 * uint32 relations, written for AMD Instinct MI355X (gfx950).
 *
 * The problem these calls state is the one of Section 2 ("Datalog and RDF"):
 * extensional facts (EDB) are loaded into relations, positive Horn clauses
 * H <- B1, ..., Bn are added, and the engine derives every intensional fact
 * (IDB) until a fixed point is reached.  The evaluation follows Sections 3-4:
 * relations are stored column-wise (one uint32 array per column, tuples in
 * insertion order, full relations kept contiguous by eager merging), and each
 * round of semi-naive evaluation hash-joins the delta of a relation against
 * hash-indexed full relations (Algorithm 1), radix-sorts the newly derived
 * tuples, removes those already in full (the difference operator of Section 4,
 * "Union and Deduplication") and appends the survivors to full.
 *
 * Conventions for every call:
 *  - Every call returns an fv_status; 0 is success, negative is an error.
 *    On error, fv_last_error(ctx) returns a NUL-terminated message that stays
 *    valid until the next call on the same context.  No C++ exception crosses
 *    this interface.
 *  - A context is not thread-safe: calls on one context must not overlap.
 *  - All GPU work is ordered on the context's stream (fv_options.stream).
 *    Calls that return host-visible results synchronise that stream.
 *  - Pointers flagged as device pointers must be HIP device memory readable by
 *    the context's device; host pointers must be ordinary host memory.
 *  - The value 0xFFFFFFFF is reserved (it marks empty hash slots) and is
 *    rejected wherever it is passed in (FV_ERESERVED).
 */
#ifndef FV_H_
#define FV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fv_ctx fv_ctx;   /* opaque; owns relations, rules and all device memory */
typedef uint32_t fv_rel;        /* relation handle: index within its context */

typedef enum {
  FV_OK = 0,
  FV_EINVAL = -1,      /* bad argument (null pointer, unknown handle, bad name) */
  FV_ENOMEM = -2,      /* device allocation failed; the context is then terminal */
  FV_EARITY = -3,      /* arity mismatch between an atom and its relation, or arity outside 1..3 */
  FV_EUNSAFE = -4,     /* a head or != variable does not occur in a body atom */
  FV_ESTATE = -5,      /* call not allowed in the current state (e.g. load after run) */
  FV_EHIP = -6,        /* a HIP runtime call failed */
  FV_ERESERVED = -7,   /* the reserved value 0xFFFFFFFF was passed in */
  FV_ETRUNC = -8,      /* export capacity smaller than the relation */
  FV_ENOTSUP = -9      /* a relation's packed tuple needs more than 64 bits even with values renumbered */
} fv_status;

/* fv_options.flags */
#define FV_PLAIN      0u   /* count-then-write joins, host loop, one sync per round */
#define FV_LEARNED    2u   /* join-cardinality predictor on (fv_options.predictor): buffers are
                              presized from its predictions and joins run in one pass without
                              a count pass; a join that overflows its buffer makes the round
                              re-run with exact count-then-write.  The result is identical. */
#define FV_TRACE      4u   /* time each kernel class with HIP events (see fv_profile);
                              kernels are then launched one by one, never as a graph */
#define FV_LOG_JOINS 16u   /* record, per join of every round, its features and true output
                              size (fv_join_trace): training data for the predictor */
#define FV_GRAPH      8u   /* capture the recursive round as a HIP graph and replay it,
                              recapturing when a buffer grows (needs a stream other than
                              the legacy null stream; ignored with FV_TRACE) */
#define FV_HOST      32u   /* evaluate on host threads instead of the GPU: the same plans and
                              operators (hash-index joins counted then written, radix sort,
                              difference by a tuple set, eager append) over host memory, as the
                              paper's CPU variant of its engine (Section 5.3, Table 3).  Chosen
                              only by this flag, never as a fallback.  Loads and exports accept
                              host or device pointers; with FV_LEARNED, FV_GRAPH or FV_LOG_JOINS
                              fv_ctx_create fails (FV_EINVAL); FV_TRACE is ignored; fv_run_batch
                              refuses it (FV_ENOTSUP) */

/* Device allocator hooks.  dev_alloc returns device memory of at least
 * `bytes` bytes usable on `stream`, or NULL on failure; dev_free releases a
 * pointer dev_alloc returned.  Both NULL: the library uses hipMalloc/hipFree. */
typedef void* (*fv_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*fv_free_fn)(void* ptr, void* stream, void* user);

/* Tuning knobs (all zero = defaults).  They change speed and memory, never
 * the result.  fv_autotune searches them; fv_tuning_load reads a stored choice. */
typedef struct {
  uint32_t radix_bits;     /* digit width of the radix sort: 8 or 11 (0: 8) */
  uint32_t fuse_dedup;     /* 1: the last radix pass takes the difference and appends to full;
                              0: a separate pass does, keeping each delta sorted (default) */
  float set_load;          /* load of the tuple set at its expected size, 0.1..0.75 (0: 0.25) */
  float index_load;        /* load of join-index tables, 0.1..0.75 (0: 0.5) */
  uint32_t max_blocks;     /* grid cap of the look-back kernels, 256..8192 (0: 2048) */
  uint32_t index_rebuild;  /* 1: rebuild the join indices of derived relations from scratch every
                              round; 0: update them with the appended rows (default) */
  uint32_t index_sort;     /* join-index construction: 0 (default) radix sort of the rows by key
                              slot for builds of at least 2^20 rows, counting by hash otherwise;
                              1 counting for every build; 2 sorting for every build (updates of
                              the indices of derived relations always count) */
  uint32_t lookahead;      /* 0 (default): enqueue each plain eager round before the previous
                              round's counters are read back, where the program allows it
                              (no join reads an index of a derived relation); 1: never */
  uint32_t dedup_ranges;   /* the difference against full: 0 (default) probes a hash set of full's
                              packed tuples; 1: Algorithm 2 -- per-column indices of full (the
                              join indices' layout, kept up to date every round), a new tuple's
                              value ranges in them, an empty range or an empty intersection of
                              the ranges proving it new; 2: full's packed tuples kept in ascending
                              order and merged with the sorted new tuples every round: in that
                              merge (ties from full first) a new tuple is one that differs from
                              the tuple before it.  Modes 1 and 2 keep no tuple set and take no
                              look-ahead. */
  uint8_t block_log2[2][4]; /* threads per block as log2 (7, 8 or 9; 0: 8) of the join kernels
                              (probe, write, one-pass join, selection: [0][b]) and of the
                              difference pass ([1][b]), per launch size bucket b: at most 2^16,
                              2^20, 2^24 rows, more */
} fv_tuning;

typedef struct {
  void* stream;            /* hipStream_t the context runs on; NULL = null stream */
  fv_alloc_fn dev_alloc;   /* optional */
  fv_free_fn dev_free;     /* optional; required when dev_alloc is set */
  void* user;              /* passed through to the hooks */
  uint32_t flags;          /* FV_* flags above */
  const fv_tuning* tuning; /* optional; copied at fv_ctx_create */
  const float* predictor;  /* FV_MLP_PARAMS floats (see fv_mlp_train); required by FV_LEARNED */
  const char* trace_only;  /* with FV_TRACE: time only this kernel class (see fv_profile names) */
} fv_options;

/* A term of an atom: a variable (is_const = 0, value = variable index within
 * the rule, 0..15) or a constant (is_const = 1, value = the uint32 constant). */
typedef struct { uint32_t value; uint32_t is_const; } fv_term;

/* An atom rel(t0, ..., t_{arity-1}). */
typedef struct { fv_rel rel; uint32_t arity; const fv_term* terms; } fv_atom;

/* A rule head :- body[0], ..., body[n_body-1], neq constraints.  `neq` holds
 * n_neq pairs of variable indices (2 * n_neq entries); pair (a, b) requires
 * the values of variables a and b to differ (the x != y of Section 5.2). */
typedef struct {
  fv_atom head;
  const fv_atom* body;
  uint32_t n_body;         /* 1..8 */
  const uint32_t* neq;
  uint32_t n_neq;          /* 0..8 */
} fv_rule;

typedef struct {
  uint32_t iterations;         /* rounds run, including the final round that derived nothing */
  uint32_t redo_rounds;        /* rounds re-run after a buffer had to grow */
  uint64_t derived_tuples;     /* sum over IDB relations of |full| at fixpoint minus loaded facts */
  uint64_t join_output_tuples; /* tuples written by joins before deduplication */
  double ms_total;             /* wall time of fv_run_fixpoint (host clock, stream synchronised) */
  uint32_t graph_captures;     /* times the recursive round was captured as a HIP graph */
  uint32_t graph_replays;      /* rounds run by replaying that graph */
  uint32_t overflows;          /* FV_LEARNED: rounds whose one-pass joins overflowed (re-run exactly) */
  uint32_t predicted_joins;    /* FV_LEARNED: joins run with a predicted output size */
  double qerror_median;        /* FV_LEARNED: median of max(m/p, p/m) over those joins (sizes + 1) */
  double qerror_max;
  uint32_t reordered_rounds;   /* FV_LEARNED: (round, rule variant) pairs run in a join order other than
                                  the default most-bound-first one, because the predictor expected
                                  fewer intermediate rows from it (bodies of three or more atoms) */
} fv_stats;

/* One kernel class in the profile returned by fv_profile (FV_TRACE only).
 * Classes named host_* are not kernels but host phases of each round, timed
 * on the host clock (launches = rounds): host_prepare (sizing, buffer growth,
 * index rebuilds before the round's kernels are enqueued), host_enqueue,
 * host_wait (counter read-back and stream sync) and host_finish; host_alloc
 * counts the device allocations (launches) and the time spent in them.  They
 * are not recorded when trace_only is set. */
typedef struct {
  char name[32];
  uint64_t launches;
  double ms;                   /* sum of kernel durations (device clock or HIP events) */
  double algo_bytes;           /* algorithmic HBM bytes these launches had to move */
  uint64_t items;              /* elements processed (rows, keys or output tuples) */
} fv_kprof;

/* Create a context.  opt may be NULL (null stream, hipMalloc, no flags).
 * The options struct is copied. */
fv_status fv_ctx_create(fv_ctx** out, const fv_options* opt);

/* Destroy a context and free all its device memory.  Safe on NULL and on a
 * context that hit an error. */
void fv_ctx_destroy(fv_ctx* ctx);

/* Text of the last error on this context ("" if none). */
const char* fv_last_error(const fv_ctx* ctx);

/* Declare a relation of the given arity (1..3) under a unique name
 * (Section 3: a relation is a set of columns of uint32 values).  The handle
 * is written to *out. */
fv_status fv_relation_create(fv_ctx* ctx, const char* name, uint32_t arity, fv_rel* out);

/* Look up a relation by name. */
fv_status fv_relation_find(fv_ctx* ctx, const char* name, fv_rel* out);

/* Append n_rows facts to a relation, given as `arity` column arrays of
 * n_rows uint32 each (Section 3, raw data arrays).  on_device != 0 means the
 * column pointers are device pointers.  The data is copied before the call
 * returns; the caller keeps ownership.  Relations are sets: duplicates are
 * removed when the fixpoint starts.  Allowed only before fv_run_fixpoint.
 * Errors: FV_EINVAL, FV_ESTATE, FV_ERESERVED (a value is 0xFFFFFFFF),
 * FV_ENOMEM, FV_EHIP. */
fv_status fv_load_columns(fv_ctx* ctx, fv_rel rel, const uint32_t* const* cols,
                          uint64_t n_rows, int on_device);

/* Add a rule (Section 2; translated into joins, selections and projections
 * as in Section 4).  The rule is validated and copied.  Allowed only before
 * fv_run_fixpoint.  Errors: FV_EARITY, FV_EUNSAFE, FV_EINVAL (variable index
 * above 15, too many atoms), FV_ERESERVED, FV_ESTATE. */
fv_status fv_add_rule(fv_ctx* ctx, const fv_rule* rule);

/* Evaluate the program to its least fixpoint by semi-naive evaluation
 * (Section 3): all rules contribute in every round, the delta of each
 * relation is joined against full relations (Algorithm 1), the new tuples are
 * radix-sorted, deduplicated against full and merged into full, until no
 * relation gains a tuple.  Runs once per context; stats may be NULL.
 * Tuples are packed column by column into 64-bit keys, each column as wide as
 * its largest possible value.  When some relation would need more than 64
 * bits (three columns of large ids), every value of the loaded facts and of
 * the rules' constants is first replaced by its rank among the distinct ones
 * (values are only compared for equality and rules create none, so the
 * fixpoint is the same up to that renaming; fv_export maps ranks back).
 * Errors: FV_ESTATE (already run), FV_ENOTSUP (still more than 64 bits: an
 * arity-3 relation over more than 2^21 distinct values), FV_ENOMEM, FV_EHIP. */
fv_status fv_run_fixpoint(fv_ctx* ctx, fv_stats* stats);

/* Batched form: evaluate n contexts that hold the same program (same
 * relations in the same order, same rules), each over its own loaded facts, as
 * one fixpoint.  Instance k's values are shifted into the id range
 * [k*stride, (k+1)*stride) of one merged namespace (stride = the power of two
 * above the largest loaded value), so every join, sort and difference launch
 * processes all instances at once.  Afterwards each context reports and exports
 * its own relations exactly as if it had run alone; fv_delta_sizes on an
 * instance context returns the merged rounds (all instances added up).  The contexts
 * must live on one device; each must be fresh (not yet run).  The merged
 * result is shared by the instances and freed with the last of them.
 * Errors: FV_EINVAL (different programs, empty batch), FV_ESTATE,
 * FV_ENOTSUP (a rule uses a constant or has a body whose atoms do not share
 * variables -- then instances could mix -- or n*stride exceeds 2^32-1), plus
 * those of fv_run_fixpoint. */
fv_status fv_run_batch(fv_ctx* const* ctxs, uint32_t n, fv_stats* stats);

/* Builds a fresh context holding the program and facts to tune on, created
 * with the options given (they carry the candidate tuning); NULL on failure.
 * The tuner runs the context to its fixpoint and destroys it. */
typedef fv_ctx* (*fv_make_ctx_fn)(const fv_options* opt, void* user);

/* Autotuner.  Coordinate search over fv_tuning: starting from the defaults,
 * each knob in turn (radix_bits {8,11}, fuse_dedup {0,1}, set_load
 * {0.25,0.5}, index_load {0.25,0.5}, max_blocks {1024,2048,4096}, index_rebuild
 * {0,1}, index_sort {0,1}, lookahead {0,1}, dedup_ranges {0,2}, then each
 * kernel class's block size per size bucket, block_log2[c][b] {7,8,9}) is set to
 * every candidate with the others at their best so far; a candidate is scored
 * by the median fv_run_fixpoint time of `reps` fresh contexts from make()
 * (reps 0 means 3).  The winner goes to *best and, if cache_path and key are
 * set, into a JSON cache file under "<gfx arch>/<key>" (other entries are
 * kept).  A candidate whose trial fails is passed over.  Errors: FV_EINVAL
 * (null arguments, a failed trial of the defaults, or a cache write;
 * fv_global_error() tells which). */
fv_status fv_autotune(fv_make_ctx_fn make, void* user, const fv_options* base, uint32_t reps,
                      const char* cache_path, const char* key, fv_tuning* best);

/* Read the tuning fv_autotune stored under key for the current GPU's
 * architecture.  FV_EINVAL if the file, or the entry, is missing. */
fv_status fv_tuning_load(const char* cache_path, const char* key, fv_tuning* out);

/* Error text of the last failed call that has no context (fv_autotune,
 * fv_tuning_load, fv_mlp_*, fv_hll_ndv). */
const char* fv_global_error(void);

/* The join-cardinality predictor: an MLP 8 -> 64 -> 64 -> 1 with ReLU whose
 * parameters are FV_MLP_PARAMS floats laid out W1[64][8] b1[64] W2[64][64]
 * b2[64] W3[1][64] b3[1] (row-major, output index first).  Inputs are the
 * 8 features of a join (see fv_join_trace), scaled by 1/16 before the first
 * layer; the output predicts log2(1 + join output size) / 16.  X is n x 8
 * row-major host memory, y has n entries.  These calls take no context: they
 * run on the current device, on opt->stream, and take their device memory
 * from opt's allocator hooks (opt may be NULL: null stream, hipMalloc).  The
 * memory is released before the call returns.  Errors: FV_EINVAL (null
 * argument, n == 0), FV_ENOMEM, FV_EHIP; fv_global_error() tells which. */
#define FV_MLP_PARAMS 4801u

/* Mean-squared-error loss of the network on (X, y) and its gradient with
 * respect to every parameter (same layout), in FP32 on the GPU. */
fv_status fv_mlp_grad(const fv_options* opt, const float* X, const float* y, uint32_t n, const float* params,
                      float* grads, float* loss);

/* Full-batch training with Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8) for
 * `steps` steps on the GPU.  init != 0 starts from He-uniform weights drawn from
 * SplitMix64(seed) and zero biases; otherwise from *params.  Writes the
 * trained parameters to params and the final loss to *loss (nullable). */
fv_status fv_mlp_train(const fv_options* opt, const float* X, const float* y, uint32_t n, uint32_t steps, float lr,
                       uint64_t seed, int init, float* params, float* loss);

/* Inference with BF16 weights and activations (round to nearest even) and
 * FP32 accumulation: yhat[i] for each row of X. */
fv_status fv_mlp_predict(const fv_options* opt, const float* X, uint32_t n, const float* params, float* yhat);

/* Distinct-value estimates of n_cols uint32 columns of n_rows values each:
 * one HyperLogLog sketch per column (Flajolet, Fusy, Gandouet and Meunier
 * 2007, the algorithm and its estimator as that paper states them; 2^12
 * registers, standard error about 1.04 / 64 = 1.6%), the same sketch kernels
 * that give the learned predictor its probe-key feature.  A value v is
 * hashed as MurmurHash3's 64-bit finalizer of v + 0x9E3779B97F4A7C15; the top
 * 12 bits pick a register, which keeps the largest 1 + (leading zeros of the
 * other 52 bits).  cols holds n_cols column pointers (device pointers if
 * on_device != 0, else host memory, copied in); estimates receives n_cols
 * doubles (host memory).  Stream, allocator and errors as for the MLP calls
 * above. */
fv_status fv_hll_ndv(const fv_options* opt, const uint32_t* const* cols, uint32_t n_cols, uint64_t n_rows,
                     int on_device, double* estimates);

/* fv_hll_ndv for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sketch kernels, with their registers and counters in a static device
 * array of 128.1 KiB that each GPU the library runs on holds until the
 * process ends.  cols is a host array of n_cols device column pointers
 * (n_cols <= FV_HLL_NOALLOC_MAX_COLS, else FV_EINVAL), estimates a device
 * array of n_cols doubles that receives the estimates.  Work is enqueued on
 * `stream` (a hipStream_t; NULL = null stream) and not waited for: read the
 * estimates after synchronising it.  The call allocates nothing, clears the
 * array with kernels (never a memset) and may be captured into a graph.
 * Calls on one GPU share its array, so calls that overlap on one GPU (two
 * streams, or two graphs in flight) race; serialise them.  Errors: FV_EINVAL,
 * FV_EHIP (fv_global_error() tells which). */
#define FV_HLL_NOALLOC_MAX_COLS 8u
fv_status fv_hll_ndv_noalloc(const uint32_t* const* cols, uint32_t n_cols, uint64_t n_rows, double* estimates,
                             void* stream);

/* Number of tuples currently in a relation (after the fixpoint: its full
 * version; before: the rows loaded so far, duplicates included). */
fv_status fv_relation_size(fv_ctx* ctx, fv_rel rel, uint64_t* n_rows);

/* Copy a relation out, sorted lexicographically by (col0, col1, col2): the
 * intensional facts derived by the fixpoint (Section 2), or a relation's
 * loaded facts, as a set.
 * cols_out holds `arity` column pointers of capacity rows each (device
 * pointers if on_device != 0).  cols_out == NULL only writes *n_rows_out.
 * If capacity < size nothing is written and FV_ETRUNC is returned with
 * *n_rows_out set.  Allowed after fv_run_fixpoint. */
fv_status fv_export(fv_ctx* ctx, fv_rel rel, uint32_t* const* cols_out,
                    uint64_t capacity, uint64_t* n_rows_out, int on_device);

/* Per-round delta sizes of the last fixpoint, summed over relations: round r
 * added out[r] tuples.  *n receives the number of rounds; up to cap entries
 * are written. */
fv_status fv_delta_sizes(fv_ctx* ctx, uint64_t* out, uint32_t cap, uint32_t* n);

/* Join trace of the last fixpoint (FV_LOG_JOINS or FV_LEARNED): one row of
 * FV_TRACE_COLS floats per join executed in a round -- the 8 predictor
 * features, then log2(1 + true output size) / 16, then the predicted output
 * size (or -1).  Up to cap rows are written to rows; *n receives the count. */
#define FV_TRACE_COLS 10u
fv_status fv_join_trace(fv_ctx* ctx, float* rows, uint32_t cap, uint32_t* n);

/* Kernel-class profile of the last fixpoint (FV_TRACE contexts): up to cap
 * entries are written, *n receives the number of classes. */
fv_status fv_profile(fv_ctx* ctx, fv_kprof* out, uint32_t cap, uint32_t* n);

#ifdef __cplusplus
}
#endif
#endif /* FV_H_ */
