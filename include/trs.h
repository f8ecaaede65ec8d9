/*
 * trs.h -- C-ABI of the MI355X term-rewriting library (libtrs.so).
 *
 * The library computes innermost normal forms of ground terms for a
 * left-linear term rewrite system, following the problem statement of
 * "Term Rewriting on GPUs" (van Eerd, Groote, Hijma, Martens, Wijs):
 *
 *   - terms, substitutions, matches and normal forms: Section 2,
 *     Definitions 1 and 2; a rule l -> r requires l not a variable,
 *     Var(r) a subset of Var(l), and every variable at most once in l;
 *   - strategy: innermost; for a head symbol the rules are tried in their
 *     given order and the first match is applied (Section 2, the derive and
 *     rewrite_f procedures);
 *   - method: Section 3 -- the term graph is stored as arrays indexed by a
 *     node index (head symbols, argument indices, normal-form flags,
 *     reference counts); in lock-step rounds every stored node whose
 *     arguments are all in normal form is matched and rewritten in place,
 *     followed by reference-count garbage collection with free-index reuse,
 *     until a round sees no node that is not in normal form.
 *
 * Encoding (all integers little-endian int32 unless stated):
 *   - symbols are numbered 0..n_sym-1; arity[s] is the arity of symbol s;
 *   - a term is its prefix (pre-order) sequence of symbol ids;
 *   - rule i occupies rule_code[rule_off[i] .. rule_off[i+1]): the prefix code
 *     of its left-hand side immediately followed by that of its right-hand
 *     side; variable k of the rule is written -1-k;
 *   - the normal form read back is the canonical serialisation: the prefix
 *     sequence of symbol ids of the term with all sharing expanded.
 *
 * Call order: trs_create -> trs_load_rules -> trs_load_terms -> trs_normalize
 * -> trs_read_nf (any number of times) ; trs_load_terms may be called again
 * to start over with new terms.  A context is used by one host thread at a
 * time; device work is issued on the stream given in trs_config.
 *
 * Errors: every call returns TRS_OK (0) or a negative trs_status; the last
 * error message of a context is available from trs_last_error().  No call
 * aborts the process.
 */
#ifndef TRS_H
#define TRS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t trs_status;

#define TRS_OK 0
#define TRS_E_ARG (-1)     /* null pointer, bad size, bad option value */
#define TRS_E_STATE (-2)   /* call out of order (e.g. normalize before terms) */
#define TRS_E_RULE (-3)    /* rule violates Definition 1 or left-linearity, or
                              arity mismatch / arity above maxarity */
#define TRS_E_TERM (-4)    /* input not ground, malformed prefix code */
#define TRS_E_POOL (-5)    /* node pool exhausted (initial load or rewriting) */
#define TRS_E_ROUNDS (-6)  /* max_rounds reached without a normal form */
#define TRS_E_HIP (-7)     /* HIP runtime error (message in trs_last_error) */
#define TRS_E_LIMIT (-8)   /* a rule exceeds the compiled-table limits */
#define TRS_E_INTERNAL (-9)

/* compiled-table limits (per rule / per system) */
#define TRS_MAX_ARITY 5      /* highest symbol arity and highest maxarity the
                               kernels are compiled for (TRS_E_LIMIT above) */
#define TRS_MAX_PATTERN 8   /* left-hand-side nodes below the root */
#define TRS_MAX_NEW 8       /* right-hand-side nodes created per rewrite */
#define TRS_MAX_RULES 256
#define TRS_MAX_SYMBOLS 4096

typedef struct trs_ctx trs_ctx;

typedef struct {
  int64_t pool_slots;  /* N: node slots in the pool, 2 .. 2^30 (slot 0 is
                          reserved; indices are int32) */
  int32_t maxarity;    /* A: argument stride of the pool, 1..TRS_MAX_ARITY;
                          0 = take the highest arity of the loaded system */
  int32_t device;      /* HIP device ordinal */
  void *hip_stream;    /* hipStream_t on which all device work is issued;
                          NULL = the library creates its own stream */
  void *dev_mem;       /* optional caller-owned device block to carve the pool
                          from (must stay valid while the context lives);
                          NULL = the library allocates */
  int64_t dev_bytes;   /* size of dev_mem in bytes */
} trs_config;

#define TRS_MODE_PLAIN 0     /* full sweep of every slot every round */
#define TRS_MODE_FRONTIER 1  /* sweep a compacted frontier; full confirmation
                                sweep before declaring a normal form */
#define TRS_MODE_LEARNED 2   /* frontier: parent notification when an
                                argument becomes a normal form, and for a
                                node found blocked the trained predictor
                                (below) decides whether it is examined again
                                next round; full confirmation sweep as in
                                TRS_MODE_FRONTIER */

typedef struct {
  int32_t mode;              /* TRS_MODE_* */
  int32_t block;             /* threads per workgroup: 64..1024, multiple of
                                64; 0 = tuned default */
  int32_t nodes_per_thread;  /* slots swept per thread per tile: 1,2,4,8,16;
                                0 = tuned default */
  int32_t rounds_per_poll;   /* rounds issued between host checks of the
                                device done flag; 0 = adaptive */
  int64_t max_rounds;        /* 0 = unlimited; else rounds 0..max_rounds-1 may
                                run, and a run that has not reached its normal
                                forms by then stops with TRS_E_ROUNDS (checked
                                on the device at every round) */
  float threshold;           /* learned mode: keep a node when p >= threshold */
  int32_t persistent;        /* 1 = one cooperative persistent kernel runs the
                                rounds with device-wide barriers; 0 = one
                                launch per round (captured in a HIP graph) */
  int32_t trace;             /* plain mode: 0 = off; k in 1..65536 = log a
                                record for a blocked node-round with
                                probability k/65536 (for training the
                                predictor; the memo shortcut is off then) */
  int64_t trace_cap;         /* records kept (0 = 1<<24); later ones dropped */
  int32_t label_horizon;     /* tracing: a record is labelled 1 when its node
                                fires or becomes a normal form within this
                                many rounds (0 = 1: the next round) */
  int32_t sweep_every;       /* learned mode: also sweep every slot every k
                                rounds (0 or -1 = never: only when the
                                frontier is empty or a round stalls); a node
                                the predictor drops is woken by the
                                notification of the argument it waits on, so
                                these sweeps are a safety net */
  int32_t max_grid;          /* most workgroups a round launch uses (0 = 8 per
                                compute unit); larger grids keep more sweep
                                tiles in flight, smaller ones fewer idle
                                workgroups in frontier rounds */
  int32_t pf_depth;          /* with 16 nodes per thread: most sweep tiles a
                                workgroup copies ahead into LDS (1..4; 0 = as
                                many as fit, at most 4; -1 = none, each tile
                                read straight into registers) */
  int32_t nf_walk;           /* frontier and learned modes, rounds that one
                                workgroup runs alone: a node that becomes a
                                normal form marks up to this many constructors
                                above it (symbols without rules whose other
                                arguments are normal forms) in the same
                                round, walking up the parent hints; a longer
                                chain goes on in the next round (0 = 256;
                                -1 = off: one round per constructor) */
  int32_t cont_passes;       /* frontier and learned modes with the walk on,
                                rounds that one workgroup runs alone: a
                                workgroup that creates a node ready at birth
                                (all arguments normal forms), or rewrites one
                                into a node that is ready again, examines it
                                in a further pass of the same round rather
                                than the next round, up to this many further
                                passes per round (0 = 64; -1 = none) */
  int32_t nf_walk_wide;      /* nf_walk for rounds that several workgroups
                                run, where a walk holds up every term's round
                                (0 = 1; -1 = off) */
  int32_t cont_passes_wide;  /* cont_passes for rounds that several
                                workgroups run (0 or -1 = none) */
  int32_t place_fresh;       /* placement of new nodes: 0 (default) = slots
                                recycled by collection first, fresh slots past
                                the extent n when none are left; k in 1..100 =
                                fresh slots first while n is below k% of the
                                pool, so that the nodes a round creates lie
                                next to each other (locality), at the price of
                                a larger extent */
} trs_opts;

typedef struct {
  int64_t rounds;        /* rewrite rounds until the confirmation round */
  int64_t rule_apps;     /* rule applications (the paper's rewritten terms) */
  int64_t node_visits;   /* slots examined, summed over rounds */
  int64_t active_visits; /* visited slots that were live and not in normal form */
  int64_t allocs;        /* nodes created */
  int64_t frees;         /* nodes returned to the free list */
  int64_t peak_slots;    /* highest slot extent n reached */
  int64_t gc_rounds;     /* rounds that collected at least one node */
  int64_t mlp_evals;     /* learned mode: predictor evaluations */
  int64_t full_sweeps;   /* frontier modes: full confirmation sweeps */
  int64_t launches;      /* kernel launches issued for the round loop */
  int64_t ready_visits;  /* active slots whose arguments were all normal forms */
  int64_t nf_set;        /* slots that became normal forms without a rule */
  int64_t rc_atomics;    /* reference-count atomic operations */
  int64_t memo_blocked;  /* active slots found still blocked by the argument
                            recorded at their previous examination */
  int64_t mlp_kept;      /* learned mode: predictor decisions that kept the node */
  int64_t trace_records; /* trace records logged (may exceed trace_cap) */
  int64_t nf_walked;     /* constructors marked normal forms by the walk of
                            trs_opts.nf_walk (not counted in nf_set) */
  int64_t last_progress_round; /* last round in which a node fired or became a
                            normal form; the rounds after it only collected
                            garbage and confirmed the normal forms */
  double device_ms;      /* device time of the round loop (HIP events) */
} trs_stats;

/* Create a context.  No device memory is touched until trs_normalize, so rule
 * and term validation also work on a host without a GPU. */
trs_status trs_create(trs_ctx **out, const trs_config *cfg);
void trs_destroy(trs_ctx *ctx);

/* Load and compile the rewrite system (Section 2, Definition 1; rule order is
 * the matching priority).  Inputs are copied; the caller keeps ownership.
 * Validates: lhs not a variable, Var(rhs) within Var(lhs), left-linear lhs,
 * well-formed prefix codes, arities within maxarity; compiles per-symbol
 * decision tables (TRS_E_LIMIT beyond the TRS_MAX_* limits). */
trs_status trs_load_rules(trs_ctx *ctx, int32_t n_sym, const int32_t *arity, int32_t n_rules,
                          const int32_t *rule_off, const int32_t *rule_code, int64_t code_len);

/* Load the ground input terms (Section 2: a term over the signature with no
 * variables; its innermost normal form is what trs_normalize computes).
 * term_code is the concatenation of the terms' prefix codes (pre-order symbol
 * ids, int32); term t occupies term_code[term_off[t] .. term_off[t+1]) and
 * term_off has n_terms + 1 entries.  Inputs are copied; the caller keeps
 * ownership.  Each term is stored as a tree of nodes (one slot per symbol
 * occurrence, Section 3's node arrays) with its own root entry, which holds
 * one reference; all terms share one node pool.  Errors: TRS_E_STATE before
 * trs_load_rules, TRS_E_ARG for null pointers or offsets outside code_len,
 * TRS_E_TERM for an empty term, a variable (code < 0), an unknown symbol or
 * a prefix code that does not parse, TRS_E_POOL if the initial graph does
 * not fit in pool_slots - 1 slots.  A failed call leaves no terms loaded. */
trs_status trs_load_terms(trs_ctx *ctx, int32_t n_terms, const int64_t *term_off,
                          const int32_t *term_code, int64_t code_len);

/* Normalise all loaded terms on the device: the round-synchronous innermost
 * method of Section 3 (every node whose arguments are all normal forms is
 * matched against its head symbol's rules in order and the first match is
 * contracted in place; reference counts are adjusted and nodes whose count
 * reaches zero are collected and their indices reused; rounds repeat until a
 * round finds no node that is not a normal form).  The result is the
 * innermost normal form of each term (Section 2, Definition 2 and the
 * derive / rewrite_f procedures), identical whatever the mode and launch
 * shape.  opts may be NULL (trs_default_opts); stats may be NULL.  Device
 * work is issued on the context's stream and complete when the call
 * returns.  Errors: TRS_E_STATE before trs_load_terms, TRS_E_ARG for option
 * values outside their documented ranges, TRS_E_POOL when the pool runs out
 * of slots, TRS_E_ROUNDS at opts->max_rounds, TRS_E_HIP for runtime errors
 * (message in trs_last_error).  After an error the pool contents are
 * unspecified; the next trs_normalize starts again from the loaded terms. */
trs_status trs_normalize(trs_ctx *ctx, const trs_opts *opts, trs_stats *stats);

/* Read back the normal form of term term_id (0 .. n_terms-1) computed by the
 * last successful trs_normalize, as its canonical serialisation: the prefix
 * sequence of symbol ids of the term with every shared node expanded (the
 * term itself of Section 2; sharing of Section 3 is not visible).  buf is
 * caller-owned host memory of cap int32 entries; with buf == NULL only
 * *len_out is set.  Errors: TRS_E_STATE before a successful trs_normalize,
 * TRS_E_ARG for a bad term_id, a null len_out or cap < length,
 * TRS_E_INTERNAL if the pool is inconsistent (a reachable node that is not a
 * normal form or a dangling index). */
trs_status trs_read_nf(trs_ctx *ctx, int32_t term_id, int32_t *buf, int64_t cap,
                       int64_t *len_out);

/* The node pool after the last successful trs_normalize, for checking the
 * method's invariants from the host (Section 3: the node arrays, the
 * reference counts and the free-index list that collection fills and
 * allocation reuses).  info receives the slot extent n (slots 1..n-1 have
 * been used; slot 0 never is), maxarity, the number of terms and the sizes
 * of the two free-index stacks.  Each other pointer is caller-owned host
 * memory, or NULL to skip that array: hss[n], args[n * maxarity]
 * (maxarity-strided; entries past a symbol's arity unspecified), state[n]
 * (bit 7: normal form; 0x00: free; bit 1 a round marker, bits 3-5 a memo),
 * rc[n], free0[info.free0], free1[info.free1] (the free slot indices) and
 * roots[n_terms] (the root slot of each term, which holds one reference).
 * Call once with NULL arrays to learn the sizes.  Copies device memory;
 * meant for tests and debugging, not for the hot path.  Errors:
 * TRS_E_STATE before a successful trs_normalize, TRS_E_ARG for a null
 * ctx or info, TRS_E_HIP for a failed copy. */
typedef struct {
  int64_t n;
  int64_t free0, free1;
  int32_t maxarity;
  int32_t n_terms;
} trs_pool_info;

trs_status trs_read_pool(trs_ctx *ctx, trs_pool_info *info, int32_t *hss, int32_t *args,
                         uint8_t *state, int32_t *rc, int32_t *free0, int32_t *free1,
                         int32_t *roots);

/* Rule applications per rule of the last trs_normalize (out[0..n_rules)). */
trs_status trs_rule_counts(trs_ctx *ctx, int64_t *out, int32_t cap);

/* Device bytes a context with this pool size and maxarity needs when the
 * caller supplies dev_mem (trs_config.dev_mem / dev_bytes).  Pure host
 * arithmetic; returns -1 for invalid sizes. */
int64_t trs_device_bytes(int64_t pool_slots, int32_t maxarity);

/* Default options (mode plain, tuned block and nodes per thread). */
void trs_default_opts(trs_opts *opts);

/* Autotuner of the launch shape (the batching step: block size and nodes
 * per thread; max_grid is part of the result).  Times complete trs_normalize
 * runs of the loaded terms under *base, walking the block x nodes-per-thread
 * grid in two stages: block sizes 64, 128, 256, 512, 1024 at 16 nodes per
 * thread, then 1, 2, 4 and 8 nodes per thread at the best block (nine runs,
 * default grid).  Plain mode, whose large rounds are classified by the scan
 * kernel and examined as lists, leaves out block 1024 and one node per
 * thread (seven runs).  *best
 * receives *base with the fastest block, nodes_per_thread and max_grid.  The
 * result is cached per context and loaded terms (a second call with the same
 * mode returns it without trials; res->trials = 0 then).  After the call the
 * context holds a completed normalisation. */
typedef struct {
  int32_t trials;       /* configurations timed by this call */
  int32_t best_block;
  int32_t best_npt;
  int32_t pad;
  double best_ms;       /* device time of the fastest trial */
  int32_t block[16], npt[16];
  double ms[16];        /* device time per trial */
  int32_t best_grid;    /* max_grid of the fastest trial (0 = default) */
  int32_t pad2;
  int32_t grid[16];
} trs_tune_result;

trs_status trs_autotune(trs_ctx *ctx, const trs_opts *base, trs_opts *best,
                        trs_tune_result *res);

/* Memory microbenchmarks of a device: the paper's comparison of aligned and
 * random-access bandwidth (Section 4, hardware table), re-measured on this
 * GPU, plus the latencies that bound one rewrite round.  Allocates and frees
 * about 2 GiB of device memory; takes a few seconds. */
typedef struct {
  double stream_read_gbps;      /* coalesced 16-byte reads of 2 GiB */
  double gather4_hbm_gops;      /* random 4-byte reads over 2 GiB, 1e9/s */
  double gather4_llc_gops;      /* random 4-byte reads over 64 MiB, 1e9/s */
  double gather1_llc_gops;      /* random 1-byte reads over 64 MiB, 1e9/s */
  double atomic_random_gops;    /* random non-returning atomic adds, 1e9/s */
  double load_latency_far_ns;   /* dependent load, 512 MiB random cycle (one
                                   wave, 64 independent chains) */
  double load_latency_near_ns;  /* dependent load, 256 KiB random cycle */
  double atomic_latency_ns;     /* dependent returning atomic (64 chains) */
  double empty_kernel_us;       /* back-to-back launch of an empty kernel */
  double copy_gbps;             /* plain device copy (bytes read + written) */
  int64_t copy_bytes;           /* bytes that copy read (and wrote) per launch */
  double clock_mhz;
  int64_t l2_bytes;
  int32_t cu_count;
  int32_t pad;
} trs_membench_result;

trs_status trs_membench(int32_t device, trs_membench_result *out);

/* ------------------------------------------------------------------------
 * Frontier predictor (TRS_MODE_LEARNED).  Not part of the paper: a small
 * network that predicts, for a node examined and found blocked in a round
 * (an argument not yet a normal form), whether it will fire or become a
 * normal form in the next round (the label horizon); only nodes it keeps
 * are examined in the next round, the others when the argument they wait on
 * becomes a normal form (parent notification) or at the next full sweep,
 * and a full sweep still confirms the normal form (so results stay exact).
 * Nodes created or rewritten blocked are left to notification alone.
 *
 *   x  = [E[sym] (16), arity/8, c_0..c_4, bucket(age)/15, 0]       (24)
 *   h1 = relu(W1 x + b1) (32);  h2 = relu(W2 h1 + b2) (32)
 *   p  = sigmoid(w3 . h2 + b3)
 *
 * c_j = 1 when argument j is a normal form or j >= arity; age = rounds since
 * the node last changed, bucket(0) = 0, bucket(a) = min(15, floor(log2 a)+1).
 * Parameters are bfloat16 (uint16 bit patterns), concatenated in the order
 * E[n_sym][16], W1[32][24], b1[32], W2[32][32], b2[32], w3[32], b3[1]
 * (row-major); arithmetic accumulates in float32.
 *
 * Trace record (uint64, written by trs_normalize with trs_opts.trace > 0):
 * sym bits 0-15, arity 16-19, c_0..c_4 bits 20-24, age bucket 25-28, label
 * bit 32 (1: the node fired or became a normal form within
 * trs_opts.label_horizon rounds; a node's later record supersedes its
 * earlier one).
 * ------------------------------------------------------------------------ */
#define TRS_MLP_EMB 16
#define TRS_MLP_DIN 24
#define TRS_MLP_H 32
#define TRS_MLP_MAX_SYM 256   /* learned mode keeps the decision table in LDS */

/* Number of bfloat16 parameters for n_sym symbols; -1 if n_sym is outside
 * 1..TRS_MLP_MAX_SYM. */
int64_t trs_mlp_param_count(int32_t n_sym);

/* Forward (and backward) pass on device `device` over n records (host
 * arrays, copied in): mean binary cross-entropy in *loss_out; if grads_out is
 * not NULL, the gradient of that mean with respect to every parameter
 * (float32, parameter order above); if probs_out is not NULL, p per record.
 * TRS_E_ARG on null inputs, n <= 0 or a record whose symbol is >= n_sym. */
trs_status trs_mlp_eval(int32_t device, int32_t n_sym, const uint16_t *params_bf16, int64_t n,
                        const uint64_t *records, double *loss_out, float *grads_out,
                        float *probs_out);

typedef struct {
  int32_t epochs;   /* passes over the training part, 1..64 */
  int32_t batch;    /* records per Adam step, >= 64 */
  float lr;         /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
  float val_frac;   /* trailing fraction of the records held out, [0, 1) */
} trs_train_opts;

typedef struct {
  int32_t epochs_run;
  int32_t pad;
  float train_loss[64];  /* mean loss over each epoch's steps */
  float val_loss[64];    /* loss on the held-out records after each epoch */
  double device_ms;      /* device time of the whole training */
} trs_train_result;

/* Train the predictor on the device with Adam on float32 master weights
 * (rounded to bfloat16 after every step) from init_bf16; the records are
 * used in the given order (shuffle them first).  Writes the trained
 * parameters to params_out. */
trs_status trs_mlp_train(int32_t device, int32_t n_sym, int64_t n, const uint64_t *records,
                         const trs_train_opts *opts, const uint16_t *init_bf16,
                         uint16_t *params_out, trs_train_result *result);

/* The predictor evaluated on the device for every input it can see:
 * probs_out[(sym * 32 + c) * 16 + bucket] (n_sym * 512 floats, may be NULL)
 * and the keep decisions p >= threshold as a bit table words_out (n_sym * 16
 * uint32; bit i of word i/32; may be NULL).  arity[sym] gives the arity fed
 * to the network. */
trs_status trs_mlp_table(int32_t device, int32_t n_sym, const int32_t *arity,
                         const uint16_t *params_bf16, float threshold, float *probs_out,
                         uint32_t *words_out);

/* trs_mlp_eval for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, arguments and results as trs_mlp_eval (host arrays,
 * copied in and out; work on the null stream, complete on return), with
 * every device buffer -- parameters, records, gradient and loss
 * accumulators, probabilities -- in a static device array of the library
 * (about 0.8 MB per device, held until the process ends).  The call makes no
 * hipMalloc or hipFree.  At most TRS_MLP_NOALLOC_MAX_RECORDS records per call
 * (TRS_E_LIMIT above).  Calls on one device share that array: calls that
 * overlap in time on the same device race and must be serialised by the
 * caller. */
#define TRS_MLP_NOALLOC_MAX_RECORDS 65536
trs_status trs_mlp_eval_noalloc(int32_t device, int32_t n_sym, const uint16_t *params_bf16,
                                int64_t n, const uint64_t *records, double *loss_out,
                                float *grads_out, float *probs_out);

/* Install predictor parameters in a context (copied; n_params must equal
 * trs_mlp_param_count of the loaded system).  Required before a
 * TRS_MODE_LEARNED trs_normalize. */
trs_status trs_set_predictor(trs_ctx *ctx, const uint16_t *params_bf16, int64_t n_params);

/* Trace records of the last trs_normalize run with trs_opts.trace > 0, in
 * the order they were logged (labels complete).  With buf == NULL only
 * *n_out is set; otherwise min(cap, count) records are copied. */
trs_status trs_read_trace(trs_ctx *ctx, uint64_t *buf, int64_t cap, int64_t *n_out);

const char *trs_status_str(trs_status s);
const char *trs_last_error(trs_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* TRS_H */
