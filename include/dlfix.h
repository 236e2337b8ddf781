/* dlfix -- semiring Datalog fixpoint engine for AMD MI355X (gfx950).
 *
 * C ABI of the shared library libdlfix.so.  Every call returns a dl_status
 * (DL_OK = 0); no C++ exception crosses this boundary.  The text of the last
 * error of an engine is available from dl_last_error().
 *
 * The library evaluates positive Datalog programs bottom-up to their least
 * fixpoint, semi-naively (Sec. 3.4: rules fire only on the facts that changed
 * in the previous iteration; Appendix A: the stable / recent / delta split of
 * the database and of every join).  Relations are columnar: an arity-n
 * relation is n integer columns plus one tag column (Sec. 3.3), held in HBM
 * as a sorted array of packed integer keys plus a tag array.  Every fact
 * carries a provenance tag from a semiring (T, 0, 1, +, x) (Sec. 3.1,
 * Sec. 3.5); a derived fact's tag is the +-sum over its derivations of the
 * x-product of the body tags.
 *
 * Threading: one engine per host thread; calls on one engine must not
 * overlap.  All device work of an engine runs on the stream given in
 * dl_options (or on a stream the engine creates).
 */
#ifndef DLFIX_H
#define DLFIX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dl_engine dl_engine; /* opaque; created by dl_load_program, freed by dl_free */

typedef enum {
  DL_OK = 0,
  DL_ERR_ARG = 1,             /* bad argument (NULL pointer, unknown relation, size mismatch) */
  DL_ERR_PARSE = 2,           /* program text does not parse */
  DL_ERR_UNSUPPORTED = 3,     /* construct outside the supported fragment (see dl_load_program) */
  DL_ERR_STATE = 4,           /* call out of order (e.g. read before run) */
  DL_ERR_NOMEM = 5,           /* device allocation failed or the workspace is full; the engine and its
                                 facts stay valid: rerun after dl_set_workspace with a larger block */
  DL_ERR_CAPACITY = 6,        /* a size exceeds an index width (e.g. > 2^32 join outputs in one round) */
  DL_ERR_PROOF_OVERFLOW = 7,  /* top-k: more than 256 probabilistic facts in one sample */
  DL_ERR_HIP = 8              /* a HIP runtime call failed */
} dl_status;

/* Provenance semirings (Sec. 3.1, Sec. 3.5).  Tags are binary32.
 *  BOOL          {false, true}, +: or, x: and.  No tag is stored.
 *  MAXMIN        [0,1], +: max, x: min.
 *  MINPLUS       [0, inf], +: min, x: + (tropical; weights as tags).
 *  ADDMULT       [0,1], +: min(1, a+b), x: a*b.
 *  DIFF_ADDMULT  ADDMULT with reverse-mode gradients (dl_backward).
 *  TOPK          up to k <= 3 proofs per fact; a proof is a set of input facts
 *                (bitset over the <= 256 probabilistic facts of its sample: one
 *                64-bit word while every sample has <= 64, else four),
 *                its probability the binary32 product of those facts'
 *                probabilities in ascending fact order.  x: pairwise unions,
 *                + : union of the lists; both keep the k most likely distinct
 *                proofs (ties: smaller bitset first).
 *  DIFF_TOPK     TOPK with the gradient of the inclusion-exclusion
 *                probability of the kept proofs.
 *  DIFF_MAXMIN   MAXMIN with gradients (Sec. 3.5): a tag is a pair (value,
 *                fact number), the value being the probability of one input
 *                fact, numbered over all relations in dl_add_facts order from
 *                0 (since the last dl_clear_facts).  x keeps the smaller value,
 *                + the larger; equal values keep the smaller fact number, so
 *                the result does not depend on evaluation order.  The
 *                derivative of a tag is 1 for its fact and 0 for all others.
 * BOOL, MAXMIN, MINPLUS, DIFF_MAXMIN and the TOPK forms have an idempotent + and are
 * iterated until no tag changes; the ADDMULT forms fix a fact's tag in the
 * iteration that first derives it (later derivations do not change it). */
typedef enum {
  DL_BOOL = 0,
  DL_MAXMIN = 1,
  DL_MINPLUS = 2,
  DL_ADDMULT = 3,
  DL_DIFF_ADDMULT = 4,
  DL_TOPK = 5,
  DL_DIFF_TOPK = 6,
  DL_DIFF_MAXMIN = 7
} dl_semiring;

typedef struct {
  int semiring;       /* dl_semiring */
  int k;              /* top-k proof count, 1..3 (ignored otherwise; 0 = 3) */
  int batched;        /* 1: every fact carries a sample id; samples never join each other (Sec. 4.3) */
  void* stream;       /* hipStream_t to run on; NULL: the engine creates its own stream */
  int dedup;          /* per-round deduplication of derived relations:
                         0 = automatic (dense-domain when the packed key domain of the relation
                             is at most 2^30 and the semiring is not a top-k form or DIFF_MAXMIN,
                             else sort-based),
                         1 = always sort-based (radix sort, unique, difference, merge),
                         2 = dense-domain wherever possible,
                         3 = hash-set (Sec. 5): each round's candidates go into a hash set that
                             folds their tags, then only the distinct keys are sorted; f32 tags
                             or none, without recorded lineage (otherwise sort-based) */
  int no_graphs;      /* 1: never replay round bodies as captured HIP graphs (0: replay where eligible;
                         the fused rounds' graphs stay in the engine from run to run while their
                         launches' arguments are unchanged, and go with dl_free) */
  int no_fused;       /* 1: never run a round as one fused launch (0: where the stratum has one
                         static-driven join whose derivations fall into per-group windows) */
  int lineage;        /* DIFF_ADDMULT derivation lineage for dl_backward:
                         0 = automatic (recorded during the run; dropped and recomputed round by
                             round in dl_backward once it would exceed lineage_budget),
                         1 = always recorded (12 bytes per discovery derivation),
                         2 = never recorded: dl_backward re-runs each round's joins on the
                             relation as it stood then (rebuilt from discovery ids) */
  size_t lineage_budget;  /* lineage = 0: bytes of recorded lineage allowed before it is dropped
                             (0: a quarter of the device memory free at creation, or of the workspace) */
  void* workspace;        /* device memory the engine keeps ALL its device buffers in (facts, relations,
                             indexes, round scratch), e.g. a torch tensor's storage; borrowed until
                             dl_free or dl_set_workspace.  The engine then never calls hipMalloc /
                             hipFree: buffers are ranges of this block, reused across iterations and
                             runs (Sec. 4.1, buffer reuse), and growing a buffer never waits for the
                             stream.  Its contents on entry do not matter.  NULL: the engine makes
                             its own hipMalloc allocations. */
  size_t workspace_bytes; /* size of `workspace` in bytes (at least 256) */
  uint64_t max_join_outputs; /* outputs of one join launch before its probe rows are split into chunks
                                (0: 2^32 - 1, the reach of the 32-bit offsets); smaller values only serve
                                to test the chunked path */
  int exact_growth;       /* 1: buffers grow to exactly the size asked (no 25% margin), so that they are
                             regrown more often (tests of the regrowth paths) */
} dl_options;

/* Result columns of dl_read_relation.  Any pointer may be NULL (not written).
 * Rows come in canonical lexicographic order (sample, col0, col1, ...). */
typedef struct {
  uint32_t* sample_ids;   /* [n] (batched engines) */
  uint32_t* columns[4];   /* columns[c][n] for c < arity */
  float* tags;            /* [n]: the tag (f32 semirings), 1.0 (BOOL), or the
                             inclusion-exclusion probability of the kept proofs (TOPK) */
  uint8_t* topk_count;    /* [n]   number of kept proofs (TOPK) */
  uint64_t* topk_bits;    /* [k*n*W], W = dl_stats.topk_words: word w of proof j of row i at
                             [(j*n + i)*W + w]; fact f of the row's sample is bit f % 64 of word f / 64 */
  float* topk_prob;       /* [k*n] binary32 proof probabilities, same layout */
  uint32_t* fact_ids;     /* [n] DIFF_MAXMIN: the number of the input fact each tag comes from
                             (not written for the other semirings) */
} dl_relation_out;

typedef struct {
  int strata;             /* strata evaluated in the last run */
  int rounds;             /* iterations over all strata (each stratum counts its final, empty one) */
  int max_rounds;         /* largest iteration count of a single stratum */
  uint64_t candidates;    /* join outputs (derivations) produced, all rounds */
  uint64_t unique;        /* distinct candidate keys after the per-round +-reduction */
  uint64_t derived;       /* tuples in derived relations at the fixpoint */
  uint64_t lineage;       /* derivations recorded for the backward pass (DIFF_ADDMULT) */
  double run_ms;          /* host wall time of the last dl_run_fixpoint */
  uint64_t device_bytes;  /* device memory currently held by the engine */
  uint32_t key_bits;      /* width of the packed keys (32 or 64) */
  uint32_t id_bits;       /* bits per column value */
  uint32_t sample_bits;   /* bits of the sample id */
  int dedup;              /* deduplication setting in force (see dl_options.dedup) */
  int orient;             /* delta-plan orientation in force: 0 auto, 1 recent-driven, 2 static-driven */
  int items;              /* join expand tile in force: outputs per thread */
  double tuned_ms;        /* median run time of the configuration dl_autotune chose */
  int lineage_mode;       /* DIFF_ADDMULT after the last run: 1 lineage recorded, 2 recomputed in
                             dl_backward (0 for the other semirings) */
  int rows;               /* row-window joins in force: 0 off, 1 for launches with many derivations
                             per window (default), 2 wherever they apply */
  uint64_t device_allocs; /* hipMalloc calls the engine has made since creation (0 with a workspace) */
  uint64_t workspace_peak;/* largest number of workspace bytes in use at once (0 without a workspace) */
  int index;              /* join indexes in force: 0 CSR offsets over the prefix domain (a hash index
                             where that domain passes 2^30), 1 hash indexes (Sec. 5) */
  int topk_words;         /* top-k forms: 64-bit words per proof set in the last run (1 while every
                             sample has at most 64 probabilistic facts, else 4: up to 256); 0 otherwise */
} dl_stats;

/* Kernel families timed by dl_profile (bit i of the mask = family i). */
typedef enum {
  DL_K_JOIN_COUNT = 0,    /* matches per probe row */
  DL_K_JOIN_EXPAND = 1,   /* load-balanced expand + gather + tag product */
  DL_K_SORT_HIST = 2,     /* radix sort: per-tile digit histograms */
  DL_K_SORT_SCATTER = 3,  /* radix sort: stable ranking + scatter */
  DL_K_SCAN = 4,          /* device-wide exclusive scans */
  DL_K_REDUCE = 5,        /* segment heads + per-key +-reduction */
  DL_K_DIFF = 6,          /* difference / +-merge against the full relation */
  DL_K_MERGE = 7,         /* merge-path merge into the full relation */
  DL_K_COMPACT = 8,       /* stream compaction, flags, lineage emission */
  DL_K_INDEX = 9,         /* index build (permute, CSR) */
  DL_K_BACKWARD = 10,     /* gradient kernels */
  DL_K_FAMILIES = 11
} dl_kernel_family;

typedef struct {
  uint64_t launches;      /* timed launches since the last dl_profile call */
  double ms;              /* summed event-to-event time of those launches */
  double bytes;           /* summed algorithmic bytes (minimum reads + writes) */
} dl_kernel_timing;

/* Parse and plan a program: the RAM program of Algorithm 1 (rules as
 * relational-algebra operators over columnar relations, Sec. 3.3; strata
 * evaluated one after the other, each to its fixpoint).
 * Text: one statement per '.'-terminated clause; '#' or '//' start comments.
 *   .input name/arity           declares an input (extensional) relation
 *   .output name/arity          optional; any derived relation can be read
 *   head(x, y) :- a(x, z), b(z, y).
 * Supported fragment: positive rules; 1 to 3 body atoms; arity 1..4;
 * variables only (no constants), pairwise distinct inside an atom; every
 * head variable occurs in the body; every body atom after the first shares a
 * variable with the atoms before it.  Strata are the strongly connected
 * components of the predicate graph, evaluated in dependency order
 * (Algorithm 1).  DIFF_ADDMULT rules have at most 2 body atoms (a recorded
 * derivation holds two body ids).
 * Anything else returns DL_ERR_UNSUPPORTED.  On success *out owns a new
 * engine (free with dl_free). */
dl_status dl_load_program(const char* program_text, const dl_options* opts, dl_engine** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * dl_load_program, but the engine keeps ALL its device buffers in the
 * library's own static array on the current device, DL_STATIC_WORKSPACE_MIB
 * MiB large, which every device the library runs on holds until the process
 * ends.  Neither this call nor any later call on the engine calls hipMalloc,
 * hipFree, hipHostMalloc or any other allocating routine, and the engine
 * creates no stream (opts->stream NULL means the null stream).
 * opts->workspace must be NULL (else DL_ERR_ARG).
 * Limits: inputs whose buffers do not fit the array give DL_ERR_NOMEM with a
 * message naming the static workspace; dl_set_workspace is refused
 * (DL_ERR_STATE).  The array is shared by all such engines on a device and
 * keeps the contents of the last one (the engine clears what must start at
 * zero): each call of dl_load_program_static hands it to the new engine, and
 * every later call on an earlier engine of that device returns DL_ERR_STATE.
 * Calls on such engines that overlap in time on one device race. */
#define DL_STATIC_WORKSPACE_MIB 128
dl_status dl_load_program_static(const char* program_text, const dl_options* opts, dl_engine** out);

/* Drop all facts and results, keep the program (and every device buffer, for
 * reuse by the next facts: Sec. 4.1, buffer reuse across runs). */
dl_status dl_clear_facts(dl_engine* e);

/* Append n facts to input relation `relation` (the extensional database F_T
 * that Algorithm 1 takes as input; one column array per attribute, Sec. 3.3
 * columnar relations; in batched engines a sample-id column, Sec. 4.3).
 * columns: `arity` pointers to n uint32 values each (SoA).
 * sample_ids: n values (batched engines; ignored otherwise, may be NULL).
 * tags: n binary32 values (probability / weight); NULL allowed for BOOL.
 * on_device: 1 if every pointer is device memory, 0 if host memory.  The data
 * is copied before the call returns.  Duplicate facts are +-merged. */
dl_status dl_add_facts(dl_engine* e, const char* relation, size_t n,
                       const uint32_t* sample_ids, const uint32_t* const* columns,
                       const float* tags, int on_device);

/* Evaluate every stratum to its fixpoint (Algorithm 1: stable = {}, recent =
 * F_T, then semi-naive iterations until an iteration adds or changes nothing;
 * Appendix A for the stable / recent / delta joins of one iteration).
 * Blocks until the result is on the device (small device-to-host reads of
 * counts, at most one per join step and per iteration).  DL_ERR_NOMEM: a
 * buffer did not fit (device memory or workspace); the facts are kept and the
 * call can be repeated, after dl_set_workspace where a workspace is used. */
dl_status dl_run_fixpoint(dl_engine* e);

/* Move the engine's device buffers into a new workspace block (p != NULL,
 * `bytes` long, contents irrelevant) or into separate hipMalloc allocations
 * (p == NULL); the previous block is no longer used when the call returns
 * (the call waits for the engine's stream).  Facts, results and indexes are
 * kept.  DL_ERR_NOMEM (nothing moved) when the live buffers do not fit.
 * This is the recovery path after a run returned DL_ERR_NOMEM (Sec. 4.1:
 * the engine's memory is one arena whose buffers are reused). */
dl_status dl_set_workspace(dl_engine* e, void* p, size_t bytes);

/* Number of tuples of a relation (after dl_run_fixpoint for derived ones):
 * |F_T| restricted to one relation at the fixpoint (Algorithm 1 result). */
dl_status dl_relation_size(dl_engine* e, const char* relation, size_t* n);

/* Copy a relation out (see dl_relation_out): the derived facts of the
 * fixpoint with their tags (Algorithm 1 result; per sample in batched
 * engines, Sec. 4.3; top-k tags as their kept proofs, Sec. 3.5).  The engine
 * keeps each relation as sorted packed keys; the columns are unpacked here
 * (Sec. 3.3 columnar layout).  `capacity` rows are available
 * in every given buffer; fewer than the relation size gives DL_ERR_ARG.
 * on_device selects device (1) or host (0) pointers for all buffers. */
dl_status dl_read_relation(dl_engine* e, const char* relation, size_t capacity,
                           const dl_relation_out* out, int on_device, size_t* n_written);

/* Point queries (a lookup of the result database, Sec. 3.3 relations held
 * sorted): for n tuples given as columns (SoA; sample ids for batched
 * engines) write rows[i] = the tuple's row in canonical order or -1 when it
 * is not in the relation, and tags[i] = its tag as in dl_read_relation (0 when
 * absent).  Either output may be NULL.  Binary search over the sorted result:
 * no copy of the relation. */
dl_status dl_lookup(dl_engine* e, const char* relation, size_t n, const uint32_t* sample_ids,
                    const uint32_t* const* columns, int64_t* rows, float* tags, int on_device);

/* Reverse mode seeded on selected rows (e.g. from dl_lookup; rows < 0 or at
 * least the relation's size are skipped): d(loss)/d(tag of row rows[i]) = grad[i].  Same accumulation as
 * dl_backward (Sec. 3.5, differentiable semirings). */
dl_status dl_backward_rows(dl_engine* e, const char* relation, size_t n, const int64_t* rows, const float* grad,
                           int on_device);

/* Reverse mode for DIFF_ADDMULT, DIFF_TOPK and DIFF_MAXMIN (Sec. 3.5: differentiable
 * provenance semirings, whose tags carry derivatives with respect to the input
 * facts' probabilities; computed here in reverse mode over the recorded or
 * recomputed derivations): grad_out[i] is d(loss)/d(tag)
 * of row i of out_relation in canonical order.  Gradients with respect to the
 * input facts' tags are accumulated (+=) into the engine until dl_zero_grad.
 * DIFF_ADDMULT sweeps the discovery derivations round by round in reverse
 * (a tuple's tag is the clamped sum over the derivations of the round that
 * found it); without recorded lineage (dl_options.lineage) each round's
 * derivations are recomputed first, which costs about one forward join pass.
 * DIFF_MAXMIN adds grad_out[i] to the fact that row i's tag comes from. */
dl_status dl_backward(dl_engine* e, const char* out_relation, const float* grad_out, int on_device);

/* Accumulated input gradients of an input relation, in dl_add_facts order
 * (the derivative of the loss with respect to each input fact's probability,
 * Sec. 3.5). */
dl_status dl_read_grad(dl_engine* e, const char* in_relation, float* grad_in, int on_device);

dl_status dl_zero_grad(dl_engine* e);

dl_status dl_get_stats(const dl_engine* e, dl_stats* out);

/* Autotuner.  Times dl_run_fixpoint on the current facts under every
 * candidate execution configuration -- deduplication (sort-based or
 * dense-domain; hash-set for the fastest sort-based one), orientation of the delta joins of 2-atom rules (recent
 * tuples probe the static side, or the static side probes an index over the
 * recent tuples), the join expand tile (1, 2, 4 or 8 outputs per thread),
 * for dense heads of static-driven joins whether derivations are folded per
 * head-key window in LDS (row windows) or scattered with global atomics, and
 * (for the fastest of those) CSR offsets or hash indexes for the joins --
 * and keeps the fastest (median of `trials` runs after a warm-up run) for
 * later runs.  All candidates compute the same relations.  If cache_path is
 * not NULL the choice is first looked up there, keyed by a hash of the program
 * text, the semiring, the key layout and log2 of the fact count, and stored
 * there (one JSON object per line) after tuning.  Ends with a run under the
 * chosen configuration. */
dl_status dl_autotune(dl_engine* e, int trials, const char* cache_path);

/* Time the kernel families in `family_mask` with HIP events recorded on the
 * engine's stream around each launch (0 switches timing off); fused rounds
 * replayed as a graph are timed by events around each replay, which count as
 * its launches.  Resets the totals; later dl_run_fixpoint and dl_backward
 * calls add to them. */
dl_status dl_profile(dl_engine* e, uint32_t family_mask);

/* Totals of one kernel family since the last dl_profile call. */
dl_status dl_get_kernel_timing(const dl_engine* e, int family, dl_kernel_timing* out);

/* Per-round sizes of the last dl_run_fixpoint (Alg. 1: one entry per
 * iteration), in order over the strata: tuples new or changed by the round,
 * its derivations (join outputs; UINT64_MAX where they were only counted in
 * total on the device: batched rounds) and info = stratum << 8 | kind, kind
 * DL_ROUND_FIRST (a stratum's first round), DL_ROUND_PLAIN (a later round of
 * separate launches), DL_ROUND_FUSED (one launch of the fused round kernel;
 * the launches of a final batch after the stratum's last round are listed
 * too and find nothing) or DL_ROUND_BATCHED (a round of a device-sized
 * batch).  For relating a kernel trace's launches to their work.  Writes
 * min(capacity, entries) entries to each array given (NULL: not written) and
 * the entry count to *n. */
#define DL_ROUND_FIRST 1
#define DL_ROUND_PLAIN 2
#define DL_ROUND_FUSED 3
#define DL_ROUND_BATCHED 4
dl_status dl_get_round_log(const dl_engine* e, size_t capacity, uint64_t* new_or_changed, uint64_t* derivations,
                           uint32_t* info, size_t* n);

/* Owned by the engine; valid until the next call on it.  Never NULL. */
const char* dl_last_error(const dl_engine* e);

void dl_free(dl_engine* e);

#ifdef __cplusplus
}
#endif
#endif /* DLFIX_H */
