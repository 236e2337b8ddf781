// Host side of the fixpoint engine: device buffers, relation store, plans.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dlfix.h"
#include "kernels.h"
#include "prof.h"
#include "program.h"

namespace dlfix {

// Raised inside the library, turned into a dl_status at the C boundary.
struct Error {
  dl_status code;
  std::string msg;
};

#define DL_HIP(call)                                                                                 \
  do {                                                                                               \
    hipError_t err_ = (call);                                                                        \
    if (err_ != hipSuccess)                                                                          \
      throw ::dlfix::Error{err_ == hipErrorOutOfMemory ? DL_ERR_NOMEM : DL_ERR_HIP,                   \
                           std::string(#call) + ": " + hipGetErrorString(err_)};                     \
  } while (0)

// A device buffer that only grows (buffer reuse across iterations, Sec. 4.1).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Host-side allocator over one device range: the caller's workspace
// (dl_options.workspace) or the library's static per-device array.  First
// fit over a free list ordered by address; a released range merges with its
// free neighbours.  Ranges are 256-byte aligned.  It makes no device call:
// releasing a range that queued kernels still read is safe because every
// later user of the range is enqueued on the same stream (Sec. 4.1 buffer
// reuse, with the arena standing in for the allocator).
struct Arena {
  char* base = nullptr;
  size_t bytes = 0;
  size_t used = 0, peak = 0;
  std::map<size_t, size_t> free_list;  // offset -> length
  void reset(void* p, size_t n);
  void* alloc(size_t n);  // nullptr when no free range is large enough
  void release(void* p, size_t n);
  size_t largest_free() const;
};

struct Table {
  DevBuf keys, tags, ids;
  size_t n = 0;
};

struct RelState {
  // input relations: facts staged as they arrive, packed at the next run
  std::vector<DevBuf> raw_cols;
  DevBuf raw_sample, raw_tags, raw_local;  // raw_local: top-k: fact id inside its sample;
                                           // differentiable max-min: fact number over all relations
  size_t nraw = 0;
  Table full, full_alt, recent;
  DevBuf cand_keys, cand_tags, cand_l, cand_r;  // this round's derivations (head rows)
  size_t ncand = 0;
  uint64_t version = 0;  // bumped whenever `full` changes (keys or tags)
  uint64_t rversion = 0; // bumped whenever `recent` changes
  // stable part (full minus recent, read under frozen tags): full_alt after
  // a round that added tuples (the merge or materialisation leaves the
  // previous state there), full itself after a round that added none
  bool stable_full = false;
  uint64_t sversion = 0;  // bumped whenever the stable part may change
  // dense-domain deduplication (derived relations with a small key domain)
  bool dense = false;
  size_t dense_keys = 0;  // size of the dense index domain (see DenseArgs)
  int dense_cols = 0;
  DevBuf dense_sbase;     // batched: first dense index of every sample (+ domain size)
  bool own_index = false;  // a plan of its own stratum joins against it
  DevBuf present, touched, dtag, did, log_keys, log_l, log_r, seg_lcount;
  DevBuf goff;                   // as a join driver: CSR over its (sample, first column) prefix
  DevBuf lb_state;               // round-end compaction: look-back statuses (kept in a reusable state)
  uint64_t goff_version = ~0ull;  // `version` it was built from
  size_t nseg = 0;         // lineage wave segments emitted this round
  Table view_full, view_recent, view_stable;  // a past round's state (lineage recomputation)
  DevBuf fact_entry;  // input facts -> entry id
  DevBuf grad;        // accumulated input gradients (per fact)
  std::vector<uint32_t> fact_slot;  // top-k: sample*64 + local id per fact (host)
  DevBuf fact_slot_d;
  uint32_t id_base = 0;  // input relations: id of entry 0
};

struct IndexState {
  Table t;           // keys permuted, tags, ids
  DevBuf off;        // CSR over the prefix
  DevBuf hash;       // or a hash index over it (HSlot[hmask + 1])
  uint32_t hmask = 0;
  bool use_hash = false;
  bool built = false;
  bool borrowed = false;  // identity permutation: t aliases the relation
  uint64_t version = ~0ull;  // relation version it was built from
};

struct LineageSeg {
  size_t off, n;
};

// Execution choices the autotuner picks among (all give the same result).
struct ExecConfig {
  int items = 2;   // join expand tile: outputs per thread (1, 2, 4, 8)
  int orient = 0;  // delta plans of 2-atom rules: 0 auto, 1 recent-driven, 2 static-driven
  int index = 0;   // indexes built for joins: 0 CSR offsets (hash above a 2^30 prefix domain), 1 hash
  int graph = 1;   // replay eligible round bodies as a captured HIP graph
  int rows = 1;    // row-window variant of the dense join where it applies
  int fused = 1;   // one launch per round (window_round) where the shape allows
};

struct Engine {
  Program prog;
  std::string text;
  ExecConfig cfg;
  dl_options opts{};
  int sr = 0;
  int k = 3;
  bool batched = false;
  bool converge = true;   // idempotent +
  bool lineage = false;   // diff add-mult
  int tag_kind = 0;       // TagKind
  size_t tag_bytes = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // device memory: hipMalloc per buffer, or ranges of one arena (workspace)
  bool use_arena = false;
  Arena arena;
  uint64_t device_allocs = 0;  // hipMalloc calls made by this engine
  // engines of dl_load_program_static: the device whose static array is the
  // arena (-1 otherwise) and the generation of that array they hold
  int static_dev = -1;
  uint64_t static_gen = 0;
  uint64_t host_words[64] = {};

  // data-dependent layout, fixed at ingest
  bool ingested = false;
  bool ran = false;
  bool key64 = false;
  int cbits = 1, sbits = 0;
  uint32_t max_id = 0, max_sample = 0;
  std::vector<uint32_t> sample_ids;  // batched: ids in use per sample (largest id + 1)
  DevBuf d_sn, d_snp;                // per sample: ids in use, padded to 32 (dense index radix)
  std::vector<RelState> rel;
  std::vector<IndexState> idx;

  // top-k: fact probabilities per sample [sample][64] and counters
  std::vector<float> qtab_h;        // top-k fact probabilities, [sample][256] (host)
  std::vector<float> qtab_up;       // the same at the stride in force, as uploaded
  std::vector<uint32_t> topk_next;
  int topk_words = 1;               // u64 words per top-k proof set in force (1: <= 64 facts per sample, 4: <= 256)
  uint32_t nfacts = 0;  // facts added since the last clear, over all relations (max-min fact numbers)
  DevBuf qtab, grad_fact;

  // lineage log (diff add-mult) and per-id tags.  Ids are handed out in
  // discovery order, so round_ids[s][i] (the first id of round i + 1 of
  // stratum s; last entry = end) also describes the relations as they stood
  // at any round: the reverse pass rebuilds them when lineage is not recorded.
  DevBuf lin_owner, lin_l, lin_r, tag_by_id, adj;
  size_t lin_n = 0;
  std::vector<LineageSeg> lin_segs;
  uint32_t next_id = 0;
  bool record = false;        // discovery derivations are being recorded
  size_t lin_budget = 0;      // bytes of recorded lineage allowed
  std::vector<std::vector<uint32_t>> round_ids;

  // round scratch
  DevBuf counts, offs, istart, alt_keys, alt_vals, vals, flags, pos, ukeys, utags,
      status, nflags, newpos, rflags, rpos, lf, lpos, nkeys, ntags, nids, tmpA_keys, tmpA_tags, tmpB_keys, tmpB_tags,
      work, unpack, qbuf,  // work: scan and radix-sort partials
      ev_keys, ev_tags, ev_l, ev_r,  // output rows of a plan with evaluation, before the condition compacts them
      wr_keys0, wr_keys1, wr_tags0, wr_tags1, wr_cnt0, wr_cnt1, wr_part;  // fused rounds: two window-layout recent sets
  uint64_t* host = nullptr;  // pinned readback words
  DevBuf dtotal;             // device words for totals
  DevBuf cs_state;           // single-pass count+scan: tile sums and flags (kept zeroed between launches)

  dl_stats stats{};
  uint64_t deferred_units = 0;  // derivations of joins whose totals stayed on the device (last run)
  uint64_t fused_units = 0;     // derivations of fused rounds (this run, added up on the host)
  // The fused rounds' graphs, one per group batch width and batch length, kept from run to
  // run while their launches' arguments stay the same (key: those bytes);
  // recs are the launches' profiling records when captured while profiling.
  struct FusedGraph {
    std::vector<unsigned char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Profiler::Rec> recs;
    bool profiled = false;
    uint32_t prof_mask = 0;  // the families timed when it was captured
    int defer_fam = -1;  // the launches' bytes per device-counted unit (Profiler::defer)
    double defer_per = 0.0;
  };
  FusedGraph fused_graph[8];
  void drop_fused_graph(FusedGraph& g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = FusedGraph{};
  }
  std::vector<uint64_t> round_log;  // rounds of the last run: (new or changed, derivations, info) triples
  void log_round(uint64_t u, uint64_t c, int stratum, int kind) {
    round_log.push_back(u);
    round_log.push_back(c);
    round_log.push_back((uint64_t)stratum << 8 | (uint64_t)kind);
  }
  int cur_stratum = 0;  // the stratum being evaluated (round log)
  uint32_t prof_mask = 0;
  dl_kernel_timing kstats[DL_K_FAMILIES]{};
  size_t device_bytes = 0;

  ~Engine();
  // memory
  void grow(DevBuf& b, size_t bytes, bool keep = false, size_t used = 0);
  void release(DevBuf& b);
  void set_workspace(void* p, size_t bytes);
  // every device buffer the engine owns (index tables that alias a relation
  // are not visited: they are re-pointed when the index is next used)
  template <typename F>
  void for_each_buf(F&& f);
  uint64_t read_total(int slot);
  void read_totals();  // all total slots into host[] (one sync)
  void sync();

  // lifecycle
  void init(const char* text, const dl_options* o);
  void add_facts(const char* relation, size_t n, const uint32_t* sample_ids, const uint32_t* const* columns,
                 const float* tags, int on_device);
  void clear_facts();
  void run();
  size_t relation_size(const char* relation);
  size_t read_relation(const char* relation, size_t capacity, const dl_relation_out* out, int on_device);
  void backward(const char* out_relation, const float* grad_out, int on_device);
  void read_grad(const char* in_relation, float* grad_in, int on_device);
  void zero_grad();
  void autotune(int trials, const char* cache_path);
  void lookup(const char* relation, size_t n, const uint32_t* sample_ids, const uint32_t* const* columns,
              int64_t* rows, float* tags, int on_device);
  void backward_rows(const char* relation, size_t n, const int64_t* rows, const float* grad, int on_device);
  std::string tune_key() const;

  int relation_id(const char* name, bool must_exist = true);
  KeyLayout layout(int ncols) const { return KeyLayout{ncols, cbits, sbits}; }
  int key_width(int ncols) const { return sbits + ncols * cbits; }
};

template <typename F>
void Engine::for_each_buf(F&& f) {
  for (auto& r : rel) {
    for (auto& c : r.raw_cols) f(c);
    for (DevBuf* b : {&r.raw_sample, &r.raw_tags, &r.raw_local}) f(*b);
    for (Table* t : {&r.full, &r.full_alt, &r.recent, &r.view_full, &r.view_recent, &r.view_stable})
      f(t->keys), f(t->tags), f(t->ids);
    for (DevBuf* b : {&r.fact_entry, &r.grad, &r.fact_slot_d, &r.cand_keys, &r.cand_tags, &r.cand_l, &r.cand_r,
                      &r.present, &r.touched, &r.dtag, &r.did, &r.log_keys, &r.log_l, &r.log_r, &r.seg_lcount,
                      &r.goff, &r.dense_sbase, &r.lb_state})
      f(*b);
  }
  for (auto& x : idx) {
    if (!x.borrowed) f(x.t.keys), f(x.t.tags), f(x.t.ids);
    f(x.off);
    f(x.hash);
  }
  for (DevBuf* b : {&d_sn, &d_snp, &qtab, &grad_fact, &lin_owner, &lin_l, &lin_r, &tag_by_id, &adj, &counts, &offs,
                    &istart, &alt_keys, &alt_vals, &vals, &flags, &pos, &ukeys, &utags, &status, &nflags, &newpos,
                    &rflags, &rpos, &lf, &lpos, &nkeys, &ntags, &nids, &tmpA_keys, &tmpA_tags, &tmpB_keys,
                    &tmpB_tags, &work, &unpack, &qbuf, &dtotal, &cs_state, &ev_keys, &ev_tags, &ev_l, &ev_r,
                    &wr_keys0, &wr_keys1, &wr_tags0, &wr_tags1, &wr_cnt0, &wr_cnt1, &wr_part})
    f(*b);
}

// Typed halves (K = packed key type), in engine_run.hip.
template <typename K>
void ingest(Engine& e);
template <typename K>
void run_fixpoint(Engine& e);
template <typename K>
size_t read_relation_t(Engine& e, int r, size_t capacity, const dl_relation_out* out, int on_device);
template <typename K>
void backward_t(Engine& e, int r, const float* grad_out, const int64_t* rows, size_t nrows);
template <typename K>
void lookup_t(Engine& e, int r, size_t n, const uint32_t* const* cols, const uint32_t* sample, int64_t* rows,
              float* tags);

}  // namespace dlfix
