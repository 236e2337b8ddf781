// Host-callable launchers of the gfx950 kernels.  Every launcher enqueues on
// `st` and never synchronises; sizes are host values.  Device pointers only.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dlfix {

template <int W>
struct TopKW;
using TopK = TopKW<1>;   // top-k proofs over up to 64 facts per sample
using TopK4 = TopKW<4>;  // over up to 256

// ------------------------------------------------------------- primitives
// Scratch words a scan of n values needs (u64 units).
size_t scan_scratch_words(size_t n);
// Exclusive prefix sum of n u32 counts (in may equal out).  The 64-bit total
// goes to *d_total; if `sentinel`, out[n] receives the (truncated) total; if
// `acc`, the total is also added to *acc.
void scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint64_t* d_total, bool sentinel,
              uint64_t* scratch, hipStream_t st,
              uint64_t* acc = nullptr);

// Stable LSD radix sort of (key, value) pairs on the low `key_bits` bits.
// Sorted data ends in (*keys, *vals); the alternates are used as ping-pong
// buffers and the pointers are swapped as needed.  vals may be NULL.
size_t radix_scratch_words(size_t n);
template <typename K>
void radix_sort(K** keys, uint32_t** vals, K** keys_alt, uint32_t** vals_alt, size_t n, int key_bits,
                uint64_t* scratch, hipStream_t st);

void iota_u32(uint32_t* out, size_t n, uint32_t start, hipStream_t st);
void fill_u32(uint32_t* out, size_t n, uint32_t v, hipStream_t st);
void fill_f32(float* out, size_t n, float v, hipStream_t st);
// out[i] = in[idx[i]] for element size `bytes` in {4, 8, sizeof(TopK), sizeof(TopK4)}.
void gather(const void* in, const uint32_t* idx, void* out, size_t n, size_t bytes, hipStream_t st);
// Max over n u32 values into *d_out (atomic max; *d_out must be initialised).
void max_u32(const uint32_t* in, size_t n, uint32_t* d_out, hipStream_t st);
// smax[sample[i]] = max(smax[...], largest column value of row i); smax must
// hold (largest sample + 1) words, cleared beforehand.
void sample_max_u32(const uint32_t* const* cols, int ncols, const uint32_t* sample, size_t n, uint32_t* smax,
                    hipStream_t st);

// ---------------------------------------------------------- relations
struct KeyLayout {  // packed key: [sample | c0 | c1 | ...], c0 most significant
  int ncols;
  int cbits;
  int sbits;
};

template <typename K>
void pack_rows(const uint32_t* const* cols, const uint32_t* sample, size_t n, KeyLayout lay, K* keys,
               hipStream_t st);
template <typename K>
void unpack_rows(const K* keys, size_t n, KeyLayout lay, uint32_t* const* cols, uint32_t* sample,
                 hipStream_t st);
// Re-pack keys with a column permutation (out column j = in column perm[j]).
template <typename K>
void permute_keys(const K* in, size_t n, KeyLayout lay, const int* perm, K* out, hipStream_t st);

// CSR offsets over the top `prefix_bits` bits (below `total_bits`) of sorted
// keys: off[v] = first row whose prefix >= v, for v in [0, 2^prefix_bits].
template <typename K>
void csr_build(const K* keys, size_t n, int total_bits, int prefix_bits, uint32_t* off, hipStream_t st);
// The same with the row count read from device memory (graph replay).
template <typename K>
void csr_build_dn(const K* keys, const uint64_t* dn, int total_bits, int prefix_bits, uint32_t* off, hipStream_t st);

// Hash index over the same prefix (Sec. 5, hash table design: open
// addressing with linear probing, row positions as the payload): one slot
// per distinct prefix of the sorted keys with its first row and row count
// (a prefix's rows are contiguous).  Memory follows the distinct prefixes,
// not the prefix domain, so any prefix width up to 62 bits is indexable.
// `mask` + 1 slots (a power of two, at least twice the rows: a probe always
// meets an empty slot).
struct alignas(16) HSlot {
  uint64_t key;  // prefix, or HSLOT_EMPTY
  uint32_t start, count;
};
constexpr uint64_t HSLOT_EMPTY = ~0ull;
template <typename K>
void hash_build(const K* keys, size_t n, int total_bits, int prefix_bits, HSlot* slots, uint32_t mask,
                hipStream_t st);

// Tag payload kinds of the relational kernels.
// TAG_VID: VTag (value, fact); TAG_TOPK4: top-k over up to 256 facts per sample
enum TagKind : int { TAG_NONE = 0, TAG_F32 = 1, TAG_TOPK = 2, TAG_VID = 3, TAG_TOPK4 = 4 };

// Expression evaluation at a plan's output (Sec. 5: a bytecode program for a
// small stack machine run by each thread on one output row; Sec. 3.3
// eval<alpha>).  ops: the EvalOp codes of program.h; an EV_SRC operand is a
// column of the driver row (>= 0) or of the index row (-1 - c); EV_CONST
// carries the value.  [0, fend) is the condition (none when fend == 0);
// computed head column c is [cbeg[c], cend[c]) (a plain column when empty).
// A computed value must be below the ids in use (`dn`, or sn[sample] in
// batched engines): it becomes a column of a packed key and a dense index.
constexpr int EVAL_MAX = 48;
constexpr int EVAL_STACK = 8;
struct EvalCode {
  const uint32_t* sn;  // batched: ids in use per sample, else NULL
  uint32_t n;          // instructions (0: nothing to evaluate)
  uint32_t fend;
  uint32_t cbeg[4], cend[4];
  uint32_t dn;
  uint8_t op[EVAL_MAX];
  int32_t arg[EVAL_MAX];
};

struct JoinArgs {
  // driver table
  const void* dkeys;
  const void* dtags;
  const uint32_t* dids;
  size_t n;
  KeyLayout dlay;
  // join prefix: driver columns forming the index prefix, in index key order
  int w;
  int jsrc[4];
  // index: CSR offsets over the prefix domain, or (hslots != NULL) a hash
  // index of hmask + 1 slots
  const uint32_t* off;
  const HSlot* hslots;
  uint32_t hmask;
  const void* ikeys;
  const void* itags;
  const uint32_t* iids;
  KeyLayout ilay;
  // output
  KeyLayout olay;
  int osrc[4];  // >= 0: driver column, < 0: index column (-1 - c)
  int sr;       // SemiringKind
  int k;        // top-k proof count
  const float* q;  // top-k: per-sample probabilities [sample][64]
  bool index_first;  // x operand order: index tag first (body order)
  int items;         // expand tile: join outputs per thread (1, 2, 4 or 8)
  uint32_t* istart;  // per driver row: first matching index row (join_count writes it when not NULL)
  // evaluation at the output (last join step or projection)
  EvalCode ev;
  uint32_t* keep;    // sort path with evaluation: per output row, 1 if it survives (else NULL)
  uint64_t* err;     // evaluation errors: a computed value outside the ids in use sets 4
};

// Differentiable max-min tags (VTag: value, fact): from the input facts'
// probabilities and numbers, their values, and the reverse pass (the gradient
// of row rows[i] -- or i -- goes to the row's fact).
struct VTag;
void vtags_from_facts(const float* q, const uint32_t* fid, size_t n, VTag* out, hipStream_t st);
void vtag_split(const VTag* t, size_t n, float* v, uint32_t* f, hipStream_t st);
void vtag_backward(const VTag* t, const int64_t* rows, const float* g, size_t n, size_t nrel, float* grad_fact,
                   hipStream_t st);

// Dense-domain deduplication state of one derived relation (key < 2^w):
// presence and "touched this round" bitmaps, a dense tag word per key and the
// list of keys touched this round.  Survivors of a join are folded into the
// dense tag with integer atomics; a derivation that cannot change the
// relation (key present under frozen tags, or no strict improvement under
// max / min) is dropped in the join itself.
enum DenseMode : int { DENSE_BOOL = 0, DENSE_ADD = 1, DENSE_MAX = 2, DENSE_MIN = 3 };
struct DenseArgs {
  uint32_t* present;   // bitmap, stable during a round
  uint32_t* touched;   // bitmap, cleared by dense_finalize
  uint32_t* dtag;      // per key: f32 bits (DENSE_ADD) or order-preserving u32 of the f32 tag
  uint32_t* did;       // per key: tuple id (lineage), written by dense_finalize
  // Lineage entries go to wave-private segments of DENSE_SEG slots: segment
  // s holds seg_lcount[s] entries at log_*[s * DENSE_SEG ...];
  // segments_lineage gathers them in segment order.
  void* log_keys;      // lineage log (DENSE_ADD with lineage): key, left id, right id
  uint32_t* log_l;
  uint32_t* log_r;
  uint32_t* seg_lcount;
  uint32_t seg_base;   // first segment of this launch
  uint64_t* overflow;  // set to 1 when a device-side total exceeds the 32-bit offsets
  int mode;
  // Dense index of a packed key: mixed radix over (col 0, ..., col last)
  // with dn ids per column and the last column padded to dnp (a multiple of
  // 32), so the keys of one (sample, col 0) prefix form a word-aligned
  // window; samples follow one another.  Order-preserving: index order is
  // key order.  With one sample dn/dnp hold the sizes; batched engines size
  // every sample by its own ids: sample s starts at sbase[s] (sbase[nsamp] =
  // domain size) with sn[s] ids per column, the last padded to snp[s].
  uint32_t dn, dnp;
  int dcols, dcbits;   // relation arity, bits per column of the packed key
  uint32_t nsamp;      // samples (1: dn / dnp, else the tables)
  const uint32_t* sbase;
  const uint32_t* sn;
  const uint32_t* snp;
  // division by dn and dnp through multiply-high and shifts (Granlund and
  // Montgomery, division by invariant integers): q = (t + ((n - t) >> s1))
  // >> s2 with t = mulhi(n, m), exact for every 32-bit n
  uint32_t dn_m, dnp_m;
  uint8_t dn_s1, dn_s2, dnp_s1, dnp_s2;
};
// Fills the multiply-high constants of DenseArgs for its dn and dnp.
void dense_divisors(DenseArgs& d);
constexpr int DENSE_SEG = 512;  // slots per wave segment (64 lanes x up to 8 rows)
// Segments a dense emission over n slots with `items` outputs per thread uses.
size_t dense_segments(size_t n, int items);
// Initial dense tag word (semiring zero) for a mode.
uint32_t dense_init_word(int mode);

// Hash-set deduplication of a round's candidates (Sec. 5, GPU hash table;
// the alternative to sorting them): every candidate is inserted into a table
// of mask + 1 slots (open addressing, linear probing; an empty slot's key is
// all ones, which no packed key narrower than K can be) and its tag folded
// into the slot's word as the dense path folds (mode: DenseMode; f32 tags or
// none).  The occupied slots then give the distinct keys, unsorted, with
// their +-folded tags (frozen sums clamped).  hset_prepare empties the table.
template <typename K>
void hset_prepare(K* hkeys, uint32_t* htags, size_t slots, int mode, hipStream_t st);
template <typename K>
void hset_insert(const K* keys, const float* tags, size_t n, K* hkeys, uint32_t* htags, uint32_t mask, int mode,
                 hipStream_t st);
template <typename K>
void hset_flags(const K* hkeys, size_t slots, uint32_t* flags, hipStream_t st);
template <typename K>
void hset_compact(const K* hkeys, const uint32_t* htags, const uint32_t* pos, size_t slots, int mode, K* okeys,
                  float* otags, hipStream_t st);

// counts[i] = number of index rows matching driver row i.
template <typename K>
void join_count(const JoinArgs& a, uint32_t* counts, hipStream_t st);  // also fills a.istart if set
// Counts and their exclusive scan (offs[0..n], total in *d_total, added to
// *acc when set) in one launch for up to CS_MAX_TILES tiles of 256 driver
// rows; false (nothing launched) otherwise or when n == 0.  `state` holds
// count_scan_state_words() words, zeroed before the first launch: two sets
// of tile statuses and a parity word; each launch works on one set and
// clears the other, so the next launch starts on a clear set; *err = 3
// reports a look-back wait that did not end.
constexpr size_t CS_MAX_TILES = 8192;
size_t count_scan_state_words();
template <typename K>
bool join_count_scan(const JoinArgs& a, uint32_t* offs, uint64_t* state, uint64_t* d_total, uint64_t* acc,
                     uint64_t* err, hipStream_t st);
// Emit every match: slot j of row i (offs = exclusive scan of counts, with
// sentinel).  Writes keys (and tags, lineage pairs if non-NULL) at out + j.
template <typename K>
void join_expand(const JoinArgs& a, int tag_kind, const uint32_t* offs, size_t total, void* okeys, void* otags,
                 uint32_t* olin_l, uint32_t* olin_r, hipStream_t st);
// The same join, emitting into a dense-domain relation (see DenseArgs).  If
// dtotal is not NULL the total is read on the device (the host passes an
// upper bound max_total for the grid) and `total` is ignored.
// Row windows of a static-driven join whose head keys start with the
// driver's (sample, first column) prefix: goff is the CSR of the driver rows
// over the packed prefix (ngroups prefixes), the head keys of a prefix fill a
// window of wkeys dense indexes (a multiple of 32, at most 8192), and
// launches with at least `from` derivations use them.
struct RowWindows {
  const uint32_t* goff;  // driver CSR over its (sample, first column) prefix: ngroups + 1 offsets
  size_t ngroups;        // 2^(sample bits + column bits)
  uint32_t wkeys;        // largest window (dense keys of one prefix)
  uint64_t from;         // derivations per launch from which windows are used
};
template <typename K>
void join_expand_dense(const JoinArgs& a, int tag_kind, const uint32_t* offs, size_t total, const uint64_t* dtotal,
                       size_t max_total, const DenseArgs& d, bool lineage, hipStream_t st,
                       const RowWindows* rw = nullptr);
template <typename K>
void project_dense(const JoinArgs& a, int tag_kind, const DenseArgs& d, bool lineage, hipStream_t st);

// Fused rounds: one launch per round for a one-plan stratum whose delta join
// is static-driven with the row-window shape and joins the recent tuples on
// their first column (see k_window_round).  The recent relation is kept in
// window layout: the rc[g] recent tuples of group g = (sample, first column)
// sit from the window's first dense index on.
struct WindowRecent {
  uint32_t* rc;  // per group: recent tuples of its window
  void* rk;      // packed keys, window g's from its first dense index on
  float* rt;     // tags (f32 semirings, else NULL), same positions
};
struct RoundArgs {
  WindowRecent cur, next;  // read in this round / written for the next one
  const uint32_t* goff;    // driver CSR over its (sample, first column) prefix
  uint32_t ngroups;        // groups (2^(sample bits + column bits))
  uint32_t win_per_key;    // a group folds in LDS when derivations * win_per_key >= window keys
                           // (0: always; ~0u: never)
  uint32_t* part;          // per workgroup: [2b] new/changed tuples, [2b + 1] derivations of the round
  uint32_t batch;          // groups per workgroup batch: RW_WAVES (one wave counts each group and does a
                           // sparse one alone) or 1 (one group per workgroup: the dense groups of large
                           // rounds spread over all workgroups instead of queueing in batches)
};
// Whether the fused round kernel takes this shape (window of at most 8192 keys),
// and its grid for `batch` groups per workgroup batch (the entries of `part`
// it writes: 2 per workgroup).
bool window_round_fits(uint32_t wkeys);
unsigned window_round_grid(uint32_t ngroups, uint32_t batch);
// Per-round totals of `rounds` fused rounds from their per-workgroup pairs
// (nb pairs a round, rounds one after the other in `part`): out[2i] = new or
// changed tuples of round i, out[2i + 1] = its derivations.
void sum_parts(const uint32_t* part, unsigned nb, unsigned rounds, uint64_t* out, hipStream_t st);
constexpr uint32_t WINDOW_ROUND_WIDE = 8;  // the wider batch (waves of the fused round's workgroup)
template <typename K>
void window_round(const JoinArgs& a, int tag_kind, const DenseArgs& d, const RoundArgs& ra, hipStream_t st);
// Sorted recent tuples with a CSR over (sample, first column) -> window layout.
template <typename K>
void to_windows(const K* keys, const float* tags, size_t n, const uint32_t* off, uint32_t ngroups,
                const DenseArgs& d, WindowRecent w, hipStream_t st);
// Pass 1 of a bitmap compaction: set-bit count of every block of a bitmap
// over `keys` dense indexes (dense_count_blocks(keys) entries).
size_t dense_count_blocks(size_t keys);
size_t dense_self_prefix_blocks();
void bitmap_block_counts(const uint32_t* bits, size_t keys, uint32_t* partial, hipStream_t st);
// Pass 2 (counts = those block counts, every block summing the ones before
// it; or, with `prefixed`, their exclusive scan -- for more than
// dense_self_prefix_blocks() blocks):
// write the touched keys in ascending order with their tags (rtags may be
// NULL), make them present, clear touched, clamp frozen sums and, with
// lineage, assign ids base.. in key order and record tags by id.  The number
// of keys goes to *d_total when d_total is not NULL, and is appended to `log`
// (log[0] = entries, then one per call) when log is not NULL.
// With `csr` (one sample, an index on the first column over the written
// keys): also write that index's CSR offsets, off[c] = slot of the first key
// with first column c for c <= n (the domain's groups are whole bitmap words:
// a group spans n^(arity-2) * np keys, a multiple of 32), so that the next
// round needs no separate index build.
struct DenseCsr {
  uint32_t* off = nullptr;
  uint32_t wwords = 0;  // bitmap words per first-column group
  uint32_t n = 0;       // groups (ids in use)
  uint32_t m = 0;       // division by wwords: multiply-high and shifts
  uint8_t s1 = 0, s2 = 0;
};
DenseCsr dense_csr(uint32_t* off, uint32_t wwords, uint32_t n);
// With `lookback` (lookback_state_words(dense_count_blocks(nkeys)) words,
// zeroed before the first launch and kept across launches; d_total must be
// set): the blocks find their first slots by a decoupled look-back over
// their published counts, so `counts` is not read -- no bitmap_block_counts
// launch is needed.
size_t lookback_state_words(size_t blocks);
template <typename K>
void dense_finalize(const DenseArgs& d, size_t nkeys, const uint32_t* counts, K* keys, float* rtags, uint32_t id_base,
                    float* tag_by_id, uint64_t* d_total, hipStream_t st, uint64_t* log = nullptr,
                    bool prefixed = false, const DenseCsr* csr = nullptr, uint64_t* lookback = nullptr);
// The round's lineage segments (d.seg_lcount entries each, pos = exclusive
// scan of those counts) compacted into (owner id, left id, right id).
template <typename K>
void segments_lineage(const DenseArgs& d, const uint32_t* pos, size_t nseg, uint32_t* owner, uint32_t* l, uint32_t* r,
                      hipStream_t st);
// Sorted keys of the set bits of the presence bitmap (counts and prefixed as
// for dense_finalize), tags and ids gathered from the dense arrays (either
// may be NULL).
size_t bitmap_words(size_t keys);
template <typename K>
void bitmap_keys(const DenseArgs& d, size_t nkeys, const uint32_t* counts, bool prefixed, K* keys, float* tags,
                 uint32_t* ids, hipStream_t st);
// Single-atom rule: re-pack driver columns as head columns, copy tags.
template <typename K>
void project_rows(const JoinArgs& a, int tag_kind, void* okeys, void* otags, uint32_t* olin_l, uint32_t* olin_r,
                  hipStream_t st);

// Segment heads of sorted keys: flags[i] = 1 iff i == 0 or key[i] != key[i-1].
template <typename K>
void head_flags(const K* keys, size_t n, uint32_t* flags, hipStream_t st);
// Reduce every run of equal keys (heads given by pos = exclusive scan of
// flags) to one row: keys_out[s], tag = +-fold in sorted order.  Tags are
// read through `perm` (sorted position -> candidate index) when non-NULL.
template <typename K>
void segment_reduce(const K* keys, const uint32_t* pos, const uint32_t* flags, size_t n, int tag_kind, int sr, int k,
                    const void* tags, const uint32_t* perm, K* keys_out, void* tags_out, size_t n_out,
                    hipStream_t st);

// For every unique candidate (sorted, distinct) find its key in the sorted
// full relation.  Converging semirings +-merge the tag into full in place.
// status[i]: 1 = new, 2 = tag changed, 0 = nothing to do.
template <typename K>
void diff_merge(const K* ukeys, const void* utags, size_t nu, const K* fkeys, void* ftags, size_t nf, int tag_kind,
                int sr, int k, bool converge, uint32_t* status, uint32_t* fpos, hipStream_t st);

// out[pos[i]] = in[i] where flag[i] (pos = exclusive scan of flags).
void compact(const void* in, const uint32_t* flags, const uint32_t* pos, size_t n, size_t bytes, void* out,
             hipStream_t st);
// flags[i] = (status[i] & mask) != 0
void status_flags(const uint32_t* status, size_t n, uint32_t mask, uint32_t* flags, hipStream_t st);
// flags[i] = 1 iff lo <= ids[i] < hi.
void range_flags(const uint32_t* ids, size_t n, uint32_t lo, uint32_t hi, uint32_t* flags, hipStream_t st);
// owner[i] = id of the row of fkeys equal to ckeys[i] when that id is in
// [lo, hi), else ~0 (fkeys sorted, fids aligned with it).
template <typename K>
void match_owner(const K* ckeys, size_t n, const K* fkeys, const uint32_t* fids, size_t F, uint32_t lo, uint32_t hi,
                 uint32_t* owner, hipStream_t st);

// Merge two sorted, disjoint relations (keys + payload) into out.
size_t merge_scratch_words(size_t na, size_t nb);
template <typename K>
void merge_sorted(const K* ak, const void* at, const uint32_t* aid, size_t na, const K* bk, const void* bt,
                  const uint32_t* bid, size_t nb, size_t tag_bytes, K* ok, void* ot, uint32_t* oid,
                  uint64_t* scratch, hipStream_t st);

// out[perm[p]] = base + (run index of sorted position p), run index =
// pos[p] + flags[p] - 1 (maps every input fact to its merged entry).
void seg_scatter(const uint32_t* pos, const uint32_t* flags, const uint32_t* perm, size_t n, uint32_t base,
                 uint32_t* out, hipStream_t st);

// Point queries against a sorted relation (query columns SoA + sample ids,
// values outside the key layout count as absent): row[i] = position in keys
// or -1, tag[i] = its tag as a float (1 for bool, inclusion-exclusion
// probability for top-k, 0 if absent).
template <typename K>
void lookup_rows(const K* keys, size_t n, const uint32_t* const* qcols, const uint32_t* qsample, size_t nq,
                 int tag_kind, const void* tags, KeyLayout lay, const float* qtab, int64_t* rows, float* qtag,
                 hipStream_t st);
// adj[ids[rows[i]]] += g[i] for 0 <= rows[i] < nrel
void scatter_add_rows(const uint32_t* ids, const int64_t* rows, const float* g, size_t n, size_t nrel, float* adj,
                      hipStream_t st);
// top-k gradient seeded on selected rows of a relation of nrel rows
template <typename K, int W>
void topk_backward_rows(const TopKW<W>* t, const K* keys, KeyLayout lay, const int64_t* rows, const float* g,
                        size_t n, size_t nrel, const float* qtab, float* grad_fact, hipStream_t st);

// ---------------------------------------------------------- tags & grads
// Top-k with W words per proof set; qtab and grad_fact are [sample][64 * W].
// Input facts -> tags: [({local_id}, q)].
template <int W>
void topk_from_facts(const float* q, const uint32_t* local_id, size_t n, TopKW<W>* out, hipStream_t st);
// Inclusion-exclusion probability of each row's kept proofs (binary64).
template <int W>
void topk_probability(const TopKW<W>* t, const uint32_t* sample, size_t n, const float* qtab, float* prob,
                      hipStream_t st);
// Proof counts, sets (word w of proof j of row i at bits[(j*n + i)*W + w])
// and probabilities.
template <int W>
void topk_split(const TopKW<W>* t, size_t n, int k, uint8_t* cnt, uint64_t* bits, float* prob, hipStream_t st);
// grad of the inclusion-exclusion probability w.r.t. fact probabilities,
// scattered into grad_fact[sample * 64 * W + fact].
template <int W>
void topk_backward(const TopKW<W>* t, const uint32_t* sample, const float* gout, size_t n, const float* qtab,
                   float* grad_fact, hipStream_t st);

// Add-mult lineage: for derivation i of tuple owner[i] with body tuples
// (l[i], r[i]): g = adj[owner] if tag[owner] < 1; adj[l] += g*tag[r];
// adj[r] += g*tag[l] (r may be ~0u: single-atom rule, adj[l] += g).
void lineage_backward(const uint32_t* owner, const uint32_t* l, const uint32_t* r, size_t n, const float* tag_by_id,
                      float* adj, hipStream_t st);
// adj[ids[i]] += g[i]
void scatter_add(const uint32_t* ids, const float* g, size_t n, float* adj, hipStream_t st);
// out[i] += adj[ids[i]] * (tag[ids[i]] < 1)
void gather_add_clamped(const uint32_t* ids, const float* adj, const float* tag_by_id, size_t n, float* out,
                        hipStream_t st);
// Lineage of new tuples.  For sorted candidate p its run is
// s = pos[p] + flags[p] - 1.  lineage_flags: lf[p] = status[s] & 1.
// lineage_emit (lpos = exclusive scan of lf): for every flagged p write
// owner = id_base + newpos[s] and the pair (cl, cr)[perm[p]] at lpos[p].
void lineage_flags(const uint32_t* pos, const uint32_t* flags, const uint32_t* status, size_t n, uint32_t* lf,
                   hipStream_t st);
void lineage_emit(const uint32_t* pos, const uint32_t* flags, const uint32_t* lf, const uint32_t* lpos,
                  const uint32_t* newpos, const uint32_t* perm, const uint32_t* cl, const uint32_t* cr, size_t n,
                  uint32_t id_base, uint32_t* owner, uint32_t* l, uint32_t* r, hipStream_t st);

}  // namespace dlfix
