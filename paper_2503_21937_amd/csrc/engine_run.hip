// The semi-naive fixpoint loop (Sec. 3.4, Algorithm 1, Appendix A) over the
// packed-key relation store, for one key width K.
//
// Per stratum: round 1 runs the base plans (rules whose body lies in lower
// strata or the input) on whole relations; every later round runs the delta
// plans, each driven by the recent tuples of one atom of the stratum.  All
// derivations of a round land in one candidate buffer per head relation
// (this replaces the paper's `append` of the three delta joins) and are then
// sorted, +-reduced per key, compared with the full relation (difference for
// frozen add-mult tags, +-merge for the converging semirings, updated only
// after every join of the round has run: Jacobi order) and merged into it.
// The new or changed tuples become the next round's recent relation; the
// stratum ends after the first round that changes nothing.
#include <algorithm>
#include <cstring>
#include <functional>

#include "dl_device.h"
#include "engine.h"
#include "prof.h"

namespace dlfix {

namespace {

// Device words of totals (64 x u64): slots 0..6 below, 8..15 = totals of a
// batch of fused rounds, 30 = id / sample maxima at ingest, 32.. = round log
// of a graph batch (count, then totals).
enum Slot { S_SCAN = 0, S_UNIQUE = 1, S_NEW = 2, S_RECENT = 3, S_LIN = 4, S_OVF = 5, S_CAND = 6, S_PART = 8, S_LOG = 32 };
constexpr int BATCH_ROUNDS = 4;  // round bodies per host synchronisation (one graph)

uint64_t* total_slot(Engine& e, int s) { return e.dtotal.as<uint64_t>() + s; }

void ensure_scratch(Engine& e, size_t words) { e.grow(e.work, (words + 16) * sizeof(uint64_t)); }

template <typename K>
void sort_pairs(Engine& e, K** kp, uint32_t** vp, size_t n, int bits) {
  e.grow(e.alt_keys, n * sizeof(K));
  ensure_scratch(e, radix_scratch_words(n));
  K* ka = e.alt_keys.as<K>();
  uint32_t* va = nullptr;
  if (vp && *vp) {
    e.grow(e.alt_vals, n * 4);
    va = e.alt_vals.as<uint32_t>();
  }
  radix_sort<K>(kp, vp, &ka, &va, n, bits, e.work.as<uint64_t>(), e.stream);
}

void scan(Engine& e, const uint32_t* in, uint32_t* out, size_t n, int slot, bool sentinel, uint64_t* acc = nullptr) {
  ensure_scratch(e, scan_scratch_words(n));
  scan_u32(in, out, n, total_slot(e, slot), sentinel, e.work.as<uint64_t>(), e.stream, acc);
}

// If a sort left its result in the engine's alternate buffer, move the
// buffers so that `owner` holds the sorted data.
void claim(DevBuf& owner, DevBuf& alt, const void* result) {
  if (result == alt.p) std::swap(owner, alt);
}

// Device-side failure flag of the dense join kernels (read with the totals).
void check_overflow(Engine& e) {
  const uint64_t f = e.host[S_OVF];
  if (f == 1) throw Error{DL_ERR_CAPACITY, "more than 2^32 join outputs in one step"};
  if (f == 3) throw Error{DL_ERR_HIP, "single-pass scan: a look-back wait did not end"};
  if (f == 4)
    throw Error{DL_ERR_CAPACITY, "a computed head value lies outside the ids in use (the largest id of the facts "
                                 "and of the program's constants)"};
  if (f) throw Error{DL_ERR_HIP, "row-window join: a derivation fell outside its window"};
}

// The plan's evaluation code (condition, computed head columns) in the
// kernels' form; limits: EVAL_MAX instructions, EVAL_STACK operands deep.
void set_eval(Engine& e, const Plan& pl, JoinArgs& a) {
  EvalCode& c = a.ev;
  c = EvalCode{};
  if (!pl.eval) return;
  auto put = [&](const std::vector<Ins>& code) {
    int depth = 0;
    for (const Ins& ins : code) {
      if (c.n >= (uint32_t)EVAL_MAX)
        throw Error{DL_ERR_UNSUPPORTED, "the expressions of a rule exceed " + std::to_string(EVAL_MAX) + " instructions"};
      c.op[c.n] = (uint8_t)ins.op;
      c.arg[c.n] = ins.arg;
      ++c.n;
      depth += (ins.op == EV_SRC || ins.op == EV_CONST) ? 1 : -1;
      if (depth > EVAL_STACK)
        throw Error{DL_ERR_UNSUPPORTED, "an expression needs more than " + std::to_string(EVAL_STACK) + " stack slots"};
    }
  };
  put(pl.filter);
  c.fend = c.n;
  for (size_t col = 0; col < pl.code.size() && col < 4; ++col) {
    c.cbeg[col] = c.n;
    put(pl.code[col]);
    c.cend[col] = c.n;
  }
  c.dn = e.max_id + 1;
  c.sn = e.batched ? e.d_sn.as<uint32_t>() : nullptr;
}

// Whether a round's L discovery derivations can be added to the recorded
// lineage.  Past the budget the whole record is dropped (memory returned) and
// the reverse pass recomputes every round's derivations instead.
bool keep_lineage(Engine& e, size_t L) {
  if ((e.lin_n + L) * 12 <= e.lin_budget) return true;
  e.record = false;
  e.lin_n = 0;
  e.lin_segs.clear();
  e.release(e.lin_owner), e.release(e.lin_l), e.release(e.lin_r);
  return false;
}

DenseArgs dense_args(Engine& e, RelState& R) {
  DenseArgs d{};
  d.present = R.present.as<uint32_t>();
  d.touched = R.touched.as<uint32_t>();
  d.dtag = R.dtag.as<uint32_t>();
  d.did = e.lineage ? R.did.as<uint32_t>() : nullptr;
  d.log_keys = R.log_keys.p;
  d.log_l = R.log_l.as<uint32_t>();
  d.log_r = R.log_r.as<uint32_t>();
  d.seg_lcount = R.seg_lcount.as<uint32_t>();
  d.seg_base = (uint32_t)R.nseg;
  d.overflow = e.dtotal.as<uint64_t>() + S_OVF;
  d.mode = e.sr == DL_BOOL ? DENSE_BOOL : !e.converge ? DENSE_ADD : e.sr == DL_MAXMIN ? DENSE_MAX : DENSE_MIN;
  d.dn = e.max_id + 1;
  d.dnp = (d.dn + 31) / 32 * 32;
  d.dcols = R.dense_cols;
  d.dcbits = e.cbits;
  dense_divisors(d);
  d.nsamp = e.batched ? (uint32_t)e.sample_ids.size() : 1u;
  d.sbase = R.dense_sbase.as<uint32_t>();
  d.sn = e.d_sn.as<uint32_t>();
  d.snp = e.d_snp.as<uint32_t>();
  return d;
}

// Dense index block of one sample for a relation of arity `ar`: n^(ar-1) x
// np keys, n = the sample's ids in use, np = n rounded up to 32.
uint64_t dense_block(uint64_t n, int ar) {
  uint64_t keys = (n + 31) / 32 * 32;
  for (int c = 0; c + 1 < ar; ++c) {
    keys *= n;
    if (keys > ((uint64_t)1 << 40)) return keys;
  }
  return keys;
}

// Dense index domain of a relation of arity `ar` (see DenseArgs): one block
// per sample, sized by the sample's own ids when batched.
uint64_t dense_domain(const Engine& e, int ar, std::vector<uint32_t>* sbase = nullptr) {
  if (!e.batched) return dense_block((uint64_t)e.max_id + 1, ar);
  uint64_t keys = 0;
  if (sbase) sbase->assign(e.sample_ids.size() + 1, 0u);
  for (size_t s = 0; s < e.sample_ids.size(); ++s) {
    if (sbase) (*sbase)[s] = (uint32_t)std::min<uint64_t>(keys, 0xffffffffu);
    keys += dense_block(e.sample_ids[s], ar);
    if (keys > ((uint64_t)1 << 40)) return keys;
  }
  if (sbase) sbase->back() = (uint32_t)std::min<uint64_t>(keys, 0xffffffffu);
  return keys;
}

// Decide the deduplication of every derived relation and reset the dense
// state (presence, touched, semiring zero in every tag word).
void setup_dense(Engine& e) {
  const size_t budget = (size_t)16 << 30;
  for (size_t r = 0; r < e.rel.size(); ++r) {
    RelState& R = e.rel[r];
    R.dense = false;
    // nullary relations (at most one tuple per sample) always take the sort path
    if (!e.prog.rels[r].derived || e.prog.rels[r].arity == 0) continue;
    const uint64_t dom = dense_domain(e, e.prog.rels[r].arity);
    const size_t keys = (size_t)std::min<uint64_t>(dom, (uint64_t)1 << 40);
    const size_t bytes = 2 * bitmap_words(keys) * 4 + (e.tag_kind == TAG_F32 ? keys * 4 : 0) + (e.lineage ? keys * 4 : 0);
    const bool fits = (e.tag_kind == TAG_NONE || e.tag_kind == TAG_F32) && dom <= ((uint64_t)1 << 31) && bytes <= budget;
    if (e.opts.dedup == 2 && !fits)
      throw Error{DL_ERR_UNSUPPORTED, "dense-domain deduplication does not fit relation " + e.prog.rels[r].name};
    R.dense = fits && e.opts.dedup != 1 && e.opts.dedup != 3;
    if (!R.dense) continue;
    R.dense_keys = keys;
    R.dense_cols = e.prog.rels[r].arity;
    const size_t lbw = lookback_state_words(dense_count_blocks(keys));
    e.grow(R.lb_state, lbw * 8);
    fill_u32(R.lb_state.as<uint32_t>(), lbw * 2, 0u, e.stream);
    if (e.batched) {
      std::vector<uint32_t> sb;
      (void)dense_domain(e, e.prog.rels[r].arity, &sb);
      e.grow(R.dense_sbase, sb.size() * 4);
      DL_HIP(hipMemcpyAsync(R.dense_sbase.p, sb.data(), sb.size() * 4, hipMemcpyHostToDevice, e.stream));
      e.sync();  // sb is a host temporary
    }
    const size_t words = bitmap_words(keys);
    e.grow(R.present, words * 4);
    e.grow(R.touched, words * 4);
    DL_HIP(hipMemsetAsync(R.present.p, 0, words * 4, e.stream));
    DL_HIP(hipMemsetAsync(R.touched.p, 0, words * 4, e.stream));
    if (e.tag_kind == TAG_F32) {
      e.grow(R.dtag, keys * 4);
      fill_u32(R.dtag.as<uint32_t>(), keys, dense_init_word(dense_args(e, R).mode), e.stream);
    }
    if (e.lineage) e.grow(R.did, keys * 4);
    R.nseg = 0;
  }
}

// Sorted full relation of a dense relation, from its presence bitmap.
template <typename K>
void materialize_full(Engine& e, RelState& R) {
  std::swap(R.full, R.full_alt);  // the previous materialisation stays as the stable part
  const size_t nb = dense_count_blocks(R.dense_keys);
  e.grow(e.flags, nb * 4);
  e.grow(e.pos, (nb + 1) * 4);
  bitmap_block_counts(R.present.as<uint32_t>(), R.dense_keys, e.flags.as<uint32_t>(), e.stream);
  scan(e, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), nb, S_SCAN, true);
  const size_t F = e.read_total(S_SCAN);
  e.grow(R.full.keys, F * sizeof(K) + 8);
  float* tags = nullptr;
  uint32_t* ids = nullptr;
  if (e.tag_kind == TAG_F32) {
    e.grow(R.full.tags, F * 4 + 8);
    tags = R.full.tags.as<float>();
  }
  if (e.lineage) {
    e.grow(R.full.ids, F * 4 + 8);
    ids = R.full.ids.as<uint32_t>();
  }
  bitmap_keys<K>(dense_args(e, R), R.dense_keys, e.pos.as<uint32_t>(), true, R.full.keys.as<K>(), tags, ids, e.stream);
  R.full.n = F;
  ++R.version;
}

const Table& index_source(const RelState& R, const IndexSpec& spec) {
  if (spec.recent) return R.recent;
  if (spec.stable) return R.stable_full ? R.full : R.full_alt;
  return R.full;
}

uint64_t index_version(const RelState& R, const IndexSpec& spec) {
  return spec.recent ? R.rversion : spec.stable ? R.sversion : R.version;
}

template <typename K>
void build_index(Engine& e, int i) {
  const IndexSpec& spec = e.prog.indexes[i];
  IndexState& ix = e.idx[i];
  RelState& R = e.rel[spec.rel];
  const Table& src = index_source(R, spec);
  const int ar = e.prog.rels[spec.rel].arity;
  const KeyLayout lay = e.layout(ar);
  const size_t n = src.n;
  const int pbits = e.sbits + spec.w * e.cbits;
  // CSR offsets need 4 bytes per prefix of the domain; a hash index 32
  // bytes per row, whatever the domain
  ix.use_hash = e.cfg.index == 1 || pbits > 30;
  if (ix.use_hash && pbits > 62) throw Error{DL_ERR_UNSUPPORTED, "join prefix wider than 62 bits (index on " + e.prog.rels[spec.rel].name + ")"};
  if (spec.identity()) {
    if (!ix.borrowed) {
      e.release(ix.t.keys), e.release(ix.t.tags), e.release(ix.t.ids);
      ix.borrowed = true;
    }
    ix.t.keys = src.keys;
    ix.t.tags = src.tags;
    ix.t.ids = src.ids;
  } else {
    if (ix.borrowed) {
      ix.t = Table{};
      ix.borrowed = false;
    }
    e.grow(ix.t.keys, n * sizeof(K) + 8);
    e.grow(e.vals, n * 4 + 4);
    permute_keys<K>(src.keys.as<K>(), n, lay, spec.perm.data(), ix.t.keys.as<K>(), e.stream);
    iota_u32(e.vals.as<uint32_t>(), n, 0, e.stream);
    K* kp = ix.t.keys.as<K>();
    uint32_t* vp = e.vals.as<uint32_t>();
    sort_pairs<K>(e, &kp, &vp, n, e.key_width(ar));
    claim(ix.t.keys, e.alt_keys, kp);
    claim(e.vals, e.alt_vals, vp);
    if (e.tag_bytes) {
      e.grow(ix.t.tags, n * e.tag_bytes + 8);
      gather(src.tags.p, e.vals.as<uint32_t>(), ix.t.tags.p, n, e.tag_bytes, e.stream);
    }
    if (e.lineage) {
      e.grow(ix.t.ids, n * 4 + 4);
      gather(src.ids.p, e.vals.as<uint32_t>(), ix.t.ids.p, n, 4, e.stream);
    }
  }
  ix.t.n = n;
  if (ix.use_hash) {
    size_t slots = 64;
    while (slots < 2 * n) slots *= 2;
    if (slots > ((size_t)1 << 32)) throw Error{DL_ERR_CAPACITY, "hash index above 2^32 slots"};
    e.grow(ix.hash, slots * sizeof(HSlot));
    ix.hmask = (uint32_t)(slots - 1);
    hash_build<K>(ix.t.keys.as<K>(), n, e.key_width(ar), pbits, ix.hash.as<HSlot>(), ix.hmask, e.stream);
  } else {
    e.grow(ix.off, (((size_t)1 << pbits) + 1) * 4);
    csr_build<K>(ix.t.keys.as<K>(), n, e.key_width(ar), pbits, ix.off.as<uint32_t>(), e.stream);
  }
  ix.built = true;
  ix.version = index_version(R, spec);
}

template <typename K>
void ensure_index(Engine& e, int i) {
  IndexState& ix = e.idx[i];
  const IndexSpec& spec = e.prog.indexes[i];
  const RelState& R = e.rel[spec.rel];
  const Table& src = index_source(R, spec);
  bool stale = !ix.built || ix.version != index_version(R, spec);
  if (ix.borrowed && ix.t.keys.p != src.keys.p) stale = true;
  if (stale) build_index<K>(e, i);
}

// Row windows (k_join_expand_rows) for a single-join plan driven by a whole
// relation whose head key starts with the driver's (sample, first column)
// prefix; a window must hold 2^5..2^13 keys.  Builds the driver's prefix CSR
// when the relation changed.  The row variant takes launches with many
// derivations per window (see `from` below).
template <typename K>
bool row_windows(Engine& e, const Plan& pl, RowWindows* rw) {
  if (pl.eval || pl.delta || pl.steps.size() != 1 || pl.steps[0].out_src.empty() || pl.steps[0].out_src[0] != 0) return false;
  const int har = e.prog.rels[pl.head_rel].arity;
  const int pbits = e.sbits + e.cbits;
  if (har < 2 || pbits > 30 || !e.rel[pl.head_rel].dense) return false;
  // window: the dense indexes of one (sample, col 0) prefix, n^(har-2) * np
  // for the sample's n ids in use; the largest window must fit LDS
  uint64_t wkeys = 0;
  auto window = [&](uint64_t n) {
    uint64_t w = (n + 31) / 32 * 32;
    for (int c = 2; c < har; ++c) w *= n;
    return w;
  };
  if (e.batched) {
    for (uint32_t n : e.sample_ids) wkeys = std::max(wkeys, window(n));
  } else {
    wkeys = window((uint64_t)e.max_id + 1);
  }
  if (wkeys > 8192) return false;
  RelState& D = e.rel[pl.driver_rel];
  if (D.full.n == 0) return false;
  const size_t groups = (size_t)1 << pbits;
  if (D.goff_version != D.version) {
    e.grow(D.goff, (groups + 1) * 4);
    csr_build<K>(D.full.keys.as<K>(), D.full.n, e.key_width(e.prog.rels[pl.driver_rel].arity), pbits,
                 D.goff.as<uint32_t>(), e.stream);
    D.goff_version = D.version;
  }
  rw->goff = D.goff.as<uint32_t>();
  rw->ngroups = groups;
  rw->wkeys = (uint32_t)wkeys;
  // at least one derivation per 12 keys of the head's dense domain: the
  // window loads and write-backs (8 bytes a key) then cost about what the
  // scattered kernel spends on that many derivations (~100 bytes of HBM
  // traffic each in latency terms); and ~128 per driver group so that a
  // group's fixed latency (bounds, barriers) is amortised
  const uint64_t per_keys = (uint64_t)e.rel[pl.head_rel].dense_keys / 12;
  const uint64_t per_group = (uint64_t)std::min(groups, D.full.n) * 128;
  rw->from = e.cfg.rows == 2 ? 0 : std::max(per_keys, per_group);
  return true;
}

struct Cur {  // the table a plan is currently expanding
  const void* keys;
  const void* tags;
  const uint32_t* ids;
  size_t n;
  int ncols;
  int minpos;  // smallest body position folded into it
};

template <typename K>
void run_plan(Engine& e, const Plan& pl) {
  const Rule& rule = e.prog.rules[pl.rule];
  RelState& D = e.rel[pl.driver_rel];
  const Table& dt = pl.delta ? D.recent : D.full;
  if (dt.n == 0) return;
  RelState& H = e.rel[pl.head_rel];
  const int har = e.prog.rels[pl.head_rel].arity;
  Cur cur{dt.keys.p, dt.tags.p, dt.ids.as<uint32_t>(), dt.n, e.prog.rels[pl.driver_rel].arity, pl.driver_atom};

  JoinArgs a{};
  a.sr = e.sr;
  a.k = e.k;
  a.q = e.qtab.as<float>();
  a.items = e.cfg.items;
  a.err = total_slot(e, S_OVF);
  set_eval(e, pl, a);
  const EvalCode ev_out = a.ev;  // applies at the plan's output only

  auto head_room = [&](size_t add) {
    const size_t used = H.ncand;
    e.grow(H.cand_keys, (used + add) * sizeof(K), true, used * sizeof(K));
    if (e.tag_bytes) e.grow(H.cand_tags, (used + add) * e.tag_bytes, true, used * e.tag_bytes);
    if (e.record) {
      e.grow(H.cand_l, (used + add) * 4, true, used * 4);
      e.grow(H.cand_r, (used + add) * 4, true, used * 4);
    }
  };
  auto out_ptrs = [&](void** ok, void** ot, uint32_t** ol, uint32_t** orr) {
    *ok = H.cand_keys.as<K>() + H.ncand;
    *ot = e.tag_bytes ? (void*)(H.cand_tags.as<uint8_t>() + H.ncand * e.tag_bytes) : nullptr;
    *ol = e.record ? H.cand_l.as<uint32_t>() + H.ncand : nullptr;
    *orr = e.record ? H.cand_r.as<uint32_t>() + H.ncand : nullptr;
  };
  // Sort path with evaluation: the output rows of n slots go to staging
  // buffers with a keep flag each; the survivors are appended to the head's
  // candidates in slot order (flag, scan, compaction).
  auto stage = [&](size_t n, void** ok, void** ot, uint32_t** ol, uint32_t** orr) {
    e.grow(e.ev_keys, n * sizeof(K) + 8);
    if (e.tag_bytes) e.grow(e.ev_tags, n * e.tag_bytes + 8);
    if (e.record) {
      e.grow(e.ev_l, n * 4 + 4);
      e.grow(e.ev_r, n * 4 + 4);
    }
    e.grow(e.flags, n * 4 + 4);
    e.grow(e.pos, (n + 1) * 4);
    a.keep = e.flags.as<uint32_t>();
    *ok = e.ev_keys.p;
    *ot = e.tag_bytes ? e.ev_tags.p : nullptr;
    *ol = e.record ? e.ev_l.as<uint32_t>() : nullptr;
    *orr = e.record ? e.ev_r.as<uint32_t>() : nullptr;
  };
  auto append_kept = [&](size_t n) {
    scan(e, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), n, S_SCAN, true);
    const size_t kept = e.read_total(S_SCAN);
    if (!kept) return;
    head_room(kept);
    void *ok, *ot;
    uint32_t *ol, *orr;
    out_ptrs(&ok, &ot, &ol, &orr);
    const uint32_t* f = e.flags.as<uint32_t>();
    const uint32_t* pos = e.pos.as<uint32_t>();
    compact(e.ev_keys.p, f, pos, n, sizeof(K), ok, e.stream);
    if (e.tag_bytes) compact(e.ev_tags.p, f, pos, n, e.tag_bytes, ot, e.stream);
    if (e.record) {
      compact(e.ev_l.p, f, pos, n, 4, ol, e.stream);
      compact(e.ev_r.p, f, pos, n, 4, orr, e.stream);
    }
    H.ncand += kept;
  };

  // Room for an emission over `add` slots: one wave segment per 256 slots;
  // returns the emission's arguments (segments start after the round's
  // earlier emissions into the same relation).
  auto dense_room = [&](size_t add, int items) {
    const size_t used = H.nseg, segs = e.record ? dense_segments(add, items) : 0;
    const size_t slots = (used + segs) * DENSE_SEG, uslots = used * DENSE_SEG;
    if (e.record) {
      e.grow(H.log_keys, slots * sizeof(K), true, uslots * sizeof(K));
      e.grow(H.log_l, slots * 4, true, uslots * 4);
      e.grow(H.log_r, slots * 4, true, uslots * 4);
      e.grow(H.seg_lcount, (used + segs) * 4, true, used * 4);
    }
    e.stats.candidates += add;
    DenseArgs d = dense_args(e, H);
    H.nseg = used + segs;
    return d;
  };

  if (pl.steps.empty()) {  // single-atom rule: permutation projection, tags copied
    a.dkeys = cur.keys;
    a.dtags = cur.tags;
    a.dids = cur.ids;
    a.n = cur.n;
    a.dlay = e.layout(cur.ncols);
    a.olay = e.layout(har);
    for (int c = 0; c < har; ++c) a.osrc[c] = pl.project[c];
    if (H.dense) {
      const DenseArgs d = dense_room(cur.n, 4);
      project_dense<K>(a, e.tag_kind, d, e.record, e.stream);
      return;
    }
    void *ok, *ot;
    uint32_t *ol, *orr;
    if (a.ev.n) {
      stage(cur.n, &ok, &ot, &ol, &orr);
      project_rows<K>(a, e.tag_kind, ok, ot, ol, orr, e.stream);
      append_kept(cur.n);
      return;
    }
    head_room(cur.n);
    out_ptrs(&ok, &ot, &ol, &orr);
    project_rows<K>(a, e.tag_kind, ok, ot, ol, orr, e.stream);
    H.ncand += cur.n;
    return;
  }

  DevBuf* tmp_keys[2] = {&e.tmpA_keys, &e.tmpB_keys};
  DevBuf* tmp_tags[2] = {&e.tmpA_tags, &e.tmpB_tags};
  // Joins whose outputs exceed the 32-bit offsets (or the max_join_outputs
  // option) run in chunks of probe rows, each chunk through the remaining
  // steps before the next one starts (depth first: the step buffers are
  // reused).  A chunk is cut from the per-row match counts read back once.
  const uint64_t limit = e.opts.max_join_outputs ? std::min<uint64_t>(e.opts.max_join_outputs, 0xffffffffull)
                                                 : 0xffffffffull;
  std::function<void(size_t, Cur)> steps_from = [&](size_t si, Cur cur) {
    const Step& step = pl.steps[si];
    a.ev = si + 1 == pl.steps.size() ? ev_out : EvalCode{};
    a.keep = nullptr;
    ensure_index<K>(e, step.index);
    const IndexState& ix = e.idx[step.index];
    const IndexSpec& spec = e.prog.indexes[step.index];
    const int iar = e.prog.rels[spec.rel].arity;
    a.dkeys = cur.keys;
    a.dtags = cur.tags;
    a.dids = cur.ids;
    a.n = cur.n;
    a.dlay = e.layout(cur.ncols);
    a.w = spec.w;
    for (int j = 0; j < spec.w; ++j) a.jsrc[j] = step.join_src[j];
    a.off = ix.use_hash ? nullptr : ix.off.as<uint32_t>();
    a.hslots = ix.use_hash ? ix.hash.as<HSlot>() : nullptr;
    a.hmask = ix.hmask;
    a.ikeys = ix.t.keys.p;
    a.itags = ix.t.tags.p;
    a.iids = ix.t.ids.as<uint32_t>();
    a.ilay = e.layout(iar);
    const int ocols = (int)step.out_vars.size();
    a.olay = e.layout(ocols);
    for (int c = 0; c < ocols; ++c) a.osrc[c] = step.out_src[c];
    a.index_first = step.body_pos < cur.minpos;
    (void)rule;

    e.grow(e.counts, cur.n * 4 + 4);
    e.grow(e.offs, (cur.n + 1) * 4);
    e.grow(e.istart, cur.n * 4 + 4);
    a.istart = e.istart.as<uint32_t>();
    const bool last = si + 1 == pl.steps.size();
    // the total stays on the device only when it cannot pass the limit
    const size_t in = std::max<size_t>(ix.t.n, 1);
    const uint64_t bound = cur.n > ((size_t)1 << 40) / in ? ((uint64_t)1 << 40) : (uint64_t)cur.n * in;
    const bool nosync = last && H.dense && !e.record && bound <= limit;
    // without a host readback the scan also adds its total to the run's
    // candidate count (collected at round end)
    if (!join_count_scan<K>(a, e.offs.as<uint32_t>(), e.cs_state.as<uint64_t>(), total_slot(e, S_SCAN),
                            nosync ? total_slot(e, S_CAND) : nullptr, total_slot(e, S_OVF), e.stream)) {
      join_count<K>(a, e.counts.as<uint32_t>(), e.stream);
      scan(e, e.counts.as<uint32_t>(), e.offs.as<uint32_t>(), cur.n, S_SCAN, true,
           nosync ? total_slot(e, S_CAND) : nullptr);
    }
    if (nosync) {
      // no host readback: the expand reads the total on the device; the
      // candidate count is collected at round end
      const DenseArgs d = dense_room(0, a.items);
      RowWindows rw{};
      const bool rows = e.cfg.rows && row_windows<K>(e, pl, &rw);
      join_expand_dense<K>(a, e.tag_kind, e.offs.as<uint32_t>(), 0, total_slot(e, S_SCAN), bound, d, false,
                           e.stream, rows ? &rw : nullptr);
      return;
    }
    const uint64_t total = e.read_total(S_SCAN);
    if (total == 0) return;
    if (total > limit) {
      // per-row match counts -> chunks of rows with at most `limit` outputs
      join_count<K>(a, e.counts.as<uint32_t>(), e.stream);
      std::vector<uint32_t> cnt(cur.n);
      DL_HIP(hipMemcpyAsync(cnt.data(), e.counts.p, cur.n * 4, hipMemcpyDeviceToHost, e.stream));
      e.sync();
      size_t r0 = 0;
      while (r0 < cur.n) {
        uint64_t acc = 0;
        size_t r1 = r0;
        while (r1 < cur.n && acc + cnt[r1] <= limit) acc += cnt[r1++];
        if (r1 == r0)
          throw Error{DL_ERR_CAPACITY, "one probe row has more than " + std::to_string(limit) + " join outputs"};
        Cur part = cur;
        part.keys = static_cast<const K*>(cur.keys) + r0;
        part.tags = cur.tags ? static_cast<const uint8_t*>(cur.tags) + r0 * e.tag_bytes : nullptr;
        part.ids = cur.ids ? cur.ids + r0 : nullptr;
        part.n = r1 - r0;
        steps_from(si, part);
        r0 = r1;
      }
      return;
    }
    if (last && H.dense) {
      const DenseArgs d = dense_room(total, a.items);
      RowWindows rw{};
      const bool rows = e.cfg.rows && row_windows<K>(e, pl, &rw);
      join_expand_dense<K>(a, e.tag_kind, e.offs.as<uint32_t>(), total, nullptr, total, d, e.record, e.stream,
                           rows ? &rw : nullptr);
      return;
    }
    if (last && H.ncand + total > 0xffffffffull)
      throw Error{DL_ERR_CAPACITY, "more than 2^32 candidate tuples in one round (sort-based deduplication)"};
    void *ok, *ot;
    uint32_t *ol = nullptr, *orr = nullptr;
    if (last && a.ev.n) {
      stage(total, &ok, &ot, &ol, &orr);
    } else if (last) {
      head_room(total);
      out_ptrs(&ok, &ot, &ol, &orr);
    } else {
      DevBuf& kb = *tmp_keys[si & 1];
      DevBuf& tb = *tmp_tags[si & 1];
      e.grow(kb, total * sizeof(K));
      if (e.tag_bytes) e.grow(tb, total * e.tag_bytes);
      ok = kb.p;
      ot = e.tag_bytes ? tb.p : nullptr;
    }
    join_expand<K>(a, e.tag_kind, e.offs.as<uint32_t>(), total, ok, ot, ol, orr, e.stream);
    if (last && a.ev.n) {
      append_kept(total);
    } else if (last) {
      H.ncand += total;
    } else {
      steps_from(si + 1, Cur{ok, ot, nullptr, total, ocols, std::min(cur.minpos, step.body_pos)});
    }
  };
  steps_from(0, cur);
}

// Dense-domain round end: the touched keys are exactly the new and changed
// tuples; sort them into the next recent relation and publish their state.
template <typename K>
size_t absorb_dense(Engine& e, int r) {
  RelState& R = e.rel[r];
  hipStream_t st = e.stream;
  const size_t nseg = R.nseg;
  R.nseg = 0;
  // touched counts per bitmap block -> positions of the new / changed tuples
  const size_t nb = dense_count_blocks(R.dense_keys);
  e.grow(e.flags, nb * 4);
  e.grow(e.pos, (nb + 1) * 4);
  DenseArgs d = dense_args(e, R);
  if (!e.lineage && R.dense_keys * (sizeof(K) + 4) <= ((size_t)1 << 30)) {
    // recent sized for the whole domain: compact first (single pass), read
    // the count after (one host sync per relation and round)
    e.grow(R.recent.keys, R.dense_keys * sizeof(K) + 8);
    if (e.tag_kind == TAG_F32) e.grow(R.recent.tags, R.dense_keys * 4 + 8);
    dense_finalize<K>(d, R.dense_keys, nullptr, R.recent.keys.as<K>(),
                      e.tag_kind == TAG_F32 ? R.recent.tags.as<float>() : nullptr, 0, nullptr, total_slot(e, S_UNIQUE),
                      st, nullptr, false, nullptr, R.lb_state.as<uint64_t>());
    e.read_totals();
    check_overflow(e);
    const size_t U = e.host[S_UNIQUE];
    R.recent.n = U;
    if (U == 0) return 0;
    e.stats.unique += U;
    ++R.version;
    ++R.rversion;
    if (R.own_index) materialize_full<K>(e, R);
    return U;
  }
  bitmap_block_counts(d.touched, R.dense_keys, e.flags.as<uint32_t>(), st);
  scan(e, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), nb, S_UNIQUE, true);
  if (e.record && nseg) {
    e.grow(e.lpos, (nseg + 1) * 4);
    scan(e, R.seg_lcount.as<uint32_t>(), e.lpos.as<uint32_t>(), nseg, S_LIN, true);
  }
  e.read_totals();
  check_overflow(e);
  const size_t U = e.host[S_UNIQUE], L = e.record && nseg ? e.host[S_LIN] : 0;
  if (U == 0) {
    R.recent.n = 0;
    return 0;
  }
  e.stats.unique += U;
  e.grow(R.recent.keys, U * sizeof(K) + 8);
  float* rtags = nullptr;
  if (e.tag_kind == TAG_F32) {
    e.grow(R.recent.tags, U * 4 + 8);
    rtags = R.recent.tags.as<float>();
  }
  const uint32_t base = e.next_id;
  if (e.lineage) e.grow(e.tag_by_id, ((size_t)base + U) * 4, true, (size_t)base * 4);
  d = dense_args(e, R);
  dense_finalize<K>(d, R.dense_keys, e.pos.as<uint32_t>(), R.recent.keys.as<K>(), rtags, base,
                    e.lineage ? e.tag_by_id.as<float>() : nullptr, nullptr, st, nullptr, true);
  if (e.lineage) {
    e.grow(R.recent.ids, U * 4 + 4);
    iota_u32(R.recent.ids.as<uint32_t>(), U, base, st);
    e.next_id = base + (uint32_t)U;
  }
  if (e.record && keep_lineage(e, L)) {
    const size_t used = e.lin_n;
    e.grow(e.lin_owner, (used + L) * 4 + 4, true, used * 4);
    e.grow(e.lin_l, (used + L) * 4 + 4, true, used * 4);
    e.grow(e.lin_r, (used + L) * 4 + 4, true, used * 4);
    if (L) {
      segments_lineage<K>(d, e.lpos.as<uint32_t>(), nseg, e.lin_owner.as<uint32_t>() + used,
                          e.lin_l.as<uint32_t>() + used, e.lin_r.as<uint32_t>() + used, st);
    }
    e.lin_segs.push_back({used, L});
    e.lin_n = used + L;
    e.stats.lineage += L;
  }
  R.recent.n = U;
  ++R.version;
  ++R.rversion;
  if (R.own_index) materialize_full<K>(e, R);
  return U;
}

template <typename K>
size_t absorb_sorted(Engine& e, int r);

// Fold a relation's round into the store; returns the size of the next
// recent relation.  Under frozen tags that is the number of new tuples, and
// none new means the stable part is the whole relation.
template <typename K>
size_t absorb(Engine& e, int r) {
  RelState& R = e.rel[r];
  const size_t n = R.dense ? absorb_dense<K>(e, r) : absorb_sorted<K>(e, r);
  R.stable_full = n == 0;
  ++R.sversion;
  return n;
}

// Deduplicate a relation's candidates and fold them into the store.
// Returns the number of tuples that are new or changed (the next recent).
template <typename K>
size_t absorb_sorted(Engine& e, int r) {
  RelState& R = e.rel[r];
  const size_t C = R.ncand;
  R.ncand = 0;
  if (C == 0) {
    R.recent.n = 0;
    return 0;
  }
  e.stats.candidates += C;
  const int ar = e.prog.rels[r].arity;
  const size_t kb = sizeof(K), tb = e.tag_bytes;
  const bool use_perm = e.tag_kind == TAG_TOPK || e.tag_kind == TAG_TOPK4 || e.tag_kind == TAG_VID || e.record;
  hipStream_t st = e.stream;

  K* kp = R.cand_keys.as<K>();
  uint32_t* vp = nullptr;
  K* uk;     // the round's distinct keys, sorted, and their +-folded tags
  void* ut;
  size_t U;
  // hash-set deduplication (f32 or no tags, no lineage record, keys below
  // the full width of K so that all ones marks an empty slot)
  const bool hset = e.opts.dedup == 3 && !use_perm && e.key_width(ar) < (int)(8 * sizeof(K));
  if (hset) {
    // 1'. candidates into a hash set at most half full, tags folded per key
    const int mode = e.tag_kind == TAG_NONE ? DENSE_BOOL
                     : e.sr == DL_MAXMIN    ? DENSE_MAX
                     : e.sr == DL_MINPLUS   ? DENSE_MIN
                                            : DENSE_ADD;
    size_t slots = 64;
    while (slots < 2 * C) slots *= 2;
    if (slots > ((size_t)1 << 32)) throw Error{DL_ERR_CAPACITY, "hash set above 2^32 slots"};
    e.grow(e.alt_keys, slots * kb);
    if (tb) e.grow(e.alt_vals, slots * 4);
    K* hk = e.alt_keys.as<K>();
    uint32_t* ht = tb ? e.alt_vals.as<uint32_t>() : nullptr;
    hset_prepare<K>(hk, ht, slots, mode, st);
    hset_insert<K>(kp, tb ? R.cand_tags.as<float>() : nullptr, C, hk, ht, (uint32_t)(slots - 1), mode, st);
    // 2'. occupied slots -> distinct keys (into the candidate buffers), sorted
    e.grow(e.flags, slots * 4);
    e.grow(e.pos, (slots + 1) * 4);
    hset_flags<K>(hk, slots, e.flags.as<uint32_t>(), st);
    scan(e, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), slots, S_UNIQUE, true);
    U = e.read_total(S_UNIQUE);
    hset_compact<K>(hk, ht, e.pos.as<uint32_t>(), slots, mode, kp, tb ? R.cand_tags.as<float>() : nullptr, st);
    vp = tb ? R.cand_tags.as<uint32_t>() : nullptr;
    sort_pairs<K>(e, &kp, &vp, U, e.key_width(ar));
    uk = kp;
    ut = vp;
  } else {
    // 1. sort the candidates by packed key (stable: derivation order kept)
    if (use_perm) {
      e.grow(e.vals, C * 4);
      iota_u32(e.vals.as<uint32_t>(), C, 0, st);
      vp = e.vals.as<uint32_t>();
    } else if (e.tag_kind == TAG_F32) {
      vp = R.cand_tags.as<uint32_t>();
    }
    sort_pairs<K>(e, &kp, &vp, C, e.key_width(ar));

    // 2. runs of equal keys -> one row each, tags +-folded in sorted order
    e.grow(e.flags, C * 4);
    e.grow(e.pos, (C + 1) * 4);
    head_flags<K>(kp, C, e.flags.as<uint32_t>(), st);
    scan(e, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), C, S_UNIQUE, true);
    U = e.read_total(S_UNIQUE);
    e.grow(e.ukeys, U * kb);
    if (tb) e.grow(e.utags, U * tb);
    const void* tsrc = use_perm ? R.cand_tags.p : (const void*)vp;
    segment_reduce<K>(kp, e.pos.as<uint32_t>(), e.flags.as<uint32_t>(), C, e.tag_kind, e.sr, e.k, tsrc,
                      use_perm ? vp : nullptr, e.ukeys.as<K>(), e.utags.p, U, st);
    uk = e.ukeys.as<K>();
    ut = e.utags.p;
  }
  e.stats.unique += U;

  // 3. difference / +-merge against the full relation
  e.grow(e.status, U * 4);
  diff_merge<K>(uk, ut, U, R.full.keys.as<K>(), R.full.tags.p, R.full.n, e.tag_kind, e.sr, e.k, e.converge,
                e.status.as<uint32_t>(), nullptr, st);
  e.grow(e.nflags, U * 4);
  e.grow(e.newpos, (U + 1) * 4);
  status_flags(e.status.as<uint32_t>(), U, 1u, e.nflags.as<uint32_t>(), st);
  scan(e, e.nflags.as<uint32_t>(), e.newpos.as<uint32_t>(), U, S_NEW, true);
  if (e.converge) {
    e.grow(e.rflags, U * 4);
    e.grow(e.rpos, (U + 1) * 4);
    status_flags(e.status.as<uint32_t>(), U, 3u, e.rflags.as<uint32_t>(), st);
    scan(e, e.rflags.as<uint32_t>(), e.rpos.as<uint32_t>(), U, S_RECENT, true);
  }
  e.read_totals();
  const size_t N = e.host[S_NEW];
  const size_t Rn = e.converge ? e.host[S_RECENT] : N;
  const uint32_t* rfl = e.converge ? e.rflags.as<uint32_t>() : e.nflags.as<uint32_t>();
  const uint32_t* rps = e.converge ? e.rpos.as<uint32_t>() : e.newpos.as<uint32_t>();

  // 4. next recent relation = new (and, converging, changed) tuples, sorted
  e.grow(R.recent.keys, Rn * kb + 8);
  compact(uk, rfl, rps, U, kb, R.recent.keys.p, st);
  if (tb) {
    e.grow(R.recent.tags, Rn * tb + 8);
    compact(ut, rfl, rps, U, tb, R.recent.tags.p, st);
  }
  R.recent.n = Rn;
  ++R.rversion;
  if (Rn && e.converge) ++R.version;  // in-place tag updates
  if (N == 0) return Rn;

  // 5. rows to merge: the new tuples
  const void* nk;
  const void* nt;
  const uint32_t* nid = nullptr;
  if (e.converge) {
    e.grow(e.nkeys, N * kb);
    compact(uk, e.nflags.as<uint32_t>(), e.newpos.as<uint32_t>(), U, kb, e.nkeys.p, st);
    if (tb) {
      e.grow(e.ntags, N * tb);
      compact(ut, e.nflags.as<uint32_t>(), e.newpos.as<uint32_t>(), U, tb, e.ntags.p, st);
    }
    nk = e.nkeys.p;
    nt = e.ntags.p;
  } else {
    nk = R.recent.keys.p;
    nt = R.recent.tags.p;
  }
  if (e.lineage) {
    // ids of the new tuples, their tags by id, and their discovery derivations
    const uint32_t base = e.next_id;
    e.grow(R.recent.ids, N * 4 + 4);
    iota_u32(R.recent.ids.as<uint32_t>(), N, base, st);
    nid = R.recent.ids.as<uint32_t>();
    e.grow(e.tag_by_id, ((size_t)base + N) * 4, true, (size_t)base * 4);
    DL_HIP(hipMemcpyAsync(e.tag_by_id.as<float>() + base, nt, N * 4, hipMemcpyDeviceToDevice, st));
    e.next_id = base + (uint32_t)N;
  }
  if (e.record) {
    e.grow(e.lf, C * 4);
    e.grow(e.lpos, (C + 1) * 4);
    lineage_flags(e.pos.as<uint32_t>(), e.flags.as<uint32_t>(), e.status.as<uint32_t>(), C, e.lf.as<uint32_t>(), st);
    scan(e, e.lf.as<uint32_t>(), e.lpos.as<uint32_t>(), C, S_LIN, true);
    const size_t L = e.read_total(S_LIN);
    if (keep_lineage(e, L)) {
      const size_t used = e.lin_n;
      e.grow(e.lin_owner, (used + L) * 4, true, used * 4);
      e.grow(e.lin_l, (used + L) * 4, true, used * 4);
      e.grow(e.lin_r, (used + L) * 4, true, used * 4);
      lineage_emit(e.pos.as<uint32_t>(), e.flags.as<uint32_t>(), e.lf.as<uint32_t>(), e.lpos.as<uint32_t>(),
                   e.newpos.as<uint32_t>(), vp, R.cand_l.as<uint32_t>(), R.cand_r.as<uint32_t>(), C,
                   e.next_id - (uint32_t)N, e.lin_owner.as<uint32_t>() + used, e.lin_l.as<uint32_t>() + used,
                   e.lin_r.as<uint32_t>() + used, st);
      e.lin_segs.push_back({used, L});
      e.lin_n = used + L;
      e.stats.lineage += L;
    }
  }

  // 6. full' = merge(full, new)
  const size_t F = R.full.n;
  e.grow(R.full_alt.keys, (F + N) * kb + 8);
  if (tb) e.grow(R.full_alt.tags, (F + N) * tb + 8);
  if (e.lineage) e.grow(R.full_alt.ids, (F + N) * 4 + 4);
  ensure_scratch(e, merge_scratch_words(F, N));
  merge_sorted<K>(R.full.keys.as<K>(), R.full.tags.p, R.full.ids.as<uint32_t>(), F, (const K*)nk, nt, nid, N, tb,
                  R.full_alt.keys.as<K>(), R.full_alt.tags.p, e.lineage ? R.full_alt.ids.as<uint32_t>() : nullptr,
                  e.work.as<uint64_t>(), st);
  std::swap(R.full, R.full_alt);
  R.full.n = F + N;
  ++R.version;
  return Rn;
}

// ------------------------------------------------ batched (graph) rounds
// A stratum whose single relation uses the dense-domain path without lineage
// and whose delta plans are all static-driven single joins against an
// identity-ordered index over the recent tuples has a round body with only
// device-side sizes: the recent index is rebuilt from the previous round's
// count (a device word), the join reads its total on the device, the round
// end compacts the touched bitmap.  Such bodies run several rounds per host
// sync (as one captured HIP graph where allowed), the host reading back one
// block of counters and the round log per batch.
std::vector<const Plan*> batch_plans(Engine& e, const Stratum& st) {
  std::vector<const Plan*> out;
  if (e.lineage || st.rels.size() != 1 || st.delta_plans.empty()) return {};
  const int r = st.rels[0];
  if (!e.rel[r].dense || e.cfg.orient == 1) return {};
  for (int p : st.delta_plans) {
    const Plan& pl = e.prog.plans[p];
    if (pl.alt < 0 || pl.eval) return {};
    const Plan& tw = e.prog.plans[pl.alt];
    if (tw.steps.size() != 1) return {};
    const IndexSpec& ix = e.prog.indexes[tw.steps[0].index];
    if (!ix.recent || !ix.identity() || ix.rel != r) return {};
    if (e.rel[tw.driver_rel].full.n == 0) return {};
    out.push_back(&tw);
  }
  return out;
}

template <typename K>
JoinArgs batch_join_args(Engine& e, const Plan& tw, RelState& R, int ar) {
  const Step& step = tw.steps[0];
  const IndexSpec& spec = e.prog.indexes[step.index];
  const RelState& D = e.rel[tw.driver_rel];
  JoinArgs a{};
  a.sr = e.sr;
  a.k = e.k;
  a.q = e.qtab.as<float>();
  a.items = e.cfg.items;
  a.dkeys = D.full.keys.p;
  a.dtags = D.full.tags.p;
  a.dids = nullptr;
  a.n = D.full.n;
  a.dlay = e.layout(e.prog.rels[tw.driver_rel].arity);
  a.w = spec.w;
  for (int j = 0; j < spec.w; ++j) a.jsrc[j] = step.join_src[j];
  a.off = e.idx[step.index].off.as<uint32_t>();
  a.ikeys = R.recent.keys.p;
  a.itags = R.recent.tags.p;
  a.iids = nullptr;
  a.ilay = e.layout(ar);
  const int ocols = (int)step.out_vars.size();
  a.olay = e.layout(ocols);
  for (int c = 0; c < ocols; ++c) a.osrc[c] = step.out_src[c];
  a.index_first = step.body_pos < tw.driver_atom;
  a.istart = e.istart.as<uint32_t>();
  return a;
}

// Whether the round end can write the recent index's CSR itself (see
// DenseCsr): one plan, one sample, an index on the first column of the
// recent tuples in key order.
bool finalize_writes_csr(const Engine& e, int r, const std::vector<const Plan*>& plans) {
  if (plans.size() != 1 || e.batched || e.prog.rels[r].arity < 2) return false;
  const IndexSpec& spec = e.prog.indexes[plans[0]->steps[0].index];
  return spec.rel == r && spec.w == 1 && spec.identity() && spec.recent;
}

// Enqueue one round body (no host interaction: capturable).  With
// `fin_csr` the previous body's round end (or the caller, before the first
// body) has written the recent index.
template <typename K>
void enqueue_round_body(Engine& e, int r, const std::vector<const Plan*>& plans, bool fin_csr) {
  RelState& R = e.rel[r];
  hipStream_t st = e.stream;
  const int ar = e.prog.rels[r].arity;
  for (const Plan* tw : plans) {
    const Step& step = tw->steps[0];
    const IndexSpec& spec = e.prog.indexes[step.index];
    const int pbits = e.sbits + spec.w * e.cbits;
    if (!fin_csr)
      csr_build_dn<K>(R.recent.keys.as<K>(), total_slot(e, S_UNIQUE), e.key_width(ar), pbits,
                      e.idx[step.index].off.as<uint32_t>(), st);
    const JoinArgs a = batch_join_args<K>(e, *tw, R, ar);
    if (!join_count_scan<K>(a, e.offs.as<uint32_t>(), e.cs_state.as<uint64_t>(), total_slot(e, S_SCAN),
                            total_slot(e, S_CAND), total_slot(e, S_OVF), st)) {
      join_count<K>(a, e.counts.as<uint32_t>(), st);
      scan_u32(e.counts.as<uint32_t>(), e.offs.as<uint32_t>(), a.n, total_slot(e, S_SCAN), true,
               e.work.as<uint64_t>(), st, total_slot(e, S_CAND));
    }
    DenseArgs d = dense_args(e, R);
    RowWindows rw{};
    const bool rows = e.cfg.rows && row_windows<K>(e, *tw, &rw);
    join_expand_dense<K>(a, e.tag_kind, e.offs.as<uint32_t>(), 0, total_slot(e, S_SCAN), (size_t)1 << 40, d, false,
                         st, rows ? &rw : nullptr);
  }
  const DenseArgs d = dense_args(e, R);
  DenseCsr csr;
  if (fin_csr) {
    const uint32_t n = e.max_id + 1;
    csr = dense_csr(e.idx[plans[0]->steps[0].index].off.as<uint32_t>(), (uint32_t)(R.dense_keys / n / 32), n);
  }
  dense_finalize<K>(d, R.dense_keys, nullptr, R.recent.keys.as<K>(),
                    e.tag_kind == TAG_F32 ? R.recent.tags.as<float>() : nullptr, 0, nullptr, total_slot(e, S_UNIQUE),
                    st, total_slot(e, S_LOG), false, fin_csr ? &csr : nullptr, R.lb_state.as<uint64_t>());
}

// Whether the rounds of a batched stratum can each run as one fused launch
// (window_round): one static-driven plan with the row-window shape whose
// index is the recent relation on its first column.  Fills rw (and builds
// the driver's prefix CSR) when they can.
template <typename K>
bool fused_eligible(Engine& e, int r, const std::vector<const Plan*>& plans, RowWindows* rw) {
  if (!e.cfg.fused || plans.size() != 1 || e.prog.rels[r].arity < 2) return false;
  const Plan& tw = *plans[0];
  const IndexSpec& spec = e.prog.indexes[tw.steps[0].index];
  if (!(spec.rel == r && spec.w == 1 && spec.identity() && spec.recent)) return false;
  if (!row_windows<K>(e, tw, rw)) return false;
  return window_round_fits(rw->wkeys);
}

// Rounds 2.. as fused launches over a window-layout recent relation (see
// k_window_round); four rounds per host synchronisation (eight while the
// rounds shrink by less than 30 % a round), as one captured
// HIP graph where allowed (timed, when profiling, by events around each
// replay).  Each batch of rounds takes a group batch width from the size of
// the last round seen, as the ratio r of the average group's derivations
// (the last round's new or changed tuples times the drivers per group, over
// the groups) to the dense threshold: 8 groups per workgroup (a wave per
// group) below r = 2, then 4 (below 4), 2 (below 16) and one group per
// workgroup -- fewer groups queue behind one workgroup's dense ones as more
// of them are dense (thresholds measured on ER graphs).  Returns the number
// of rounds run.
template <typename K>
int fused_rounds(Engine& e, const Stratum& st, const Plan& tw, const RowWindows& rw) {
  const int r = st.rels[0];
  RelState& R = e.rel[r];
  const int ar = e.prog.rels[r].arity;
  const size_t keys = R.dense_keys;
  // groups of the rounds: one engine's ids in use (groups past the largest
  // id have no driver rows), a batched engine's whole (sample, id) prefix
  const uint32_t ng = e.batched ? (uint32_t)rw.ngroups : (uint32_t)std::min<uint64_t>(rw.ngroups, (uint64_t)e.max_id + 1);
  const bool f32 = e.tag_kind == TAG_F32;
  DevBuf* rk[2] = {&e.wr_keys0, &e.wr_keys1};
  DevBuf* rt[2] = {&e.wr_tags0, &e.wr_tags1};
  DevBuf* rc[2] = {&e.wr_cnt0, &e.wr_cnt1};
  for (int i = 0; i < 2; ++i) {
    e.grow(*rk[i], keys * sizeof(K) + 8);
    if (f32) e.grow(*rt[i], keys * 4 + 8);
    e.grow(*rc[i], (size_t)ng * 4 + 4);
  }
  // group batch widths (groups per workgroup batch) a batch of rounds can take
  constexpr int NW = 4;
  const uint32_t widths[NW] = {WINDOW_ROUND_WIDE, WINDOW_ROUND_WIDE / 2, WINDOW_ROUND_WIDE / 4, 1};
  unsigned nbw[NW], nbmax = 0;
  for (int m = 0; m < NW; ++m) nbmax = std::max(nbmax, nbw[m] = window_round_grid(ng, widths[m]));
  // a batch is BATCH_ROUNDS rounds, or twice that while the rounds shrink
  // slowly; both even, so that a batch ends with the recent tuples back in
  // window set 0
  constexpr int LONG_ROUNDS = 2 * BATCH_ROUNDS;
  static_assert(BATCH_ROUNDS % 2 == 0, "a batch ends in window set 0");
  e.grow(e.wr_part, (size_t)LONG_ROUNDS * nbmax * 2 * 4);
  // round 1's recent tuples (sorted) into window layout, through their CSR
  // over (sample, first column)
  const int ir = tw.steps[0].index;
  IndexState& ix = e.idx[ir];
  e.grow(ix.off, (rw.ngroups + 1) * 4);
  csr_build<K>(R.recent.keys.as<K>(), R.recent.n, e.key_width(ar), e.sbits + e.cbits, ix.off.as<uint32_t>(), e.stream);
  const DenseArgs d = dense_args(e, R);
  WindowRecent w[2];
  for (int i = 0; i < 2; ++i)
    w[i] = WindowRecent{rc[i]->as<uint32_t>(), rk[i]->p, f32 ? rt[i]->as<float>() : nullptr};
  to_windows<K>(R.recent.keys.as<K>(), f32 ? R.recent.tags.as<float>() : nullptr, R.recent.n, ix.off.as<uint32_t>(), ng,
                d, w[0], e.stream);
  const JoinArgs a = batch_join_args<K>(e, tw, R, ar);
  RoundArgs ra{};
  ra.goff = rw.goff;
  ra.ngroups = ng;
  ra.win_per_key = e.cfg.rows == 0 ? ~0u : e.cfg.rows == 2 ? 0u : 12u;
  e.sync();
  // Every round writes its workgroups' counts to its own part of wr_part;
  // after a batch one small launch adds them up per round into the total
  // slots, which the host reads back with the others.
  static_assert(S_PART + 2 * LONG_ROUNDS <= 30, "batch totals overlap other slots");
  auto enqueue_rounds = [&](int m, int len) {
    ra.batch = widths[m];
    for (int i = 0; i < len; ++i) {
      ra.cur = w[i & 1];
      ra.next = w[(i + 1) & 1];
      ra.part = e.wr_part.as<uint32_t>() + (size_t)i * nbw[m] * 2;
      window_round<K>(a, e.tag_kind, d, ra, e.stream);
    }
  };
  auto enqueue_readback = [&](int m, int len) {
    sum_parts(e.wr_part.as<uint32_t>(), nbw[m], (unsigned)len, total_slot(e, S_PART), e.stream);
    DL_HIP(hipMemcpyAsync(e.host, e.dtotal.p, 64 * sizeof(uint64_t), hipMemcpyDeviceToHost, e.stream));
  };
  // The graph holds the rounds' launches only, so that two events around a
  // replay time exactly them when profiling (events recorded inside a graph
  // carry no time): the launches' records (family, bytes) are kept from the
  // capture and counted once per replay.  A graph is captured once per batch
  // shape (gi = width m, plus NW for a long batch) and kept in the engine for
  // later runs while every argument of its launches is the same.
  static_assert(2 * NW <= (int)(sizeof(e.fused_graph) / sizeof(e.fused_graph[0])), "a cached graph per shape");
  bool tried[2 * NW] = {};
  hipEvent_t span[2] = {nullptr, nullptr};
  if (g_prof) {
    span[0] = g_prof->get();
    span[1] = g_prof->get();
  }
  auto graph_key = [&](int gi) {
    const int m = gi % NW, len = gi < NW ? BATCH_ROUNDS : LONG_ROUNDS;
    std::vector<unsigned char> k;
    auto put = [&](const void* p, size_t n) {
      const unsigned char* c = static_cast<const unsigned char*>(p);
      k.insert(k.end(), c, c + n);
    };
    RoundArgs rk = ra;  // what enqueue_rounds sets per round: from w, wr_part and the width
    rk.cur = rk.next = WindowRecent{};
    rk.part = nullptr;
    rk.batch = widths[m];
    const void* part = e.wr_part.p;
    const int tk = e.tag_kind;
    put(&a, sizeof a);
    put(&d, sizeof d);
    put(&rk, sizeof rk);
    put(w, sizeof w);
    put(&part, sizeof part);
    put(&nbw[m], sizeof nbw[m]);
    put(&len, sizeof len);
    put(&tk, sizeof tk);
    put(&e.stream, sizeof e.stream);
    return k;
  };
  auto release = [&] {
    for (int gi = 0; gi < 2 * NW; ++gi) e.drop_fused_graph(e.fused_graph[gi]);
  };
  auto capture = [&](int gi) {  // the batch body of shape gi as a graph, once
    tried[gi] = true;
    if (!e.cfg.graph) return;
    Engine::FusedGraph& G = e.fused_graph[gi];
    std::vector<unsigned char> key = graph_key(gi);
    // the last run's graph fits: same arguments and, when timing, captured
    // while timing the same families
    const bool fits = G.exec && G.key == key && (!g_prof || (G.profiled && G.prof_mask == g_prof->mask));
    if (fits) {
      if (g_prof && G.defer_fam >= 0) g_prof->defer(G.defer_fam, G.defer_per);  // as its launchers did
      return;
    }
    e.drop_fused_graph(G);
    if (hipStreamBeginCapture(e.stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
      (void)hipGetLastError();
      return;
    }
    const size_t m0 = g_prof ? g_prof->recs.size() : 0;
    bool ok = true;
    try {
      enqueue_rounds(gi % NW, gi < NW ? BATCH_ROUNDS : LONG_ROUNDS);
    } catch (...) {
      ok = false;
    }
    if (hipStreamEndCapture(e.stream, &G.graph) != hipSuccess || !G.graph) ok = false;
    if (ok && hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0) != hipSuccess) ok = false;
    if (g_prof) {  // the launches' records, without their (captured) events' times
      if (ok) G.recs.assign(g_prof->recs.begin() + (std::ptrdiff_t)m0, g_prof->recs.end());
      g_prof->recs.resize(m0);
    }
    if (!ok) {
      e.drop_fused_graph(G);
      (void)hipGetLastError();
      return;
    }
    G.key = std::move(key);
    G.profiled = g_prof != nullptr;
    if (g_prof) {
      G.prof_mask = g_prof->mask;
      G.defer_fam = g_prof->deferred_fam;
      G.defer_per = g_prof->deferred_per;
    }
  };
  // the dense threshold of a group (derivations); the forced settings take
  // one width throughout
  const double per_group = (double)a.n / std::max<uint32_t>(ng, 1u);
  const double dense = ra.win_per_key == ~0u ? -1.0 : (double)rw.wkeys / std::max(ra.win_per_key, 1u);
  uint64_t last = R.recent.n, before = 0;  // the last two rounds' new or changed tuples
  int rounds = 0;
  bool done = false;
  while (!done) {
    int m = 0;
    if (dense >= 0 && ra.win_per_key == 0) {
      m = NW - 1;
    } else if (dense >= 0) {
      const double r = (double)last * per_group / ng / dense;
      m = r < 2.0 ? 0 : r < 4.0 ? 1 : r < 16.0 ? 2 : 3;
    }
    // a long batch while the rounds shrink by less than 30 % a round (a long
    // tail: fewer host synchronisations, and few rounds run past the end)
    const bool lng = last < before && (double)last >= 0.7 * (double)before;
    const int len = lng ? LONG_ROUNDS : BATCH_ROUNDS, gi = m + (lng ? NW : 0);
    if (!tried[gi]) capture(gi);
    hipGraphExec_t exec = e.cfg.graph ? e.fused_graph[gi].exec : nullptr;
    const bool timed = exec && span[0] && span[1];
    if (timed) DL_HIP(hipEventRecord(span[0], e.stream));
    if (exec) DL_HIP(hipGraphLaunch(exec, e.stream));
    else enqueue_rounds(m, len);
    if (timed) DL_HIP(hipEventRecord(span[1], e.stream));
    enqueue_readback(m, len);
    e.sync();
    if (timed) {
      float ms = 0.0f;
      DL_HIP(hipEventElapsedTime(&ms, span[0], span[1]));
      Profiler::fold_span(e.fused_graph[gi].recs, ms, e.kstats);
    }
    if (e.host[S_OVF]) {
      release();
      check_overflow(e);
    }
    for (int i = 0; i < len; ++i) {
      const uint64_t U = e.host[S_PART + 2 * i], C = e.host[S_PART + 2 * i + 1];
      e.log_round(U, C, e.cur_stratum, DL_ROUND_FUSED);
      if (done) continue;  // launched after the last round: found nothing
      ++rounds;
      ++R.version;
      ++R.rversion;
      e.stats.unique += U;
      e.fused_units += C;
      done = U == 0;
      before = last;
      last = U;
    }
  }
  R.recent.n = 0;
  ix.built = false;
  return rounds;  // the graphs stay for the next run
}

// Rounds 2.. of an eligible stratum in batches of device-sized round bodies;
// returns the number of rounds run (the last one changed nothing).
template <typename K>
int batch_rounds(Engine& e, const Stratum& st, const std::vector<const Plan*>& plans) {
  const int r = st.rels[0];
  RelState& R = e.rel[r];
  {
    RowWindows frw{};
    if (fused_eligible<K>(e, r, plans, &frw)) return fused_rounds<K>(e, st, *plans[0], frw);
  }
  // every buffer the body touches at its final size, before any batch (and capture)
  const size_t keys = R.dense_keys;
  e.grow(R.recent.keys, keys * sizeof(K) + 8, true, R.recent.n * sizeof(K));
  if (e.tag_kind == TAG_F32) e.grow(R.recent.tags, keys * 4 + 8, true, R.recent.n * 4);
  size_t words = scan_scratch_words(dense_count_blocks(R.dense_keys));
  for (const Plan* tw : plans) {
    const size_t n = e.rel[tw->driver_rel].full.n;
    e.grow(e.counts, n * 4 + 4);
    e.grow(e.offs, (n + 1) * 4);
    e.grow(e.istart, n * 4 + 4);
    words = std::max(words, scan_scratch_words(n));
    const IndexSpec& spec = e.prog.indexes[tw->steps[0].index];
    e.grow(e.idx[tw->steps[0].index].off, (((size_t)1 << (e.sbits + spec.w * e.cbits)) + 1) * 4);
    RowWindows rw{};
    if (e.cfg.rows) (void)row_windows<K>(e, *tw, &rw);  // builds the driver's prefix CSR outside the graph
  }
  ensure_scratch(e, words);
  const size_t nb = dense_count_blocks(R.dense_keys);
  e.grow(e.flags, nb * 4);
  e.grow(e.pos, (nb + 1) * 4);
  // the first body's recent index (later ones come from the round ends)
  const bool fin_csr = finalize_writes_csr(e, r, plans);
  if (fin_csr) {
    const int ir = plans[0]->steps[0].index;
    csr_build<K>(R.recent.keys.as<K>(), R.recent.n, e.key_width(e.prog.rels[r].arity), e.sbits + e.cbits,
                 e.idx[ir].off.as<uint32_t>(), e.stream);
  }
  e.sync();

  // Rounds go in batches of BATCH_ROUNDS round bodies: the host syncs once
  // per batch and reads each round's new-tuple count from the round log;
  // rounds after the fixpoint in a batch find an empty recent relation and
  // change nothing.  A batch is one captured HIP graph, or -- while kernels
  // are timed (events inside graphs cannot be timed) or when capture is
  // refused -- the same launches enqueued directly.
  auto enqueue_batch = [&] {
    fill_u32(reinterpret_cast<uint32_t*>(total_slot(e, S_LOG)), 2, 0u, e.stream);  // log entries = 0
    for (int i = 0; i < BATCH_ROUNDS; ++i) enqueue_round_body<K>(e, r, plans, fin_csr);
    DL_HIP(hipMemcpyAsync(e.host, e.dtotal.p, 64 * sizeof(uint64_t), hipMemcpyDeviceToHost, e.stream));
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto release = [&] {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  };
  if (e.cfg.graph && !g_prof && hipStreamBeginCapture(e.stream, hipStreamCaptureModeRelaxed) == hipSuccess) {
    bool ok = true;
    try {
      enqueue_batch();
    } catch (...) {
      ok = false;
    }
    if (hipStreamEndCapture(e.stream, &graph) != hipSuccess || !graph) ok = false;
    if (ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) ok = false;
    if (!ok) {
      release();
      (void)hipGetLastError();
    }
  } else {
    (void)hipGetLastError();
  }
  int rounds = 0;
  bool done = false;
  while (!done) {
    if (exec) DL_HIP(hipGraphLaunch(exec, e.stream));
    else enqueue_batch();
    e.sync();
    if (e.host[S_OVF]) {
      release();
      check_overflow(e);
    }
    const uint64_t* log = e.host + S_LOG;
    for (uint64_t i = 0; i < log[0] && !done; ++i) {
      const size_t U = log[1 + i];
      e.log_round(U, ~0ull, e.cur_stratum, DL_ROUND_BATCHED);
      ++rounds;
      ++R.version;
      ++R.rversion;
      e.stats.unique += U;
      done = U == 0;
    }
  }
  R.recent.n = 0;
  release();
  for (const Plan* tw : plans) e.idx[tw->steps[0].index].built = false;
  return rounds;
}

}  // namespace

template <typename K>
void ingest(Engine& e) {
  hipStream_t st = e.stream;
  if (e.sr == DL_TOPK || e.sr == DL_DIFF_TOPK) {
    // proof sets of one word while every sample has at most 64 probabilistic
    // facts, else of four (256)
    uint32_t most = 0;
    for (uint32_t c : e.topk_next) most = std::max(most, c);
    const int W = most > 64 ? 4 : 1;
    e.topk_words = W;
    e.tag_kind = W == 4 ? TAG_TOPK4 : TAG_TOPK;
    e.tag_bytes = W == 4 ? sizeof(TopK4) : sizeof(TopK);
    const size_t ns = std::max<size_t>(e.topk_next.size(), 1), qs = 64 * (size_t)W;
    e.qtab_up.assign(ns * qs, 0.0f);
    for (size_t s = 0; s < e.topk_next.size(); ++s)
      for (size_t i = 0; i < qs; ++i) e.qtab_up[s * qs + i] = e.qtab_h[s * 256 + i];
    e.grow(e.qtab, ns * qs * 4);
    DL_HIP(hipMemcpyAsync(e.qtab.p, e.qtab_up.data(), ns * qs * 4, hipMemcpyHostToDevice, st));
    e.grow(e.grad_fact, ns * qs * 4);
    DL_HIP(hipMemsetAsync(e.grad_fact.p, 0, ns * qs * 4, st));
  } else if (e.tag_kind == TAG_VID) {  // input gradients by fact number
    const size_t q = (size_t)e.nfacts + 1;
    e.grow(e.grad_fact, q * 4);
    DL_HIP(hipMemsetAsync(e.grad_fact.p, 0, q * 4, st));
  }
  uint32_t id = 0;
  for (size_t r = 0; r < e.rel.size(); ++r) {
    if (!e.prog.rels[r].input) continue;
    RelState& R = e.rel[r];
    const size_t n = R.nraw;
    const int ar = e.prog.rels[r].arity;
    R.id_base = id;
    R.full.n = 0;
    R.recent.n = 0;
    ++R.version;
    if (n == 0) continue;
    const KeyLayout lay = e.layout(ar);
    // pack, sort with the fact index as payload, +-merge duplicate facts
    e.grow(R.cand_keys, n * sizeof(K));
    std::vector<const uint32_t*> cols(ar);
    for (int c = 0; c < ar; ++c) cols[c] = R.raw_cols[c].as<uint32_t>();
    pack_rows<K>(cols.data(), R.raw_sample.as<uint32_t>(), n, lay, R.cand_keys.as<K>(), st);
    e.grow(e.vals, n * 4);
    iota_u32(e.vals.as<uint32_t>(), n, 0, st);
    K* kp = R.cand_keys.as<K>();
    uint32_t* vp = e.vals.as<uint32_t>();
    sort_pairs<K>(e, &kp, &vp, n, e.key_width(ar));
    e.grow(e.flags, n * 4);
    e.grow(e.pos, (n + 1) * 4);
    head_flags<K>(kp, n, e.flags.as<uint32_t>(), st);
    scan(e, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), n, S_UNIQUE, true);
    const size_t U = e.read_total(S_UNIQUE);
    const void* ftags = nullptr;
    if (e.tag_kind == TAG_F32) {
      ftags = R.raw_tags.p;
    } else if (e.tag_kind == TAG_TOPK) {
      e.grow(R.cand_tags, n * sizeof(TopK));
      topk_from_facts<1>(R.raw_tags.as<float>(), R.raw_local.as<uint32_t>(), n, R.cand_tags.as<TopK>(), st);
      ftags = R.cand_tags.p;
    } else if (e.tag_kind == TAG_TOPK4) {
      e.grow(R.cand_tags, n * sizeof(TopK4));
      topk_from_facts<4>(R.raw_tags.as<float>(), R.raw_local.as<uint32_t>(), n, R.cand_tags.as<TopK4>(), st);
      ftags = R.cand_tags.p;
    } else if (e.tag_kind == TAG_VID) {
      e.grow(R.cand_tags, n * sizeof(VTag));
      vtags_from_facts(R.raw_tags.as<float>(), R.raw_local.as<uint32_t>(), n, R.cand_tags.as<VTag>(), st);
      ftags = R.cand_tags.p;
    }
    e.grow(R.full.keys, U * sizeof(K) + 8);
    if (e.tag_bytes) e.grow(R.full.tags, U * e.tag_bytes + 8);
    segment_reduce<K>(kp, e.pos.as<uint32_t>(), e.flags.as<uint32_t>(), n, e.tag_kind, e.sr, e.k, ftags, vp,
                      R.full.keys.as<K>(), R.full.tags.p, U, st);
    R.full.n = U;
    e.grow(R.fact_entry, n * 4);
    seg_scatter(e.pos.as<uint32_t>(), e.flags.as<uint32_t>(), vp, n, id, R.fact_entry.as<uint32_t>(), st);
    if (e.lineage) {
      e.grow(R.full.ids, U * 4 + 4);
      iota_u32(R.full.ids.as<uint32_t>(), U, id, st);
    }
    e.grow(R.grad, n * 4);
    DL_HIP(hipMemsetAsync(R.grad.p, 0, n * 4, st));
    id += (uint32_t)U;
  }
  if (e.lineage) {
    e.grow(e.tag_by_id, (size_t)id * 4 + 4);
    for (size_t r = 0; r < e.rel.size(); ++r) {
      RelState& R = e.rel[r];
      if (e.prog.rels[r].input && R.full.n)
        DL_HIP(hipMemcpyAsync(e.tag_by_id.as<float>() + R.id_base, R.full.tags.p, R.full.n * 4,
                              hipMemcpyDeviceToDevice, st));
    }
  }
  for (auto& x : e.idx) x.built = false;
  e.sync();
}

template <typename K>
void run_fixpoint(Engine& e) {
  e.stats.strata = 0;
  e.stats.rounds = 0;
  e.stats.max_rounds = 0;
  e.stats.candidates = 0;
  e.stats.unique = 0;
  e.stats.lineage = 0;
  e.stats.derived = 0;
  uint32_t edb = 0;
  for (size_t r = 0; r < e.rel.size(); ++r) {
    RelState& R = e.rel[r];
    R.ncand = 0;
    if (e.prog.rels[r].input) {
      edb += (uint32_t)R.full.n;
    } else {
      R.full.n = 0;
      R.full_alt.n = 0;
      R.recent.n = 0;
      R.stable_full = false;
      ++R.version;
      ++R.sversion;
    }
  }
  e.next_id = edb;
  e.fused_units = 0;
  e.round_log.clear();
  e.lin_n = 0;
  e.lin_segs.clear();
  e.record = e.lineage && e.lin_budget > 0;
  e.round_ids.clear();
  DL_HIP(hipMemsetAsync(e.dtotal.p, 0, 32 * sizeof(uint64_t), e.stream));
  setup_dense(e);
  // derivations so far: counted on the host, on the device (read with the
  // totals every round reads) and in fused rounds
  e.host[S_CAND] = 0;
  auto derivations = [&] { return e.stats.candidates + e.host[S_CAND] + e.fused_units; };
  e.cur_stratum = 0;
  for (const Stratum& st : e.prog.strata) {
    int rounds = 1;
    std::vector<uint32_t> ids{e.next_id};
    uint64_t d0 = derivations();
    for (int p : st.base_plans) run_plan<K>(e, e.prog.plans[p]);
    size_t changed = 0;
    for (int r : st.rels) changed += absorb<K>(e, r);
    e.log_round(changed, derivations() - d0, e.cur_stratum, DL_ROUND_FIRST);
    if (changed) {
      const std::vector<const Plan*> gp = batch_plans(e, st);
      const int gr = gp.empty() ? 0 : batch_rounds<K>(e, st, gp);
      if (gr > 0) {
        rounds += gr;
        changed = 0;
      }
    }
    while (changed && !st.delta_plans.empty()) {
      ++rounds;
      d0 = derivations();
      for (int p : st.delta_plans) {
        const Plan& pl = e.prog.plans[p];
        // orientation: by default dense heads take the static-driven twin
        // (outputs grouped by the static side: coalesced dense accesses)
        const bool twin = pl.alt >= 0 && (e.cfg.orient == 2 || (e.cfg.orient == 0 && e.rel[pl.head_rel].dense));
        run_plan<K>(e, twin ? e.prog.plans[pl.alt] : pl);
      }
      changed = 0;
      ids.push_back(e.next_id);
      for (int r : st.rels) changed += absorb<K>(e, r);
      e.log_round(changed, derivations() - d0, e.cur_stratum, DL_ROUND_PLAIN);
    }
    ids.push_back(e.next_id);
    if (e.lineage) e.round_ids.push_back(std::move(ids));
    if (changed) ++rounds;  // non-recursive stratum: its second round derives nothing
    for (int r : st.rels) {
      if (e.rel[r].dense) materialize_full<K>(e, e.rel[r]);
      e.rel[r].recent.n = 0;
    }
    e.stats.strata += 1;
    e.stats.rounds += rounds;
    e.stats.max_rounds = std::max(e.stats.max_rounds, rounds);
    ++e.cur_stratum;
  }
  for (size_t r = 0; r < e.rel.size(); ++r)
    if (e.prog.rels[r].derived) e.stats.derived += e.rel[r].full.n;
  e.read_totals();
  check_overflow(e);
  e.stats.candidates += e.host[S_CAND] + e.fused_units;
  e.deferred_units = e.host[S_CAND] + e.fused_units;
  e.stats.lineage_mode = !e.lineage ? 0 : e.record ? 1 : 2;
}

template <typename K>
size_t read_relation_t(Engine& e, int r, size_t capacity, const dl_relation_out* out, int on_device) {
  (void)capacity;
  RelState& R = e.rel[r];
  const size_t n = R.full.n;
  if (n == 0) return 0;
  hipStream_t st = e.stream;
  const int ar = e.prog.rels[r].arity;
  const KeyLayout lay = e.layout(ar);
  // device staging: columns + sample (u32 each), tags (f32), fact numbers, top-k parts
  const bool topk = e.tag_kind == TAG_TOPK || e.tag_kind == TAG_TOPK4;
  const size_t W = topk ? (size_t)e.topk_words : 1;
  const size_t words = (size_t)(ar + 1) * n + 2 * n + (size_t)e.k * n * (2 * W + 1) + n;
  e.grow(e.unpack, words * 4 + 64);
  uint32_t* base = e.unpack.as<uint32_t>();
  uint32_t* dcols[4] = {nullptr, nullptr, nullptr, nullptr};
  uint32_t* dsample = base + (size_t)ar * n;
  float* dtag = reinterpret_cast<float*>(dsample + n);
  uint32_t* dfid = reinterpret_cast<uint32_t*>(dtag + n);
  uint64_t* dbits = reinterpret_cast<uint64_t*>(((uintptr_t)(dfid + n) + 7) & ~(uintptr_t)7);
  float* dprob = reinterpret_cast<float*>(dbits + (size_t)e.k * n * W);
  uint8_t* dcnt = reinterpret_cast<uint8_t*>(dprob + (size_t)e.k * n);
  for (int c = 0; c < ar; ++c) dcols[c] = on_device ? out->columns[c] : (out->columns[c] ? base + (size_t)c * n : nullptr);
  uint32_t* samp = on_device ? out->sample_ids : (out->sample_ids ? dsample : nullptr);
  const bool need_sample = topk && e.batched;
  uint32_t* samp_k = samp ? samp : (need_sample ? dsample : nullptr);
  unpack_rows<K>(R.full.keys.as<K>(), n, lay, dcols, e.batched ? samp_k : nullptr, st);
  if (!e.batched && samp) DL_HIP(hipMemsetAsync(samp, 0, n * 4, st));
  float* tg = out->tags ? (on_device ? out->tags : dtag) : nullptr;
  uint32_t* fi = e.tag_kind == TAG_VID && out->fact_ids ? (on_device ? out->fact_ids : dfid) : nullptr;
  if (fi) vtag_split(R.full.tags.as<VTag>(), n, nullptr, fi, st);
  if (tg) {
    if (e.tag_kind == TAG_F32) DL_HIP(hipMemcpyAsync(tg, R.full.tags.p, n * 4, hipMemcpyDeviceToDevice, st));
    else if (e.tag_kind == TAG_NONE) fill_f32(tg, n, 1.0f, st);
    else if (e.tag_kind == TAG_VID) vtag_split(R.full.tags.as<VTag>(), n, tg, nullptr, st);
    else if (e.tag_kind == TAG_TOPK)
      topk_probability<1>(R.full.tags.as<TopK>(), e.batched ? samp_k : nullptr, n, e.qtab.as<float>(), tg, st);
    else
      topk_probability<4>(R.full.tags.as<TopK4>(), e.batched ? samp_k : nullptr, n, e.qtab.as<float>(), tg, st);
  }
  uint8_t* oc = nullptr;
  uint64_t* ob = nullptr;
  float* op = nullptr;
  if (topk) {
    oc = out->topk_count ? (on_device ? out->topk_count : dcnt) : nullptr;
    ob = out->topk_bits ? (on_device ? out->topk_bits : dbits) : nullptr;
    op = out->topk_prob ? (on_device ? out->topk_prob : dprob) : nullptr;
    if ((oc || ob || op) && W == 1) topk_split<1>(R.full.tags.as<TopK>(), n, e.k, oc, ob, op, st);
    else if (oc || ob || op) topk_split<4>(R.full.tags.as<TopK4>(), n, e.k, oc, ob, op, st);
  }
  if (!on_device) {
    auto d2h = [&](void* dst, const void* src, size_t bytes) {
      if (dst) DL_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    };
    for (int c = 0; c < ar; ++c) d2h(out->columns[c], dcols[c], n * 4);
    if (out->sample_ids) {
      if (e.batched) d2h(out->sample_ids, dsample, n * 4);
      else std::memset(out->sample_ids, 0, n * 4);
    }
    d2h(out->tags, dtag, n * 4);
    if (fi) d2h(out->fact_ids, dfid, n * 4);
    if (topk) {
      d2h(out->topk_count, dcnt, n);
      d2h(out->topk_bits, dbits, (size_t)e.k * n * W * 8);
      d2h(out->topk_prob, dprob, (size_t)e.k * n * 4);
    }
  }
  e.sync();
  return n;
}

template <typename K>
void lookup_t(Engine& e, int r, size_t n, const uint32_t* const* cols, const uint32_t* sample, int64_t* rows,
              float* tags) {
  const RelState& R = e.rel[r];
  lookup_rows<K>(R.full.keys.as<K>(), R.full.n, cols, sample, n, e.tag_kind, R.full.tags.p,
                 e.layout(e.prog.rels[r].arity), e.qtab.as<float>(), rows, tags, e.stream);
}

// ------------------------------------------------- lineage recomputation
// Rows of `src` whose id lies in [lo, hi), in key order, into `dst`.
template <typename K>
void select_ids(Engine& e, const Table& src, uint32_t lo, uint32_t hi, Table& dst) {
  const size_t n = src.n;
  dst.n = 0;
  if (n == 0 || lo >= hi) return;
  hipStream_t st = e.stream;
  e.grow(e.flags, n * 4);
  e.grow(e.pos, (n + 1) * 4);
  range_flags(src.ids.as<uint32_t>(), n, lo, hi, e.flags.as<uint32_t>(), st);
  scan(e, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), n, S_SCAN, true);
  const size_t m = e.read_total(S_SCAN);
  e.grow(dst.keys, m * sizeof(K) + 8);
  e.grow(dst.tags, m * 4 + 8);
  e.grow(dst.ids, m * 4 + 8);
  compact(src.keys.p, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), n, sizeof(K), dst.keys.p, st);
  compact(src.tags.p, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), n, 4, dst.tags.p, st);
  compact(src.ids.p, e.flags.as<uint32_t>(), e.pos.as<uint32_t>(), n, 4, dst.ids.p, st);
  dst.n = m;
}

// Put the relations of stratum `si` into (or back from) the state they had
// when the joins of round `round` (1-based) ran: full = ids below the round's
// first id, recent = the previous round's ids, stable = older ids.
template <typename K>
void swap_views(Engine& e, const Stratum& st, int si, int round, bool enter) {
  const std::vector<uint32_t>& ids = e.round_ids[si];
  for (int r : st.rels) {
    RelState& R = e.rel[r];
    if (enter) {
      const uint32_t b = ids[round - 1], a = round >= 2 ? ids[round - 2] : b;
      select_ids<K>(e, R.full, 0, b, R.view_full);
      select_ids<K>(e, R.full, a, b, R.view_recent);
      select_ids<K>(e, R.full, 0, a, R.view_stable);
    }
    std::swap(R.full, R.view_full);
    std::swap(R.recent, R.view_recent);
    std::swap(R.full_alt, R.view_stable);
    R.stable_full = false;  // a view's stable part is explicit
    ++R.version;
    ++R.rversion;
    ++R.sversion;
  }
}

// Reverse sweep without recorded lineage: for each round, newest first,
// re-run its joins on the relations as they stood, keep the derivations
// whose head was discovered in that round, and push the adjoints through
// them.
template <typename K>
void recompute_backward(Engine& e) {
  hipStream_t st = e.stream;
  const bool saved_record = e.record;
  for (size_t si = e.prog.strata.size(); si-- > 0;) {
    const Stratum& S = e.prog.strata[si];
    const std::vector<uint32_t>& ids = e.round_ids[si];
    const int rounds = (int)ids.size() - 1;
    std::vector<bool> dense(e.rel.size());
    for (int r : S.rels) dense[r] = e.rel[r].dense;
    for (int round = rounds; round >= 1; --round) {
      const uint32_t lo = ids[round - 1], hi = ids[round];
      if (lo == hi) continue;
      swap_views<K>(e, S, (int)si, round, true);
      e.record = true;
      for (int r : S.rels) {
        e.rel[r].dense = false;
        e.rel[r].ncand = 0;
      }
      try {
        for (int p : round == 1 ? S.base_plans : S.delta_plans) run_plan<K>(e, e.prog.plans[p]);
      } catch (...) {
        swap_views<K>(e, S, (int)si, round, false);
        for (int r : S.rels) e.rel[r].dense = dense[r], e.rel[r].ncand = 0;
        e.record = saved_record;
        throw;
      }
      swap_views<K>(e, S, (int)si, round, false);
      e.record = saved_record;
      for (int r : S.rels) {
        RelState& H = e.rel[r];
        H.dense = dense[r];
        const size_t c = H.ncand;
        H.ncand = 0;
        if (!c) continue;
        e.grow(e.lin_owner, c * 4 + 4);
        match_owner<K>(H.cand_keys.as<K>(), c, H.full.keys.as<K>(), H.full.ids.as<uint32_t>(), H.full.n, lo, hi,
                       e.lin_owner.as<uint32_t>(), st);
        lineage_backward(e.lin_owner.as<uint32_t>(), H.cand_l.as<uint32_t>(), H.cand_r.as<uint32_t>(), c,
                         e.tag_by_id.as<float>(), e.adj.as<float>(), st);
      }
    }
  }
}

template <typename K>
void backward_t(Engine& e, int r, const float* gout, const int64_t* rows, size_t nrows) {
  RelState& R = e.rel[r];
  const size_t n = R.full.n;
  hipStream_t st = e.stream;
  if (e.sr == DL_DIFF_TOPK && rows) {
    if (e.topk_words == 1)
      topk_backward_rows<K, 1>(R.full.tags.as<TopK>(), R.full.keys.as<K>(), e.layout(e.prog.rels[r].arity), rows,
                               gout, nrows, n, e.qtab.as<float>(), e.grad_fact.as<float>(), st);
    else
      topk_backward_rows<K, 4>(R.full.tags.as<TopK4>(), R.full.keys.as<K>(), e.layout(e.prog.rels[r].arity), rows,
                               gout, nrows, n, e.qtab.as<float>(), e.grad_fact.as<float>(), st);
    return;
  }
  if (e.sr == DL_DIFF_MAXMIN) {  // the gradient of a row goes to the fact its tag comes from
    vtag_backward(R.full.tags.as<VTag>(), rows, gout, rows ? nrows : n, n, e.grad_fact.as<float>(), st);
    return;
  }
  if (e.sr == DL_DIFF_TOPK) {
    uint32_t* samp = nullptr;
    if (e.batched && n) {
      e.grow(e.vals, n * 4);
      samp = e.vals.as<uint32_t>();
      uint32_t* cols[4] = {nullptr, nullptr, nullptr, nullptr};
      unpack_rows<K>(R.full.keys.as<K>(), n, e.layout(e.prog.rels[r].arity), cols, samp, st);
    }
    if (e.topk_words == 1)
      topk_backward<1>(R.full.tags.as<TopK>(), samp, gout, n, e.qtab.as<float>(), e.grad_fact.as<float>(), st);
    else
      topk_backward<4>(R.full.tags.as<TopK4>(), samp, gout, n, e.qtab.as<float>(), e.grad_fact.as<float>(), st);
    return;
  }
  // diff add-mult: seed, sweep the recorded derivations in reverse, collect
  const size_t ids = e.next_id;
  e.grow(e.adj, ids * 4 + 4);
  DL_HIP(hipMemsetAsync(e.adj.p, 0, ids * 4 + 4, st));
  if (rows) scatter_add_rows(R.full.ids.as<uint32_t>(), rows, gout, nrows, n, e.adj.as<float>(), st);
  else scatter_add(R.full.ids.as<uint32_t>(), gout, n, e.adj.as<float>(), st);
  if (e.record) {
    for (size_t i = e.lin_segs.size(); i-- > 0;) {
      const LineageSeg& s = e.lin_segs[i];
      lineage_backward(e.lin_owner.as<uint32_t>() + s.off, e.lin_l.as<uint32_t>() + s.off,
                       e.lin_r.as<uint32_t>() + s.off, s.n, e.tag_by_id.as<float>(), e.adj.as<float>(), st);
    }
  } else {
    recompute_backward<K>(e);
  }
  for (size_t q = 0; q < e.rel.size(); ++q) {
    if (!e.prog.rels[q].input || !e.rel[q].nraw) continue;
    gather_add_clamped(e.rel[q].fact_entry.as<uint32_t>(), e.adj.as<float>(), e.tag_by_id.as<float>(),
                       e.rel[q].nraw, e.rel[q].grad.as<float>(), st);
  }
}

template void ingest<uint32_t>(Engine&);
template void ingest<uint64_t>(Engine&);
template void run_fixpoint<uint32_t>(Engine&);
template void run_fixpoint<uint64_t>(Engine&);
template size_t read_relation_t<uint32_t>(Engine&, int, size_t, const dl_relation_out*, int);
template size_t read_relation_t<uint64_t>(Engine&, int, size_t, const dl_relation_out*, int);
template void backward_t<uint32_t>(Engine&, int, const float*, const int64_t*, size_t);
template void backward_t<uint64_t>(Engine&, int, const float*, const int64_t*, size_t);
template void lookup_t<uint32_t>(Engine&, int, size_t, const uint32_t* const*, const uint32_t*, int64_t*, float*);
template void lookup_t<uint64_t>(Engine&, int, size_t, const uint32_t* const*, const uint32_t*, int64_t*, float*);

}  // namespace dlfix
