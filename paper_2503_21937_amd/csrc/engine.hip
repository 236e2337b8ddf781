// Engine lifecycle, fact staging, device memory and the C ABI (dlfix.h).
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "dl_device.h"
#include "engine.h"
#include "prof.h"

namespace dlfix {

thread_local Profiler* g_prof = nullptr;

namespace {
// Installs a profiler for one engine call when timing is on; folds the event
// times into the engine's per-family totals when the call is done.
struct ProfScope {
  Engine& e;
  Profiler p;
  bool on;
  explicit ProfScope(Engine& eng) : e(eng), on(eng.prof_mask != 0) {
    if (!on) return;
    p.mask = e.prof_mask;
    g_prof = &p;
  }
  void finish() {
    if (!on) return;
    g_prof = nullptr;
    on = false;
    e.sync();
    if (p.deferred_fam >= 0) e.kstats[p.deferred_fam].bytes += p.deferred_per * (double)e.deferred_units;
    Profiler::fold(p.recs, e.kstats);
  }
  ~ProfScope() {
    if (on) g_prof = nullptr;
  }
};
}  // namespace

Engine::~Engine() {
  for (FusedGraph& g : fused_graph) drop_fused_graph(g);
  // arena ranges belong to the caller's workspace (or the static array)
  if (!use_arena) for_each_buf([](DevBuf& b) {
      if (b.p) (void)hipFree(b.p);
      b.p = nullptr;
    });
  if (host && host != host_words) (void)hipHostFree(host);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// ------------------------------------------------------------- arena
namespace {
constexpr size_t ARENA_ALIGN = 256;
size_t align_up(size_t n) { return (n + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN; }
}  // namespace

void Arena::reset(void* p, size_t n) {
  // the first range starts at the first aligned address inside [p, p + n)
  const uintptr_t a = (reinterpret_cast<uintptr_t>(p) + ARENA_ALIGN - 1) & ~(uintptr_t)(ARENA_ALIGN - 1);
  const size_t skip = (size_t)(a - reinterpret_cast<uintptr_t>(p));
  base = reinterpret_cast<char*>(a);
  bytes = n > skip ? (n - skip) / ARENA_ALIGN * ARENA_ALIGN : 0;
  used = peak = 0;
  free_list.clear();
  if (bytes) free_list[0] = bytes;
}

void* Arena::alloc(size_t n) {
  n = align_up(std::max<size_t>(n, 1));
  for (auto it = free_list.begin(); it != free_list.end(); ++it) {
    if (it->second < n) continue;
    const size_t off = it->first, len = it->second;
    free_list.erase(it);
    if (len > n) free_list[off + n] = len - n;
    used += n;
    peak = std::max(peak, used);
    return base + off;
  }
  return nullptr;
}

void Arena::release(void* p, size_t n) {
  if (!p) return;
  n = align_up(std::max<size_t>(n, 1));
  size_t off = (size_t)(static_cast<char*>(p) - base);
  used -= n;
  auto next = free_list.lower_bound(off);
  if (next != free_list.end() && off + n == next->first) {  // merge with the range after
    n += next->second;
    next = free_list.erase(next);
  }
  if (next != free_list.begin()) {  // merge with the range before
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += n;
      return;
    }
  }
  free_list[off] = n;
}

size_t Arena::largest_free() const {
  size_t m = 0;
  for (const auto& f : free_list) m = std::max(m, f.second);
  return m;
}

void Engine::grow(DevBuf& b, size_t bytes, bool keep, size_t used) {
  if (bytes <= b.cap) return;
  size_t cap = std::max<size_t>(opts.exact_growth ? bytes : bytes + bytes / 4, 256);
  void* p = nullptr;
  if (use_arena) {
    cap = align_up(cap);
    p = arena.alloc(cap);
    if (!p) {  // no room for the growth margin: the exact size
      cap = align_up(bytes);
      p = arena.alloc(cap);
    }
    if (!p)
      throw Error{DL_ERR_NOMEM,
                  std::string(static_dev >= 0 ? "the library's static workspace" : "workspace") +
                      " exhausted: a buffer of " + std::to_string(bytes) + " bytes does not fit (" +
                      std::to_string(arena.used) + " of " + std::to_string(arena.bytes) +
                      " bytes in use, largest free range " + std::to_string(arena.largest_free()) + "); " +
                      (static_dev >= 0 ? "the input is beyond what an engine of dl_load_program_static can hold"
                                       : "give the engine a larger workspace (dl_set_workspace)")};
  } else {
    hipError_t err = hipMalloc(&p, cap);
    if (err != hipSuccess) {
      (void)hipGetLastError();
      throw Error{DL_ERR_NOMEM, "device allocation of " + std::to_string(cap) + " bytes failed"};
    }
    ++device_allocs;
  }
  if (keep && used && b.p) DL_HIP(hipMemcpyAsync(p, b.p, used, hipMemcpyDeviceToDevice, stream));
  if (b.p) {
    if (use_arena) {
      arena.release(b.p, b.cap);  // later users of the range are ordered after the copy on the stream
    } else {
      DL_HIP(hipStreamSynchronize(stream));  // the old buffer may still be read by queued work
      DL_HIP(hipFree(b.p));
    }
    device_bytes -= b.cap;
  }
  b.p = p;
  b.cap = cap;
  device_bytes += cap;
}

void Engine::release(DevBuf& b) {
  if (b.p) {
    if (use_arena) {
      arena.release(b.p, b.cap);
    } else {
      DL_HIP(hipStreamSynchronize(stream));
      DL_HIP(hipFree(b.p));
    }
    device_bytes -= b.cap;
  }
  b.p = nullptr;
  b.cap = 0;
}

// Move every live buffer into a new home: the range [p, p + n) (p != NULL)
// or separate hipMalloc allocations (p == NULL).  On failure nothing moves.
void Engine::set_workspace(void* p, size_t n) {
  if (static_dev >= 0) throw Error{DL_ERR_STATE, "an engine of dl_load_program_static keeps the static workspace"};
  if (p && n < ARENA_ALIGN) throw Error{DL_ERR_ARG, "workspace below 256 bytes"};
  sync();
  Arena na;
  if (p) na.reset(p, n);
  struct Move {
    DevBuf* b;
    void* to;
  };
  std::vector<Move> moves;
  auto undo = [&] {
    if (!p)
      for (auto& m : moves) (void)hipFree(m.to);
  };
  try {
    for_each_buf([&](DevBuf& b) {
      if (!b.p) return;
      void* q = nullptr;
      if (p) {
        q = na.alloc(b.cap);
        if (!q)
          throw Error{DL_ERR_NOMEM, "the new workspace (" + std::to_string(n) + " bytes) cannot hold the engine's " +
                                        std::to_string(device_bytes) + " bytes of live buffers"};
      } else {
        if (hipMalloc(&q, b.cap) != hipSuccess) {
          (void)hipGetLastError();
          throw Error{DL_ERR_NOMEM, "device allocation of " + std::to_string(b.cap) + " bytes failed"};
        }
        ++device_allocs;
      }
      moves.push_back(Move{&b, q});
    });
  } catch (...) {
    undo();
    throw;
  }
  for (auto& m : moves) DL_HIP(hipMemcpyAsync(m.to, m.b->p, m.b->cap, hipMemcpyDeviceToDevice, stream));
  sync();
  for (auto& m : moves) {
    if (!use_arena) DL_HIP(hipFree(m.b->p));
    m.b->p = m.to;
    if (p) m.b->cap = align_up(m.b->cap);
  }
  for (auto& x : idx)
    if (x.borrowed) {  // aliases of moved relation buffers: re-pointed at the next use
      x.t = Table{};
      x.built = false;
    }
  use_arena = p != nullptr;
  arena = na;
  if (!use_arena) arena = Arena{};
  device_bytes = 0;
  for_each_buf([&](DevBuf& b) { device_bytes += b.cap; });
  stats.device_bytes = device_bytes;
}

void Engine::sync() { DL_HIP(hipStreamSynchronize(stream)); }

void Engine::read_totals() {
  DL_HIP(hipMemcpyAsync(host, dtotal.p, 32 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
  sync();
}

uint64_t Engine::read_total(int slot) {
  DL_HIP(hipMemcpyAsync(host, dtotal.as<uint64_t>() + slot, sizeof(uint64_t), hipMemcpyDeviceToHost, stream));
  sync();
  return host[0];
}

int Engine::relation_id(const char* name, bool must_exist) {
  if (!name) throw Error{DL_ERR_ARG, "relation name is NULL"};
  int r = prog.find(name);
  if (r < 0 && must_exist) throw Error{DL_ERR_ARG, std::string("unknown relation ") + name};
  return r;
}

void Engine::init(const char* program_text, const dl_options* o) {
  text = program_text;
  opts = *o;
  sr = o->semiring;
  if (sr < DL_BOOL || sr > DL_DIFF_MAXMIN) throw Error{DL_ERR_ARG, "unknown semiring"};
  k = o->k == 0 ? 3 : o->k;
  if ((sr == DL_TOPK || sr == DL_DIFF_TOPK) && (k < 1 || k > 3)) throw Error{DL_ERR_ARG, "k must be 1..3"};
  batched = o->batched != 0;
  converge = !(sr == DL_ADDMULT || sr == DL_DIFF_ADDMULT);
  lineage = sr == DL_DIFF_ADDMULT;
  tag_kind = sr == DL_BOOL                       ? TAG_NONE
             : (sr == DL_TOPK || sr == DL_DIFF_TOPK) ? TAG_TOPK
             : sr == DL_DIFF_MAXMIN                  ? TAG_VID
                                                     : TAG_F32;
  tag_bytes = tag_kind == TAG_NONE ? 0 : tag_kind == TAG_F32 ? 4 : tag_kind == TAG_VID ? sizeof(VTag) : sizeof(TopK);
  std::string perr;
  int rc = parse_and_plan(program_text, !converge, lineage, prog, perr);
  if (rc) throw Error{(dl_status)rc, perr};
  rel.assign(prog.rels.size(), RelState{});
  for (size_t r = 0; r < prog.rels.size(); ++r) rel[r].raw_cols.assign(prog.rels[r].arity, DevBuf{});
  idx.assign(prog.indexes.size(), IndexState{});
  if (o->dedup < 0 || o->dedup > 3) throw Error{DL_ERR_ARG, "dedup must be 0, 1, 2 or 3"};
  cfg.graph = o->no_graphs ? 0 : 1;
  cfg.fused = o->no_fused ? 0 : 1;
  for (const Plan& pl : prog.plans)
    for (const Step& st : pl.steps) {
      const IndexSpec& ix = prog.indexes[st.index];
      if (!ix.recent && prog.rels[ix.rel].derived && prog.rels[ix.rel].stratum == prog.rels[pl.head_rel].stratum)
        rel[ix.rel].own_index = true;
    }
  if (o->stream || static_dev >= 0) {
    stream = (hipStream_t)o->stream;  // static engines never create a stream: NULL is the null stream
  } else {
    DL_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    own_stream = true;
  }
  if (static_dev >= 0) {  // the arena over the static array was set by the caller
    host = host_words;    // readback words in the engine itself (no pinned allocation)
  } else {
    if (o->workspace) {
      if (o->workspace_bytes < ARENA_ALIGN) throw Error{DL_ERR_ARG, "workspace below 256 bytes"};
      use_arena = true;
      arena.reset(o->workspace, o->workspace_bytes);
    }
    DL_HIP(hipHostMalloc((void**)&host, 64 * sizeof(uint64_t), hipHostMallocDefault));
  }
  grow(dtotal, 64 * sizeof(uint64_t));
  grow(cs_state, count_scan_state_words() * sizeof(uint64_t));
  fill_u32(cs_state.as<uint32_t>(), count_scan_state_words() * 2, 0u, stream);
  if (o->lineage < 0 || o->lineage > 2) throw Error{DL_ERR_ARG, "lineage must be 0, 1 or 2"};
  if (o->lineage == 0 && o->lineage_budget) {
    lin_budget = o->lineage_budget;
  } else if (o->lineage == 0 && use_arena) {
    lin_budget = arena.bytes / 4;
  } else if (o->lineage == 0) {
    size_t free_b = 0, total_b = 0;
    DL_HIP(hipMemGetInfo(&free_b, &total_b));
    lin_budget = free_b / 4;
  } else {
    lin_budget = o->lineage == 1 ? SIZE_MAX : 0;
  }
}

void Engine::clear_facts() {
  for (auto& r : rel) {
    r.nraw = 0;
    r.fact_slot.clear();
    r.full.n = r.full_alt.n = r.recent.n = 0;
  }
  for (auto& x : idx) x.built = false;
  qtab_h.clear();
  topk_next.clear();
  nfacts = 0;
  ingested = false;
  ran = false;
}

void Engine::add_facts(const char* relation, size_t n, const uint32_t* sample_ids, const uint32_t* const* columns,
                       const float* tags, int on_device) {
  int r = relation_id(relation);
  if (!prog.rels[r].input) throw Error{DL_ERR_ARG, std::string(relation) + " is not an input relation"};
  if (n == 0) return;
  const int ar = prog.rels[r].arity;
  if (!columns) throw Error{DL_ERR_ARG, "columns is NULL"};
  for (int c = 0; c < ar; ++c)
    if (!columns[c]) throw Error{DL_ERR_ARG, "a column pointer is NULL"};
  if (batched && !sample_ids) throw Error{DL_ERR_ARG, "batched engine needs sample ids"};
  if (sr != DL_BOOL && !tags) throw Error{DL_ERR_ARG, "this semiring needs tags"};
  if (tag_kind == TAG_VID && n >= (size_t)UINT32_MAX - nfacts)  // UINT32_MAX: the fact number of x's identity
    throw Error{DL_ERR_CAPACITY, "more than 2^32 - 2 facts"};
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  RelState& R = rel[r];
  const bool topk = sr == DL_TOPK || sr == DL_DIFF_TOPK;
  std::vector<uint32_t> samp_h;
  std::vector<float> q_h;
  std::vector<uint32_t> local_h;
  if (topk) {  // fact ids inside each sample, in add order (host bookkeeping)
    samp_h.assign(n, 0);
    q_h.assign(n, 0.0f);
    if (batched) DL_HIP(hipMemcpy(samp_h.data(), sample_ids, n * 4, on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    DL_HIP(hipMemcpy(q_h.data(), tags, n * 4, on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    std::vector<uint32_t> next = topk_next;
    local_h.assign(n, 0);
    for (size_t i = 0; i < n; ++i) {
      uint32_t s = samp_h[i];
      if (s >= next.size()) next.resize((size_t)s + 1, 0);
      if (next[s] >= 256)
        throw Error{DL_ERR_PROOF_OVERFLOW, "sample " + std::to_string(s) + " has more than 256 probabilistic facts"};
      local_h[i] = next[s]++;
    }
    topk_next = next;
    if (qtab_h.size() < topk_next.size() * 256) qtab_h.resize(topk_next.size() * 256, 0.0f);
    for (size_t i = 0; i < n; ++i) {
      qtab_h[(size_t)samp_h[i] * 256 + local_h[i]] = q_h[i];
      R.fact_slot.push_back(samp_h[i] * 256 + local_h[i]);  // at the stride in force when read
    }
  }
  const size_t old = R.nraw;
  for (int c = 0; c < ar; ++c) {
    grow(R.raw_cols[c], (old + n) * 4, true, old * 4);
    DL_HIP(hipMemcpyAsync(R.raw_cols[c].as<uint32_t>() + old, columns[c], n * 4, kind, stream));
  }
  if (batched) {
    grow(R.raw_sample, (old + n) * 4, true, old * 4);
    DL_HIP(hipMemcpyAsync(R.raw_sample.as<uint32_t>() + old, sample_ids, n * 4, kind, stream));
  }
  if (tag_kind != TAG_NONE) {
    grow(R.raw_tags, (old + n) * 4, true, old * 4);
    DL_HIP(hipMemcpyAsync(R.raw_tags.as<float>() + old, tags, n * 4, kind, stream));
  }
  if (topk) {
    grow(R.raw_local, (old + n) * 4, true, old * 4);
    DL_HIP(hipMemcpyAsync(R.raw_local.as<uint32_t>() + old, local_h.data(), n * 4, hipMemcpyHostToDevice, stream));
  } else if (tag_kind == TAG_VID) {  // fact numbers continue over calls and relations
    grow(R.raw_local, (old + n) * 4, true, old * 4);
    iota_u32(R.raw_local.as<uint32_t>() + old, n, nfacts, stream);
    nfacts += (uint32_t)n;
  }
  R.nraw = old + n;
  sync();  // host staging vectors go out of scope
  ingested = false;
  ran = false;
}

static int bits_for(uint32_t maxv) {
  int b = 1;
  while (b < 32 && (uint64_t)maxv >= (1ull << b)) ++b;
  return b;
}

void Engine::run() {
  auto t0 = std::chrono::steady_clock::now();
  ran = false;  // a run that fails part way leaves no result to read
  ProfScope prof(*this);
  if (!ingested) {
    // id domain and sample domain from the facts
    uint32_t* dmax = reinterpret_cast<uint32_t*>(dtotal.as<uint64_t>() + 30);
    DL_HIP(hipMemsetAsync(dmax, 0, 8, stream));
    for (size_t r = 0; r < rel.size(); ++r) {
      for (auto& c : rel[r].raw_cols) max_u32(c.as<uint32_t>(), rel[r].nraw, dmax, stream);
      if (batched) max_u32(rel[r].raw_sample.as<uint32_t>(), rel[r].nraw, dmax + 1, stream);
    }
    DL_HIP(hipMemcpyAsync(host, dmax, 8, hipMemcpyDeviceToHost, stream));
    sync();
    uint32_t maxid = (uint32_t)host[0], maxs = (uint32_t)(host[0] >> 32);
    max_id = std::max(maxid, prog.max_const);  // program constants belong to the id domain
    max_sample = batched ? maxs : 0;
    sample_ids.clear();
    if (batched) {  // ids in use per sample: the dense domains size every sample by its own ids
      const size_t ns = (size_t)maxs + 1;
      grow(d_sn, ns * 4 + 4);
      grow(d_snp, ns * 4 + 4);
      DL_HIP(hipMemsetAsync(d_sn.p, 0, ns * 4, stream));
      for (size_t r = 0; r < rel.size(); ++r) {
        std::vector<const uint32_t*> cols;
        for (auto& c : rel[r].raw_cols) cols.push_back(c.as<uint32_t>());
        sample_max_u32(cols.data(), (int)cols.size(), rel[r].raw_sample.as<uint32_t>(), rel[r].nraw,
                       d_sn.as<uint32_t>(), stream);
      }
      sample_ids.resize(ns);
      DL_HIP(hipMemcpyAsync(sample_ids.data(), d_sn.p, ns * 4, hipMemcpyDeviceToHost, stream));
      sync();
      std::vector<uint32_t> np(ns);
      for (size_t s = 0; s < ns; ++s) {
        sample_ids[s] = std::max(sample_ids[s] + 1, prog.max_const + 1);
        np[s] = (sample_ids[s] + 31) / 32 * 32;
      }
      DL_HIP(hipMemcpyAsync(d_sn.p, sample_ids.data(), ns * 4, hipMemcpyHostToDevice, stream));
      DL_HIP(hipMemcpyAsync(d_snp.p, np.data(), ns * 4, hipMemcpyHostToDevice, stream));
      sync();
    }
    cbits = bits_for(maxid);
    sbits = batched ? bits_for(maxs) : 0;
    int width = key_width(prog.max_cols);
    if (width > 64)
      throw Error{DL_ERR_UNSUPPORTED, "packed keys need " + std::to_string(width) + " bits (more than 64)"};
    key64 = width > 32;
    stats.key_bits = key64 ? 64 : 32;
    stats.id_bits = (uint32_t)cbits;
    stats.sample_bits = (uint32_t)sbits;
    if (key64) ingest<uint64_t>(*this);
    else ingest<uint32_t>(*this);
    ingested = true;
  }
  if (key64) run_fixpoint<uint64_t>(*this);
  else run_fixpoint<uint32_t>(*this);
  prof.finish();
  ran = true;
  stats.run_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  stats.device_bytes = device_bytes;
  stats.dedup = opts.dedup;
  stats.orient = cfg.orient;
  stats.items = cfg.items;
  stats.rows = cfg.rows;
  stats.index = cfg.index;
  stats.topk_words = (sr == DL_TOPK || sr == DL_DIFF_TOPK) ? topk_words : 0;
}

size_t Engine::relation_size(const char* relation) {
  int r = relation_id(relation);
  if (!ran) throw Error{DL_ERR_STATE, "run the fixpoint first"};
  return rel[r].full.n;
}

size_t Engine::read_relation(const char* relation, size_t capacity, const dl_relation_out* out, int on_device) {
  int r = relation_id(relation);
  if (!ran) throw Error{DL_ERR_STATE, "run the fixpoint first"};
  if (!out) throw Error{DL_ERR_ARG, "out is NULL"};
  if (capacity < rel[r].full.n) throw Error{DL_ERR_ARG, "capacity below the relation size"};
  return key64 ? read_relation_t<uint64_t>(*this, r, capacity, out, on_device)
               : read_relation_t<uint32_t>(*this, r, capacity, out, on_device);
}

void Engine::backward(const char* out_relation, const float* grad_out, int on_device) {
  int r = relation_id(out_relation);
  if (!ran) throw Error{DL_ERR_STATE, "run the fixpoint first"};
  if (sr != DL_DIFF_ADDMULT && sr != DL_DIFF_TOPK && sr != DL_DIFF_MAXMIN)
    throw Error{DL_ERR_STATE, "backward needs a differentiable semiring"};
  const size_t n = rel[r].full.n;
  if (n && !grad_out) throw Error{DL_ERR_ARG, "grad_out is NULL"};
  grow(unpack, n * 4 + 4);
  if (n)
    DL_HIP(hipMemcpyAsync(unpack.p, grad_out, n * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          stream));
  ProfScope prof(*this);
  if (key64) backward_t<uint64_t>(*this, r, unpack.as<float>(), nullptr, 0);
  else backward_t<uint32_t>(*this, r, unpack.as<float>(), nullptr, 0);
  prof.finish();
  sync();
}

void Engine::backward_rows(const char* relation, size_t n, const int64_t* rows, const float* grad, int on_device) {
  int r = relation_id(relation);
  if (!ran) throw Error{DL_ERR_STATE, "run the fixpoint first"};
  if (sr != DL_DIFF_ADDMULT && sr != DL_DIFF_TOPK && sr != DL_DIFF_MAXMIN)
    throw Error{DL_ERR_STATE, "backward needs a differentiable semiring"};
  if (n && (!rows || !grad)) throw Error{DL_ERR_ARG, "rows or grad is NULL"};
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  grow(qbuf, n * 12 + 16);
  int64_t* drows = qbuf.as<int64_t>();
  float* dgrad = reinterpret_cast<float*>(drows + n);
  if (n) {
    DL_HIP(hipMemcpyAsync(drows, rows, n * 8, k, stream));
    DL_HIP(hipMemcpyAsync(dgrad, grad, n * 4, k, stream));
  }
  ProfScope prof(*this);
  if (key64) backward_t<uint64_t>(*this, r, dgrad, drows, n);
  else backward_t<uint32_t>(*this, r, dgrad, drows, n);
  prof.finish();
  sync();
}

void Engine::lookup(const char* relation, size_t n, const uint32_t* sample_ids, const uint32_t* const* columns,
                    int64_t* rows, float* tags, int on_device) {
  int r = relation_id(relation);
  if (!ran) throw Error{DL_ERR_STATE, "run the fixpoint first"};
  const int ar = prog.rels[r].arity;
  if (n == 0) return;
  if (!columns) throw Error{DL_ERR_ARG, "columns is NULL"};
  for (int c = 0; c < ar; ++c)
    if (!columns[c]) throw Error{DL_ERR_ARG, "a column pointer is NULL"};
  if (batched && !sample_ids) throw Error{DL_ERR_ARG, "batched engine needs sample ids"};
  // stage inputs and outputs on the device
  const size_t in_words = (size_t)(ar + 1) * n;
  grow(qbuf, in_words * 4 + n * 12 + 64);
  uint32_t* base = qbuf.as<uint32_t>();
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const uint32_t* dcols[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int c = 0; c < ar; ++c) {
    DL_HIP(hipMemcpyAsync(base + (size_t)c * n, columns[c], n * 4, k, stream));
    dcols[c] = base + (size_t)c * n;
  }
  const uint32_t* dsample = nullptr;
  if (batched) {
    DL_HIP(hipMemcpyAsync(base + (size_t)ar * n, sample_ids, n * 4, k, stream));
    dsample = base + (size_t)ar * n;
  }
  int64_t* drows = reinterpret_cast<int64_t*>(((uintptr_t)(base + in_words) + 7) & ~(uintptr_t)7);
  float* dtags = reinterpret_cast<float*>(drows + n);
  if (key64) lookup_t<uint64_t>(*this, r, n, dcols, dsample, drows, dtags);
  else lookup_t<uint32_t>(*this, r, n, dcols, dsample, drows, dtags);
  const hipMemcpyKind back = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (rows) DL_HIP(hipMemcpyAsync(rows, drows, n * 8, back, stream));
  if (tags) DL_HIP(hipMemcpyAsync(tags, dtags, n * 4, back, stream));
  sync();
}

void Engine::read_grad(const char* in_relation, float* grad_in, int on_device) {
  int r = relation_id(in_relation);
  if (!prog.rels[r].input) throw Error{DL_ERR_ARG, "not an input relation"};
  if (!ran) throw Error{DL_ERR_STATE, "run the fixpoint first"};
  RelState& R = rel[r];
  if (!R.nraw) return;
  if (!grad_in) throw Error{DL_ERR_ARG, "grad_in is NULL"};
  grow(R.grad, R.nraw * 4);
  std::vector<uint32_t> slots;
  if (sr == DL_TOPK || sr == DL_DIFF_TOPK) {
    // grad_fact is [sample][64 * W]; gather the slots of this relation's facts
    const uint32_t qs = 64u * (uint32_t)topk_words;
    slots.resize(R.nraw);
    for (size_t i = 0; i < R.nraw; ++i) slots[i] = (R.fact_slot[i] >> 8) * qs + (R.fact_slot[i] & 255u);
    grow(R.fact_slot_d, R.nraw * 4);
    DL_HIP(hipMemcpyAsync(R.fact_slot_d.p, slots.data(), R.nraw * 4, hipMemcpyHostToDevice, stream));
    gather(grad_fact.p, R.fact_slot_d.as<uint32_t>(), R.grad.p, R.nraw, 4, stream);
  } else if (tag_kind == TAG_VID) {  // grad_fact is indexed by fact number
    gather(grad_fact.p, R.raw_local.as<uint32_t>(), R.grad.p, R.nraw, 4, stream);
  }
  DL_HIP(hipMemcpyAsync(grad_in, R.grad.p, R.nraw * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        stream));
  sync();
}

void Engine::zero_grad() {
  for (auto& R : rel)
    if (R.grad.p) DL_HIP(hipMemsetAsync(R.grad.p, 0, R.grad.cap, stream));
  if (grad_fact.p) DL_HIP(hipMemsetAsync(grad_fact.p, 0, grad_fact.cap, stream));
  sync();
}

// ------------------------------------------------------------- autotuner
// Key of a tuning decision: the program, the semiring, the packed key width
// and the input size class (log2 of the fact count).
std::string Engine::tune_key() const {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the program text
  for (unsigned char c : text) h = (h ^ c) * 1099511628211ull;
  size_t facts = 0;
  for (const auto& r : rel) facts += r.nraw;
  int lg = 0;
  while (((size_t)1 << lg) < facts) ++lg;
  char buf[160];
  std::snprintf(buf, sizeof buf, "%016llx/sr%d/k%d/b%d/key%d/id%d/s%d/f%d", (unsigned long long)h, sr, k,
                (int)batched, key64 ? 64 : 32, cbits, sbits, lg);
  return buf;
}

namespace {
struct Tuned {
  int dedup, orient, items, rows, index;
  double ms;
};

bool cache_lookup(const char* path, const std::string& key, Tuned* t) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {  // later lines override earlier ones
    char k[200];
    Tuned x{};
    x.rows = 1;
    x.index = 0;
    const bool ok =
        std::sscanf(line,
                    "{\"key\": \"%199[^\"]\", \"dedup\": %d, \"orient\": %d, \"items\": %d, \"rows\": %d, \"index\": %d, "
                    "\"ms\": %lf",
                    k, &x.dedup, &x.orient, &x.items, &x.rows, &x.index, &x.ms) == 7 ||
        std::sscanf(line, "{\"key\": \"%199[^\"]\", \"dedup\": %d, \"orient\": %d, \"items\": %d, \"rows\": %d, \"ms\": %lf",
                    k, &x.dedup, &x.orient, &x.items, &x.rows, &x.ms) == 6 ||
        std::sscanf(line, "{\"key\": \"%199[^\"]\", \"dedup\": %d, \"orient\": %d, \"items\": %d, \"ms\": %lf",
                    k, &x.dedup, &x.orient, &x.items, &x.ms) == 5;
    if (ok && key == k) {
      *t = x;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const Tuned& t) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"key\": \"%s\", \"dedup\": %d, \"orient\": %d, \"items\": %d, \"rows\": %d, \"index\": %d, "
               "\"ms\": %.4f}\n",
               key.c_str(), t.dedup, t.orient, t.items, t.rows, t.index, t.ms);
  std::fclose(f);
}
}  // namespace

// Time the fixpoint under every candidate configuration on the current facts
// (median of `trials` runs after one warm-up run) and keep the fastest.
void Engine::autotune(int trials, const char* cache_path) {
  if (trials < 1) trials = 1;
  if (!ingested) run();  // fixes the key layout the decision is keyed on
  const std::string key = tune_key();
  Tuned best{opts.dedup, cfg.orient, cfg.items, cfg.rows, cfg.index, 1e300};
  if (cache_path && cache_lookup(cache_path, key, &best)) {
    opts.dedup = best.dedup;
    cfg.orient = best.orient;
    cfg.items = best.items;
    cfg.rows = best.rows;
    cfg.index = best.index;
    stats.tuned_ms = best.ms;
    run();  // results of the cached configuration
    return;
  }
  bool twins = false;
  for (const Plan& pl : prog.plans) twins = twins || pl.alt >= 0;
  const int saved_dedup = opts.dedup;
  const ExecConfig saved = cfg;
  cfg.index = 0;
  Tuned best1{1, 0, 2, 1, 0, 1e300};  // the fastest sort-based configuration
  // median of `trials` runs after a warm-up run; false when the
  // configuration does not apply (e.g. no dense domain)
  auto time_config = [&](double* med) {
    std::vector<double> ms;
    try {
      run();
      for (int t = 0; t < trials; ++t) {
        run();
        ms.push_back(stats.run_ms);
      }
    } catch (const Error& x) {
      if (x.code == DL_ERR_UNSUPPORTED) return false;
      opts.dedup = saved_dedup;
      cfg = saved;
      throw;
    }
    std::sort(ms.begin(), ms.end());
    *med = ms[ms.size() / 2];
    return true;
  };
  for (int dedup : {1, 2}) {
    for (int orient : {1, 2}) {
      if (orient == 2 && !twins) continue;
      for (int items : {1, 2, 4, 8}) {
        // row windows only exist for dense heads of static-driven joins
        for (int rows : {1, 0}) {
          if (rows == 0 && (dedup != 2 || orient != 2)) continue;
          opts.dedup = dedup;
          cfg.orient = orient;
          cfg.items = items;
          cfg.rows = rows;
          double med;
          if (!time_config(&med)) break;  // e.g. no dense domain
          if (med < best.ms) best = Tuned{dedup, orient, items, rows, 0, med};
          if (dedup == 1 && med < best1.ms) best1 = Tuned{dedup, orient, items, rows, 0, med};
        }
      }
    }
  }
  // the fastest sort-based configuration with hash-set deduplication
  if (best1.ms < 1e300) {
    opts.dedup = 3;
    cfg.orient = best1.orient;
    cfg.items = best1.items;
    cfg.rows = best1.rows;
    double med;
    if (time_config(&med) && med < best.ms) best = Tuned{3, best1.orient, best1.items, best1.rows, 0, med};
  }
  // the fastest configuration with hash indexes instead of CSR offsets
  if (best.ms < 1e300) {
    opts.dedup = best.dedup;
    cfg.orient = best.orient;
    cfg.items = best.items;
    cfg.rows = best.rows;
    cfg.index = 1;
    double med;
    if (time_config(&med) && med < best.ms) {
      best.index = 1;
      best.ms = med;
    }
  }
  opts.dedup = best.dedup;
  cfg.orient = best.orient;
  cfg.items = best.items;
  cfg.rows = best.rows;
  cfg.index = best.index;
  stats.tuned_ms = best.ms;
  if (cache_path) cache_store(cache_path, key, best);
  run();  // leave the results of the chosen configuration in place
}

}  // namespace dlfix

// ---------------------------------------------------------------- C ABI
using dlfix::Engine;
using dlfix::Error;

struct dl_engine {
  Engine e;
};

// ------------------------------------------------------ static workspace
// Device memory the library itself holds for callers that cannot allocate
// (dl_load_program_static): one array on every device the library runs on,
// kept until the process ends.  In host code `scratch` is only a stand-in
// for the symbol: its device address comes from hipGetSymbolAddress, once
// per device with that device current, and only that address is used.
constexpr size_t STATIC_WORKSPACE_BYTES = (size_t)DL_STATIC_WORKSPACE_MIB << 20;
static __device__ __align__(256) uint8_t scratch[STATIC_WORKSPACE_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
struct StaticSlot {
  void* ptr = nullptr;  // device address of `scratch` on this device
  uint64_t gen = 0;     // bumped by every dl_load_program_static on this device
};
std::mutex g_static_mu;
StaticSlot g_static[MAX_DEVICES];

// The current device's array (resolved on first use) and a new generation.
void static_claim(int* dev, void** ptr, uint64_t* gen) {
  DL_HIP(hipGetDevice(dev));
  if (*dev < 0 || *dev >= MAX_DEVICES) throw Error{DL_ERR_ARG, "device ordinal beyond the static workspace table"};
  std::lock_guard<std::mutex> lk(g_static_mu);
  StaticSlot& s = g_static[*dev];
  if (!s.ptr) {
    void* p = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (rc != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error{DL_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(rc)};
    }
    s.ptr = p;
  }
  *ptr = s.ptr;
  *gen = ++s.gen;
}

// Whether a static engine still holds its device's array.
bool static_current(const Engine& e) {
  if (e.static_dev < 0) return true;
  std::lock_guard<std::mutex> lk(g_static_mu);
  return g_static[e.static_dev].gen == e.static_gen;
}
}  // namespace

template <typename F>
static dl_status guard(dl_engine* h, F&& f) {
  if (!h) return DL_ERR_ARG;
  try {
    h->e.err.clear();
    if (!static_current(h->e))
      throw Error{DL_ERR_STATE, "a later dl_load_program_static on this device took over the static workspace"};
    f();
    return DL_OK;
  } catch (const Error& x) {
    h->e.err = x.msg;
    return x.code;
  } catch (const std::bad_alloc&) {
    h->e.err = "host allocation failed";
    return DL_ERR_NOMEM;
  } catch (const std::exception& x) {
    h->e.err = x.what();
    return DL_ERR_HIP;
  }
}

static thread_local std::string g_load_error;

extern "C" {

dl_status dl_load_program(const char* program_text, const dl_options* opts, dl_engine** out) {
  if (!out) return DL_ERR_ARG;
  *out = nullptr;
  if (!program_text || !opts) {
    g_load_error = "program text or options is NULL";
    return DL_ERR_ARG;
  }
  dl_engine* h = nullptr;
  try {
    h = new dl_engine();
    h->e.init(program_text, opts);
  } catch (const Error& x) {
    g_load_error = x.msg;
    delete h;
    return x.code;
  } catch (const std::exception& x) {
    g_load_error = x.what();
    delete h;
    return DL_ERR_HIP;
  }
  *out = h;
  return DL_OK;
}

dl_status dl_load_program_static(const char* program_text, const dl_options* opts, dl_engine** out) {
  if (!out) return DL_ERR_ARG;
  *out = nullptr;
  if (!program_text || !opts || opts->workspace) {
    g_load_error = opts && opts->workspace ? "dl_load_program_static takes no workspace (it uses the static one)"
                                           : "program text or options is NULL";
    return DL_ERR_ARG;
  }
  dl_engine* h = nullptr;
  try {
    int dev = 0;
    void* ptr = nullptr;
    uint64_t gen = 0;
    static_claim(&dev, &ptr, &gen);
    h = new dl_engine();
    h->e.static_dev = dev;
    h->e.static_gen = gen;
    h->e.use_arena = true;
    h->e.arena.reset(ptr, STATIC_WORKSPACE_BYTES);
    h->e.init(program_text, opts);
  } catch (const Error& x) {
    g_load_error = x.msg;
    delete h;
    return x.code;
  } catch (const std::exception& x) {
    g_load_error = x.what();
    delete h;
    return DL_ERR_HIP;
  }
  *out = h;
  return DL_OK;
}

dl_status dl_clear_facts(dl_engine* h) {
  return guard(h, [&] { h->e.clear_facts(); });
}

dl_status dl_add_facts(dl_engine* h, const char* relation, size_t n, const uint32_t* sample_ids,
                       const uint32_t* const* columns, const float* tags, int on_device) {
  return guard(h, [&] { h->e.add_facts(relation, n, sample_ids, columns, tags, on_device); });
}

dl_status dl_run_fixpoint(dl_engine* h) {
  return guard(h, [&] { h->e.run(); });
}

dl_status dl_set_workspace(dl_engine* h, void* p, size_t bytes) {
  return guard(h, [&] { h->e.set_workspace(p, bytes); });
}

dl_status dl_relation_size(dl_engine* h, const char* relation, size_t* n) {
  return guard(h, [&] {
    if (!n) throw Error{DL_ERR_ARG, "n is NULL"};
    *n = h->e.relation_size(relation);
  });
}

dl_status dl_read_relation(dl_engine* h, const char* relation, size_t capacity, const dl_relation_out* out,
                           int on_device, size_t* n_written) {
  return guard(h, [&] {
    size_t n = h->e.read_relation(relation, capacity, out, on_device);
    if (n_written) *n_written = n;
  });
}

dl_status dl_backward(dl_engine* h, const char* out_relation, const float* grad_out, int on_device) {
  return guard(h, [&] { h->e.backward(out_relation, grad_out, on_device); });
}

dl_status dl_lookup(dl_engine* h, const char* relation, size_t n, const uint32_t* sample_ids,
                    const uint32_t* const* columns, int64_t* rows, float* tags, int on_device) {
  return guard(h, [&] { h->e.lookup(relation, n, sample_ids, columns, rows, tags, on_device); });
}

dl_status dl_backward_rows(dl_engine* h, const char* relation, size_t n, const int64_t* rows, const float* grad,
                           int on_device) {
  return guard(h, [&] { h->e.backward_rows(relation, n, rows, grad, on_device); });
}

dl_status dl_read_grad(dl_engine* h, const char* in_relation, float* grad_in, int on_device) {
  return guard(h, [&] { h->e.read_grad(in_relation, grad_in, on_device); });
}

dl_status dl_zero_grad(dl_engine* h) {
  return guard(h, [&] { h->e.zero_grad(); });
}

dl_status dl_get_stats(const dl_engine* h, dl_stats* out) {
  if (!h || !out) return DL_ERR_ARG;
  *out = h->e.stats;
  out->device_allocs = h->e.device_allocs;
  out->workspace_peak = h->e.use_arena ? h->e.arena.peak : 0;
  out->device_bytes = h->e.device_bytes;
  return DL_OK;
}

dl_status dl_autotune(dl_engine* h, int trials, const char* cache_path) {
  return guard(h, [&] { h->e.autotune(trials, cache_path); });
}

dl_status dl_profile(dl_engine* h, uint32_t family_mask) {
  return guard(h, [&] {
    h->e.prof_mask = family_mask & ((1u << DL_K_FAMILIES) - 1);
    for (auto& k : h->e.kstats) k = dl_kernel_timing{};
  });
}

dl_status dl_get_kernel_timing(const dl_engine* h, int family, dl_kernel_timing* out) {
  if (!h || !out || family < 0 || family >= DL_K_FAMILIES) return DL_ERR_ARG;
  *out = h->e.kstats[family];
  return DL_OK;
}

dl_status dl_get_round_log(const dl_engine* h, size_t capacity, uint64_t* new_or_changed, uint64_t* derivations,
                           uint32_t* info, size_t* n) {
  if (!h || !n) return DL_ERR_ARG;
  const std::vector<uint64_t>& log = h->e.round_log;
  *n = log.size() / 3;
  for (size_t i = 0; i < std::min(capacity, *n); ++i) {
    if (new_or_changed) new_or_changed[i] = log[3 * i];
    if (derivations) derivations[i] = log[3 * i + 1];
    if (info) info[i] = (uint32_t)log[3 * i + 2];
  }
  return DL_OK;
}

const char* dl_last_error(const dl_engine* h) {
  if (!h) return g_load_error.c_str();
  return h->e.err.c_str();
}

void dl_free(dl_engine* h) { delete h; }

}  // extern "C"
