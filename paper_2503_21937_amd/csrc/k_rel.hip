// Relational kernels for gfx950: key packing, CSR index build, index join
// (count / load-balanced expand with the offset tile staged in LDS, fused
// column gather and x of the tags), +-reduction of equal keys, the
// difference / +-merge against the full relation, merge-path merge, and the
// tag and gradient kernels.
#include "prof.h"
#include "rel_device.h"

namespace dlfix {

// Bytes of one tag of a kind (algorithmic byte counts of the kernels).
static double tag_size(int tk) {
  switch (tk) {
    case TAG_NONE: return 0.0;
    case TAG_F32: return 4.0;
    case TAG_VID: return (double)sizeof(VTag);
    case TAG_TOPK: return (double)sizeof(TopK);
    default: return (double)sizeof(TopK4);
  }
}

template <typename K>
__global__ void k_pack(const uint32_t* c0, const uint32_t* c1, const uint32_t* c2, const uint32_t* c3,
                       const uint32_t* sample, size_t n, KeyLayout l, K* keys) {
  GRID_STRIDE(i, n) {
    uint32_t v[4] = {c0 ? c0[i] : 0u, c1 ? c1[i] : 0u, c2 ? c2[i] : 0u, c3 ? c3[i] : 0u};
    keys[i] = key_make<K>(sample ? sample[i] : 0u, v, l);
  }
}

template <typename K>
void pack_rows(const uint32_t* const* cols, const uint32_t* sample, size_t n, KeyLayout l, K* keys, hipStream_t st) {
  if (!n) return;
  const uint32_t* c[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int i = 0; i < l.ncols; ++i) c[i] = cols[i];
  k_pack<K><<<grid_for(n), BLOCK, 0, st>>>(c[0], c[1], c[2], c[3], l.sbits ? sample : nullptr, n, l, keys);
}

template <typename K>
__global__ void k_unpack(const K* keys, size_t n, KeyLayout l, uint32_t* c0, uint32_t* c1, uint32_t* c2, uint32_t* c3,
                         uint32_t* sample) {
  GRID_STRIDE(i, n) {
    K k = keys[i];
    if (c0) c0[i] = key_col(k, 0, l);
    if (c1) c1[i] = key_col(k, 1, l);
    if (c2) c2[i] = key_col(k, 2, l);
    if (c3) c3[i] = key_col(k, 3, l);
    if (sample) sample[i] = key_sample(k, l);
  }
}

template <typename K>
void unpack_rows(const K* keys, size_t n, KeyLayout l, uint32_t* const* cols, uint32_t* sample, hipStream_t st) {
  if (!n) return;
  uint32_t* c[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int i = 0; i < l.ncols; ++i) c[i] = cols[i];
  k_unpack<K><<<grid_for(n), BLOCK, 0, st>>>(keys, n, l, c[0], c[1], c[2], c[3], sample);
}

struct Perm4 {
  int p[4];
};

template <typename K>
__global__ void k_permute(const K* in, size_t n, KeyLayout l, Perm4 perm, K* out) {
  GRID_STRIDE(i, n) {
    K k = in[i];
    uint32_t v[4];
    for (int c = 0; c < l.ncols; ++c) v[c] = key_col(k, perm.p[c], l);
    out[i] = key_make<K>(key_sample(k, l), v, l);
  }
}

template <typename K>
void permute_keys(const K* in, size_t n, KeyLayout l, const int* perm, K* out, hipStream_t st) {
  if (!n) return;
  Perm4 p{{0, 0, 0, 0}};
  for (int i = 0; i < l.ncols; ++i) p.p[i] = perm[i];
  k_permute<K><<<grid_for(n), BLOCK, 0, st>>>(in, n, l, p, out);
}

// ------------------------------------------------------------------ CSR
template <typename K>
__global__ void k_csr(const K* __restrict__ keys, size_t n_h, const uint64_t* __restrict__ dn, int shift,
                      uint64_t domain, uint32_t* __restrict__ off) {
  const size_t n = dn ? (size_t)*dn : n_h;
  GRID_STRIDE(v, domain + 1) {
    size_t lo = 0, hi = n;  // first row with prefix >= v
    while (lo < hi) {
      size_t mid = (lo + hi) >> 1;
      if (((uint64_t)keys[mid] >> shift) < v) lo = mid + 1;
      else hi = mid;
    }
    off[v] = (uint32_t)lo;
  }
}

// Small domains: one wave per prefix, a 64-ary search (each step the lanes
// probe evenly spaced keys and a ballot narrows the range 64-fold), so the
// latency is ~log64(n) dependent loads instead of log2(n) -- the per-prefix
// searches of a small domain are too few to hide a long chain.
template <typename K>
__global__ __launch_bounds__(BLOCK) void k_csr_wave(const K* __restrict__ keys, size_t n_h,
                                                    const uint64_t* __restrict__ dn, int shift, uint64_t domain,
                                                    uint32_t* __restrict__ off) {
  const size_t n = dn ? (size_t)*dn : n_h;
  const size_t lane = (size_t)lane_id();
  for (uint64_t v = ((size_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE; v <= domain;
       v += (size_t)gridDim.x * NWAVES) {  // uniform per wave
    size_t lo = 0, hi = n;  // first row with prefix >= v lies in [lo, hi]
    while (hi - lo > (size_t)WAVE) {
      const size_t step = (hi - lo + WAVE - 1) / WAVE;
      const size_t pos = lo + lane * step;
      const bool below = pos < hi && ((uint64_t)keys[pos] >> shift) < v;
      const uint32_t cnt = (uint32_t)__popcll(ballot(below));  // `below` holds on a prefix of the lanes
      if (cnt == 0) {
        hi = lo;
        break;
      }
      const size_t nlo = lo + (cnt - 1) * step + 1, nhi = lo + cnt * step;
      lo = nlo;
      hi = nhi < hi ? nhi : hi;
    }
    const size_t pos = lo + lane;
    const bool below = pos < hi && ((uint64_t)keys[pos] >> shift) < v;
    const size_t r = lo + (size_t)__popcll(ballot(below));
    if (lane == 0) off[v] = (uint32_t)r;
  }
}

constexpr uint64_t CSR_WAVE_DOMAIN = 1ull << 16;  // up to here a wave per prefix

template <typename K>
static void csr_launch(const K* keys, size_t n, const uint64_t* dn, int shift, uint64_t domain, uint32_t* off,
                       hipStream_t st) {
  if (domain < CSR_WAVE_DOMAIN) {
    const size_t waves = domain + 1;
    const size_t blocks = (waves + NWAVES - 1) / NWAVES;
    k_csr_wave<K><<<(unsigned)(blocks < 8192 ? blocks : 8192), BLOCK, 0, st>>>(keys, n, dn, shift, domain, off);
  } else {
    k_csr<K><<<grid_for(domain + 1), BLOCK, 0, st>>>(keys, n, dn, shift, domain, off);
  }
}

template <typename K>
void csr_build(const K* keys, size_t n, int total_bits, int prefix_bits, uint32_t* off, hipStream_t st) {
  uint64_t domain = 1ull << prefix_bits;
  DL_PROF_BEGIN(9, st);
  csr_launch<K>(keys, n, nullptr, total_bits - prefix_bits, domain, off, st);
  DL_PROF_END(9, st, (domain + 1) * 4.0 + (double)n * sizeof(K));
}

template <typename K>
void csr_build_dn(const K* keys, const uint64_t* dn, int total_bits, int prefix_bits, uint32_t* off, hipStream_t st) {
  uint64_t domain = 1ull << prefix_bits;
  csr_launch<K>(keys, 0, dn, total_bits - prefix_bits, domain, off, st);
}

// Hash index build in two launches over the sorted keys: the first row of
// every prefix run claims a slot (compare-and-swap on the empty key, then
// the next slot on a collision) and records itself as the run's start; the
// last row of the run then finds that slot and writes the row count.
template <typename K>
__global__ void k_hash_insert(const K* __restrict__ keys, size_t n, int shift, HSlot* __restrict__ slots,
                              uint32_t mask) {
  GRID_STRIDE(i, n) {
    const uint64_t p = (uint64_t)keys[i] >> shift;
    if (i > 0 && ((uint64_t)keys[i - 1] >> shift) == p) continue;
    for (uint32_t h = hash_slot(p, mask);; h = (h + 1) & mask) {
      const unsigned long long old =
          atomicCAS(reinterpret_cast<unsigned long long*>(&slots[h].key), (unsigned long long)HSLOT_EMPTY,
                    (unsigned long long)p);
      if (old == HSLOT_EMPTY) {
        slots[h].start = (uint32_t)i;
        break;
      }
    }
  }
}

template <typename K>
__global__ void k_hash_count(const K* __restrict__ keys, size_t n, int shift, HSlot* __restrict__ slots,
                             uint32_t mask) {
  GRID_STRIDE(i, n) {
    const uint64_t p = (uint64_t)keys[i] >> shift;
    if (i + 1 < n && ((uint64_t)keys[i + 1] >> shift) == p) continue;
    for (uint32_t h = hash_slot(p, mask);; h = (h + 1) & mask) {
      if (slots[h].key == p) {
        slots[h].count = (uint32_t)i + 1u - slots[h].start;
        break;
      }
    }
  }
}

template <typename K>
void hash_build(const K* keys, size_t n, int total_bits, int prefix_bits, HSlot* slots, uint32_t mask,
                hipStream_t st) {
  fill_u32(reinterpret_cast<uint32_t*>(slots), ((size_t)mask + 1) * 4, 0xffffffffu, st);  // every key empty
  if (!n) return;
  const int shift = total_bits - prefix_bits;
  DL_PROF_BEGIN(9, st);
  k_hash_insert<K><<<grid_for(n), BLOCK, 0, st>>>(keys, n, shift, slots, mask);
  k_hash_count<K><<<grid_for(n), BLOCK, 0, st>>>(keys, n, shift, slots, mask);
  DL_PROF_END(9, st, ((double)mask + 1) * 16.0 + 2.0 * (double)n * sizeof(K));
}

// ------------------------------------------------------------------ joins
template <typename K>
__global__ void k_join_count(JoinArgs a, uint32_t* __restrict__ counts) {
  const K* dk = (const K*)a.dkeys;
  GRID_STRIDE(i, a.n) {
    uint32_t b, c;
    index_range(a, join_prefix(dk[i], a), &b, &c);
    counts[i] = c;
    if (a.istart) a.istart[i] = b;
  }
}

template <typename K>
void join_count(const JoinArgs& a, uint32_t* counts, hipStream_t st) {
  if (!a.n) return;
  DL_PROF_BEGIN(0, st);
  k_join_count<K><<<grid_for(a.n), BLOCK, 0, st>>>(a, counts);
  DL_PROF_END(0, st, a.n * (sizeof(K) + 12.0));
}


// Join counts and their exclusive scan in one launch (single-pass scan).
// Workgroup b counts the matches of its tile of CS_TILE driver rows and gets
// the sum of the tiles before it by a decoupled look-back (block_lookback),
// then writes its offsets; the last tile writes the total.  Launches
// alternate between two status sets (a parity word after them): the last
// workgroup, whose look-back ends only once every other workgroup has
// published (and so has read the parity), clears the set of the previous
// launch (all of whose workgroups have ended) and flips the parity, so the
// set a launch starts on is always clear.
constexpr int CS_ITEMS = 1;
constexpr int CS_TILE = BLOCK * CS_ITEMS;

size_t count_scan_state_words() { return CS_MAX_TILES * 2 + 2; }

template <typename K>
__global__ __launch_bounds__(BLOCK) void k_join_count_scan(JoinArgs a, uint32_t* __restrict__ offs,
                                                           uint64_t* __restrict__ state, uint64_t* __restrict__ d_total,
                                                           uint64_t* __restrict__ acc, uint64_t* __restrict__ err) {
  __shared__ uint64_t tmp[NWAVES], sh[2 * NWAVES];
  uint64_t* parity = state + 2 * CS_MAX_TILES;
  const uint32_t par = (uint32_t)__hip_atomic_load(parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u;
  uint64_t* stat = state + par * CS_MAX_TILES;
  const K* dk = (const K*)a.dkeys;
  const size_t base = (size_t)blockIdx.x * CS_TILE + (size_t)threadIdx.x * CS_ITEMS;
  uint32_t c[CS_ITEMS], st[CS_ITEMS];
  uint64_t s = 0;
#pragma unroll
  for (int q = 0; q < CS_ITEMS; ++q) {
    const size_t i = base + q;
    c[q] = 0;
    st[q] = 0;
    if (i < a.n) index_range(a, join_prefix(dk[i], a), &st[q], &c[q]);
    s += c[q];
  }
  uint64_t tot;
  const uint64_t ex = block_exclusive_scan(s, tmp, &tot);
  const uint64_t carry = block_lookback(stat, tot, sh, err);
  uint64_t run = carry + ex;
#pragma unroll
  for (int q = 0; q < CS_ITEMS; ++q) {
    if (base + q < a.n) {
      offs[base + q] = (uint32_t)run;
      if (a.istart) a.istart[base + q] = st[q];
    }
    run += c[q];
  }
  if (blockIdx.x == gridDim.x - 1) {
    if (threadIdx.x == 0) {
      const uint64_t total = carry + tot;
      *d_total = total;
      offs[a.n] = (uint32_t)total;
      if (acc) *acc += total;
    }
    uint64_t* prev = state + (1u - par) * CS_MAX_TILES;
    for (size_t i = threadIdx.x; i < CS_MAX_TILES; i += BLOCK)
      __hip_atomic_store(prev + i, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) __hip_atomic_store(parity, (uint64_t)(1u - par), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename K>
bool join_count_scan(const JoinArgs& a, uint32_t* offs, uint64_t* state, uint64_t* d_total, uint64_t* acc,
                     uint64_t* err, hipStream_t st) {
  const size_t nt = (a.n + CS_TILE - 1) / CS_TILE;
  if (a.n == 0 || nt > CS_MAX_TILES) return false;
  DL_PROF_BEGIN(0, st);
  k_join_count_scan<K><<<(unsigned)nt, BLOCK, 0, st>>>(a, offs, state, d_total, acc, err);
  DL_PROF_END(0, st, a.n * (sizeof(K) + 12.0));
  return true;
}

template <typename K, int TK, int EXP_ITEMS>
__global__ __launch_bounds__(BLOCK) void k_join_expand(JoinArgs a, const uint32_t* __restrict__ offs, size_t total,
                                                       K* __restrict__ okeys, typename TagOf<TK>::T* __restrict__ otags,
                                                       uint32_t* __restrict__ ol, uint32_t* __restrict__ orr) {
  using T = typename TagOf<TK>::T;
  constexpr int EXP_TILE = BLOCK * EXP_ITEMS;
  __shared__ uint32_t s_row[EXP_TILE];
  __shared__ uint32_t s_wave[NWAVES];
  __shared__ size_t s_r[2];
  const K* dk = (const K*)a.dkeys;
  const K* ik = (const K*)a.ikeys;
  const T* dt = (const T*)a.dtags;
  const T* it = (const T*)a.itags;
  const size_t s0 = (size_t)blockIdx.x * EXP_TILE;
  const size_t s1 = s0 + EXP_TILE < total ? s0 + EXP_TILE : total;  // exclusive
  tile_rows<EXP_ITEMS>(offs, a.n, s0, s1, s_row, s_wave, s_r);
#pragma unroll
  for (int it_ = 0; it_ < EXP_ITEMS; ++it_) {
    const size_t j = s0 + (size_t)it_ * BLOCK + threadIdx.x;
    if (j >= s1) break;
    const size_t row = s_row[j - s0];
    const uint32_t base = offs[row];
    const K dkey = dk[row];
    uint32_t first, cnt;
    if (a.istart) first = a.istart[row];  // written by the count
    else index_range(a, join_prefix(dkey, a), &first, &cnt);
    const uint32_t irow = first + ((uint32_t)j - base);
    const K ikey = ik[irow];
    uint32_t v[4];
    const bool ok = out_cols<K>(a, dkey, ikey, v);
    if (a.keep) a.keep[j] = ok ? 1u : 0u;
    const uint32_t sample = key_sample(dkey, a.dlay);
    okeys[j] = key_make<K>(sample, v, a.olay);
    if constexpr (TK != TAG_NONE) {
      T x = dt[row], y = it[irow];
      otags[j] = a.index_first ? tag_otimes<TK>(y, x, a, sample) : tag_otimes<TK>(x, y, a, sample);
    }
    if (ol) {
      ol[j] = a.dids[row];
      orr[j] = a.iids[irow];
    }
  }
}

template <typename K>
void join_expand(const JoinArgs& a, int tk, const uint32_t* offs, size_t total, void* okeys, void* otags, uint32_t* ol,
                 uint32_t* orr, hipStream_t st) {
  if (!total) return;
  const int items = a.items == 1 || a.items == 2 || a.items == 8 ? a.items : 4;
  const size_t nb = (total + (size_t)BLOCK * items - 1) / ((size_t)BLOCK * items);
  const double tb = tag_size(tk);
  // algorithmic bytes of a join: probe rows read once (key + tag), every
  // derivation once (key + tag, plus its two lineage ids when recorded)
  const double bytes = total * (sizeof(K) + tb + (ol ? 8.0 : 0.0)) + a.n * (sizeof(K) + tb);
#define DL_EXPAND(IT)                                                                                          \
  if (tk == TAG_NONE)                                                                                          \
    k_join_expand<K, TAG_NONE, IT><<<nb, BLOCK, 0, st>>>(a, offs, total, (K*)okeys, (NoTag*)otags, ol, orr);  \
  else if (tk == TAG_F32)                                                                                      \
    k_join_expand<K, TAG_F32, IT><<<nb, BLOCK, 0, st>>>(a, offs, total, (K*)okeys, (float*)otags, ol, orr);   \
  else if (tk == TAG_VID)                                                                                      \
    k_join_expand<K, TAG_VID, IT><<<nb, BLOCK, 0, st>>>(a, offs, total, (K*)okeys, (VTag*)otags, ol, orr);    \
  else if (tk == TAG_TOPK)                                                                                     \
    k_join_expand<K, TAG_TOPK, IT><<<nb, BLOCK, 0, st>>>(a, offs, total, (K*)okeys, (TopK*)otags, ol, orr);   \
  else                                                                                                         \
    k_join_expand<K, TAG_TOPK4, IT><<<nb, BLOCK, 0, st>>>(a, offs, total, (K*)okeys, (TopK4*)otags, ol, orr);
  DL_PROF_BEGIN(1, st);
  switch (items) {
    case 1: DL_EXPAND(1) break;
    case 2: DL_EXPAND(2) break;
    case 8: DL_EXPAND(8) break;
    default: DL_EXPAND(4) break;
  }
#undef DL_EXPAND
  DL_PROF_END(1, st, bytes);
}

template <typename K, int TK>
__global__ void k_project(JoinArgs a, K* __restrict__ okeys, typename TagOf<TK>::T* __restrict__ otags,
                          uint32_t* __restrict__ ol, uint32_t* __restrict__ orr) {
  using T = typename TagOf<TK>::T;
  const K* dk = (const K*)a.dkeys;
  GRID_STRIDE(i, a.n) {
    K dkey = dk[i];
    uint32_t v[4];
    const bool ok = out_cols<K>(a, dkey, dkey, v);  // sources are driver columns only
    if (a.keep) a.keep[i] = ok ? 1u : 0u;
    okeys[i] = key_make<K>(key_sample(dkey, a.dlay), v, a.olay);
    if constexpr (TK != TAG_NONE) otags[i] = ((const T*)a.dtags)[i];
    if (ol) {
      ol[i] = a.dids[i];
      orr[i] = ~0u;
    }
  }
}

template <typename K>
void project_rows(const JoinArgs& a, int tk, void* okeys, void* otags, uint32_t* ol, uint32_t* orr, hipStream_t st) {
  if (!a.n) return;
  if (tk == TAG_NONE)
    k_project<K, TAG_NONE><<<grid_for(a.n), BLOCK, 0, st>>>(a, (K*)okeys, (NoTag*)otags, ol, orr);
  else if (tk == TAG_F32)
    k_project<K, TAG_F32><<<grid_for(a.n), BLOCK, 0, st>>>(a, (K*)okeys, (float*)otags, ol, orr);
  else if (tk == TAG_VID)
    k_project<K, TAG_VID><<<grid_for(a.n), BLOCK, 0, st>>>(a, (K*)okeys, (VTag*)otags, ol, orr);
  else if (tk == TAG_TOPK)
    k_project<K, TAG_TOPK><<<grid_for(a.n), BLOCK, 0, st>>>(a, (K*)okeys, (TopK*)otags, ol, orr);
  else
    k_project<K, TAG_TOPK4><<<grid_for(a.n), BLOCK, 0, st>>>(a, (K*)okeys, (TopK4*)otags, ol, orr);
}

// ------------------------------------------------------------- reduction
template <typename K>
__global__ void k_head_flags(const K* __restrict__ keys, size_t n, uint32_t* __restrict__ flags) {
  GRID_STRIDE(i, n) flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

template <typename K>
void head_flags(const K* keys, size_t n, uint32_t* flags, hipStream_t st) {
  if (!n) return;
  DL_PROF_BEGIN(5, st);
  k_head_flags<K><<<grid_for(n), BLOCK, 0, st>>>(keys, n, flags);
  DL_PROF_END(5, st, n * (sizeof(K) + 4.0));
}

template <typename K, int TK>
__global__ void k_segment_reduce(const K* __restrict__ keys, const uint32_t* __restrict__ pos,
                                 const uint32_t* __restrict__ flags, size_t n, int sr, int k,
                                 const typename TagOf<TK>::T* __restrict__ tags, const uint32_t* __restrict__ perm,
                                 K* __restrict__ kout, typename TagOf<TK>::T* __restrict__ tout) {
  using T = typename TagOf<TK>::T;
  GRID_STRIDE(i, n) {
    if (!flags[i]) continue;
    const uint32_t s = pos[i];
    kout[s] = keys[i];
    if constexpr (TK != TAG_NONE) {
      T acc = tags[perm ? perm[i] : i];
      for (size_t j = i + 1; j < n && !flags[j]; ++j) {
        T x = tags[perm ? perm[j] : j];
        if constexpr (TK == TAG_F32) acc = f_oplus(sr, acc, x);
        else if constexpr (TK == TAG_VID) acc = vtag_pick(acc, x, true);
        else acc = topk_oplus(acc, x, k);
      }
      tout[s] = acc;
    }
  }
}

template <typename K>
void segment_reduce(const K* keys, const uint32_t* pos, const uint32_t* flags, size_t n, int tk, int sr, int k,
                    const void* tags, const uint32_t* perm, K* kout, void* tout, size_t nout, hipStream_t st) {
  if (!n) return;
  const double tb = tag_size(tk);
  DL_PROF_BEGIN(5, st);
  if (tk == TAG_NONE)
    k_segment_reduce<K, TAG_NONE><<<grid_for(n), BLOCK, 0, st>>>(keys, pos, flags, n, sr, k, (const NoTag*)tags, perm,
                                                                 kout, (NoTag*)tout);
  else if (tk == TAG_F32)
    k_segment_reduce<K, TAG_F32><<<grid_for(n), BLOCK, 0, st>>>(keys, pos, flags, n, sr, k, (const float*)tags, perm,
                                                                kout, (float*)tout);
  else if (tk == TAG_VID)
    k_segment_reduce<K, TAG_VID><<<grid_for(n), BLOCK, 0, st>>>(keys, pos, flags, n, sr, k, (const VTag*)tags, perm,
                                                                kout, (VTag*)tout);
  else if (tk == TAG_TOPK)
    k_segment_reduce<K, TAG_TOPK><<<grid_for(n), BLOCK, 0, st>>>(keys, pos, flags, n, sr, k, (const TopK*)tags, perm,
                                                                 kout, (TopK*)tout);
  else
    k_segment_reduce<K, TAG_TOPK4><<<grid_for(n), BLOCK, 0, st>>>(keys, pos, flags, n, sr, k, (const TopK4*)tags,
                                                                  perm, kout, (TopK4*)tout);
  DL_PROF_END(5, st, n * (sizeof(K) + 8.0 + tb + (perm ? 4.0 : 0.0)) + nout * (sizeof(K) + tb));
}

// ------------------------------------------------- difference / +-merge
constexpr int DIFF_ITEMS = 4;
constexpr int DIFF_TILE = BLOCK * DIFF_ITEMS;
constexpr int DIFF_LDS = 4096;

template <typename K>
__device__ __forceinline__ size_t lower_bound_k(const K* a, size_t lo, size_t hi, K x) {
  while (lo < hi) {
    size_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename K, int TK>
__global__ __launch_bounds__(BLOCK) void k_diff(const K* __restrict__ uk, typename TagOf<TK>::T* __restrict__ ut,
                                                size_t nu, const K* __restrict__ fk,
                                                typename TagOf<TK>::T* __restrict__ ft, size_t nf, int sr, int k,
                                                int converge, uint32_t* __restrict__ status,
                                                uint32_t* __restrict__ fpos) {
  using T = typename TagOf<TK>::T;
  __shared__ K s_f[DIFF_LDS];
  __shared__ size_t s_lo, s_hi;
  const size_t u0 = (size_t)blockIdx.x * DIFF_TILE;
  const size_t u1 = u0 + DIFF_TILE < nu ? u0 + DIFF_TILE : nu;
  if (threadIdx.x == 0) {
    s_lo = lower_bound_k(fk, 0, nf, uk[u0]);
    size_t hi = lower_bound_k(fk, s_lo, nf, uk[u1 - 1]);
    s_hi = hi < nf ? hi + 1 : nf;  // include the possible match of the last key
  }
  __syncthreads();
  const size_t lo = s_lo, hi = s_hi, span = hi - lo;
  const bool staged = span <= (size_t)DIFF_LDS;
  if (staged)
    for (size_t i = threadIdx.x; i < span; i += BLOCK) s_f[i] = fk[lo + i];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < DIFF_ITEMS; ++r) {
    const size_t i = u0 + (size_t)r * BLOCK + threadIdx.x;
    if (i >= u1) break;
    const K key = uk[i];
    size_t f;
    bool found;
    if (staged) {
      size_t l = lower_bound_k(s_f, 0, span, key);
      f = lo + l;
      found = l < span && s_f[l] == key;
    } else {
      f = lower_bound_k(fk, lo, hi, key);
      found = f < hi && fk[f] == key;
    }
    if (fpos) fpos[i] = (uint32_t)f;
    uint32_t s = found ? 0u : 1u;
    if constexpr (TK != TAG_NONE) {
      if (found && converge) {
        T old = ft[f];
        T nw;
        if constexpr (TK == TAG_F32) {
          nw = f_oplus(sr, old, ut[i]);
          if (__float_as_uint(nw) != __float_as_uint(old)) s = 2u;
        } else if constexpr (TK == TAG_VID) {
          nw = vtag_pick(old, ut[i], true);
          if (__float_as_uint(nw.v) != __float_as_uint(old.v) || nw.f != old.f) s = 2u;
        } else {
          nw = topk_oplus(old, ut[i], k);
          if (!topk_same(nw, old)) s = 2u;
        }
        if (s == 2u) {
          ft[f] = nw;
          ut[i] = nw;
        }
      }
    }
    status[i] = s;
  }
}

template <typename K>
void diff_merge(const K* uk, const void* ut, size_t nu, const K* fk, void* ft, size_t nf, int tk, int sr, int k,
                bool converge, uint32_t* status, uint32_t* fpos, hipStream_t st) {
  if (!nu) return;
  size_t nb = (nu + DIFF_TILE - 1) / DIFF_TILE;
  const double tb = tag_size(tk);
  DL_PROF_BEGIN(6, st);
  if (tk == TAG_NONE)
    k_diff<K, TAG_NONE><<<nb, BLOCK, 0, st>>>(uk, (NoTag*)ut, nu, fk, (NoTag*)ft, nf, sr, k, converge, status, fpos);
  else if (tk == TAG_F32)
    k_diff<K, TAG_F32><<<nb, BLOCK, 0, st>>>(uk, (float*)ut, nu, fk, (float*)ft, nf, sr, k, converge, status, fpos);
  else if (tk == TAG_VID)
    k_diff<K, TAG_VID><<<nb, BLOCK, 0, st>>>(uk, (VTag*)ut, nu, fk, (VTag*)ft, nf, sr, k, converge, status, fpos);
  else if (tk == TAG_TOPK)
    k_diff<K, TAG_TOPK><<<nb, BLOCK, 0, st>>>(uk, (TopK*)ut, nu, fk, (TopK*)ft, nf, sr, k, converge, status, fpos);
  else
    k_diff<K, TAG_TOPK4><<<nb, BLOCK, 0, st>>>(uk, (TopK4*)ut, nu, fk, (TopK4*)ft, nf, sr, k, converge, status, fpos);
  DL_PROF_END(6, st, nu * (sizeof(K) + tb + 4.0) + (double)nf * sizeof(K));
}

// ------------------------------------------------------------ merge path
constexpr int MERGE_ITEMS = 8;
constexpr int MERGE_TILE = BLOCK * MERGE_ITEMS;

size_t merge_scratch_words(size_t na, size_t nb) { return (na + nb + MERGE_TILE - 1) / MERGE_TILE + 2; }

// Number of A elements among the first `diag` outputs (A first on ties).
template <typename K>
__device__ __forceinline__ size_t merge_path(const K* a, size_t na, const K* b, size_t nb, size_t diag) {
  size_t lo = diag > nb ? diag - nb : 0;
  size_t hi = diag < na ? diag : na;
  while (lo < hi) {
    size_t mid = (lo + hi) >> 1;
    if (a[mid] <= b[diag - 1 - mid]) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

template <typename K>
__global__ void k_merge_partition(const K* a, size_t na, const K* b, size_t nb, size_t ntiles, uint64_t* split) {
  GRID_STRIDE(t, ntiles + 1) {
    size_t diag = t * (size_t)MERGE_TILE;
    if (diag > na + nb) diag = na + nb;
    split[t] = merge_path(a, na, b, nb, diag);
  }
}

template <typename K>
__global__ __launch_bounds__(BLOCK) void k_merge(const K* __restrict__ ak, const uint8_t* __restrict__ at,
                                                 const uint32_t* __restrict__ aid, size_t na,
                                                 const K* __restrict__ bk, const uint8_t* __restrict__ bt,
                                                 const uint32_t* __restrict__ bid, size_t nb, int tag_bytes,
                                                 const uint64_t* __restrict__ split, K* __restrict__ ok,
                                                 uint8_t* __restrict__ ot, uint32_t* __restrict__ oid) {
  __shared__ K s_k[MERGE_TILE];
  __shared__ uint16_t s_src[MERGE_TILE];
  const size_t t = blockIdx.x;
  const size_t d0 = t * (size_t)MERGE_TILE;
  const size_t d1 = d0 + MERGE_TILE < na + nb ? d0 + MERGE_TILE : na + nb;
  const size_t a0 = split[t], a1 = split[t + 1];
  const size_t b0 = d0 - a0, b1 = d1 - a1;
  const int nta = (int)(a1 - a0), ntb = (int)(b1 - b0), cnt = nta + ntb;
  for (int i = threadIdx.x; i < nta; i += BLOCK) s_k[i] = ak[a0 + i];
  for (int i = threadIdx.x; i < ntb; i += BLOCK) s_k[nta + i] = bk[b0 + i];
  __syncthreads();
  const K* sa = s_k;
  const K* sb = s_k + nta;
  const int d = threadIdx.x * MERGE_ITEMS;
  uint16_t mine[MERGE_ITEMS];
  if (d < cnt) {
    int lo = d > ntb ? d - ntb : 0, hi = d < nta ? d : nta;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (sa[mid] <= sb[d - 1 - mid]) lo = mid + 1;
      else hi = mid;
    }
    int ai = lo, bi = d - lo;
#pragma unroll
    for (int s = 0; s < MERGE_ITEMS; ++s) {
      if (d + s >= cnt) break;
      bool takeA = bi >= ntb || (ai < nta && sa[ai] <= sb[bi]);
      mine[s] = takeA ? (uint16_t)ai++ : (uint16_t)(nta + bi++);
    }
  }
  __syncthreads();
  if (d < cnt) {
#pragma unroll
    for (int s = 0; s < MERGE_ITEMS; ++s)
      if (d + s < cnt) s_src[d + s] = mine[s];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < cnt; i += BLOCK) {
    const int src = s_src[i];
    const size_t o = d0 + i;
    ok[o] = s_k[src];
    const bool fromA = src < nta;
    const size_t g = fromA ? a0 + src : b0 + (src - nta);
    if (oid) oid[o] = fromA ? aid[g] : bid[g];
    if (tag_bytes == 4) {
      reinterpret_cast<uint32_t*>(ot)[o] = reinterpret_cast<const uint32_t*>(fromA ? at : bt)[g];
    } else if (tag_bytes == 8) {
      reinterpret_cast<uint64_t*>(ot)[o] = reinterpret_cast<const uint64_t*>(fromA ? at : bt)[g];
    } else if (tag_bytes == (int)sizeof(TopK)) {
      reinterpret_cast<TopK*>(ot)[o] = reinterpret_cast<const TopK*>(fromA ? at : bt)[g];
    } else if (tag_bytes == (int)sizeof(TopK4)) {
      reinterpret_cast<TopK4*>(ot)[o] = reinterpret_cast<const TopK4*>(fromA ? at : bt)[g];
    }
  }
}

template <typename K>
void merge_sorted(const K* ak, const void* at, const uint32_t* aid, size_t na, const K* bk, const void* bt,
                  const uint32_t* bid, size_t nb, size_t tag_bytes, K* ok, void* ot, uint32_t* oid, uint64_t* scratch,
                  hipStream_t st) {
  if (na + nb == 0) return;
  size_t ntiles = (na + nb + MERGE_TILE - 1) / MERGE_TILE;
  k_merge_partition<K><<<grid_for(ntiles + 1), BLOCK, 0, st>>>(ak, na, bk, nb, ntiles, scratch);
  DL_PROF_BEGIN(7, st);
  k_merge<K><<<ntiles, BLOCK, 0, st>>>(ak, (const uint8_t*)at, aid, na, bk, (const uint8_t*)bt, bid, nb, (int)tag_bytes,
                                      scratch, ok, (uint8_t*)ot, oid);
  DL_PROF_END(7, st, 2.0 * (na + nb) * (sizeof(K) + tag_bytes + (oid ? 4.0 : 0.0)));
}

// ---------------------------------------------------------------- lineage
__global__ void k_lineage_flags(const uint32_t* __restrict__ pos, const uint32_t* __restrict__ flags,
                                const uint32_t* __restrict__ status, size_t n, uint32_t* __restrict__ lf) {
  GRID_STRIDE(p, n) lf[p] = status[pos[p] + flags[p] - 1] & 1u;
}

void lineage_flags(const uint32_t* pos, const uint32_t* flags, const uint32_t* status, size_t n, uint32_t* lf,
                   hipStream_t st) {
  if (n) k_lineage_flags<<<grid_for(n), BLOCK, 0, st>>>(pos, flags, status, n, lf);
}

__global__ void k_lineage_emit(const uint32_t* __restrict__ pos, const uint32_t* __restrict__ flags,
                               const uint32_t* __restrict__ lf, const uint32_t* __restrict__ lpos,
                               const uint32_t* __restrict__ newpos, const uint32_t* __restrict__ perm,
                               const uint32_t* __restrict__ cl, const uint32_t* __restrict__ cr, size_t n,
                               uint32_t id_base, uint32_t* __restrict__ owner, uint32_t* __restrict__ l,
                               uint32_t* __restrict__ r) {
  GRID_STRIDE(p, n) {
    if (!lf[p]) continue;
    uint32_t s = pos[p] + flags[p] - 1;
    uint32_t o = lpos[p];
    uint32_t c = perm[p];
    owner[o] = id_base + newpos[s];
    l[o] = cl[c];
    r[o] = cr[c];
  }
}

void lineage_emit(const uint32_t* pos, const uint32_t* flags, const uint32_t* lf, const uint32_t* lpos,
                  const uint32_t* newpos, const uint32_t* perm, const uint32_t* cl, const uint32_t* cr, size_t n,
                  uint32_t id_base, uint32_t* owner, uint32_t* l, uint32_t* r, hipStream_t st) {
  if (n)
    k_lineage_emit<<<grid_for(n), BLOCK, 0, st>>>(pos, flags, lf, lpos, newpos, perm, cl, cr, n, id_base, owner, l,
                                                  r);
}

__global__ void k_seg_scatter(const uint32_t* __restrict__ pos, const uint32_t* __restrict__ flags,
                              const uint32_t* __restrict__ perm, size_t n, uint32_t base, uint32_t* __restrict__ out) {
  GRID_STRIDE(p, n) out[perm[p]] = base + pos[p] + flags[p] - 1;
}

void seg_scatter(const uint32_t* pos, const uint32_t* flags, const uint32_t* perm, size_t n, uint32_t base,
                 uint32_t* out, hipStream_t st) {
  if (n) k_seg_scatter<<<grid_for(n), BLOCK, 0, st>>>(pos, flags, perm, n, base, out);
}

// ------------------------------------------------------------- gradients
__global__ void k_lineage_backward(const uint32_t* __restrict__ owner, const uint32_t* __restrict__ l,
                                   const uint32_t* __restrict__ r, size_t n, const float* __restrict__ tag,
                                   float* adj) {
  GRID_STRIDE(i, n) {
    const uint32_t o = owner[i];
    if (o == ~0u) continue;          // recomputed derivation of an older tuple
    if (!(tag[o] < 1.0f)) continue;  // clamp: d min(1, s)/ds = 0 once s >= 1
    const float g = adj[o];
    if (g == 0.0f) continue;
    const uint32_t a = l[i], b = r[i];
    if (b == ~0u) {
      atomicAdd(&adj[a], g);
    } else {
      atomicAdd(&adj[a], __fmul_rn(g, tag[b]));
      atomicAdd(&adj[b], __fmul_rn(g, tag[a]));
    }
  }
}

void lineage_backward(const uint32_t* owner, const uint32_t* l, const uint32_t* r, size_t n, const float* tag,
                      float* adj, hipStream_t st) {
  if (!n) return;
  DL_PROF_BEGIN(10, st);
  k_lineage_backward<<<grid_for(n), BLOCK, 0, st>>>(owner, l, r, n, tag, adj);
  DL_PROF_END(10, st, n * 28.0);
}

__global__ void k_scatter_add(const uint32_t* __restrict__ ids, const float* __restrict__ g, size_t n, float* adj) {
  GRID_STRIDE(i, n) atomicAdd(&adj[ids[i]], g[i]);
}

void scatter_add(const uint32_t* ids, const float* g, size_t n, float* adj, hipStream_t st) {
  if (n) k_scatter_add<<<grid_for(n), BLOCK, 0, st>>>(ids, g, n, adj);
}

__global__ void k_gather_add_clamped(const uint32_t* __restrict__ ids, const float* __restrict__ adj,
                                     const float* __restrict__ tag, size_t n, float* __restrict__ out) {
  GRID_STRIDE(i, n) {
    uint32_t id = ids[i];
    if (tag[id] < 1.0f) out[i] += adj[id];
  }
}

void gather_add_clamped(const uint32_t* ids, const float* adj, const float* tag, size_t n, float* out, hipStream_t st) {
  if (n) k_gather_add_clamped<<<grid_for(n), BLOCK, 0, st>>>(ids, adj, tag, n, out);
}

// ------------------------------------------------------------------ top-k
// W 64-bit words per proof set; a sample's fact probabilities are the 64 * W
// floats at qtab + sample * 64 * W.
template <int W>
__global__ void k_topk_from_facts(const float* __restrict__ q, const uint32_t* __restrict__ local, size_t n,
                                  TopKW<W>* __restrict__ out) {
  GRID_STRIDE(i, n) {
    TopKW<W> t = topk_empty<W>();
    t.cnt = 1;
    t.b[local[i] >> 6] = 1ull << (local[i] & 63u);
    t.p[0] = q[i];
    out[i] = t;
  }
}

template <int W>
void topk_from_facts(const float* q, const uint32_t* local, size_t n, TopKW<W>* out, hipStream_t st) {
  if (n) k_topk_from_facts<W><<<grid_for(n), BLOCK, 0, st>>>(q, local, n, out);
}

// P = sum over non-empty subsets S of the kept proofs of (-1)^(|S|+1) times
// the product of the probabilities of the facts in their union.  With
// skip_bit >= 0: adds to *dP the derivative of P by that fact's probability.
template <int W>
__device__ double incl_excl(const TopKW<W>& t, const float* q, int skip_bit, double* dP) {
  double P = 0;
  for (uint32_t S = 1; S < (1u << t.cnt); ++S) {
    uint64_t u[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      u[w] = 0;
      for (uint32_t i = 0; i < t.cnt; ++i)
        if (S >> i & 1u) u[w] |= t.b[i * W + w];
    }
    double prod = 1.0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      uint64_t b = u[w];
      while (b) {
        const int i = w * 64 + __builtin_ctzll(b);
        if (i != skip_bit) prod *= (double)q[i];
        b &= b - 1;
      }
    }
    double sign = (__popc(S) & 1) ? 1.0 : -1.0;
    if (skip_bit < 0) P += sign * prod;
    else if (u[skip_bit >> 6] >> (skip_bit & 63) & 1ull) *dP += sign * prod;
  }
  return P;
}

template <int W>
__global__ void k_topk_prob(const TopKW<W>* __restrict__ t, const uint32_t* __restrict__ sample, size_t n,
                            const float* __restrict__ qtab, float* __restrict__ prob) {
  GRID_STRIDE(i, n) {
    const float* q = qtab + (size_t)(sample ? sample[i] : 0u) * 64 * W;
    prob[i] = (float)incl_excl<W>(t[i], q, -1, nullptr);
  }
}

template <int W>
void topk_probability(const TopKW<W>* t, const uint32_t* sample, size_t n, const float* qtab, float* prob,
                      hipStream_t st) {
  if (n) k_topk_prob<W><<<grid_for(n), BLOCK, 0, st>>>(t, sample, n, qtab, prob);
}

// word w of proof j of row i at bits[(j * n + i) * W + w]
template <int W>
__global__ void k_topk_split(const TopKW<W>* __restrict__ t, size_t n, int k, uint8_t* cnt, uint64_t* bits,
                             float* prob) {
  GRID_STRIDE(i, n) {
    const TopKW<W> x = t[i];
    if (cnt) cnt[i] = (uint8_t)x.cnt;
    for (int j = 0; j < k; ++j) {
      if (bits)
        for (int w = 0; w < W; ++w) bits[((size_t)j * n + i) * W + w] = (uint32_t)j < x.cnt ? x.b[j * W + w] : 0ull;
      if (prob) prob[(size_t)j * n + i] = (uint32_t)j < x.cnt ? x.p[j] : 0.0f;
    }
  }
}

template <int W>
void topk_split(const TopKW<W>* t, size_t n, int k, uint8_t* cnt, uint64_t* bits, float* prob, hipStream_t st) {
  if (n) k_topk_split<W><<<grid_for(n), BLOCK, 0, st>>>(t, n, k, cnt, bits, prob);
}

// The gradient of one row's probability: every fact of its kept proofs
// gets g * dP/dq (proofs held fixed); grad is [sample][64 * W].
template <int W>
__device__ void topk_row_backward(const TopKW<W>& x, uint32_t s, float g, const float* __restrict__ qtab,
                                  float* grad) {
  const float* q = qtab + (size_t)s * 64 * W;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint64_t all = 0;
    for (uint32_t j = 0; j < x.cnt; ++j) all |= x.b[j * W + w];
    while (all) {
      const int bit = w * 64 + __builtin_ctzll(all);
      all &= all - 1;
      double d = 0;
      incl_excl<W>(x, q, bit, &d);
      atomicAdd(&grad[(size_t)s * 64 * W + bit], (float)((double)g * d));
    }
  }
}

template <int W>
__global__ void k_topk_backward(const TopKW<W>* __restrict__ t, const uint32_t* __restrict__ sample,
                                const float* __restrict__ gout, size_t n, const float* __restrict__ qtab,
                                float* grad) {
  GRID_STRIDE(i, n) {
    const float g = gout[i];
    if (g == 0.0f) continue;
    topk_row_backward<W>(t[i], sample ? sample[i] : 0u, g, qtab, grad);
  }
}

template <int W>
void topk_backward(const TopKW<W>* t, const uint32_t* sample, const float* gout, size_t n, const float* qtab,
                   float* grad, hipStream_t st) {
  if (n) k_topk_backward<W><<<grid_for(n), BLOCK, 0, st>>>(t, sample, gout, n, qtab, grad);
}

// ------------------------------------------------------------ point queries
struct QCols {
  const uint32_t* c[4];
  const uint32_t* sample;
};

template <typename K>
__global__ void k_lookup(const K* __restrict__ keys, size_t n, QCols qc, size_t nq, int tk,
                         const void* __restrict__ tags, KeyLayout lay, const float* __restrict__ qtab,
                         int64_t* __restrict__ rows, float* __restrict__ qtag) {
  GRID_STRIDE(i, nq) {
    uint32_t v[4];
    bool ok = true;
    for (int c = 0; c < lay.ncols; ++c) {
      v[c] = qc.c[c][i];
      ok = ok && ((uint64_t)v[c] >> lay.cbits) == 0;
    }
    const uint32_t smp = qc.sample ? qc.sample[i] : 0u;
    ok = ok && (lay.sbits ? ((uint64_t)smp >> lay.sbits) == 0 : smp == 0);
    const K q = key_make<K>(smp, v, lay);
    size_t lo = 0, hi = ok ? n : 0;
    while (lo < hi) {
      size_t mid = (lo + hi) >> 1;
      if (keys[mid] < q) lo = mid + 1;
      else hi = mid;
    }
    const bool found = ok && lo < n && keys[lo] == q;
    if (rows) rows[i] = found ? (int64_t)lo : -1;
    if (qtag) {
      float t = 0.0f;
      if (found) {
        if (tk == TAG_F32) t = ((const float*)tags)[lo];
        else if (tk == TAG_VID) t = ((const VTag*)tags)[lo].v;
        else if (tk == TAG_NONE) t = 1.0f;
        else if (tk == TAG_TOPK)
          t = (float)incl_excl<1>(((const TopK*)tags)[lo], qtab + (size_t)key_sample(q, lay) * 64, -1, nullptr);
        else
          t = (float)incl_excl<4>(((const TopK4*)tags)[lo], qtab + (size_t)key_sample(q, lay) * 256, -1, nullptr);
      }
      qtag[i] = t;
    }
  }
}

template <typename K>
void lookup_rows(const K* keys, size_t n, const uint32_t* const* qcols, const uint32_t* qsample, size_t nq, int tk,
                 const void* tags, KeyLayout lay, const float* qtab, int64_t* rows, float* qtag, hipStream_t st) {
  if (!nq) return;
  QCols qc{{nullptr, nullptr, nullptr, nullptr}, qsample};
  for (int c = 0; c < lay.ncols; ++c) qc.c[c] = qcols[c];
  k_lookup<K><<<grid_for(nq), BLOCK, 0, st>>>(keys, n, qc, nq, tk, tags, lay, qtab, rows, qtag);
}

// Owner of each recomputed derivation: the id of its head tuple if that id
// lies in [lo, hi) (the tuple was discovered in the round being replayed),
// else ~0 (a derivation of an older tuple, ignored under frozen tags).
template <typename K>
__global__ void k_match_owner(const K* __restrict__ ckeys, size_t n, const K* __restrict__ fkeys,
                              const uint32_t* __restrict__ fids, size_t F, uint32_t lo, uint32_t hi,
                              uint32_t* __restrict__ owner) {
  GRID_STRIDE(i, n) {
    const K q = ckeys[i];
    size_t a = 0, b = F;
    while (a < b) {
      size_t mid = (a + b) >> 1;
      if (fkeys[mid] < q) a = mid + 1;
      else b = mid;
    }
    uint32_t o = ~0u;
    if (a < F && fkeys[a] == q) {
      const uint32_t id = fids[a];
      if (id >= lo && id < hi) o = id;
    }
    owner[i] = o;
  }
}

template <typename K>
void match_owner(const K* ckeys, size_t n, const K* fkeys, const uint32_t* fids, size_t F, uint32_t lo, uint32_t hi,
                 uint32_t* owner, hipStream_t st) {
  if (n) k_match_owner<K><<<grid_for(n), BLOCK, 0, st>>>(ckeys, n, fkeys, fids, F, lo, hi, owner);
}
template void match_owner<uint32_t>(const uint32_t*, size_t, const uint32_t*, const uint32_t*, size_t, uint32_t,
                                    uint32_t, uint32_t*, hipStream_t);
template void match_owner<uint64_t>(const uint64_t*, size_t, const uint64_t*, const uint32_t*, size_t, uint32_t,
                                    uint32_t, uint32_t*, hipStream_t);

__global__ void k_scatter_add_rows(const uint32_t* __restrict__ ids, const int64_t* __restrict__ rows,
                                   const float* __restrict__ g, size_t n, size_t nrel, float* adj) {
  GRID_STRIDE(i, n) {
    if (rows[i] >= 0 && (uint64_t)rows[i] < nrel) atomicAdd(&adj[ids[rows[i]]], g[i]);
  }
}

void scatter_add_rows(const uint32_t* ids, const int64_t* rows, const float* g, size_t n, size_t nrel, float* adj,
                      hipStream_t st) {
  if (n) k_scatter_add_rows<<<grid_for(n), BLOCK, 0, st>>>(ids, rows, g, n, nrel, adj);
}

template <typename K, int W>
__global__ void k_topk_backward_rows(const TopKW<W>* __restrict__ t, const K* __restrict__ keys, KeyLayout lay,
                                     const int64_t* __restrict__ rows, const float* __restrict__ gout, size_t n,
                                     size_t nrel, const float* __restrict__ qtab, float* grad) {
  GRID_STRIDE(i, n) {
    const float g = gout[i];
    if (g == 0.0f || rows[i] < 0 || (uint64_t)rows[i] >= nrel) continue;
    const size_t r = (size_t)rows[i];
    topk_row_backward<W>(t[r], key_sample(keys[r], lay), g, qtab, grad);
  }
}

template <typename K, int W>
void topk_backward_rows(const TopKW<W>* t, const K* keys, KeyLayout lay, const int64_t* rows, const float* g,
                        size_t n, size_t nrel, const float* qtab, float* grad_fact, hipStream_t st) {
  if (n) k_topk_backward_rows<K, W><<<grid_for(n), BLOCK, 0, st>>>(t, keys, lay, rows, g, n, nrel, qtab, grad_fact);
}

// -------------------------------------------------- differentiable max-min
// Input facts' tags: (probability, fact number).
__global__ void k_vtags_from_facts(const float* __restrict__ q, const uint32_t* __restrict__ fid, size_t n,
                                   VTag* __restrict__ out) {
  GRID_STRIDE(i, n) out[i] = VTag{q[i], fid[i]};
}
void vtags_from_facts(const float* q, const uint32_t* fid, size_t n, VTag* out, hipStream_t st) {
  if (n) k_vtags_from_facts<<<grid_for(n), BLOCK, 0, st>>>(q, fid, n, out);
}

// The values and the fact numbers of n tags (either output may be NULL).
__global__ void k_vtag_split(const VTag* __restrict__ t, size_t n, float* __restrict__ v, uint32_t* __restrict__ f) {
  GRID_STRIDE(i, n) {
    const VTag x = t[i];
    if (v) v[i] = x.v;
    if (f) f[i] = x.f;
  }
}
void vtag_split(const VTag* t, size_t n, float* v, uint32_t* f, hipStream_t st) {
  if (n && (v || f)) k_vtag_split<<<grid_for(n), BLOCK, 0, st>>>(t, n, v, f);
}

// Reverse mode: a tag equals the probability of its fact, so the gradient
// of row i (rows[i] when given, else i; rows outside [0, nrel) are skipped)
// goes to that fact.
__global__ void k_vtag_backward(const VTag* __restrict__ t, const int64_t* __restrict__ rows,
                                const float* __restrict__ g, size_t n, size_t nrel, float* __restrict__ grad_fact) {
  GRID_STRIDE(i, n) {
    const int64_t r = rows ? rows[i] : (int64_t)i;
    if (r >= 0 && (uint64_t)r < nrel) atomicAdd(grad_fact + t[r].f, g[i]);
  }
}
void vtag_backward(const VTag* t, const int64_t* rows, const float* g, size_t n, size_t nrel, float* grad_fact,
                   hipStream_t st) {
  if (!n) return;
  DL_PROF_BEGIN(10, st);
  k_vtag_backward<<<grid_for(n), BLOCK, 0, st>>>(t, rows, g, n, nrel, grad_fact);
  DL_PROF_END(10, st, n * 16.0);
}

// ------------------------------------------------------- instantiations
#define INST(K)                                                                                                      \
  template void pack_rows<K>(const uint32_t* const*, const uint32_t*, size_t, KeyLayout, K*, hipStream_t);         \
  template void unpack_rows<K>(const K*, size_t, KeyLayout, uint32_t* const*, uint32_t*, hipStream_t);             \
  template void permute_keys<K>(const K*, size_t, KeyLayout, const int*, K*, hipStream_t);                        \
  template void csr_build<K>(const K*, size_t, int, int, uint32_t*, hipStream_t);                                   \
  template void csr_build_dn<K>(const K*, const uint64_t*, int, int, uint32_t*, hipStream_t);                       \
  template void hash_build<K>(const K*, size_t, int, int, HSlot*, uint32_t, hipStream_t);                          \
  template void join_count<K>(const JoinArgs&, uint32_t*, hipStream_t);                                             \
  template bool join_count_scan<K>(const JoinArgs&, uint32_t*, uint64_t*, uint64_t*, uint64_t*, uint64_t*, hipStream_t);                                             \
  template void join_expand<K>(const JoinArgs&, int, const uint32_t*, size_t, void*, void*, uint32_t*, uint32_t*,   \
                               hipStream_t);                                                                         \
  template void project_rows<K>(const JoinArgs&, int, void*, void*, uint32_t*, uint32_t*, hipStream_t);             \
  template void head_flags<K>(const K*, size_t, uint32_t*, hipStream_t);                                            \
  template void segment_reduce<K>(const K*, const uint32_t*, const uint32_t*, size_t, int, int, int, const void*,  \
                                  const uint32_t*, K*, void*, size_t, hipStream_t);                                          \
  template void diff_merge<K>(const K*, const void*, size_t, const K*, void*, size_t, int, int, int, bool,          \
                              uint32_t*, uint32_t*, hipStream_t);                                                   \
  template void merge_sorted<K>(const K*, const void*, const uint32_t*, size_t, const K*, const void*,              \
                                const uint32_t*, size_t, size_t, K*, void*, uint32_t*, uint64_t*, hipStream_t);

#define INST2(K)                                                                                                 \
  template void lookup_rows<K>(const K*, size_t, const uint32_t* const*, const uint32_t*, size_t, int,           \
                               const void*, KeyLayout, const float*, int64_t*, float*, hipStream_t);                                                    \
  template void topk_backward_rows<K, 1>(const TopK*, const K*, KeyLayout, const int64_t*, const float*, size_t,  \
                                         size_t, const float*, float*, hipStream_t);                               \
  template void topk_backward_rows<K, 4>(const TopK4*, const K*, KeyLayout, const int64_t*, const float*, size_t, \
                                         size_t, const float*, float*, hipStream_t);

#define INST_W(W)                                                                                                \
  template void topk_from_facts<W>(const float*, const uint32_t*, size_t, TopKW<W>*, hipStream_t);                \
  template void topk_probability<W>(const TopKW<W>*, const uint32_t*, size_t, const float*, float*, hipStream_t);  \
  template void topk_split<W>(const TopKW<W>*, size_t, int, uint8_t*, uint64_t*, float*, hipStream_t);            \
  template void topk_backward<W>(const TopKW<W>*, const uint32_t*, const float*, size_t, const float*, float*,    \
                                 hipStream_t);

INST_W(1)
INST_W(4)
INST(uint32_t)
INST(uint64_t)
INST2(uint32_t)
INST2(uint64_t)

}  // namespace dlfix
