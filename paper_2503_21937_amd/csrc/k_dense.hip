// Dense-domain deduplication for gfx950: when a derived relation's packed
// keys fit a small domain, its membership and tags live in flat arrays
// indexed by key.  The join kernel then tests every derivation against them,
// drops the ones that cannot change the relation, folds the rest into the
// dense tag with exact integer atomics (max / min on an order-preserving
// encoding of binary32, or float add for frozen add-mult sums), and appends
// each key the first time it is touched in the round (wave-aggregated
// append).  Only the touched keys are sorted afterwards.
#include "prof.h"
#include "rel_device.h"

namespace dlfix {

// binary32 -> u32 with the same order (negative values below positive ones)
__device__ __forceinline__ uint32_t to_ordered(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

uint32_t dense_init_word(int mode) {
  switch (mode) {
    case DENSE_MAX: return 0x80000000u;          // ordered(+0.0f): max-min zero
    case DENSE_MIN: return 0x7f800000u | 0x80000000u;  // ordered(+inf): min-plus zero
    default: return 0u;                          // add-mult sums start at 0.0f
  }
}

static int norm_items(int items) { return items == 1 || items == 2 || items == 8 ? items : 4; }

size_t dense_segments(size_t n, int items) {
  const size_t tile = (size_t)BLOCK * norm_items(items);
  return (n + tile - 1) / tile * NWAVES;
}

// Per-wave append cursor into the wave's private lineage segment (no
// atomics; the order inside a segment is slot order).
struct WaveSeg {
  uint32_t ln = 0;
};

// Called by every lane of the wave; `act` marks lanes holding a derivation.
template <typename K>
__device__ __forceinline__ void dense_emit(const DenseArgs& d, WaveSeg& ws, size_t seg, bool act, K key, float t,
                                           uint32_t l, uint32_t r, bool lineage) {
  // The presence, touched and tag words are loaded together up front and
  // every atomic is issued without waiting for its result.  A derivation
  // marks its key touched when it beats the tag it read: that value is no
  // older than the round's start and tags only move one way inside a round,
  // so the final tag then differs from the round-start tag; conversely the
  // first derivation to write the final value saw a smaller one.  A stale
  // touched word only costs a redundant atomicOr.
  bool keep = false, logit = false;
  if (act) {
    const uint64_t kk = (uint64_t)key;
    const size_t w = kk >> 5;
    const uint32_t bit = 1u << (kk & 31);
    const uint32_t pw = d.present[w];
    const uint32_t tw = d.touched[w];
    const bool present = (pw & bit) != 0u;
    switch (d.mode) {
      case DENSE_BOOL:
        keep = !present;
        break;
      case DENSE_ADD:
        if (!present) {
          atomicAdd(reinterpret_cast<float*>(d.dtag) + kk, t);
          keep = true;
          logit = lineage;
        }
        break;
      case DENSE_MAX: {
        const uint32_t o = to_ordered(t), cur = d.dtag[kk];
        if (o > cur) {
          atomicMax(d.dtag + kk, o);
          keep = true;
        }
        keep = keep || !present;
        break;
      }
      default: {  // DENSE_MIN
        const uint32_t o = to_ordered(t), cur = d.dtag[kk];
        if (o < cur) {
          atomicMin(d.dtag + kk, o);
          keep = true;
        }
        keep = keep || !present;
        break;
      }
    }
    if (keep && !(tw & bit)) atomicOr(d.touched + w, bit);
  }
  if (lineage) {
    const uint64_t lm = ballot(logit);
    if (logit) {
      const size_t o = seg * DENSE_SEG + ws.ln + rank_below(lm);
      reinterpret_cast<K*>(d.log_keys)[o] = key;
      d.log_l[o] = l;
      d.log_r[o] = r;
    }
    ws.ln += (uint32_t)__popcll(lm);
  }
}

__device__ __forceinline__ void dense_close(const DenseArgs& d, const WaveSeg& ws, size_t seg, bool lineage) {
  if (lineage && lane_id() == 0) d.seg_lcount[seg] = ws.ln;
}

// Each wave handles DX_ITEMS rows of 64 join outputs per block and owns one
// lineage segment (DX_ITEMS * 64 <= DENSE_SEG).
// Tiles of BLOCK * DX_ITEMS join outputs; a block loops over tiles
// (tile, tile + gridDim.x, ...).  The total comes from `total`, or from
// device memory (`dtotal`) when the host did not read it back: then the grid
// is a fixed size and blocks beyond the last tile exit at once.
template <typename K, int TK, int DX_ITEMS>
__global__ __launch_bounds__(BLOCK) void k_join_expand_dense(JoinArgs a, const uint32_t* __restrict__ offs,
                                                             size_t total_h, const uint64_t* __restrict__ dtotal,
                                                             DenseArgs d, int lineage) {
  using T = typename TagOf<TK>::T;
  constexpr int DX_TILE = BLOCK * DX_ITEMS;
  static_assert(DX_ITEMS * WAVE <= DENSE_SEG, "a wave's outputs must fit its segment");
  __shared__ uint32_t s_row[DX_TILE];
  __shared__ uint32_t s_wave[NWAVES];
  __shared__ size_t s_r[2];
  const K* dk = (const K*)a.dkeys;
  const K* ik = (const K*)a.ikeys;
  const T* dt = (const T*)a.dtags;
  const T* it = (const T*)a.itags;
  const size_t total = dtotal ? (size_t)*dtotal : total_h;
  if (total > 0xffffffffull) {  // offsets are 32-bit: refuse, the host reports it
    if (blockIdx.x == 0 && threadIdx.x == 0 && d.overflow) *d.overflow = 1;
    return;
  }
  const size_t ntiles = (total + DX_TILE - 1) / DX_TILE;
  for (size_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {  // uniform per block
    const size_t s0 = tile * DX_TILE;
    const size_t s1 = s0 + DX_TILE < total ? s0 + DX_TILE : total;
    tile_rows<DX_ITEMS>(offs, a.n, s0, s1, s_row, s_wave, s_r);
    const size_t seg = d.seg_base + tile * NWAVES + threadIdx.x / WAVE;
    WaveSeg ws;
    for (int it_ = 0; it_ < DX_ITEMS; ++it_) {
      const size_t j = s0 + (size_t)it_ * BLOCK + threadIdx.x;
      if (s0 + (size_t)it_ * BLOCK >= s1) break;  // uniform across the block
      const bool act = j < s1;
      K okey = 0;
      float t = 0.0f;
      uint32_t l = 0, r = 0;
      if (act) {
        const size_t row = s_row[j - s0];
        const uint32_t base = offs[row];
        const K dkey = dk[row];
        const uint64_t p = join_prefix(dkey, a);
        const uint32_t irow = a.off[p] + ((uint32_t)j - base);
        const K ikey = ik[irow];
        uint32_t v[4];
        for (int c = 0; c < a.olay.ncols; ++c) {
          int s = a.osrc[c];
          v[c] = s >= 0 ? key_col(dkey, s, a.dlay) : key_col(ikey, -1 - s, a.ilay);
        }
        const uint32_t sample = key_sample(dkey, a.dlay);
        okey = key_make<K>(sample, v, a.olay);
        if constexpr (TK == TAG_F32) {
          const float x = dt[row], y = it[irow];
          t = a.index_first ? f_otimes(a.sr, y, x) : f_otimes(a.sr, x, y);
        }
        if (lineage) {
          l = a.dids[row];
          r = a.iids[irow];
        }
      }
      dense_emit<K>(d, ws, seg, act, okey, t, l, r, lineage != 0);
    }
    dense_close(d, ws, seg, lineage != 0);
    __syncthreads();  // s_row is rebuilt for the next tile
  }
}

template <typename K>
void join_expand_dense(const JoinArgs& a, int tk, const uint32_t* offs, size_t total, const uint64_t* dtotal,
                       size_t max_total, const DenseArgs& d, bool lineage, hipStream_t st) {
  const int items = norm_items(a.items);
  const size_t tile = (size_t)BLOCK * items;
  size_t nb;
  if (dtotal) {  // total unknown on the host: bounded, fixed-size grid
    const size_t need = (max_total + tile - 1) / tile;
    nb = need < 4096 ? need : 4096;
    if (nb == 0) return;
  } else {
    if (!total) return;
    nb = (total + tile - 1) / tile;
  }
  const double tb = tk == TAG_F32 ? 4.0 : 0.0;
  const double lin = lineage ? 4.0 : 0.0;
  // per derivation: index row read, presence word and dense tag read; per probe row: driver row + offset
  const double per = (sizeof(K) + tb + lin + 4.0 + tb);
  const double bytes = (dtotal ? 0.0 : total * per) + a.n * (sizeof(K) + tb + lin + 4.0);
#define DL_DEXPAND(IT)                                                                                         \
  if (tk == TAG_F32)                                                                                           \
    k_join_expand_dense<K, TAG_F32, IT><<<nb, BLOCK, 0, st>>>(a, offs, total, dtotal, d, lineage ? 1 : 0);     \
  else                                                                                                         \
    k_join_expand_dense<K, TAG_NONE, IT><<<nb, BLOCK, 0, st>>>(a, offs, total, dtotal, d, lineage ? 1 : 0);
  DL_PROF_BEGIN(1, st);
  switch (items) {
    case 1: DL_DEXPAND(1) break;
    case 2: DL_DEXPAND(2) break;
    case 8: DL_DEXPAND(8) break;
    default: DL_DEXPAND(4) break;
  }
#undef DL_DEXPAND
  DL_PROF_END(1, st, bytes);
  if (dtotal) DL_PROF_DEFER(1, st, dtotal, per);
}

constexpr int PX_ITEMS = 4;  // projection: rows per thread (fixed tile)
constexpr int PX_TILE = BLOCK * PX_ITEMS;

template <typename K, int TK>
__global__ __launch_bounds__(BLOCK) void k_project_dense(JoinArgs a, DenseArgs d, int lineage) {
  const K* dk = (const K*)a.dkeys;
  const size_t seg = d.seg_base + (size_t)blockIdx.x * NWAVES + threadIdx.x / WAVE;
  WaveSeg ws;
  for (int it_ = 0; it_ < PX_ITEMS; ++it_) {
    const size_t i0 = (size_t)blockIdx.x * PX_TILE + (size_t)it_ * BLOCK;
    if (i0 >= a.n) break;  // uniform across the block
    const size_t i = i0 + threadIdx.x;
    const bool act = i < a.n;
    K okey = 0;
    float t = 0.0f;
    uint32_t l = 0;
    if (act) {
      const K dkey = dk[i];
      uint32_t v[4];
      for (int c = 0; c < a.olay.ncols; ++c) v[c] = key_col(dkey, a.osrc[c], a.dlay);
      okey = key_make<K>(key_sample(dkey, a.dlay), v, a.olay);
      if constexpr (TK == TAG_F32) t = ((const float*)a.dtags)[i];
      if (lineage) l = a.dids[i];
    }
    dense_emit<K>(d, ws, seg, act, okey, t, l, ~0u, lineage != 0);
  }
  dense_close(d, ws, seg, lineage != 0);
}

template <typename K>
void project_dense(const JoinArgs& a, int tk, const DenseArgs& d, bool lineage, hipStream_t st) {
  if (!a.n) return;
  const size_t nb = (a.n + PX_TILE - 1) / PX_TILE;
  if (tk == TAG_F32)
    k_project_dense<K, TAG_F32><<<nb, BLOCK, 0, st>>>(a, d, lineage ? 1 : 0);
  else
    k_project_dense<K, TAG_NONE><<<nb, BLOCK, 0, st>>>(a, d, lineage ? 1 : 0);
}

// Round end: the touched bits are exactly the new and changed tuples.  A
// bitmap is compacted in key order in two passes: per-block popcount sums
// (bitmap_block_counts), their exclusive scan, then an emission pass in which
// every wave walks BM_ITEMS groups of 64 consecutive words (one word per lane:
// coalesced) and expands their set bits cooperatively, so that consecutive
// lanes write consecutive keys whatever the bit density (wave_expand_bits).
// dense_finalize also makes the touched tuples present, clears touched,
// clamps frozen sums and, with lineage, hands out ids in key order.
constexpr int BM_ITEMS = 16;
constexpr int BM_TILE = BLOCK * BM_ITEMS;
constexpr int BM_WAVE_WORDS = WAVE * BM_ITEMS;

size_t dense_count_blocks(int w) { return (bitmap_words(w) + BM_TILE - 1) / BM_TILE; }

__global__ void k_acc_total(const uint64_t* __restrict__ src, uint64_t* __restrict__ acc) { *acc += *src; }

void accumulate_total(const uint64_t* src, uint64_t* acc, hipStream_t st) { k_acc_total<<<1, 1, 0, st>>>(src, acc); }

__global__ __launch_bounds__(BLOCK) void k_block_counts(const uint32_t* __restrict__ bits, size_t words,
                                                        uint32_t* __restrict__ partial) {
  __shared__ uint32_t tmp[NWAVES];
  const size_t base = (size_t)blockIdx.x * BM_TILE + threadIdx.x;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i) {
    const size_t wi = base + (size_t)i * BLOCK;
    if (wi < words) c += (uint32_t)__popc(bits[wi]);
  }
  c = wave_sum(c);
  if (lane_id() == 0) tmp[threadIdx.x / WAVE] = c;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = tmp[0] + tmp[1] + tmp[2] + tmp[3];
}

void bitmap_block_counts(const uint32_t* bits, int w, uint32_t* partial, hipStream_t st) {
  const size_t words = bitmap_words(w);
  DL_PROF_BEGIN(6, st);
  k_block_counts<<<dense_count_blocks(w), BLOCK, 0, st>>>(bits, words, partial);
  DL_PROF_END(6, st, words * 4.0);
}

// Position of the n-th (from 0) set bit of x, which has more than n.
__device__ __forceinline__ uint32_t select_bit(uint32_t x, uint32_t n) {
  uint32_t pos = 0;
#pragma unroll
  for (int sh = 16; sh > 0; sh >>= 1) {
    const uint32_t low = (uint32_t)__popc(x & ((1u << sh) - 1u));
    if (n >= low) {
      n -= low;
      x >>= sh;
      pos += sh;
    }
  }
  return pos;
}

// The set bits of 64 words, word wbase + lane in each lane, become slots
// base, base + 1, ... in key order: f(slot, key) runs with consecutive
// lanes on consecutive slots (source lane by a binary search over the wave's
// inclusive popcount scan, bit by rank select).  Called by the whole wave;
// returns the number of bits.
template <typename F>
__device__ __forceinline__ uint32_t wave_expand_bits(uint32_t x, uint64_t wbase, uint32_t base, F&& f) {
  const uint32_t cnt = (uint32_t)__popc(x);
  const uint32_t incl = wave_inclusive_scan(cnt);
  const uint32_t excl = incl - cnt;
  const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
  for (uint32_t j0 = 0; j0 < total; j0 += WAVE) {  // uniform across the wave
    const uint32_t j = j0 + (uint32_t)lane_id();
    int src = 0;  // lanes whose inclusive count is <= j
#pragma unroll
    for (int step = WAVE / 2; step > 0; step >>= 1) {
      const uint32_t v = __shfl(incl, src + step - 1, WAVE);
      if (v <= j) src += step;
    }
    const uint32_t word = __shfl(x, src, WAVE);
    const uint32_t before = __shfl(excl, src, WAVE);
    if (j < total) f(base + j, ((wbase + (uint64_t)src) << 5) | select_bit(word, j - before));
  }
  return total;
}

template <typename K>
__global__ __launch_bounds__(BLOCK) void k_dense_finalize(DenseArgs d, size_t words, const uint32_t* __restrict__ bpos,
                                                          K* __restrict__ keys, float* __restrict__ rtags,
                                                          uint32_t id_base, float* __restrict__ tag_by_id) {
  __shared__ uint32_t s_tot[NWAVES];
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  const size_t w0 = (size_t)blockIdx.x * BM_TILE + (size_t)wv * BM_WAVE_WORDS;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i) {
    const size_t wi = w0 + (size_t)i * WAVE + lane;
    if (wi < words) c += (uint32_t)__popc(d.touched[wi]);
  }
  c = wave_sum(c);
  if (lane == 0) s_tot[wv] = c;
  __syncthreads();
  if (c == 0) return;  // wave-uniform; no barrier follows
  uint32_t o = bpos[blockIdx.x];
  for (int i = 0; i < wv; ++i) o += s_tot[i];
  for (int i = 0; i < BM_ITEMS; ++i) {
    const size_t wb = w0 + (size_t)i * WAVE;
    const size_t wi = wb + lane;
    const uint32_t x = wi < words ? d.touched[wi] : 0u;
    if (!__ballot(x != 0u)) continue;
    if (x) {
      d.present[wi] |= x;
      d.touched[wi] = 0u;
    }
    o += wave_expand_bits(x, wb, o, [&](uint32_t slot, uint64_t kk) {
      keys[slot] = (K)kk;
      float t = 1.0f;
      if (d.mode == DENSE_ADD) {
        t = fminf(1.0f, __uint_as_float(d.dtag[kk]));
        d.dtag[kk] = __float_as_uint(t);
      } else if (d.mode != DENSE_BOOL) {
        t = from_ordered(d.dtag[kk]);
      }
      if (rtags) rtags[slot] = t;
      if (d.did) {
        d.did[kk] = id_base + slot;
        tag_by_id[id_base + slot] = t;
      }
    });
  }
}

template <typename K>
void dense_finalize(const DenseArgs& d, int w, const uint32_t* bpos, K* keys, float* rtags, uint32_t id_base,
                    float* tag_by_id, hipStream_t st) {
  const size_t words = bitmap_words(w);
  DL_PROF_BEGIN(6, st);
  k_dense_finalize<K><<<dense_count_blocks(w), BLOCK, 0, st>>>(d, words, bpos, keys, rtags, id_base, tag_by_id);
  DL_PROF_END(6, st, words * 12.0);
}

template <typename K>
__global__ void k_dense_owners(DenseArgs d, const K* __restrict__ keys, size_t n, uint32_t* __restrict__ owner) {
  GRID_STRIDE(i, n) owner[i] = d.did[(uint64_t)keys[i]];
}

template <typename K>
void dense_owners(const DenseArgs& d, const K* keys, size_t n, uint32_t* owner, hipStream_t st) {
  if (n) k_dense_owners<K><<<grid_for(n), BLOCK, 0, st>>>(d, keys, n, owner);
}

// One block per segment: copy its elements to their compacted position.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_segments_compact(const T* __restrict__ in, const uint32_t* __restrict__ cnt,
                                                            const uint32_t* __restrict__ pos, size_t nseg,
                                                            T* __restrict__ out) {
  for (size_t s = blockIdx.x; s < nseg; s += gridDim.x) {
    const uint32_t c = cnt[s], o = pos[s];
    for (uint32_t i = threadIdx.x; i < c; i += BLOCK) out[o + i] = in[s * DENSE_SEG + i];
  }
}

void segments_compact(const void* in, const uint32_t* cnt, const uint32_t* pos, size_t nseg, size_t bytes, void* out,
                      hipStream_t st) {
  if (!nseg) return;
  const unsigned g = (unsigned)(nseg < 65536 ? nseg : 65536);
  DL_PROF_BEGIN(8, st);
  if (bytes == 4)
    k_segments_compact<uint32_t><<<g, BLOCK, 0, st>>>((const uint32_t*)in, cnt, pos, nseg, (uint32_t*)out);
  else
    k_segments_compact<uint64_t><<<g, BLOCK, 0, st>>>((const uint64_t*)in, cnt, pos, nseg, (uint64_t*)out);
  DL_PROF_END(8, st, nseg * 8.0);
}

size_t bitmap_words(int w) { return w >= 5 ? (size_t)1 << (w - 5) : 1; }

// Sorted keys of the present bits (one block per BM_TILE words, block
// offsets from bitmap_block_counts + scan), with their tags and ids.
template <typename K>
__global__ __launch_bounds__(BLOCK) void k_bitmap_keys(DenseArgs d, size_t words, const uint32_t* __restrict__ bpos,
                                                       K* __restrict__ keys, float* __restrict__ tags,
                                                       uint32_t* __restrict__ ids) {
  __shared__ uint32_t s_tot[NWAVES];
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  const size_t w0 = (size_t)blockIdx.x * BM_TILE + (size_t)wv * BM_WAVE_WORDS;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i) {
    const size_t wi = w0 + (size_t)i * WAVE + lane;
    if (wi < words) c += (uint32_t)__popc(d.present[wi]);
  }
  c = wave_sum(c);
  if (lane == 0) s_tot[wv] = c;
  __syncthreads();
  if (c == 0) return;  // wave-uniform; no barrier follows
  uint32_t o = bpos[blockIdx.x];
  for (int i = 0; i < wv; ++i) o += s_tot[i];
  for (int i = 0; i < BM_ITEMS; ++i) {
    const size_t wb = w0 + (size_t)i * WAVE;
    const size_t wi = wb + lane;
    const uint32_t x = wi < words ? d.present[wi] : 0u;
    if (!__ballot(x != 0u)) continue;
    o += wave_expand_bits(x, wb, o, [&](uint32_t slot, uint64_t kk) {
      keys[slot] = (K)kk;
      if (tags) {
        const uint32_t v = d.dtag[kk];
        tags[slot] = d.mode == DENSE_ADD ? __uint_as_float(v) : d.mode == DENSE_BOOL ? 1.0f : from_ordered(v);
      }
      if (ids) ids[slot] = d.did[kk];
    });
  }
}

template <typename K>
void bitmap_keys(const DenseArgs& d, int w, const uint32_t* bpos, K* keys, float* tags, uint32_t* ids, hipStream_t st) {
  const size_t words = bitmap_words(w);
  DL_PROF_BEGIN(6, st);
  k_bitmap_keys<K><<<dense_count_blocks(w), BLOCK, 0, st>>>(d, words, bpos, keys, tags, ids);
  DL_PROF_END(6, st, words * 4.0);
}

#define INST(K)                                                                                                       \
  template void join_expand_dense<K>(const JoinArgs&, int, const uint32_t*, size_t, const uint64_t*, size_t,     \
                                     const DenseArgs&, bool, hipStream_t);                                                                   \
  template void project_dense<K>(const JoinArgs&, int, const DenseArgs&, bool, hipStream_t);                        \
  template void dense_finalize<K>(const DenseArgs&, int, const uint32_t*, K*, float*, uint32_t, float*, hipStream_t);       \
  template void dense_owners<K>(const DenseArgs&, const K*, size_t, uint32_t*, hipStream_t);                                  \
  template void bitmap_keys<K>(const DenseArgs&, int, const uint32_t*, K*, float*, uint32_t*, hipStream_t);

INST(uint32_t)
INST(uint64_t)

}  // namespace dlfix
