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
  bool keep = false, logit = false;
  if (act) {
    const uint64_t kk = (uint64_t)key;
    const size_t w = kk >> 5;
    const uint32_t bit = 1u << (kk & 31);
    const bool present = (d.present[w] & bit) != 0u;
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
        const uint32_t o = to_ordered(t);
        if (o > d.dtag[kk]) keep = o > atomicMax(d.dtag + kk, o);
        keep = keep || !present;
        break;
      }
      default: {  // DENSE_MIN
        const uint32_t o = to_ordered(t);
        if (o < d.dtag[kk]) keep = o < atomicMin(d.dtag + kk, o);
        keep = keep || !present;
        break;
      }
    }
    if (keep && !(d.touched[w] & bit)) atomicOr(d.touched + w, bit);
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

// Round end: the touched bits are exactly the new and changed tuples.  The
// bitmap is compacted in key order in two passes over the touched words:
// per-block popcount sums (dense_touched_counts), their exclusive scan, then
// dense_finalize, where every thread scans its BM_ITEMS consecutive words
// inside the block and writes their keys in ascending order.  The touched
// tuples become present, touched is cleared, frozen sums are clamped.
constexpr int BM_ITEMS = 16;
constexpr int BM_TILE = BLOCK * BM_ITEMS;

size_t dense_count_blocks(int w) { return (bitmap_words(w) + BM_TILE - 1) / BM_TILE; }

__global__ void k_acc_total(const uint64_t* __restrict__ src, uint64_t* __restrict__ acc) { *acc += *src; }

void accumulate_total(const uint64_t* src, uint64_t* acc, hipStream_t st) { k_acc_total<<<1, 1, 0, st>>>(src, acc); }

__global__ __launch_bounds__(BLOCK) void k_touched_counts(const uint32_t* __restrict__ bits, size_t words,
                                                          uint32_t* __restrict__ partial) {
  __shared__ uint32_t tmp[NWAVES];
  const size_t base = (size_t)blockIdx.x * BM_TILE + (size_t)threadIdx.x * BM_ITEMS;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i)
    if (base + i < words) c += (uint32_t)__popc(bits[base + i]);
  c = wave_sum(c);
  if (lane_id() == 0) tmp[threadIdx.x / WAVE] = c;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = tmp[0] + tmp[1] + tmp[2] + tmp[3];
}

void dense_touched_counts(const DenseArgs& d, int w, uint32_t* partial, hipStream_t st) {
  const size_t words = bitmap_words(w);
  DL_PROF_BEGIN(6, st);
  k_touched_counts<<<dense_count_blocks(w), BLOCK, 0, st>>>(d.touched, words, partial);
  DL_PROF_END(6, st, words * 4.0);
}

template <typename K>
__global__ __launch_bounds__(BLOCK) void k_dense_finalize(DenseArgs d, size_t words, const uint32_t* __restrict__ bpos,
                                                          K* __restrict__ keys, float* __restrict__ rtags,
                                                          uint32_t id_base, float* __restrict__ tag_by_id) {
  __shared__ uint32_t tmp[NWAVES];
  const size_t base = (size_t)blockIdx.x * BM_TILE + (size_t)threadIdx.x * BM_ITEMS;
  uint32_t b[BM_ITEMS];
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i) {
    b[i] = base + i < words ? d.touched[base + i] : 0u;
    c += (uint32_t)__popc(b[i]);
  }
  uint32_t tot;
  uint32_t o = bpos[blockIdx.x] + block_exclusive_scan(c, tmp, &tot);
  if (c == 0) return;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i) {
    uint32_t x = b[i];
    if (!x) continue;
    const size_t wi = base + i;
    d.present[wi] |= x;
    d.touched[wi] = 0u;
    while (x) {
      const int bit = __builtin_ctz(x);
      x &= x - 1;
      const uint64_t kk = ((uint64_t)wi << 5) | (uint64_t)bit;
      keys[o] = (K)kk;
      float t = 1.0f;
      if (d.mode == DENSE_ADD) {
        t = fminf(1.0f, __uint_as_float(d.dtag[kk]));
        d.dtag[kk] = __float_as_uint(t);
      } else if (d.mode != DENSE_BOOL) {
        t = from_ordered(d.dtag[kk]);
      }
      if (rtags) rtags[o] = t;
      if (d.did) {
        d.did[kk] = id_base + o;
        tag_by_id[id_base + o] = t;
      }
      ++o;
    }
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

__global__ void k_popc(const uint32_t* __restrict__ bits, size_t words, uint32_t* __restrict__ counts) {
  GRID_STRIDE(i, words) counts[i] = (uint32_t)__popc(bits[i]);
}

void bitmap_popcounts(const uint32_t* bits, size_t words, uint32_t* counts, hipStream_t st) {
  if (words) k_popc<<<grid_for(words), BLOCK, 0, st>>>(bits, words, counts);
}

template <typename K>
__global__ void k_bitmap_keys(DenseArgs d, size_t words, const uint32_t* __restrict__ pos, K* __restrict__ keys,
                              float* __restrict__ tags, uint32_t* __restrict__ ids) {
  GRID_STRIDE(wi, words) {
    uint32_t b = d.present[wi];
    uint32_t o = pos[wi];
    while (b) {
      const int i = __builtin_ctz(b);
      b &= b - 1;
      const uint64_t kk = ((uint64_t)wi << 5) | (uint64_t)i;
      keys[o] = (K)kk;
      if (tags) {
        const uint32_t x = d.dtag[kk];
        tags[o] = d.mode == DENSE_ADD ? __uint_as_float(x) : d.mode == DENSE_BOOL ? 1.0f : from_ordered(x);
      }
      if (ids) ids[o] = d.did[kk];
      ++o;
    }
  }
}

template <typename K>
void bitmap_keys(const DenseArgs& d, int w, const uint32_t* pos, K* keys, float* tags, uint32_t* ids, hipStream_t st) {
  const size_t words = bitmap_words(w);
  k_bitmap_keys<K><<<grid_for(words), BLOCK, 0, st>>>(d, words, pos, keys, tags, ids);
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
