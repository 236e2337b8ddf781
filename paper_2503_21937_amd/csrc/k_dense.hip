// Dense-domain deduplication for gfx950: when a derived relation's packed
// keys fit a small domain, its membership and tags live in flat arrays
// indexed by key.  The join kernel then tests every derivation against them,
// drops the ones that cannot change the relation, folds the rest into the
// dense tag with exact integer atomics (max / min on an order-preserving
// encoding of binary32, or float add for frozen add-mult sums), and appends
// each key the first time it is touched in the round (wave-aggregated
// append).  Only the touched keys are sorted afterwards.
#include <type_traits>

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

__device__ __forceinline__ uint32_t dense_init_word_dev(int mode) {
  return mode == DENSE_MAX ? 0x80000000u : mode == DENSE_MIN ? (0x7f800000u | 0x80000000u) : 0u;
}

uint32_t dense_init_word(int mode) {
  switch (mode) {
    case DENSE_MAX: return 0x80000000u;          // ordered(+0.0f): max-min zero
    case DENSE_MIN: return 0x7f800000u | 0x80000000u;  // ordered(+inf): min-plus zero
    default: return 0u;                          // add-mult sums start at 0.0f
  }
}

static int norm_items(int items) { return items == 1 || items == 2 || items == 8 ? items : 4; }

// Packed key -> dense index (mixed radix, see DenseArgs) and back.  Dense
// domains hold fewer than 2^32 keys.
template <typename K>
__device__ __forceinline__ uint32_t dense_index(const DenseArgs& d, K key) {
  const uint64_t k = (uint64_t)key;
  const uint32_t mask = (1u << d.dcbits) - 1u;
  const uint32_t s = (uint32_t)(k >> (d.dcols * d.dcbits));
  uint32_t base = 0, n = d.dn, np = d.dnp;
  if (d.nsamp > 1) {
    base = d.sbase[s];
    n = d.sn[s];
    np = d.snp[s];
  }
  uint32_t idx = 0;
  for (int c = 0; c + 1 < d.dcols; ++c) idx = idx * n + ((uint32_t)(k >> ((d.dcols - 1 - c) * d.dcbits)) & mask);
  return base + idx * np + ((uint32_t)k & mask);
}

static void divisor(uint32_t dv, uint32_t* m, uint8_t* s1, uint8_t* s2) {
  int l = 0;
  while (l < 32 && ((uint64_t)1 << l) < dv) ++l;  // l = ceil(log2 dv)
  *m = (uint32_t)(((((uint64_t)1 << l) - dv) << 32) / dv + 1);
  *s1 = (uint8_t)(l < 1 ? l : 1);
  *s2 = (uint8_t)(l > 1 ? l - 1 : 0);
}

void dense_divisors(DenseArgs& d) {
  divisor(d.dn, &d.dn_m, &d.dn_s1, &d.dn_s2);
  divisor(d.dnp, &d.dnp_m, &d.dnp_s1, &d.dnp_s2);
}

__device__ __forceinline__ uint32_t fast_div(uint32_t n, uint32_t m, uint32_t s1, uint32_t s2) {
  const uint32_t t = __umulhi(n, m);
  return (t + ((n - t) >> s1)) >> s2;
}

// Sample whose dense block holds idx (batched engines).
__device__ __forceinline__ uint32_t dense_sample(const DenseArgs& d, uint32_t idx) {
  uint32_t lo = 0, hi = d.nsamp;  // sbase[lo] <= idx < sbase[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (d.sbase[mid] <= idx) lo = mid;
    else hi = mid;
  }
  return lo;
}

// idx -> packed key; `s_from` is a sample at or before idx's (batched), so
// that a run of nearby indexes walks forward instead of searching.
template <typename K>
__device__ __forceinline__ K dense_key(const DenseArgs& d, uint32_t idx, uint32_t s_from = ~0u) {
  if (d.nsamp > 1) {  // the sample whose block holds idx, then its own radix
    uint32_t lo;
    if (s_from == ~0u) {
      lo = dense_sample(d, idx);
    } else {
      lo = s_from;
      while (lo + 1 < d.nsamp && d.sbase[lo + 1] <= idx) ++lo;
    }
    const uint32_t n = d.sn[lo], np = d.snp[lo];
    uint32_t r = idx - d.sbase[lo];
    uint64_t k = r % np;
    r /= np;
    for (int c = 1; c < d.dcols; ++c) {
      k |= (uint64_t)(r % n) << (c * d.dcbits);
      r /= n;
    }
    return (K)(k | ((uint64_t)lo << (d.dcols * d.dcbits)));
  }
  uint32_t q = fast_div(idx, d.dnp_m, d.dnp_s1, d.dnp_s2);
  uint64_t k = idx - q * d.dnp;
  idx = q;
  for (int c = 1; c < d.dcols; ++c) {
    q = fast_div(idx, d.dn_m, d.dn_s1, d.dn_s2);
    k |= (uint64_t)(idx - q * d.dn) << (c * d.dcbits);
    idx = q;
  }
  return (K)(k | ((uint64_t)idx << (d.dcols * d.dcbits)));
}

size_t dense_segments(size_t n, int items) {
  const size_t tile = (size_t)BLOCK * norm_items(items);
  return (n + tile - 1) / tile * NWAVES;
}

// Per-wave append cursor into the wave's private lineage segment (no
// atomics; the order inside a segment is slot order).
struct WaveSeg {
  uint32_t ln = 0;
};

// Words a derivation's update depends on, loaded before any update of the
// tile is issued (so that the loads of several derivations overlap).
struct DenseProbe {
  uint32_t pw = 0, tw = 0, cur = 0;
};

template <typename K>
__device__ __forceinline__ DenseProbe dense_load(const DenseArgs& d, bool act, K key) {
  DenseProbe pr;
  if (act) {
    const uint32_t kk = dense_index(d, key);
    pr.pw = d.present[kk >> 5];
    pr.tw = d.touched[kk >> 5];
    if (d.mode == DENSE_MAX || d.mode == DENSE_MIN) pr.cur = d.dtag[kk];
  }
  return pr;
}

// Called by every lane of the wave; `act` marks lanes holding a derivation.
// Every atomic is issued without waiting for its result.  A derivation marks
// its key touched when it beats the tag it read: that value is no older than
// the round's start and tags only move one way inside a round, so the final
// tag then differs from the round-start tag; conversely the first
// derivation to write the final value saw a smaller one.  A stale touched
// word only costs a redundant atomicOr.
template <typename K>
__device__ __forceinline__ void dense_apply(const DenseArgs& d, WaveSeg& ws, size_t seg, bool act, K key, float t,
                                            uint32_t l, uint32_t r, bool lineage, const DenseProbe& pr) {
  bool keep = false, logit = false;
  if (act) {
    const uint32_t kk = dense_index(d, key);
    const size_t w = kk >> 5;
    const uint32_t bit = 1u << (kk & 31);
    const bool present = (pr.pw & bit) != 0u;
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
        if (o > pr.cur) {
          atomicMax(d.dtag + kk, o);
          keep = true;
        }
        keep = keep || !present;
        break;
      }
      default: {  // DENSE_MIN
        const uint32_t o = to_ordered(t);
        if (o < pr.cur) {
          atomicMin(d.dtag + kk, o);
          keep = true;
        }
        keep = keep || !present;
        break;
      }
    }
    if (keep && !(pr.tw & bit)) atomicOr(d.touched + w, bit);
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

template <typename K>
__device__ __forceinline__ void dense_emit(const DenseArgs& d, WaveSeg& ws, size_t seg, bool act, K key, float t,
                                           uint32_t l, uint32_t r, bool lineage) {
  dense_apply<K>(d, ws, seg, act, key, t, l, r, lineage, dense_load<K>(d, act, key));
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
// FM >= 0: the specialised variant (32-bit keys, one sample, binary head of
// a driver column and an index column, no lineage, dense mode FM with its
// semiring's product): the dense index is c0 * dnp + c1, computed from the
// two columns without building the packed key.
template <typename K, int TK, int DX_ITEMS, int FM>
__global__ __launch_bounds__(BLOCK) void k_join_expand_dense(JoinArgs a, const uint32_t* __restrict__ offs,
                                                             size_t total_h, const uint64_t* __restrict__ dtotal,
                                                             DenseArgs d, int lineage_arg, uint64_t skip_at) {
  using T = typename TagOf<TK>::T;
  constexpr bool FAST = FM >= 0;
  const int lineage = FAST ? 0 : lineage_arg;
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
  if (total >= skip_at) return;  // the row-window kernel takes this launch
  const size_t ntiles = (total + DX_TILE - 1) / DX_TILE;
  for (size_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {  // uniform per block
    const size_t s0 = tile * DX_TILE;
    const size_t s1 = s0 + DX_TILE < total ? s0 + DX_TILE : total;
    tile_rows<DX_ITEMS>(offs, a.n, s0, s1, s_row, s_wave, s_r);
    const size_t seg = d.seg_base + tile * NWAVES + threadIdx.x / WAVE;
    WaveSeg ws;
    // The items of a thread go through each dependent step together (probe
    // row -> CSR offset -> index row -> dense words), so that their loads
    // overlap instead of paying one memory latency per item and step.
    bool act[DX_ITEMS];
    uint32_t row[DX_ITEMS], irow[DX_ITEMS], base[DX_ITEMS];
    K dkey[DX_ITEMS], okey[DX_ITEMS];
    float t[DX_ITEMS];
#pragma unroll
    for (int q = 0; q < DX_ITEMS; ++q) {
      const size_t j = s0 + (size_t)q * BLOCK + threadIdx.x;
      act[q] = j < s1;
      row[q] = act[q] ? s_row[j - s0] : 0u;
    }
#pragma unroll
    for (int q = 0; q < DX_ITEMS; ++q) {
      base[q] = act[q] ? offs[row[q]] : 0u;
      dkey[q] = act[q] ? dk[row[q]] : (K)0;
      irow[q] = act[q] ? a.istart[row[q]] : 0u;
    }
#pragma unroll
    for (int q = 0; q < DX_ITEMS; ++q) {
      const uint32_t j = (uint32_t)(s0 + (size_t)q * BLOCK + threadIdx.x);
      irow[q] += j - base[q];
    }
    if constexpr (FAST) {
      // column 0 from the driver key, column 1 from the index key
      const uint32_t sh0 = (uint32_t)((a.dlay.ncols - 1 - a.osrc[0]) * a.dlay.cbits);
      const uint32_t sh1 = (uint32_t)((a.ilay.ncols - 1 - (-1 - a.osrc[1])) * a.ilay.cbits);
      const uint32_t m0 = cmask(a.dlay.cbits), m1 = cmask(a.ilay.cbits);
      uint32_t kk[DX_ITEMS];
      float tt[DX_ITEMS];
#pragma unroll
      for (int q = 0; q < DX_ITEMS; ++q) {
        kk[q] = 0;
        tt[q] = 0.0f;
        if (act[q]) {
          const K ikey = ik[irow[q]];
          kk[q] = (((uint32_t)dkey[q] >> sh0) & m0) * d.dnp + (((uint32_t)ikey >> sh1) & m1);
          if constexpr (TK == TAG_F32) {
            const float x = dt[row[q]], y = it[irow[q]];
            const float p = a.index_first ? y : x, r = a.index_first ? x : y;
            tt[q] = FM == DENSE_ADD ? __fmul_rn(p, r) : FM == DENSE_MAX ? fminf(p, r) : __fadd_rn(p, r);
          }
        }
      }
      uint32_t pw[DX_ITEMS], tw[DX_ITEMS], cur[DX_ITEMS];
#pragma unroll
      for (int q = 0; q < DX_ITEMS; ++q) {
        pw[q] = tw[q] = cur[q] = 0;
        if (act[q]) {
          pw[q] = d.present[kk[q] >> 5];
          tw[q] = d.touched[kk[q] >> 5];
          if constexpr (FM == DENSE_MAX || FM == DENSE_MIN) cur[q] = d.dtag[kk[q]];
        }
      }
#pragma unroll
      for (int q = 0; q < DX_ITEMS; ++q) {
        if (!act[q]) continue;
        const uint32_t bit = 1u << (kk[q] & 31);
        const bool present = (pw[q] & bit) != 0u;
        bool keep;
        if constexpr (FM == DENSE_BOOL) {
          keep = !present;
        } else if constexpr (FM == DENSE_ADD) {
          keep = !present;
          if (keep) atomicAdd(reinterpret_cast<float*>(d.dtag) + kk[q], tt[q]);
        } else if constexpr (FM == DENSE_MAX) {
          const uint32_t o = to_ordered(tt[q]);
          keep = o > cur[q];
          if (keep) atomicMax(d.dtag + kk[q], o);
          keep = keep || !present;
        } else {
          const uint32_t o = to_ordered(tt[q]);
          keep = o < cur[q];
          if (keep) atomicMin(d.dtag + kk[q], o);
          keep = keep || !present;
        }
        if (keep && !(tw[q] & bit)) atomicOr(d.touched + (kk[q] >> 5), bit);
      }
      __syncthreads();  // s_row is rebuilt for the next tile
      continue;
    }
#pragma unroll
    for (int q = 0; q < DX_ITEMS; ++q) {
      okey[q] = 0;
      t[q] = 0.0f;
      if (act[q]) {
        const K ikey = ik[irow[q]];
        uint32_t v[4];
        act[q] = out_cols<K>(a, dkey[q], ikey, v);  // with evaluation: the condition and computed columns
        okey[q] = key_make<K>(key_sample(dkey[q], a.dlay), v, a.olay);
        if constexpr (TK == TAG_F32) {
          const float x = dt[row[q]], y = it[irow[q]];
          t[q] = a.index_first ? f_otimes(a.sr, y, x) : f_otimes(a.sr, x, y);
        }
      }
    }
    DenseProbe pr[DX_ITEMS];
#pragma unroll
    for (int q = 0; q < DX_ITEMS; ++q) pr[q] = dense_load<K>(d, act[q], okey[q]);
#pragma unroll
    for (int q = 0; q < DX_ITEMS; ++q) {
      if (s0 + (size_t)q * BLOCK >= s1) break;  // uniform across the block
      uint32_t l = 0, r = 0;
      if (lineage && act[q]) {
        l = a.dids[row[q]];
        r = a.iids[irow[q]];
      }
      dense_apply<K>(d, ws, seg, act[q], okey[q], t[q], l, r, lineage != 0, pr[q]);
    }
    dense_close(d, ws, seg, lineage != 0);
    __syncthreads();  // s_row is rebuilt for the next tile
  }
}

// Row-window variant for static-driven joins whose head key starts with the
// driver's (sample, first column) prefix p: all derivations of the driver
// rows with prefix p land in one window of the head's dense indexes (the
// keys with that prefix).  One workgroup owns one window at a time: it loads
// the window's presence bits and tags into LDS, folds every derivation of the
// group there with LDS atomics (duplicates across the group's driver rows
// meet in LDS), and writes back only the entries it changed, with plain
// coalesced stores (no other workgroup of the launch touches the window).
// This trades one streaming pass over the windows for scattered global
// atomics and pays off when the launch has many derivations per window: the
// host sets the threshold `from`; a launch whose total is only known on the
// device reads it and, below the threshold, runs load-balanced scattered
// tiles itself (one launch per join either way).
constexpr int RW_BITS = 13;  // largest window: 8192 keys (32 KB of tags)
constexpr int RW_KEYS = 1 << RW_BITS;
constexpr int RW_ROWS = 255;   // driver rows of a group staged in LDS (4 workgroups fit a CU)
constexpr int RW_BLOCK = 512;  // 8 waves: the window's LDS is shared by more waves
constexpr int RW_WAVES = RW_BLOCK / WAVE;
constexpr int SPARSE_ITEMS = 2;  // fused rounds: derivations per lane in flight in a sparse group
static_assert(RW_KEYS / 32 <= RW_WAVES * WAVE, "a wave's share of a window's mark words fits its lanes");

// FM >= 0 selects the specialised variant for the most common shape: 32-bit
// keys, one sample, a binary head whose second column comes from the index
// row, no lineage, and the dense mode FM with its semiring's product (min for
// DENSE_MAX, + for DENSE_MIN, * for DENSE_ADD); FM = -1 is the general one.
template <typename K, int TK, int RX_ITEMS, int FM>
__global__ __launch_bounds__(RW_BLOCK, 8) void k_join_expand_rows(JoinArgs a, const uint32_t* __restrict__ offs,
                                                               size_t total_h, const uint64_t* __restrict__ dtotal,
                                                               DenseArgs d, RowWindows rw, int lineage_arg) {
  using T = typename TagOf<TK>::T;
  constexpr bool FAST = FM >= 0;
  const int lineage = FAST ? 0 : lineage_arg;
  constexpr int TILE = RW_BLOCK * RX_ITEMS;
  // window tags; in a launch below the threshold, the tile's slot -> row map
  __shared__ uint32_t s_tag[RW_KEYS];
  __shared__ uint32_t s_pres[RW_KEYS / 32];
  __shared__ uint32_t s_new[RW_KEYS / 32];
  // per driver row of the group: first output slot, index row of the first
  // output minus that slot (mod 2^32), key and tag
  __shared__ uint32_t s_offs[RW_ROWS + 1];
  __shared__ uint32_t s_ibase[RW_ROWS];
  __shared__ K s_dkey[RW_ROWS];
  __shared__ float s_dtag[TK == TAG_F32 ? RW_ROWS : 1];
  __shared__ uint32_t s_did[RW_ROWS];  // lineage: driver row ids
  __shared__ __align__(8) uint32_t s_cpre[RW_ROWS + 1];  // chunks of 64 outputs before each row
  const size_t total = dtotal ? (size_t)*dtotal : total_h;
  if (total > 0xffffffffull) {  // offsets are 32-bit: refuse, the host reports it
    if (blockIdx.x == 0 && threadIdx.x == 0 && d.overflow) *d.overflow = 1;
    return;
  }
  const K* dk = (const K*)a.dkeys;
  const K* ik = (const K*)a.ikeys;
  const T* dt = (const T*)a.dtags;
  const T* it = (const T*)a.itags;
  // Output columns 1.. (column 0 is the group's): which key holds each and
  // at which shift, fixed for the launch, so a derivation extracts them with
  // one shift and mask apiece.
  const int nc = FAST ? 2 : a.olay.ncols;
  bool from_index[4];
  uint32_t shf[4], msk[4];
#pragma unroll
  for (int c = 1; c < (FAST ? 2 : 4); ++c) {
    const int s = c < nc ? a.osrc[c] : 0;
    from_index[c] = s < 0;
    const KeyLayout& l = s < 0 ? a.ilay : a.dlay;
    shf[c] = (uint32_t)((l.ncols - 1 - (s < 0 ? -1 - s : s)) * l.cbits);
    msk[c] = cmask(l.cbits);
  }
  if (total < rw.from) {
    // Too few derivations for windows (the total is only known on the
    // device): scattered dense updates over load-balanced tiles of
    // RW_BLOCK * RX_ITEMS outputs, as k_join_expand_dense does (no lineage:
    // the host launches this kernel below the threshold only without it).
    if (lineage) return;
    uint32_t* s_row = s_tag;
    uint32_t* s_wv = s_cpre;
    size_t* s_r = reinterpret_cast<size_t*>(s_cpre + 2 * RW_WAVES);
    const size_t ntiles = (total + TILE - 1) / TILE;
    for (size_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {  // uniform per block
      const size_t t0 = tile * TILE;
      const size_t t1 = t0 + TILE < total ? t0 + TILE : total;
      tile_rows<RX_ITEMS, RW_BLOCK>(offs, a.n, t0, t1, s_row, s_wv, s_r);
      bool act[RX_ITEMS];
      uint32_t row[RX_ITEMS], irow[RX_ITEMS];
      K dkey[RX_ITEMS], ikey[RX_ITEMS];
      float x[RX_ITEMS], y[RX_ITEMS];
#pragma unroll
      for (int q = 0; q < RX_ITEMS; ++q) {
        const size_t j = t0 + (size_t)q * RW_BLOCK + threadIdx.x;
        act[q] = j < t1;
        row[q] = act[q] ? s_row[j - t0] : 0u;
      }
#pragma unroll
      for (int q = 0; q < RX_ITEMS; ++q) {
        const uint32_t j = (uint32_t)(t0 + (size_t)q * RW_BLOCK + threadIdx.x);
        dkey[q] = act[q] ? dk[row[q]] : (K)0;
        irow[q] = act[q] ? a.istart[row[q]] + (j - offs[row[q]]) : 0u;
        x[q] = 0.0f;
        if constexpr (TK == TAG_F32) x[q] = act[q] ? dt[row[q]] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < RX_ITEMS; ++q) {
        ikey[q] = act[q] ? ik[irow[q]] : (K)0;
        y[q] = 0.0f;
        if constexpr (TK == TAG_F32) y[q] = act[q] ? it[irow[q]] : 0.0f;
      }
      uint32_t kk[RX_ITEMS];
      float tt[RX_ITEMS];
#pragma unroll
      for (int q = 0; q < RX_ITEMS; ++q) {
        // the head key's dense index (mixed radix) and the derivation's tag
        kk[q] = 0;
        tt[q] = 0.0f;
        if (act[q]) {
          if constexpr (FAST) {
            kk[q] = ((uint32_t)dkey[q] >> (uint32_t)((a.dlay.ncols - 1) * a.dlay.cbits) & cmask(a.dlay.cbits)) * d.dnp +
                    (((uint32_t)ikey[q] >> shf[1]) & msk[1]);
          } else {
            uint32_t v[4];
            for (int c = 0; c < a.olay.ncols; ++c) {
              const int sc = a.osrc[c];
              v[c] = sc >= 0 ? key_col(dkey[q], sc, a.dlay) : key_col(ikey[q], -1 - sc, a.ilay);
            }
            kk[q] = dense_index(d, key_make<K>(key_sample(dkey[q], a.dlay), v, a.olay));
          }
          if constexpr (TK == TAG_F32) tt[q] = a.index_first ? f_otimes(a.sr, y[q], x[q]) : f_otimes(a.sr, x[q], y[q]);
        }
      }
      uint32_t pw[RX_ITEMS], tw[RX_ITEMS], cur[RX_ITEMS];
#pragma unroll
      for (int q = 0; q < RX_ITEMS; ++q) {
        pw[q] = tw[q] = cur[q] = 0;
        if (act[q]) {
          pw[q] = d.present[kk[q] >> 5];
          tw[q] = d.touched[kk[q] >> 5];
          if (d.mode == DENSE_MAX || d.mode == DENSE_MIN) cur[q] = d.dtag[kk[q]];
        }
      }
#pragma unroll
      for (int q = 0; q < RX_ITEMS; ++q) {
        if (!act[q]) continue;
        const uint32_t bit = 1u << (kk[q] & 31);
        const bool present = (pw[q] & bit) != 0u;
        const int mode = FAST ? FM : d.mode;
        bool keep = false;
        if (mode == DENSE_BOOL) {
          keep = !present;
        } else if (mode == DENSE_ADD) {
          keep = !present;
          if (keep) atomicAdd(reinterpret_cast<float*>(d.dtag) + kk[q], tt[q]);
        } else if (mode == DENSE_MAX) {
          const uint32_t o = to_ordered(tt[q]);
          keep = o > cur[q];
          if (keep) atomicMax(d.dtag + kk[q], o);
          keep = keep || !present;
        } else {
          const uint32_t o = to_ordered(tt[q]);
          keep = o < cur[q];
          if (keep) atomicMin(d.dtag + kk[q], o);
          keep = keep || !present;
        }
        if (keep && !(tw[q] & bit)) atomicOr(d.touched + (kk[q] >> 5), bit);
      }
      __syncthreads();  // s_row is rebuilt for the next tile
    }
    return;
  }
  const uint32_t pmask = (1u << d.dcbits) - 1u;
  // The next group's driver rows are fetched while the current one is
  // processed (its CSR bounds at the top, their output slots after the
  // window load), so a group starts without waiting on those loads.
  size_t g = blockIdx.x;
  uint32_t r0 = 0, r1 = 0, s0 = 0, s1 = 0;
  if (g < rw.ngroups) {
    r0 = rw.goff[g];
    r1 = rw.goff[g + 1];
    s0 = offs[r0];
    s1 = offs[r1];
  }
  for (; g < rw.ngroups; g += gridDim.x) {  // uniform per block
    const size_t gn = g + gridDim.x;
    uint32_t nr0 = 0, nr1 = 0, ns0 = 0, ns1 = 0;
    if (gn < rw.ngroups) {
      nr0 = rw.goff[gn];
      nr1 = rw.goff[gn + 1];
    }
    if (r0 == r1 || s0 == s1) {  // nothing to derive in this group
      if (gn < rw.ngroups) {
        ns0 = offs[nr0];
        ns1 = offs[nr1];
      }
      r0 = nr0, r1 = nr1, s0 = ns0, s1 = ns1;
      continue;
    }
    const uint32_t nr = r1 - r0;
    const bool lds_rows = nr <= (uint32_t)RW_ROWS;  // else rows are read from global memory
    // window of the prefix (sample, col 0): dense indexes kb .. kb + W - 1,
    // W = n^(arity-2) * np for the sample's n and np (a multiple of 32)
    const uint32_t gs = (uint32_t)(g >> d.dcbits), c0 = (uint32_t)g & pmask;
    uint32_t gn_ = d.dn, gnp = d.dnp, gbase = 0;
    if (!FAST && d.nsamp > 1) {
      gn_ = d.sn[gs];
      gnp = d.snp[gs];
      gbase = d.sbase[gs];
    }
    uint32_t W = gnp;
    for (int c = 2; c < nc; ++c) W *= gn_;
    const uint64_t kb = (uint64_t)gbase + (uint64_t)c0 * W;
    const uint32_t NWD = W / 32;
    const size_t wb = kb >> 5;
    for (uint32_t i = threadIdx.x; i < NWD; i += RW_BLOCK) {
      s_pres[i] = d.present[wb + i];
      s_new[i] = 0u;
    }
    if constexpr (TK == TAG_F32) {
      // 16-byte loads, several in flight per thread (the window is
      // W >= 32 keys long and W-aligned, hence 128-byte aligned)
      const uint4* src = reinterpret_cast<const uint4*>(d.dtag + kb);
      uint4* dst = reinterpret_cast<uint4*>(s_tag);
#pragma unroll 4
      for (uint32_t i = threadIdx.x; i < W / 4; i += RW_BLOCK) dst[i] = src[i];
    }
    if (gn < rw.ngroups) {
      ns0 = offs[nr0];
      ns1 = offs[nr1];
    }
    if (lds_rows) {
      for (uint32_t i = threadIdx.x; i <= nr; i += RW_BLOCK) {
        const uint32_t o = offs[r0 + i];
        s_offs[i] = o;
        if (i < nr) {
          const K key = dk[r0 + i];
          s_dkey[i] = key;
          s_ibase[i] = a.istart[r0 + i] - o;
          if constexpr (TK == TAG_F32) s_dtag[i] = dt[r0 + i];
          if (lineage) s_did[i] = a.dids[r0 + i];
        }
      }
    }
    __syncthreads();
    // One derivation whose index row (key ikey, tag y) is already loaded:
    // fold it into the window; with lineage, log it if it is a discovery
    // (called by whole waves: the segment claims are ballots).  A wave loads
    // the index rows of all its chunks first, so their latencies overlap.
    // A derivation marks its key when it makes it present or improves its
    // tag: it then beats the value it read, and the final value beats the
    // key's value before the launch, so the window's atomics need no result.
    auto fold = [&](bool act, uint32_t j, K dkey, K ikey, float x, float y, uint32_t irow, uint32_t lrow) {
      bool logit = false;
      K okey = 0;
      if (act) {
        // offset in the window of the prefix (sample, v[0]): the remaining
        // columns in mixed radix (n per middle column, np for the last)
        uint32_t v[4], lk = 0;
#pragma unroll
        for (int c = 1; c < 4; ++c) {
          if (c < nc) {
            v[c] = (uint32_t)((uint64_t)(from_index[c] ? ikey : dkey) >> shf[c]) & msk[c];
            lk = lk * (c + 1 < nc ? gn_ : gnp) + v[c];
          }
        }
        if (lk >= W) {  // the host only picks this kernel when every key lies in its window
          if (d.overflow) *d.overflow = 2;
        } else {
          const uint32_t loc = lk;
          const uint32_t wi = loc >> 5, bit = 1u << (loc & 31);
          bool mark = false;
          if constexpr (TK == TAG_F32) {
            const float t = a.index_first ? f_otimes(a.sr, y, x) : f_otimes(a.sr, x, y);
            if (d.mode == DENSE_ADD) {
              if (!(s_pres[wi] & bit)) {
                atomicAdd(reinterpret_cast<float*>(s_tag) + loc, t);
                mark = true;
                logit = lineage != 0;
              }
            } else {
              // an absent key holds the semiring zero: the presence bit only
              // matters for a derivation that does not beat that zero
              const uint32_t o = to_ordered(t), zero = dense_init_word_dev(d.mode);
              if (d.mode == DENSE_MAX) {
                mark = o > s_tag[loc];
                if (mark) atomicMax(s_tag + loc, o);
                else if (o <= zero) mark = !(s_pres[wi] & bit);
              } else {
                mark = o < s_tag[loc];
                if (mark) atomicMin(s_tag + loc, o);
                else if (o >= zero) mark = !(s_pres[wi] & bit);
              }
            }
          } else {
            mark = !(s_pres[wi] & bit);
          }
          if (mark) atomicOr(s_new + wi, bit);
          if (logit) {
            v[0] = key_col(dkey, 0, a.dlay);
            okey = key_make<K>(key_sample(dkey, a.dlay), v, a.olay);
          }
        }
      }
      if (lineage) {
        // discovery derivations go to the segment of their output slot
        // (DENSE_SEG slots each); a wave's lanes hold consecutive slots, so
        // they touch at most two segments, each claimed with one atomic add
        const uint32_t sj = j / DENSE_SEG;
        const uint32_t s_first = __shfl(sj, 0, WAVE);
        const uint64_t lm = ballot(logit);
        const uint64_t second = ballot(sj != s_first);
        const uint64_t m1 = lm & ~second, m2 = lm & second;
        uint32_t b1 = 0, b2 = 0;
        const int lane = lane_id();
        if (m1 && lane == __builtin_ctzll(m1))
          b1 = atomicAdd(d.seg_lcount + d.seg_base + s_first, (uint32_t)__popcll(m1));
        if (m2 && lane == __builtin_ctzll(m2))
          b2 = atomicAdd(d.seg_lcount + d.seg_base + s_first + 1, (uint32_t)__popcll(m2));
        b1 = __shfl(b1, m1 ? __builtin_ctzll(m1) : 0, WAVE);
        b2 = __shfl(b2, m2 ? __builtin_ctzll(m2) : 0, WAVE);
        if (logit) {
          const bool in2 = (second >> lane) & 1ull;
          const uint32_t p = in2 ? b2 + rank_below(m2) : b1 + rank_below(m1);
          const size_t o = (size_t)(d.seg_base + sj) * DENSE_SEG + p;
          reinterpret_cast<K*>(d.log_keys)[o] = okey;
          d.log_l[o] = lrow;
          d.log_r[o] = a.iids[irow];
        }
      }
    };
    // Specialised fold (FAST): the head's second column is the index row's
    // column at shf[1]; the product and the merge are fixed by FM.
    auto fold_fast = [&](bool act, K ikey, float x, float y) {
      if (!act) return;
      const uint32_t loc = (uint32_t)((uint64_t)ikey >> shf[1]) & msk[1];
      if (loc >= W) {  // the host only picks this kernel when every key lies in its window
        if (d.overflow) *d.overflow = 2;
        return;
      }
      const uint32_t wi = loc >> 5, bit = 1u << (loc & 31);
      const float p = a.index_first ? y : x, r = a.index_first ? x : y;  // body order of the operands
      bool mark;
      if constexpr (FM == DENSE_BOOL) {
        mark = !(s_pres[wi] & bit);
      } else if constexpr (FM == DENSE_ADD) {
        mark = !(s_pres[wi] & bit);
        if (mark) atomicAdd(reinterpret_cast<float*>(s_tag) + loc, __fmul_rn(p, r));
      } else if constexpr (FM == DENSE_MAX) {
        const uint32_t o = to_ordered(fminf(p, r));
        mark = o > s_tag[loc];
        if (mark) atomicMax(s_tag + loc, o);
        else if (o <= 0x80000000u) mark = !(s_pres[wi] & bit);  // does not beat the zero +0.0
      } else {
        const uint32_t o = to_ordered(__fadd_rn(p, r));
        mark = o < s_tag[loc];
        if (mark) atomicMin(s_tag + loc, o);
        else if (o >= (0x7f800000u | 0x80000000u)) mark = !(s_pres[wi] & bit);  // does not beat +inf
      }
      if (mark) atomicOr(s_new + wi, bit);
    };
    if (lds_rows) {
      // Chunks of 64 consecutive outputs of one driver row; every wave takes
      // a contiguous range of chunks and walks the rows along it (a wave's
      // lanes share the row: its key, tag and index base are LDS broadcasts).
      if (threadIdx.x < WAVE) {  // chunk counts of the rows, scanned by one wave
        uint32_t cnt[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t i = (uint32_t)threadIdx.x * 4 + k;
          cnt[k] = i < nr ? (s_offs[i + 1] - s_offs[i] + WAVE - 1) / WAVE : 0u;
          sum += cnt[k];
        }
        uint32_t run = wave_inclusive_scan(sum) - sum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t i = (uint32_t)threadIdx.x * 4 + k;
          if (i <= nr) s_cpre[i] = run;
          run += cnt[k];
        }
      }
      __syncthreads();
      // wave-uniform (scalar) chunk bounds: the compiler cannot see that
      // threadIdx.x / WAVE is the same on every lane
      const uint32_t nch = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_cpre[nr]);
      const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
      const uint32_t lane = (uint32_t)lane_id();
      const uint32_t per = (nch + RW_WAVES - 1) / RW_WAVES;
      uint32_t c = wv * per;
      const uint32_t ce = c + per < nch ? c + per : nch;
      // the row state is uniform per wave: read from LDS into scalars
      auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
      uint32_t lo = 0;
      if (c < ce) {  // the row of chunk c: s_cpre[lo] <= c < s_cpre[lo + 1]
        uint32_t hi = nr;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (uni(s_cpre[mid]) <= c) lo = mid;
          else hi = mid;
        }
      }
      for (; c < ce; c += RX_ITEMS) {  // uniform per wave
        bool act[RX_ITEMS];
        uint32_t jj[RX_ITEMS], irow[RX_ITEMS], lrow[RX_ITEMS];
        K dkey[RX_ITEMS], ikey[RX_ITEMS];
        float x[RX_ITEMS], y[RX_ITEMS];
#pragma unroll
        for (int q = 0; q < RX_ITEMS; ++q) {
          const uint32_t cq = c + (uint32_t)q;
          if (cq < ce)
            while (uni(s_cpre[lo + 1]) <= cq) ++lo;  // empty rows own no chunk
          const uint32_t j = uni(s_offs[lo]) + (cq - uni(s_cpre[lo])) * WAVE + lane;
          act[q] = cq < ce && j < uni(s_offs[lo + 1]);
          jj[q] = j;
          if constexpr (sizeof(K) == 8)
            dkey[q] = ((K)uni((uint32_t)(s_dkey[lo] >> 32)) << 32) | (K)uni((uint32_t)s_dkey[lo]);
          else
            dkey[q] = (K)uni((uint32_t)s_dkey[lo]);
          irow[q] = uni(s_ibase[lo]) + j;
          x[q] = 0.0f;
          if constexpr (TK == TAG_F32) x[q] = __uint_as_float(uni(__float_as_uint(s_dtag[lo])));
          lrow[q] = lineage ? uni(s_did[lo]) : 0u;
        }
#pragma unroll
        for (int q = 0; q < RX_ITEMS; ++q) {
          ikey[q] = act[q] ? ik[irow[q]] : (K)0;
          y[q] = 0.0f;
          if constexpr (TK == TAG_F32) y[q] = act[q] ? it[irow[q]] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < RX_ITEMS; ++q) {
          if constexpr (FAST) fold_fast(act[q], ikey[q], x[q], y[q]);
          else if (c + (uint32_t)q < ce) fold(act[q], jj[q], dkey[q], ikey[q], x[q], y[q], irow[q], lrow[q]);
        }
      }
    } else {
      // many driver rows: each output searches its row among the group's
      // offsets in global memory
      for (uint32_t t0 = s0; t0 < s1; t0 += TILE) {
        bool act[RX_ITEMS];
        uint32_t jj[RX_ITEMS], irow[RX_ITEMS], lrow[RX_ITEMS];
        K dkey[RX_ITEMS], ikey[RX_ITEMS];
        float x[RX_ITEMS], y[RX_ITEMS];
#pragma unroll
        for (int q = 0; q < RX_ITEMS; ++q) {
          const uint32_t j = t0 + (uint32_t)(q * RW_BLOCK) + threadIdx.x;
          act[q] = j < s1;
          uint32_t lo = 0, hi = nr;  // invariant: start(lo) <= j < start(hi)
          while (act[q] && hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (offs[r0 + mid] <= j) lo = mid;
            else hi = mid;
          }
          const uint32_t r = r0 + lo;
          jj[q] = j;
          dkey[q] = act[q] ? dk[r] : (K)0;
          irow[q] = act[q] ? a.istart[r] + (j - offs[r]) : 0u;
          x[q] = 0.0f;
          if constexpr (TK == TAG_F32) x[q] = act[q] ? dt[r] : 0.0f;
          lrow[q] = (lineage && act[q]) ? a.dids[r] : 0u;
        }
#pragma unroll
        for (int q = 0; q < RX_ITEMS; ++q) {
          ikey[q] = act[q] ? ik[irow[q]] : (K)0;
          y[q] = 0.0f;
          if constexpr (TK == TAG_F32) y[q] = act[q] ? it[irow[q]] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < RX_ITEMS; ++q) {
          if constexpr (FAST) fold_fast(act[q], ikey[q], x[q], y[q]);
          else if (t0 + (uint32_t)(q * RW_BLOCK) < s1)  // uniform across the block
            fold(act[q], jj[q], dkey[q], ikey[q], x[q], y[q], irow[q], lrow[q]);
        }
      }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < NWD; i += RW_BLOCK) {
      const uint32_t nb = s_new[i];
      if (nb) d.touched[wb + i] |= nb;
    }
    if constexpr (TK == TAG_F32) {
      // four keys per thread: one 16-byte store when any of them changed (an
      // unchanged key is rewritten with the value it had at the launch's
      // start: no other workgroup writes this window)
      uint4* dst = reinterpret_cast<uint4*>(d.dtag + kb);
      const uint4* src = reinterpret_cast<const uint4*>(s_tag);
      for (uint32_t i = threadIdx.x; i < W / 4; i += RW_BLOCK)
        if ((s_new[i >> 3] >> ((i & 7) * 4)) & 0xfu) dst[i] = src[i];
    }
    __syncthreads();  // the window's LDS is reloaded for the next group
    r0 = nr0, r1 = nr1, s0 = ns0, s1 = ns1;
  }
}

template <typename K>
void join_expand_dense(const JoinArgs& a, int tk, const uint32_t* offs, size_t total, const uint64_t* dtotal,
                       size_t max_total, const DenseArgs& d, bool lineage, hipStream_t st, const RowWindows* rw) {
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
  // algorithmic bytes of a join: every probe row read once (key + tag), every
  // derivation once (key + tag, and a lineage pair of two 4-byte ids when
  // recorded); the dense words a derivation is folded into are not counted
  const double tb = tk == TAG_F32 ? 4.0 : 0.0;
  const double per = sizeof(K) + tb + (lineage ? 8.0 : 0.0);
  const double bytes = (dtotal ? 0.0 : total * per) + a.n * (sizeof(K) + tb);
  // row windows: one launch of the row-window kernel, which reads the total
  // and falls back to scattered tiles below the threshold when the total is
  // only known on the device (with lineage the total is known on the host)
  const bool rows = rw && !a.ev.n && rw->wkeys <= (uint32_t)RW_KEYS && (!lineage || !dtotal) &&
                    (dtotal || total >= rw->from);
  if (rows && lineage) fill_u32(d.seg_lcount + d.seg_base, dense_segments(total, items), 0u, st);
  const uint64_t skip_at = ~0ull;
  // one workgroup per group (up to 16384; beyond, workgroups loop): the
  // dispatcher hands the next group to whichever CU frees a slot first, which
  // balances groups of very different sizes; with a device total, at least
  // as many workgroups as the fallback's tiles need (up to 4096)
  unsigned nrb = rows ? (unsigned)(rw->ngroups < 16384 ? rw->ngroups : 16384) : 0u;
  if (rows && dtotal) {
    const size_t rtile = (size_t)RW_BLOCK * items, need = (max_total + rtile - 1) / rtile;
    const unsigned ns = (unsigned)(need < 4096 ? need : 4096);
    nrb = nrb > ns ? nrb : ns;
  }
  // the specialised variants (see k_join_expand_rows, k_join_expand_dense)
  int fm = -1;
  if (sizeof(K) == 4 && d.nsamp <= 1 && !lineage && !a.ev.n && a.olay.ncols == 2 && a.osrc[0] >= 0 &&
      a.osrc[1] < 0) {
    if (tk == TAG_NONE && d.mode == DENSE_BOOL) fm = DENSE_BOOL;
    else if (tk == TAG_F32 && d.mode == DENSE_ADD && (a.sr == SR_ADDMULT || a.sr == SR_DIFF_ADDMULT)) fm = DENSE_ADD;
    else if (tk == TAG_F32 && d.mode == DENSE_MAX && a.sr == SR_MAXMIN) fm = DENSE_MAX;
    else if (tk == TAG_F32 && d.mode == DENSE_MIN && a.sr == SR_MINPLUS) fm = DENSE_MIN;
  }
#define DL_ROWS(TK, IT, FM) \
  k_join_expand_rows<K, TK, IT, FM><<<nrb, RW_BLOCK, 0, st>>>(a, offs, total, dtotal, d, *rw, lineage ? 1 : 0)
#define DL_SCAT(TK, IT, FM)                                                                                  \
  k_join_expand_dense<K, TK, IT, FM><<<nb, BLOCK, 0, st>>>(a, offs, total, dtotal, d, lineage ? 1 : 0, skip_at)
#define DL_DEXPAND(IT)                                                                                               \
  if (tk == TAG_F32) {                                                                                               \
    if (!rows) {                                                                                                     \
      if constexpr (sizeof(K) == 4) {                                                                                \
        if (fm == DENSE_MAX) DL_SCAT(TAG_F32, IT, DENSE_MAX);                                                        \
        else if (fm == DENSE_MIN) DL_SCAT(TAG_F32, IT, DENSE_MIN);                                                   \
        else if (fm == DENSE_ADD) DL_SCAT(TAG_F32, IT, DENSE_ADD);                                                   \
        else DL_SCAT(TAG_F32, IT, -1);                                                                               \
      } else {                                                                                                       \
        DL_SCAT(TAG_F32, IT, -1);                                                                                    \
      }                                                                                                              \
    }                                                                                                                \
    if (rows) {                                                                                                      \
      if constexpr (sizeof(K) == 4) {                                                                                \
        if (fm == DENSE_MAX) DL_ROWS(TAG_F32, IT, DENSE_MAX);                                                        \
        else if (fm == DENSE_MIN) DL_ROWS(TAG_F32, IT, DENSE_MIN);                                                   \
        else if (fm == DENSE_ADD) DL_ROWS(TAG_F32, IT, DENSE_ADD);                                                   \
        else DL_ROWS(TAG_F32, IT, -1);                                                                               \
      } else {                                                                                                       \
        DL_ROWS(TAG_F32, IT, -1);                                                                                    \
      }                                                                                                              \
    }                                                                                                                \
  } else {                                                                                                           \
    if (!rows) {                                                                                                     \
      if constexpr (sizeof(K) == 4) {                                                                                \
        if (fm == DENSE_BOOL) DL_SCAT(TAG_NONE, IT, DENSE_BOOL);                                                     \
        else DL_SCAT(TAG_NONE, IT, -1);                                                                              \
      } else {                                                                                                       \
        DL_SCAT(TAG_NONE, IT, -1);                                                                                   \
      }                                                                                                              \
    }                                                                                                                \
    if (rows) {                                                                                                      \
      if constexpr (sizeof(K) == 4) {                                                                                \
        if (fm == DENSE_BOOL) DL_ROWS(TAG_NONE, IT, DENSE_BOOL);                                                     \
        else DL_ROWS(TAG_NONE, IT, -1);                                                                              \
      } else {                                                                                                       \
        DL_ROWS(TAG_NONE, IT, -1);                                                                                   \
      }                                                                                                              \
    }                                                                                                                \
  }
  DL_PROF_BEGIN(1, st);
  switch (items) {
    case 1: DL_DEXPAND(1) break;
    case 2: DL_DEXPAND(2) break;
    case 8: DL_DEXPAND(8) break;
    default: DL_DEXPAND(4) break;
  }
#undef DL_DEXPAND
#undef DL_ROWS
#undef DL_SCAT
  DL_PROF_END(1, st, bytes);
  if (dtotal) DL_PROF_DEFER(1, per);
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
    K okey = 0;
    float t = 0.0f;
    uint32_t l = 0;
    bool act = i < a.n;
    if (act) {
      const K dkey = dk[i];
      uint32_t v[4];
      act = out_cols<K>(a, dkey, dkey, v);  // sources are driver columns only
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
constexpr int BM_ITEMS = 2;
constexpr int BM_TILE = BLOCK * BM_ITEMS;
constexpr int BM_WAVE_WORDS = WAVE * BM_ITEMS;

size_t dense_count_blocks(size_t keys) { return (bitmap_words(keys) + BM_TILE - 1) / BM_TILE; }

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

void bitmap_block_counts(const uint32_t* bits, size_t keys, uint32_t* partial, hipStream_t st) {
  const size_t words = bitmap_words(keys);
  DL_PROF_BEGIN(6, st);
  k_block_counts<<<dense_count_blocks(keys), BLOCK, 0, st>>>(bits, words, partial);
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
// base, base + 1, ... in index order: f(slot, index, aux, bit) runs with
// consecutive lanes on consecutive slots (source lane by a binary search over
// the wave's inclusive popcount scan, bit by rank select); aux is the source
// lane's `aux` value.  Called by the whole wave; returns the number of bits.
template <typename F>
__device__ __forceinline__ uint32_t wave_expand_bits(uint32_t x, uint64_t wbase, uint32_t base, uint64_t aux, F&& f) {
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
    const uint64_t ax = ((uint64_t)(uint32_t)__shfl((uint32_t)(aux >> 32), src, WAVE) << 32) |
                        (uint32_t)__shfl((uint32_t)aux, src, WAVE);
    const uint32_t bit = select_bit(word, j - before);
    if (j < total) f(base + j, ((wbase + (uint64_t)src) << 5) | bit, ax, bit);
  }
  return total;
}

// The block's first output slot.  `counts` holds the blocks' counts (from
// bitmap_block_counts) and the block sums the earlier ones itself instead of
// a separate scan launch -- or, with `prefixed`, counts already holds the
// exclusive scan (large bitmaps: the per-block sums would grow quadratically).
// The last block also writes the grand total.  Every wave of the block must
// call it (one barrier).
constexpr size_t BM_SELF_PREFIX_MAX = 2048;  // blocks up to which each block sums its own prefix
size_t dense_self_prefix_blocks() { return BM_SELF_PREFIX_MAX; }

__device__ __forceinline__ uint32_t block_first_slot(const uint32_t* __restrict__ counts, int prefixed,
                                                     uint32_t own_wave_count, uint32_t* s_tot, uint32_t* s_pre,
                                                     uint64_t* d_total, uint64_t* log = nullptr) {
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  uint32_t pre = 0;
  if (prefixed) {
    if (threadIdx.x == 0) pre = counts[blockIdx.x];
  } else {
    for (size_t i = threadIdx.x; i < blockIdx.x; i += BLOCK) pre += counts[i];
  }
  pre = wave_sum(pre);
  if (lane == 0) {
    s_tot[wv] = own_wave_count;
    s_pre[wv] = pre;
  }
  __syncthreads();
  uint32_t o = 0, all = 0;
  for (int i = 0; i < NWAVES; ++i) {
    o += s_pre[i] + (i < wv ? s_tot[i] : 0u);
    all += s_tot[i];
  }
  if (d_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    uint32_t p = 0;
    for (int i = 0; i < NWAVES; ++i) p += s_pre[i];
    *d_total = (uint64_t)p + all;
    if (log) log[1 + log[0]++] = (uint64_t)p + all;  // round log: count, then one total per round
  }
  return o;
}

DenseCsr dense_csr(uint32_t* off, uint32_t wwords, uint32_t n) {
  DenseCsr c;
  c.off = off;
  c.wwords = wwords;
  c.n = n;
  divisor(wwords, &c.m, &c.s1, &c.s2);
  return c;
}

// The block's first output slot in a single pass (no separate count
// launch): a decoupled look-back over the blocks' touched counts
// (block_lookback).  Launches alternate between two status sets (a parity
// word after them); the last block, whose look-back ends only after every
// other block has published (and so has read the parity), clears the
// previous launch's set and flips the parity.  The last block also writes
// the grand total (and the round log).
size_t lookback_state_words(size_t blocks) { return 2 * blocks + 1; }

__device__ __forceinline__ uint32_t block_first_slot_published(uint64_t* lb, size_t cap, uint32_t own_wave_count,
                                                               uint32_t* s_tot, uint64_t* sh, uint64_t* d_total,
                                                               uint64_t* log, uint64_t* err) {
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  const uint32_t par = (uint32_t)__hip_atomic_load(lb + 2 * cap, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1u;
  uint64_t* stat = lb + par * cap;
  if (lane == 0) s_tot[wv] = own_wave_count;
  __syncthreads();
  const uint32_t own = s_tot[0] + s_tot[1] + s_tot[2] + s_tot[3];
  const uint32_t base = (uint32_t)block_lookback(stat, own, sh, err);
  if (blockIdx.x == gridDim.x - 1) {  // every block has published: clear the other set, flip
    uint64_t* prev = lb + (1u - par) * cap;
    for (size_t i = threadIdx.x; i < gridDim.x; i += BLOCK)
      __hip_atomic_store(prev + i, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) {
      __hip_atomic_store(lb + 2 * cap, (uint64_t)(1u - par), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *d_total = (uint64_t)base + own;
      if (log) log[1 + log[0]++] = (uint64_t)base + own;
    }
  }
  uint32_t o = base;
  for (int i = 0; i < wv; ++i) o += s_tot[i];
  return o;
}

template <typename K>
__global__ __launch_bounds__(BLOCK) void k_dense_finalize(DenseArgs d, size_t words, const uint32_t* __restrict__ counts,
                                                          K* __restrict__ keys, float* __restrict__ rtags,
                                                          uint32_t id_base, float* __restrict__ tag_by_id,
                                                          uint64_t* __restrict__ d_total, uint64_t* __restrict__ log,
                                                          int prefixed, DenseCsr csr, uint64_t* __restrict__ lb,
                                                          size_t lb_cap) {
  __shared__ uint32_t s_tot[NWAVES], s_pre[NWAVES];
  __shared__ uint64_t s_lb[2 * NWAVES];
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  const size_t w0 = (size_t)blockIdx.x * BM_TILE + (size_t)wv * BM_WAVE_WORDS;
  uint32_t b[BM_ITEMS];  // the lane's words, loaded together
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i) {
    const size_t wi = w0 + (size_t)i * WAVE + lane;
    b[i] = wi < words ? d.touched[wi] : 0u;
    c += (uint32_t)__popc(b[i]);
  }
  c = wave_sum(c);
  uint32_t o = lb ? block_first_slot_published(lb, lb_cap, c, s_tot, s_lb, d_total, log, d.overflow)
                  : block_first_slot(counts, prefixed, c, s_tot, s_pre, d_total, log);
  if (csr.off) {
    // group starts: a word wi with wi % wwords == 0 opens first-column group
    // wi / wwords, whose first key (if any) gets the slot after every set bit
    // of the words before it
    uint32_t run = o;
#pragma unroll
    for (int i = 0; i < BM_ITEMS; ++i) {
      const uint32_t cnt = (uint32_t)__popc(b[i]);
      const uint32_t incl = wave_inclusive_scan(cnt);
      const size_t wi = w0 + (size_t)i * WAVE + lane;
      if (wi < words) {
        const uint32_t q = fast_div((uint32_t)wi, csr.m, csr.s1, csr.s2);
        if ((uint32_t)wi == q * csr.wwords) csr.off[q] = run + incl - cnt;
      }
      run += __shfl(incl, WAVE - 1, WAVE);
    }
    if (blockIdx.x == gridDim.x - 1 && lane == WAVE - 1 && wv == NWAVES - 1) csr.off[csr.n] = run;
  }
  if (c == 0) return;  // wave-uniform; no barrier follows
  // batched: the sample of the wave's first word, searched once
  const uint32_t s_hint = d.nsamp > 1 ? __shfl(lane == 0 ? dense_sample(d, (uint32_t)(w0 << 5)) : 0u, 0, WAVE) : ~0u;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i) {
    const uint32_t x = b[i];
    if (!__ballot(x != 0u)) continue;
    const size_t wb = w0 + (size_t)i * WAVE;
    if (x) {
      d.present[wb + lane] |= x;
      d.touched[wb + lane] = 0u;
    }
    // a word's 32 indexes share all columns but the last (dnp is a multiple
    // of 32): one index-to-key conversion per word, the bit adds to the key
    const uint64_t kbase = x ? (uint64_t)dense_key<K>(d, (uint32_t)((wb + lane) << 5), s_hint) : 0ull;
    o += wave_expand_bits(x, wb, o, kbase, [&](uint32_t slot, uint64_t kk, uint64_t kb, uint32_t bit) {
      keys[slot] = (K)(kb + bit);
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
void dense_finalize(const DenseArgs& d, size_t nkeys, const uint32_t* counts, K* keys, float* rtags, uint32_t id_base,
                    float* tag_by_id, uint64_t* d_total, hipStream_t st, uint64_t* log, bool prefixed,
                    const DenseCsr* csr, uint64_t* lookback) {
  const size_t words = bitmap_words(nkeys);
  const size_t nb = dense_count_blocks(nkeys);
  DL_PROF_BEGIN(6, st);
  k_dense_finalize<K><<<nb, BLOCK, 0, st>>>(d, words, counts, keys, rtags, id_base, tag_by_id, d_total, log,
                                            prefixed ? 1 : 0, csr ? *csr : DenseCsr{}, lookback, nb);
  DL_PROF_END(6, st, words * 12.0);
}

// One wave per lineage segment (segments are short): its entries go to
// their compacted position as (owner id, left id, right id), the owner found
// through the dense id of the logged head key (assigned by this round's
// dense_finalize).
template <typename K>
__global__ __launch_bounds__(BLOCK) void k_segments_lineage(DenseArgs d, const uint32_t* __restrict__ pos, size_t nseg,
                                                            uint32_t* __restrict__ owner, uint32_t* __restrict__ l,
                                                            uint32_t* __restrict__ r) {
  const K* lk = reinterpret_cast<const K*>(d.log_keys);
  const size_t w0 = (size_t)blockIdx.x * NWAVES + threadIdx.x / WAVE, ws = (size_t)gridDim.x * NWAVES;
  for (size_t s = w0; s < nseg; s += ws) {
    const uint32_t c = d.seg_lcount[s], o = pos[s];
    for (uint32_t i = (uint32_t)lane_id(); i < c; i += WAVE) {
      const size_t src = s * DENSE_SEG + i;
      owner[o + i] = d.did[dense_index(d, lk[src])];
      l[o + i] = d.log_l[src];
      r[o + i] = d.log_r[src];
    }
  }
}

template <typename K>
void segments_lineage(const DenseArgs& d, const uint32_t* pos, size_t nseg, uint32_t* owner, uint32_t* l, uint32_t* r,
                      hipStream_t st) {
  if (!nseg) return;
  const size_t blocks = (nseg + NWAVES - 1) / NWAVES;
  const unsigned g = (unsigned)(blocks < 65536 ? blocks : 65536);
  DL_PROF_BEGIN(8, st);
  k_segments_lineage<K><<<g, BLOCK, 0, st>>>(d, pos, nseg, owner, l, r);
  DL_PROF_END(8, st, nseg * 8.0);
}

size_t bitmap_words(size_t keys) { return (keys + 31) / 32; }

// Sorted keys of the present bits (one block per BM_TILE words, block
// offsets from bitmap_block_counts + scan), with their tags and ids.
template <typename K>
__global__ __launch_bounds__(BLOCK) void k_bitmap_keys(DenseArgs d, size_t words, const uint32_t* __restrict__ counts,
                                                       int prefixed, K* __restrict__ keys, float* __restrict__ tags,
                                                       uint32_t* __restrict__ ids) {
  __shared__ uint32_t s_tot[NWAVES], s_pre[NWAVES];
  __shared__ uint64_t s_lb[2 * NWAVES];
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  const size_t w0 = (size_t)blockIdx.x * BM_TILE + (size_t)wv * BM_WAVE_WORDS;
  uint32_t b[BM_ITEMS];
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i) {
    const size_t wi = w0 + (size_t)i * WAVE + lane;
    b[i] = wi < words ? d.present[wi] : 0u;
    c += (uint32_t)__popc(b[i]);
  }
  c = wave_sum(c);
  uint32_t o = block_first_slot(counts, prefixed, c, s_tot, s_pre, nullptr);
  if (c == 0) return;  // wave-uniform; no barrier follows
  const uint32_t s_hint = d.nsamp > 1 ? __shfl(lane == 0 ? dense_sample(d, (uint32_t)(w0 << 5)) : 0u, 0, WAVE) : ~0u;
#pragma unroll
  for (int i = 0; i < BM_ITEMS; ++i) {
    const uint32_t x = b[i];
    if (!__ballot(x != 0u)) continue;
    const size_t wb = w0 + (size_t)i * WAVE;
    const uint64_t kbase = x ? (uint64_t)dense_key<K>(d, (uint32_t)((wb + lane) << 5), s_hint) : 0ull;
    o += wave_expand_bits(x, wb, o, kbase, [&](uint32_t slot, uint64_t kk, uint64_t kb, uint32_t bit) {
      keys[slot] = (K)(kb + bit);
      if (tags) {
        const uint32_t v = d.dtag[kk];
        tags[slot] = d.mode == DENSE_ADD ? __uint_as_float(v) : d.mode == DENSE_BOOL ? 1.0f : from_ordered(v);
      }
      if (ids) ids[slot] = d.did[kk];
    });
  }
}

template <typename K>
void bitmap_keys(const DenseArgs& d, size_t nkeys, const uint32_t* counts, bool prefixed, K* keys, float* tags,
                 uint32_t* ids, hipStream_t st) {
  const size_t words = bitmap_words(nkeys);
  DL_PROF_BEGIN(6, st);
  k_bitmap_keys<K><<<dense_count_blocks(nkeys), BLOCK, 0, st>>>(d, words, counts, prefixed ? 1 : 0, keys, tags, ids);
  DL_PROF_END(6, st, words * 4.0);
}

// ------------------------------------------------------------ fused rounds
// One launch per round (count, join and round-end compaction together) for a
// one-plan stratum whose delta join is static-driven with the row-window
// shape -- the head key starts with the driver's (sample, first column)
// prefix g -- and joins the recent tuples on their first column.  All
// derivations of the driver rows of group g land in window g of the head,
// which therefore belongs to whichever workgroup takes g: no other workgroup
// reads or writes it during the round.  The recent relation lives in window
// layout (WindowRecent), written by the previous round, so a driver row's
// matches are read straight from its recent group; the counts and offsets a
// group needs come from those group counts (no global scan).  A group with
// many derivations for its window's size folds them in LDS over the staged
// window (as k_join_expand_rows); a sparse one folds them with global
// atomics on its window without staging it.  The workgroup then writes the
// window's new or changed tuples as the group's recent tuples for the next
// round (in key order), makes them present and adds their count to the
// workgroup's own slot of the round's counts (the host adds them up).  Every
// read of a round is of the previous round's recent tuples or of the group's
// own window (Jacobi order), and two window-layout buffers alternate.
//
// Workgroups take batches of groups (every grid-th batch): in a batch of
// RW_WAVES groups each wave sums one group's derivation count and does a
// sparse group alone, and the dense groups are then processed by the whole
// workgroup one after the other; in a batch of one group (large rounds, where
// most groups are dense) the first wave counts and the dense groups spread
// over all workgroups.

// Window of group g (first dense index, keys) of the relation of DenseArgs.
__device__ __forceinline__ uint32_t group_window(const DenseArgs& d, uint32_t g, uint32_t* W) {
  const uint32_t s = g >> d.dcbits, c0 = g & ((1u << d.dcbits) - 1u);
  uint32_t n = d.dn, np = d.dnp, base = 0;
  if (d.nsamp > 1) {
    base = d.sbase[s];
    n = d.sn[s];
    np = d.snp[s];
  }
  uint32_t w = np;
  for (int c = 2; c < d.dcols; ++c) w *= n;
  *W = w;
  return base + c0 * w;
}

// Whether group g is a (sample, id) prefix of the dense domain: the groups
// of a round cover whole powers of two of samples and ids, and only these
// have a window (a group with driver rows always has one).
__device__ __forceinline__ bool group_in_domain(const DenseArgs& d, uint32_t g) {
  const uint32_t s = g >> d.dcbits, c0 = g & ((1u << d.dcbits) - 1u);
  if (d.nsamp > 1) return s < d.nsamp && c0 < d.sn[s];
  return s == 0 && c0 < d.dn;
}

bool window_round_fits(uint32_t wkeys) { return wkeys <= (uint32_t)RW_KEYS; }

// Workgroups of a fused round: one per batch of `batch` groups (up to
// 16384; beyond, each takes every grid-th batch), so that the dispatcher
// hands batches to CUs as they free up.
unsigned window_round_grid(uint32_t ngroups, uint32_t batch) {
  return (unsigned)std::min<size_t>(16384, ((size_t)ngroups + batch - 1) / batch);
}
static_assert(WINDOW_ROUND_WIDE == (uint32_t)RW_WAVES, "the wide batch is one group per wave");

template <typename K, int TK, int RX_ITEMS, int FM>
__global__ __launch_bounds__(RW_BLOCK, 6) void k_window_round(JoinArgs a, DenseArgs d, RoundArgs ra) {
  constexpr bool FAST = FM >= 0;
  constexpr int WAVE_MARKS = RW_KEYS / RW_WAVES;  // per-wave mark words in s_tag (>= RW_KEYS / 32)
  __shared__ __align__(16) uint32_t s_tag[RW_KEYS];  // dense group: its window's tags; sparse groups: per-wave marks
  __shared__ uint32_t s_pres[RW_KEYS / 32];
  __shared__ uint32_t s_new[RW_KEYS / 32];
  __shared__ uint32_t s_offs[RW_ROWS + 1];  // per chunk row: first local output slot
  __shared__ uint32_t s_ibase[RW_ROWS];     // recent position of the row's first match minus that slot
  __shared__ K s_dkey[RW_ROWS];
  __shared__ float s_dtag[TK == TAG_F32 ? RW_ROWS : 1];
  __shared__ __align__(8) uint32_t s_cpre[RW_ROWS + 1];  // 64-output chunks before each row
  __shared__ uint32_t s_gd[RW_WAVES];  // derivations of the batch's dense groups (0: none)
  __shared__ uint32_t s_ws[RW_WAVES];
  __shared__ uint32_t s_sum[2];         // the workgroup's new/changed tuples and derivations
  // rows of each wave's group as the wave phase read them (groups of at
  // most WAVE driver rows): key, tag, recent count and recent base
  __shared__ K s_ck[RW_WAVES][WAVE];
  __shared__ float s_ct[RW_WAVES][TK == TAG_F32 ? WAVE : 1];
  __shared__ uint32_t s_cc[RW_WAVES][WAVE], s_cb[RW_WAVES][WAVE];
  static_assert(WAVE_MARKS >= RW_KEYS / 32, "a wave's marks must cover a window");
  const K* dk = (const K*)a.dkeys;
  const float* dt = (const float*)a.dtags;
  const K* ik = (const K*)ra.cur.rk;
  const float* it = ra.cur.rt;
  const uint32_t lane = (uint32_t)lane_id();
  const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
  auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
  // head columns 1..: which key holds each, at which shift (fixed per launch)
  const int nc = FAST ? 2 : a.olay.ncols;
  bool from_index[4];
  uint32_t shf[4], msk[4];
#pragma unroll
  for (int c = 1; c < (FAST ? 2 : 4); ++c) {
    const int s = c < nc ? a.osrc[c] : 0;
    from_index[c] = s < 0;
    const KeyLayout& l = s < 0 ? a.ilay : a.dlay;
    shf[c] = (uint32_t)((l.ncols - 1 - (s < 0 ? -1 - s : s)) * l.cbits);
    msk[c] = cmask(l.cbits);
  }
  // recent group of a driver row: (sample, joined column)
  const uint32_t jshift = (uint32_t)((a.dlay.ncols - 1 - a.jsrc[0]) * a.dlay.cbits), jmask = cmask(a.dlay.cbits);
  auto recent_group = [&](K dkey) -> uint32_t {
    const uint32_t y = (uint32_t)((uint64_t)dkey >> jshift) & jmask;
    return a.dlay.sbits ? (key_sample(dkey, a.dlay) << d.dcbits) | y : y;
  };
  const int mode = FAST ? FM : d.mode;
  const uint32_t zero = dense_init_word_dev(mode);
  // offset of a derivation's head key in its window (the head key's columns
  // after the first, in the window's mixed radix)
  auto head_loc = [&](K dkey, K ikey) -> uint32_t {
    if constexpr (FAST) {
      return (uint32_t)((uint64_t)ikey >> shf[1]) & msk[1];
    } else {
      const uint32_t s = key_sample(dkey, a.dlay);
      const uint32_t gn = d.nsamp > 1 ? d.sn[s] : d.dn, gnp = d.nsamp > 1 ? d.snp[s] : d.dnp;
      uint32_t loc = 0;
#pragma unroll
      for (int c = 1; c < 4; ++c)
        if (c < nc)
          loc = loc * (c + 1 < nc ? gn : gnp) + ((uint32_t)((uint64_t)(from_index[c] ? ikey : dkey) >> shf[c]) & msk[c]);
      return loc;
    }
  };
  // the derivation's tag: the product of the body tags in body order
  auto product = [&](float x, float y) -> float {
    const float p = a.index_first ? y : x, r = a.index_first ? x : y;
    if constexpr (FAST) return FM == DENSE_ADD ? __fmul_rn(p, r) : FM == DENSE_MAX ? fminf(p, r) : __fadd_rn(p, r);
    else return f_otimes(a.sr, p, r);
  };
  // One derivation folded into its window: `tw` the key's tag word and
  // `pres()` its presence (LDS in a staged window, global memory otherwise),
  // read only where the outcome depends on it (max / min: a tag that does
  // not beat the current one); true when it makes the key present or
  // improves its tag.
  auto fold_word = [&](uint32_t* tw, auto&& pres, float t) -> bool {
    if (mode == DENSE_ADD) {
      const bool p = pres();
      if (!p) atomicAdd(reinterpret_cast<float*>(tw), t);
      return !p;
    }
    const uint32_t o = to_ordered(t), cur = *tw;
    if (mode == DENSE_MAX) {
      if (o > cur) {
        atomicMax(tw, o);
        return true;
      }
      return o <= zero && !pres();  // does not beat the zero: new only if absent
    }
    if (o < cur) {
      atomicMin(tw, o);
      return true;
    }
    return o >= zero && !pres();
  };
  // A window's marked keys become group g's recent tuples of the next round
  // (in key order): emitted by one wave over words [w0, w1) of `marks`
  // (64 at a time, coalesced writes) starting at slot `base`; returns the
  // number emitted.  Tags come from the staged window (`win`) or from the
  // dense tag words; frozen sums are clamped.
  auto emit = [&](uint32_t g, uint32_t kb, const uint32_t* marks, uint32_t w0, uint32_t w1, uint32_t base,
                  bool win) -> uint32_t {
    // presence: a staged window's words are in s_pres (only this workgroup
    // writes them during the round), so they are stored, not read again
    K* nk = reinterpret_cast<K*>(ra.next.rk) + kb;
    float* nt = ra.next.rt ? ra.next.rt + kb : nullptr;
    const uint32_t c0 = g & ((1u << d.dcbits) - 1u);
    const size_t wb = kb >> 5;
    uint32_t run = base;
    for (uint32_t q0 = w0; q0 < w1; q0 += WAVE) {  // uniform
      const uint32_t wi = q0 + lane;
      const uint32_t xw = wi < w1 ? marks[wi] : 0u;
      if (xw) {
        if (win) d.present[wb + wi] = s_pres[wi] | xw;
        else d.present[wb + wi] |= xw;
      }
      run += wave_expand_bits(xw, wb + q0, run, 0ull, [&](uint32_t slot, uint64_t kk, uint64_t, uint32_t) {
        const uint32_t loc = (uint32_t)kk - kb;
        if constexpr (FAST) nk[slot] = (K)(((uint64_t)c0 << a.olay.cbits) | loc);
        else nk[slot] = dense_key<K>(d, (uint32_t)kk);
        if constexpr (TK == TAG_F32) {
          const uint32_t v = win ? s_tag[loc] : __hip_atomic_load(d.dtag + kk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          float t;
          if (mode == DENSE_ADD) {
            t = fminf(1.0f, __uint_as_float(v));  // the frozen tag: the clamped sum of the round
            if (!win) d.dtag[kk] = __float_as_uint(t);
          } else {
            t = from_ordered(v);
          }
          nt[slot] = t;
        }
      });
    }
    return run - base;
  };

  // A dense group's window into LDS by waves w0 .. w0 + nw - 1 (uniform):
  // its presence words in 256-byte pieces and (float tags) its tag words in
  // 1 KB pieces, each piece a wave's loads written straight into LDS (lane
  // l's 4 or 16 bytes at the piece's LDS base + 4 l or 16 l), so that no
  // registers hold the data and all of a wave's pieces are in flight
  // together.  A window is W-aligned, W a multiple of 32; the barrier after
  // staging waits for the loads.
  auto stage = [&](uint32_t kb, uint32_t W, uint32_t w0, uint32_t nw) {
    uint32_t l = lane;
    // made opaque here: otherwise the per-lane addresses are hoisted out of
    // the batch loop and spilled to scratch memory, for want of registers
    asm volatile("" : "+v"(l));
    const uint32_t NWD = W / 32;
    for (uint32_t c = wv - w0; c * WAVE < NWD; c += nw) {  // uniform
      const uint32_t q = c * WAVE + l;
      if (q < NWD)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(d.present + (kb >> 5) + q),
                                         (__attribute__((address_space(3))) void*)(s_pres + c * WAVE), 4, 0, 0);
    }
    if constexpr (TK == TAG_F32) {
      const uint4* src = reinterpret_cast<const uint4*>(d.dtag + kb);
      const uint32_t NQ = W / 4;
      for (uint32_t c = wv - w0; c * WAVE < NQ; c += nw) {  // uniform
        const uint32_t q = c * WAVE + l;
        if (q < NQ)
          __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + q),
                                           (__attribute__((address_space(3))) void*)(s_tag + c * WAVE * 4), 16, 0, 0);
      }
    }
  };

  if (threadIdx.x < 2) s_sum[threadIdx.x] = 0u;
  // batches of B groups, every gridDim.x-th to this workgroup (no shared
  // counter: same-address atomics from every CU serialise)
  const uint32_t B = ra.batch;  // 1 or RW_WAVES
  for (uint32_t g0 = blockIdx.x * B; g0 < ra.ngroups; g0 += gridDim.x * B) {
    __syncthreads();  // s_gd and the wave marks of the previous batch are no longer read
    if (B == 1 && wv != 0 && group_in_domain(d, g0)) {
      // one group per batch (large rounds: most groups are dense): the
      // other waves stage its window while the first wave counts (only a
      // group of the domain has one)
      uint32_t W;
      const uint32_t kb = group_window(d, g0, &W);
      stage(kb, W, 1, RW_WAVES - 1);
    }
    {
      // Wave phase: wave wv (< B) takes group g0 + wv.  It counts the group's
      // derivations; a sparse group is done by the wave alone (global
      // atomics on its window, marks in the wave's LDS words, emission), a
      // dense one is left for the whole workgroup.
      const uint32_t g = wv < B ? g0 + wv : ra.ngroups;
      uint32_t D = 0, r0 = 0, r1 = 0;
      // the lane's row (the first WAVE rows of the group): key, tag,
      // recent group count and base, kept for the folds below
      K rkey = 0;
      float rtag = 0.0f;
      uint32_t rcnt = 0, rbase = 0;
      if (g < ra.ngroups) {
        r0 = uni(ra.goff[g]);
        r1 = uni(ra.goff[g + 1]);
        if (r0 + lane < r1) {
          rkey = dk[r0 + lane];
          if constexpr (TK == TAG_F32) rtag = dt[r0 + lane];
          const uint32_t gy = recent_group(rkey);
          uint32_t wy;
          rcnt = ra.cur.rc[gy];
          rbase = group_window(d, gy, &wy);
        }
        D = rcnt;
        for (uint32_t r = r0 + WAVE + lane; r < r1; r += WAVE) D += ra.cur.rc[recent_group(dk[r])];
        D = uni(wave_sum(D));
      }
      uint32_t dense = 0;
      if (g < ra.ngroups && D == 0) {
        if (lane == 0) ra.next.rc[g] = 0u;
      } else if (g < ra.ngroups) {
        uint32_t W;
        const uint32_t kb = group_window(d, g, &W);
        if (ra.win_per_key != ~0u && (uint64_t)D * ra.win_per_key >= W) {
          dense = D;
          s_ck[wv][lane] = rkey;  // the workgroup phase takes the rows from here
          if constexpr (TK == TAG_F32) s_ct[wv][lane] = rtag;
          s_cc[wv][lane] = rcnt;
          s_cb[wv][lane] = rbase;
        } else {
          // the wave's mark words (the first wave of a one-group batch marks
          // in s_new: the other waves are staging s_tag)
          uint32_t* marks = B == 1 ? s_new : s_tag + wv * WAVE_MARKS;
          const uint32_t NWD = W / 32;
          const size_t wb = kb >> 5;
          for (uint32_t i = lane; i < NWD; i += WAVE) marks[i] = 0u;
          // One derivation folded into the group's window in global memory.
          auto fold_sparse = [&](K dkey, float x, K ikey, float y) {
            const uint32_t loc = head_loc(dkey, ikey);
            if (loc >= W) {  // the host only picks this kernel when every key lies in its window
              if (d.overflow) *d.overflow = 2;
              return;
            }
            const uint32_t wi = loc >> 5, bit = 1u << (loc & 31);
            auto pres = [&] { return (d.present[wb + wi] & bit) != 0u; };
            bool mark;
            if constexpr (TK == TAG_F32) mark = fold_word(d.dtag + kb + loc, pres, product(x, y));
            else mark = !pres();
            if (mark) atomicOr(marks + wi, bit);
          };
          // The derivations of the first WAVE rows (held by the lanes since
          // the count) spread over the lanes as one list, SPARSE_ITEMS per
          // lane at a time, whatever the rows' sizes: each lane finds its
          // derivation's row by a binary search over the rows' running
          // counts, so all loads of a step are in flight together.
          {
            const uint32_t incl = wave_inclusive_scan(rcnt);  // rcnt is 0 past the group's rows
            const uint32_t excl = incl - rcnt;
            const uint32_t D64 = uni(__shfl(incl, WAVE - 1, WAVE));
            for (uint32_t j0 = 0; j0 < D64; j0 += WAVE * SPARSE_ITEMS) {  // uniform
              uint32_t row[SPARSE_ITEMS];
              K ikey[SPARSE_ITEMS];
              float y[SPARSE_ITEMS];
#pragma unroll
              for (int q = 0; q < SPARSE_ITEMS; ++q) {
                const uint32_t j = j0 + (uint32_t)q * WAVE + lane;
                uint32_t lo = 0;  // rows whose running count is <= j
#pragma unroll
                for (uint32_t step = WAVE / 2; step >= 1; step >>= 1)
                  if (__shfl(incl, (int)(lo + step - 1), WAVE) <= j) lo += step;
                row[q] = lo;
                const uint32_t idx = __shfl(rbase, (int)(lo & (WAVE - 1)), WAVE) + j -
                                     __shfl(excl, (int)(lo & (WAVE - 1)), WAVE);
                const bool act = j < D64;
                ikey[q] = act ? ik[idx] : (K)0;
                y[q] = 0.0f;
                if constexpr (TK == TAG_F32) y[q] = act ? it[idx] : 0.0f;
              }
#pragma unroll
              for (int q = 0; q < SPARSE_ITEMS; ++q) {
                const int src = (int)(row[q] & (WAVE - 1));
                K dkey;
                if constexpr (sizeof(K) == 8)
                  dkey = ((K)__shfl((uint32_t)(rkey >> 32), src, WAVE) << 32) | (K)__shfl((uint32_t)rkey, src, WAVE);
                else
                  dkey = (K)__shfl((uint32_t)rkey, src, WAVE);
                float x = 0.0f;
                if constexpr (TK == TAG_F32) x = __shfl(rtag, src, WAVE);
                if (j0 + (uint32_t)q * WAVE + lane < D64) fold_sparse(dkey, x, ikey[q], y[q]);
              }
            }
          }
          for (uint32_t r = r0 + WAVE; r < r1; ++r) {  // rows past the first WAVE: one at a time
            const K dkey = dk[r];
            float x = 0.0f;
            if constexpr (TK == TAG_F32) x = dt[r];
            const uint32_t gy = recent_group(dkey);
            uint32_t wy;
            const uint32_t cnt = uni(ra.cur.rc[gy]);
            const uint32_t base = group_window(d, gy, &wy);
            for (uint32_t i = lane; i < cnt; i += WAVE) {
              float y = 0.0f;
              if constexpr (TK == TAG_F32) y = it[base + i];
              fold_sparse(dkey, x, ik[base + i], y);
            }
          }
          const uint32_t total = emit(g, kb, marks, 0, NWD, 0, false);
          if (lane == 0) {
            ra.next.rc[g] = total;
            atomicAdd(s_sum, total);
            atomicAdd(s_sum + 1, D);
          }
        }
      }
      if (lane == 0) s_gd[wv] = dense;
    }
    __syncthreads();
    // Workgroup phase: the batch's dense groups, one at a time, folded in
    // LDS over the staged window.
    for (uint32_t w = 0; w < (uint32_t)RW_WAVES; ++w) {
      const uint32_t D = s_gd[w];
      if (!D) continue;  // uniform
      const uint32_t g = g0 + w;
      uint32_t W;
      const uint32_t kb = group_window(d, g, &W);
      const uint32_t NWD = W / 32;
      for (uint32_t i = threadIdx.x; i < NWD; i += RW_BLOCK) s_new[i] = 0u;
      if (B != 1) stage(kb, W, 0, RW_WAVES);  // else staged during the wave phase
      const uint32_t r0 = uni(ra.goff[g]), r1 = uni(ra.goff[g + 1]);
      for (uint32_t q0 = r0; q0 < r1; q0 += RW_ROWS) {  // uniform
        const uint32_t nr = r1 - q0 < (uint32_t)RW_ROWS ? r1 - q0 : (uint32_t)RW_ROWS;
        __syncthreads();  // the window is staged; the previous chunk's rows are no longer read
        if (threadIdx.x < WAVE) {
          // the chunk's rows (4 per lane): recent group counts, their local
          // output offsets and 64-output chunk counts, scanned by one wave;
          // a group of at most WAVE rows comes from the wave phase's copy
          uint32_t cnt[4], base[4], sum = 0, csum = 0;
          const bool cached = r1 - r0 <= (uint32_t)WAVE;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t i = lane * 4 + k;
            cnt[k] = base[k] = 0;
            if (i < nr) {
              K key;
              if (cached) {
                key = s_ck[w][i];
                cnt[k] = s_cc[w][i];
                base[k] = s_cb[w][i];
                if constexpr (TK == TAG_F32) s_dtag[i] = s_ct[w][i];
              } else {
                key = dk[q0 + i];
                const uint32_t gy = recent_group(key);
                uint32_t wy;
                cnt[k] = ra.cur.rc[gy];
                base[k] = group_window(d, gy, &wy);
                if constexpr (TK == TAG_F32) s_dtag[i] = dt[q0 + i];
              }
              s_dkey[i] = key;
            }
            sum += cnt[k];
            csum += (cnt[k] + WAVE - 1) / WAVE;
          }
          uint32_t run = wave_inclusive_scan(sum) - sum, crun = wave_inclusive_scan(csum) - csum;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const uint32_t i = lane * 4 + k;
            if (i <= nr) {
              s_offs[i] = run;
              s_cpre[i] = crun;
            }
            if (i < nr) s_ibase[i] = base[k] - run;
            run += cnt[k];
            crun += (cnt[k] + WAVE - 1) / WAVE;
          }
        }
        __syncthreads();
        // every wave takes a contiguous range of 64-output chunks and walks
        // the rows along it (row state uniform per wave)
        const uint32_t nch = uni(s_cpre[nr]);
        const uint32_t per = (nch + RW_WAVES - 1) / RW_WAVES;
        uint32_t c = wv * per;
        const uint32_t ce = c + per < nch ? c + per : nch;
        uint32_t lo = 0;
        if (c < ce) {  // the row of chunk c: s_cpre[lo] <= c < s_cpre[lo + 1]
          uint32_t hi = nr;
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (uni(s_cpre[mid]) <= c) lo = mid;
            else hi = mid;
          }
        }
        // the current row's chunk and output ranges, recent base, key and
        // tag, held in scalar registers until a chunk past its end
        uint32_t r_c0 = 0, r_cend = 0, r_off = 0, r_oend = 0, r_ib = 0;
        K r_key = 0;
        float r_tag = 0.0f;
        auto load_row = [&](uint32_t l) {
          r_c0 = uni(s_cpre[l]);
          r_cend = uni(s_cpre[l + 1]);
          r_off = uni(s_offs[l]);
          r_oend = uni(s_offs[l + 1]);
          r_ib = uni(s_ibase[l]);
          if constexpr (sizeof(K) == 8)
            r_key = ((K)uni((uint32_t)(s_dkey[l] >> 32)) << 32) | (K)uni((uint32_t)s_dkey[l]);
          else
            r_key = (K)uni((uint32_t)s_dkey[l]);
          if constexpr (TK == TAG_F32) r_tag = __uint_as_float(uni(__float_as_uint(s_dtag[l])));
        };
        if (c < ce) load_row(lo);
        for (; c < ce; c += RX_ITEMS) {  // uniform per wave
          bool act[RX_ITEMS];
          uint32_t irow[RX_ITEMS];
          K dkey[RX_ITEMS], ikey[RX_ITEMS];
          float x[RX_ITEMS], y[RX_ITEMS];
#pragma unroll
          for (int q = 0; q < RX_ITEMS; ++q) {
            const uint32_t cq = c + (uint32_t)q;
            if (cq < ce && cq >= r_cend) {
              do ++lo;
              while (uni(s_cpre[lo + 1]) <= cq);  // empty rows own no chunk
              load_row(lo);
            }
            const uint32_t j = r_off + (cq - r_c0) * WAVE + lane;
            act[q] = cq < ce && j < r_oend;
            dkey[q] = r_key;
            irow[q] = r_ib + j;
            x[q] = r_tag;
          }
#pragma unroll
          for (int q = 0; q < RX_ITEMS; ++q) {
            ikey[q] = act[q] ? ik[irow[q]] : (K)0;
            y[q] = 0.0f;
            if constexpr (TK == TAG_F32) y[q] = act[q] ? it[irow[q]] : 0.0f;
          }
#pragma unroll
          for (int q = 0; q < RX_ITEMS; ++q) {
            if (!act[q]) continue;
            const uint32_t loc = head_loc(dkey[q], ikey[q]);
            if (loc >= W) {
              if (d.overflow) *d.overflow = 2;
              continue;
            }
            const uint32_t wi = loc >> 5, bit = 1u << (loc & 31);
            auto pres = [&] { return (s_pres[wi] & bit) != 0u; };
            bool mark;
            if constexpr (TK == TAG_F32 && (FM == DENSE_MAX || FM == DENSE_MIN)) {
              const uint32_t o = to_ordered(product(x[q], y[q]));
              if constexpr (FM == DENSE_MAX) mark = o > atomicMax(s_tag + loc, o) || (o <= zero && !pres());
              else mark = o < atomicMin(s_tag + loc, o) || (o >= zero && !pres());
            } else if constexpr (TK == TAG_F32) {
              mark = fold_word(s_tag + loc, pres, product(x[q], y[q]));
            } else {
              mark = !pres();
            }
            if (mark) atomicOr(s_new + wi, bit);
          }
        }
      }
      __syncthreads();
      // the window's marked keys: per-wave word counts -> slots, emission
      // by every wave over its share of the words (NWD / RW_WAVES, rounded
      // up), tags written back where changed
      const uint32_t per = (NWD + RW_WAVES - 1) / RW_WAVES;  // <= RW_KEYS / 32 / RW_WAVES <= WAVE
      const uint32_t e0 = min(wv * per, NWD), e1 = min(e0 + per, NWD);
      const uint32_t xw = e0 + lane < e1 ? s_new[e0 + lane] : 0u;
      const uint32_t cw = wave_sum((uint32_t)__popc(xw));
      if (lane == 0) s_ws[wv] = cw;
      __syncthreads();
      uint32_t before = 0, total = 0;
#pragma unroll
      for (int i = 0; i < RW_WAVES; ++i) {
        const uint32_t t = s_ws[i];
        before += (uint32_t)i < wv ? t : 0u;
        total += t;
      }
      if (e0 < e1) (void)emit(g, kb, s_new, e0, e1, before, true);
      if constexpr (TK == TAG_F32) {
        // write the window back four keys at a time where any changed (an
        // unchanged key gets the value it had: nothing else writes it);
        // frozen sums are clamped here
        uint4* dst = reinterpret_cast<uint4*>(d.dtag + kb);
        const uint4* src = reinterpret_cast<const uint4*>(s_tag);
        for (uint32_t i = threadIdx.x; i < W / 4; i += RW_BLOCK) {
          const uint32_t nb = (s_new[i >> 3] >> ((i & 7) * 4)) & 0xfu;
          if (!nb) continue;
          uint4 v = src[i];
          if (mode == DENSE_ADD) {
            if (nb & 1u) v.x = __float_as_uint(fminf(1.0f, __uint_as_float(v.x)));
            if (nb & 2u) v.y = __float_as_uint(fminf(1.0f, __uint_as_float(v.y)));
            if (nb & 4u) v.z = __float_as_uint(fminf(1.0f, __uint_as_float(v.z)));
            if (nb & 8u) v.w = __float_as_uint(fminf(1.0f, __uint_as_float(v.w)));
          }
          dst[i] = v;
        }
      }
      if (threadIdx.x == 0) {
        ra.next.rc[g] = total;
        atomicAdd(s_sum, total);
        atomicAdd(s_sum + 1, D);
      }
      __syncthreads();  // the window's LDS is reused by the next group
    }
  }
  // the workgroup's counts of the round (the host adds them up)
  __syncthreads();
  if (threadIdx.x == 0) {
    ra.part[2 * blockIdx.x] = s_sum[0];
    ra.part[2 * blockIdx.x + 1] = s_sum[1];
  }
}

template <typename K>
void window_round(const JoinArgs& a, int tk, const DenseArgs& d, const RoundArgs& ra, hipStream_t st) {
  const unsigned nb = window_round_grid(ra.ngroups, ra.batch);
  int fm = -1;
  if (sizeof(K) == 4 && d.nsamp <= 1 && a.olay.ncols == 2 && a.osrc[0] >= 0 && a.osrc[1] < 0) {
    if (tk == TAG_NONE && d.mode == DENSE_BOOL) fm = DENSE_BOOL;
    else if (tk == TAG_F32 && d.mode == DENSE_ADD && (a.sr == SR_ADDMULT || a.sr == SR_DIFF_ADDMULT)) fm = DENSE_ADD;
    else if (tk == TAG_F32 && d.mode == DENSE_MAX && a.sr == SR_MAXMIN) fm = DENSE_MAX;
    else if (tk == TAG_F32 && d.mode == DENSE_MIN && a.sr == SR_MINPLUS) fm = DENSE_MIN;
  }
  const int items = a.items >= 4 ? 4 : a.items >= 2 ? 2 : 1;
#define DL_WR(TK, IT, FM) k_window_round<K, TK, IT, FM><<<nb, RW_BLOCK, 0, st>>>(a, d, ra)
#define DL_WR_ITEMS(TK, FM)               \
  if (items == 1) DL_WR(TK, 1, FM);       \
  else if (items == 2) DL_WR(TK, 2, FM);  \
  else DL_WR(TK, 4, FM);
  DL_PROF_BEGIN(1, st);
  if (tk == TAG_F32) {
    if constexpr (sizeof(K) == 4) {
      if (fm == DENSE_MAX) { DL_WR_ITEMS(TAG_F32, DENSE_MAX) }
      else if (fm == DENSE_MIN) { DL_WR_ITEMS(TAG_F32, DENSE_MIN) }
      else if (fm == DENSE_ADD) { DL_WR_ITEMS(TAG_F32, DENSE_ADD) }
      else { DL_WR_ITEMS(TAG_F32, -1) }
    } else {
      DL_WR_ITEMS(TAG_F32, -1)
    }
  } else {
    if constexpr (sizeof(K) == 4) {
      if (fm == DENSE_BOOL) { DL_WR_ITEMS(TAG_NONE, DENSE_BOOL) }
      else { DL_WR_ITEMS(TAG_NONE, -1) }
    } else {
      DL_WR_ITEMS(TAG_NONE, -1)
    }
  }
#undef DL_WR_ITEMS
#undef DL_WR
  // algorithmic bytes: every driver row read once (key + tag), every
  // derivation once (its recent row's key + tag; counted on the device)
  const double per = sizeof(K) + (tk == TAG_F32 ? 4.0 : 0.0);
  DL_PROF_END(1, st, a.n * per);
  DL_PROF_DEFER(1, per);
}

// Totals of a batch of fused rounds: workgroup i adds up round i's
// per-workgroup (new or changed, derivations) pairs (nb of them, from
// part + 2 nb i) into out[2i] and out[2i + 1].
__global__ __launch_bounds__(BLOCK) void k_sum_parts(const uint32_t* __restrict__ part, unsigned nb,
                                                     uint64_t* __restrict__ out) {
  __shared__ uint64_t s_u[NWAVES], s_c[NWAVES];
  const uint2* p = reinterpret_cast<const uint2*>(part) + (size_t)blockIdx.x * nb;
  uint64_t u = 0, c = 0;
  for (unsigned b = threadIdx.x; b < nb; b += BLOCK) {
    const uint2 v = p[b];
    u += v.x;
    c += v.y;
  }
  u = wave_sum<uint64_t>(u);
  c = wave_sum<uint64_t>(c);
  const int wv = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    s_u[wv] = u;
    s_c[wv] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tu = 0, tc = 0;
    for (int i = 0; i < NWAVES; ++i) {
      tu += s_u[i];
      tc += s_c[i];
    }
    out[2 * blockIdx.x] = tu;
    out[2 * blockIdx.x + 1] = tc;
  }
}

void sum_parts(const uint32_t* part, unsigned nb, unsigned rounds, uint64_t* out, hipStream_t st) {
  k_sum_parts<<<rounds, BLOCK, 0, st>>>(part, nb, out);
}

// Window layout of a sorted relation: group g's rows (off[g] .. off[g+1])
// go to its window's first dense indexes; every group's count is written.
template <typename K>
__global__ void k_to_windows(const K* __restrict__ keys, const float* __restrict__ tags, size_t n,
                             const uint32_t* __restrict__ off, uint32_t ngroups, DenseArgs d, WindowRecent w) {
  GRID_STRIDE(i, (size_t)ngroups) w.rc[i] = off[i + 1] - off[i];
  const int shift = (d.dcols - 1) * d.dcbits;
  GRID_STRIDE(i, n) {
    const K k = keys[i];
    const uint32_t g = (uint32_t)((uint64_t)k >> shift);  // (sample, first column)
    uint32_t W;
    const uint32_t dst = group_window(d, g, &W) + (uint32_t)i - off[g];
    reinterpret_cast<K*>(w.rk)[dst] = k;
    if (tags) w.rt[dst] = tags[i];
  }
}

template <typename K>
void to_windows(const K* keys, const float* tags, size_t n, const uint32_t* off, uint32_t ngroups,
                const DenseArgs& d, WindowRecent w, hipStream_t st) {
  k_to_windows<K><<<grid_for(std::max<size_t>(n, ngroups)), BLOCK, 0, st>>>(keys, tags, n, off, ngroups, d, w);
}

// ------------------------------------------------- hash-set deduplication
template <typename K>
void hset_prepare(K* hkeys, uint32_t* htags, size_t slots, int mode, hipStream_t st) {
  fill_u32(reinterpret_cast<uint32_t*>(hkeys), slots * (sizeof(K) / 4), 0xffffffffu, st);
  if (htags) fill_u32(htags, slots, dense_init_word(mode), st);
}

template <typename K>
__global__ void k_hset_insert(const K* __restrict__ keys, const float* __restrict__ tags, size_t n,
                              K* __restrict__ hkeys, uint32_t* __restrict__ htags, uint32_t mask, int mode) {
  using U = std::conditional_t<sizeof(K) == 8, unsigned long long, unsigned int>;
  const K empty = (K)~(K)0;
  GRID_STRIDE(i, n) {
    const K k = keys[i];
    uint32_t h = hash_slot((uint64_t)k, mask);
    for (;; h = (h + 1) & mask) {
      K cur = hkeys[h];
      if (cur == empty) cur = (K)atomicCAS(reinterpret_cast<U*>(hkeys + h), (U)empty, (U)k);
      if (cur == empty || cur == k) break;  // claimed, or the key's slot
    }
    if (!htags) continue;
    const float t = tags[i];
    if (mode == DENSE_ADD) atomicAdd(reinterpret_cast<float*>(htags + h), t);
    else if (mode == DENSE_MAX) atomicMax(htags + h, to_ordered(t));
    else atomicMin(htags + h, to_ordered(t));
  }
}

template <typename K>
void hset_insert(const K* keys, const float* tags, size_t n, K* hkeys, uint32_t* htags, uint32_t mask, int mode,
                 hipStream_t st) {
  if (!n) return;
  DL_PROF_BEGIN(5, st);
  k_hset_insert<K><<<grid_for(n), BLOCK, 0, st>>>(keys, tags, n, hkeys, htags, mask, mode);
  DL_PROF_END(5, st, (double)n * (sizeof(K) + (htags ? 4.0 : 0.0)));
}

template <typename K>
__global__ void k_hset_flags(const K* __restrict__ hkeys, size_t slots, uint32_t* __restrict__ flags) {
  GRID_STRIDE(i, slots) flags[i] = hkeys[i] != (K)~(K)0 ? 1u : 0u;
}

template <typename K>
void hset_flags(const K* hkeys, size_t slots, uint32_t* flags, hipStream_t st) {
  k_hset_flags<K><<<grid_for(slots), BLOCK, 0, st>>>(hkeys, slots, flags);
}

template <typename K>
__global__ void k_hset_compact(const K* __restrict__ hkeys, const uint32_t* __restrict__ htags,
                               const uint32_t* __restrict__ pos, size_t slots, int mode, K* __restrict__ okeys,
                               float* __restrict__ otags) {
  GRID_STRIDE(i, slots) {
    if (pos[i + 1] == pos[i]) continue;  // empty slot
    const uint32_t o = pos[i];
    okeys[o] = hkeys[i];
    if (otags) {
      const uint32_t w = htags[i];
      otags[o] = mode == DENSE_ADD ? fminf(1.0f, __uint_as_float(w)) : from_ordered(w);
    }
  }
}

template <typename K>
void hset_compact(const K* hkeys, const uint32_t* htags, const uint32_t* pos, size_t slots, int mode, K* okeys,
                  float* otags, hipStream_t st) {
  DL_PROF_BEGIN(8, st);
  k_hset_compact<K><<<grid_for(slots), BLOCK, 0, st>>>(hkeys, htags, pos, slots, mode, okeys, otags);
  DL_PROF_END(8, st, (double)slots * (sizeof(K) + 4.0));
}

#define INST(K)                                                                                                       \
  template void join_expand_dense<K>(const JoinArgs&, int, const uint32_t*, size_t, const uint64_t*, size_t,     \
                                     const DenseArgs&, bool, hipStream_t, const RowWindows*);                                                \
  template void project_dense<K>(const JoinArgs&, int, const DenseArgs&, bool, hipStream_t);                        \
  template void dense_finalize<K>(const DenseArgs&, size_t, const uint32_t*, K*, float*, uint32_t, float*, uint64_t*,        \
                                  hipStream_t, uint64_t*, bool, const DenseCsr*, uint64_t*);                                \
  template void segments_lineage<K>(const DenseArgs&, const uint32_t*, size_t, uint32_t*, uint32_t*, uint32_t*,            \
                                    hipStream_t);                                                                          \
  template void bitmap_keys<K>(const DenseArgs&, size_t, const uint32_t*, bool, K*, float*, uint32_t*, hipStream_t); \
  template void window_round<K>(const JoinArgs&, int, const DenseArgs&, const RoundArgs&, hipStream_t);               \
  template void to_windows<K>(const K*, const float*, size_t, const uint32_t*, uint32_t, const DenseArgs&,             \
                              WindowRecent, hipStream_t);                                                              \
  template void hset_prepare<K>(K*, uint32_t*, size_t, int, hipStream_t);                                              \
  template void hset_insert<K>(const K*, const float*, size_t, K*, uint32_t*, uint32_t, int, hipStream_t);             \
  template void hset_flags<K>(const K*, size_t, uint32_t*, hipStream_t);                                                \
  template void hset_compact<K>(const K*, const uint32_t*, const uint32_t*, size_t, int, K*, float*, hipStream_t);

INST(uint32_t)
INST(uint64_t)

}  // namespace dlfix
