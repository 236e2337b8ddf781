// Device helpers shared by the relational kernels: packed-key fields, the
// join prefix of a probe row, tag types per payload kind, searches.
#pragma once
#include "dl_device.h"
#include "kernels.h"
#include "program.h"  // EvalOp codes

namespace dlfix {

#define GRID_STRIDE(i, n) \
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

static inline unsigned grid_for(size_t n, size_t per_block = BLOCK) {
  size_t b = (n + per_block - 1) / per_block;
  return (unsigned)(b < 65536 ? (b ? b : 1) : 65536);
}

// ------------------------------------------------------------ key helpers
__device__ __forceinline__ uint32_t cmask(int cbits) { return (uint32_t)((1ull << cbits) - 1); }

template <typename K>
__device__ __forceinline__ uint32_t key_col(K key, int c, const KeyLayout& l) {
  return (uint32_t)((uint64_t)key >> ((l.ncols - 1 - c) * l.cbits)) & cmask(l.cbits);
}
template <typename K>
__device__ __forceinline__ uint32_t key_sample(K key, const KeyLayout& l) {
  return l.sbits ? (uint32_t)((uint64_t)key >> (l.ncols * l.cbits)) : 0u;
}
template <typename K>
__device__ __forceinline__ K key_make(uint32_t sample, const uint32_t* cols, const KeyLayout& l) {
  uint64_t k = l.sbits ? (uint64_t)sample << (l.ncols * l.cbits) : 0ull;
  for (int c = 0; c < l.ncols; ++c) k |= (uint64_t)cols[c] << ((l.ncols - 1 - c) * l.cbits);
  return (K)k;
}

// Runs instructions [b, e) of the evaluation code on one output row (driver
// key dkey, index key ikey) with a fixed-size stack in thread-local memory;
// returns false when a division by zero voids the row.  The instruction
// stream is the same for every lane.
template <typename K>
__device__ bool eval_run(const EvalCode& c, uint32_t b, uint32_t e, K dkey, const KeyLayout& dl, K ikey,
                         const KeyLayout& il, uint32_t* out) {
  uint32_t st[EVAL_STACK];
  int sp = 0;
  for (uint32_t i = b; i < e; ++i) {
    const int op = c.op[i];
    const int32_t a = c.arg[i];
    if (op == EV_SRC) {
      st[sp++] = a >= 0 ? key_col(dkey, a, dl) : key_col(ikey, -1 - a, il);
      continue;
    }
    if (op == EV_CONST) {
      st[sp++] = (uint32_t)a;
      continue;
    }
    const uint32_t y = st[--sp], x = st[--sp];
    uint32_t r;
    switch (op) {
      case EV_ADD: r = x + y; break;
      case EV_SUB: r = x - y; break;
      case EV_MUL: r = x * y; break;
      case EV_DIV:
        if (!y) return false;
        r = x / y;
        break;
      case EV_MOD:
        if (!y) return false;
        r = x % y;
        break;
      case EV_EQ: r = x == y; break;
      case EV_NE: r = x != y; break;
      case EV_LT: r = x < y; break;
      case EV_LE: r = x <= y; break;
      case EV_GT: r = x > y; break;
      case EV_GE: r = x >= y; break;
      default: r = (x != 0u) & (y != 0u); break;  // EV_AND
    }
    st[sp++] = r;
  }
  *out = st[0];
  return true;
}

// The output row's columns v[0 .. olay.ncols) from the plain sources (osrc)
// and, with evaluation, the computed ones; false when the row is filtered
// out or a division by zero voids it.  A computed value outside the ids in
// use drops the row and reports error 4.
template <typename K>
__device__ __forceinline__ bool out_cols(const JoinArgs& a, K dkey, K ikey, uint32_t* v) {
  for (int c = 0; c < a.olay.ncols; ++c) {
    const int s = a.osrc[c];
    v[c] = s >= 0 ? key_col(dkey, s, a.dlay) : key_col(ikey, -1 - s, a.ilay);
  }
  if (!a.ev.n) return true;
  uint32_t f = 1;
  if (a.ev.fend && (!eval_run<K>(a.ev, 0, a.ev.fend, dkey, a.dlay, ikey, a.ilay, &f) || !f)) return false;
  for (int c = 0; c < a.olay.ncols; ++c) {
    if (a.ev.cbeg[c] == a.ev.cend[c]) continue;
    uint32_t x;
    if (!eval_run<K>(a.ev, a.ev.cbeg[c], a.ev.cend[c], dkey, a.dlay, ikey, a.ilay, &x)) return false;
    if (x >= (a.ev.sn ? a.ev.sn[key_sample(dkey, a.dlay)] : a.ev.dn)) {
      if (a.err) *a.err = 4;
      return false;
    }
    v[c] = x;
  }
  return true;
}

// Slot of a prefix in a hash index: the 64-bit finaliser of MurmurHash3
// (public domain: xor-shift, multiply, twice), masked.
__device__ __forceinline__ uint32_t hash_slot(uint64_t p, uint32_t mask) {
  p ^= p >> 33;
  p *= 0xff51afd7ed558ccdull;
  p ^= p >> 33;
  p *= 0xc4ceb9fe1a85ec53ull;
  p ^= p >> 33;
  return (uint32_t)p & mask;
}

// First index row and row count of join prefix p: CSR offsets, or a probe
// of the hash index (linear from the prefix's slot to its slot or an empty
// one; the table is at most half full).
__device__ __forceinline__ void index_range(const JoinArgs& a, uint64_t p, uint32_t* start, uint32_t* count) {
  if (a.hslots) {
    for (uint32_t h = hash_slot(p, a.hmask);; h = (h + 1) & a.hmask) {
      const HSlot s = a.hslots[h];
      if (s.key == p) {
        *start = s.start;
        *count = s.count;
        return;
      }
      if (s.key == HSLOT_EMPTY) {
        *start = 0;
        *count = 0;
        return;
      }
    }
  }
  *start = a.off[p];
  *count = a.off[p + 1] - *start;
}

template <typename K>
__device__ __forceinline__ uint64_t join_prefix(K dkey, const JoinArgs& a) {
  uint64_t p = a.ilay.sbits ? (uint64_t)key_sample(dkey, a.dlay) << (a.w * a.ilay.cbits) : 0ull;
  for (int j = 0; j < a.w; ++j) p |= (uint64_t)key_col(dkey, a.jsrc[j], a.dlay) << ((a.w - 1 - j) * a.ilay.cbits);
  return p;
}

template <int TK>
struct TagOf {
  using T = NoTag;
};
template <>
struct TagOf<TAG_F32> {
  using T = float;
};
template <>
struct TagOf<TAG_TOPK> {
  using T = TopK;
};
template <>
struct TagOf<TAG_VID> {
  using T = VTag;
};
template <>
struct TagOf<TAG_TOPK4> {
  using T = TopK4;
};

template <int TK>
__device__ __forceinline__ typename TagOf<TK>::T tag_otimes(const typename TagOf<TK>::T& x,
                                                           const typename TagOf<TK>::T& y, const JoinArgs& a,
                                                           uint32_t sample) {
  if constexpr (TK == TAG_F32) {
    return f_otimes(a.sr, x, y);
  } else if constexpr (TK == TAG_TOPK) {
    return topk_otimes(x, y, a.k, a.q + (size_t)sample * 64);
  } else if constexpr (TK == TAG_TOPK4) {
    return topk_otimes(x, y, a.k, a.q + (size_t)sample * 256);
  } else if constexpr (TK == TAG_VID) {
    return vtag_pick(x, y, false);
  } else {
    return NoTag{};
  }
}

__device__ __forceinline__ size_t upper_bound_u32(const uint32_t* a, size_t n, uint32_t x) {
  size_t lo = 0, hi = n;
  while (lo < hi) {
    size_t mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// upper_bound by a whole wave: first index i in [0, n] with a[i] > x (a
// sorted).  Each step the 64 lanes probe evenly spaced positions and a ballot
// narrows the range 64-fold, so a search costs ~log64(n) dependent loads
// instead of log2(n).  Must be called by all lanes; the result is uniform.
__device__ __forceinline__ size_t wave_upper_bound(const uint32_t* a, size_t n, uint32_t x) {
  const size_t lane = (size_t)lane_id();
  size_t lo = 0, hi = n;  // every a[i] with i < lo is <= x; the answer lies in [lo, hi]
  while (hi - lo > (size_t)WAVE) {
    const size_t step = (hi - lo + WAVE - 1) / WAVE;
    const size_t pos = lo + lane * step;
    const bool le = pos < hi && a[pos] <= x;
    const uint32_t cnt = (uint32_t)__popcll(ballot(le));  // le holds on a prefix of the lanes
    if (cnt == 0) return lo;
    const size_t nlo = lo + (cnt - 1) * step + 1, nhi = lo + cnt * step;
    lo = nlo;
    hi = nhi < hi ? nhi : hi;
  }
  const size_t pos = lo + lane;
  const bool le = pos < hi && a[pos] <= x;
  return lo + (size_t)__popcll(ballot(le));
}

// Owning probe row of every output slot of the tile [s0, s1) of a
// load-balanced expansion (offs = exclusive scan of the match counts, with
// sentinel offs[n] = total): every row with matches marks the slot where its
// outputs start, then an inclusive max-scan over the tile carries each row
// id over its slots (rows without matches mark nothing, so the last marked
// row at or before a slot owns it).  Result: s_row[t] for t < s1 - s0.
// Must be called by the whole BS-thread block; s_row holds BS * ITEMS,
// s_wave BS / WAVE.
template <int ITEMS, int BS = BLOCK>
__device__ __forceinline__ void tile_rows(const uint32_t* __restrict__ offs, size_t n, size_t s0, size_t s1,
                                          uint32_t* s_row, uint32_t* s_wave, size_t* s_r) {
  constexpr int TILE = BS * ITEMS;
  const int wv = threadIdx.x / WAVE;
  if (wv < 2) {  // wave 0 finds the tile's first row, wave 1 its last
    const size_t r = wave_upper_bound(offs, n + 1, (uint32_t)(wv == 0 ? s0 : s1 - 1)) - 1;
    if (lane_id() == 0) s_r[wv] = r;
  }
  for (int t = threadIdx.x; t < TILE; t += BS) s_row[t] = 0u;
  __syncthreads();
  const size_t r0 = s_r[0], r1 = s_r[1];
  if (threadIdx.x == 0) s_row[0] = (uint32_t)r0;
  for (size_t r = r0 + 1 + threadIdx.x; r <= r1; r += BS) {
    const uint32_t o = offs[r];
    if (o < s1 && offs[r + 1] > o) s_row[o - s0] = (uint32_t)r;
  }
  __syncthreads();
  // inclusive max-scan over the tile: blocked per thread, then across threads
  uint32_t v[ITEMS];
  uint32_t m = 0;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    v[i] = s_row[threadIdx.x * ITEMS + i];
    m = v[i] > m ? v[i] : m;
    v[i] = m;
  }
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  uint32_t inc = m;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    uint32_t t = __shfl_up(inc, d, WAVE);
    if (lane >= d) inc = t > inc ? t : inc;
  }
  if (lane == WAVE - 1) s_wave[w] = inc;
  uint32_t before = __shfl_up(inc, 1, WAVE);
  if (lane == 0) before = 0;
  __syncthreads();
  for (int i = 0; i < w; ++i) before = s_wave[i] > before ? s_wave[i] : before;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) s_row[threadIdx.x * ITEMS + i] = v[i] > before ? v[i] : before;
  __syncthreads();
}

}  // namespace dlfix
