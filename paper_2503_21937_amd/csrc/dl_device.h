// Device-side building blocks for gfx950 (CDNA4, wave64): wave ballots,
// mbcnt ranks, wave/block scans, packed-key helpers and the provenance tag
// algebra.  Included by the .hip kernel sources only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dlfix {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;  // 4 waves per workgroup
constexpr int NWAVES = BLOCK / WAVE;

__device__ __forceinline__ int lane_id() { return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Inclusive scan across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T t = __shfl_up(v, d, WAVE);
    if (lane >= d) v += t;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
  return v;
}

// Exclusive scan over a 256-thread block; returns the block total in *total.
// `tmp` is __shared__ storage of NWAVES elements.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* tmp, T* total) {
  const int lane = lane_id();
  const int w = threadIdx.x / WAVE;
  T inc = wave_inclusive_scan(v);
  if (lane == WAVE - 1) tmp[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < NWAVES; ++i) {
    T t = tmp[i];
    if (i < w) before += t;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

// Decoupled look-back of a single-pass scan across the workgroups of a
// launch (Merrill and Garland's chained scan, with a whole block reading a
// window of predecessors at a time).  Each workgroup's status is one 64-bit
// word, flag and value together (so a relaxed load sees both): LB_AGG = the
// block's own sum is published, LB_INC = its inclusive prefix is published.
// Block b publishes LB_AGG | agg, then reads the statuses of the BLOCK
// workgroups before it (each thread one word, spinning until that word has a
// flag), adds everything from the latest LB_INC in the window on, and moves
// one window further back only when the window holds no LB_INC; finally it
// publishes LB_INC | (prefix + agg).  Block 0 publishes LB_INC at once, so a
// window that reaches it always ends the walk, and the work per block is
// bounded by how far the last published prefix lags behind -- not by b, as
// when every block sums all of its predecessors.  Waits are only on
// lower-numbered workgroups, which are dispatched earlier and publish before
// they wait, so they end; they are bounded besides (*err = 3 if a spin runs
// out, never expected).  When it returns, every block before b has published
// (an LB_INC at block j implies that all blocks up to j have).  Returns the
// exclusive prefix of block b to every thread.  Called by all threads of a
// BLOCK-thread workgroup; `sh` is __shared__ storage of 2 * NWAVES words.
constexpr uint64_t LB_AGG = 1ull << 62;
constexpr uint64_t LB_INC = 1ull << 63;
constexpr uint64_t LB_VAL = LB_AGG - 1;

__device__ __forceinline__ uint64_t block_lookback(uint64_t* stat, uint64_t agg, uint64_t* sh,
                                                   uint64_t* err) {
  const uint32_t b = blockIdx.x;
  if (b == 0) {
    if (threadIdx.x == 0) __hip_atomic_store(stat, LB_INC | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (threadIdx.x == 0) __hip_atomic_store(stat + b, LB_AGG | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int lane = lane_id(), wv = threadIdx.x / WAVE;
  uint64_t pre = 0;
  for (int64_t end = b;; end -= BLOCK) {
    const int64_t i = end - BLOCK + (int64_t)threadIdx.x;
    uint64_t v = 0;
    if (i >= 0) {
      uint32_t spins = 0;
      while (!((v = __hip_atomic_load(stat + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & (LB_AGG | LB_INC))) {
        if (++spins > (1u << 24)) {
          *err = 3;
          v = LB_INC;  // end the walk; the result is reported as failed
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    // latest inclusive prefix in the window (position in the block), -1 if none
    const uint64_t m = __ballot(i >= 0 && (v & LB_INC));
    if (lane == 0) sh[wv] = m ? (uint64_t)(wv * WAVE + 63 - __builtin_clzll(m)) + 1 : 0;
    __syncthreads();
    int64_t hi = -1;
#pragma unroll
    for (int w = 0; w < NWAVES; ++w)
      if (sh[w]) hi = (int64_t)sh[w] - 1;
    const uint64_t mine = wave_sum<uint64_t>(i >= 0 && (int64_t)threadIdx.x >= hi ? (v & LB_VAL) : 0ull);
    if (lane == 0) sh[NWAVES + wv] = mine;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NWAVES; ++w) pre += sh[NWAVES + w];
    __syncthreads();  // sh is rewritten by the next window
    if (hi >= 0) break;
  }
  if (threadIdx.x == 0) __hip_atomic_store(stat + b, LB_INC | (pre + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return pre;
}

// ---------------------------------------------------------------- tag types
// Bool: presence is the tag (nothing stored).
struct NoTag {};

// Top-k proofs, k <= 3: sets of the sample's probabilistic facts (W 64-bit
// words each, fact f at bit f % 64 of word f / 64; proof i's words at
// b[i*W .. i*W + W - 1]) with their binary32 probabilities, best first.
// W = 1 covers 64 facts per sample, W = 4 covers 256.
template <int W>
struct TopKW {
  static constexpr int WORDS = W;
  uint64_t b[3 * W];
  float p[3];
  uint32_t cnt;
};
using TopK = TopKW<1>;
using TopK4 = TopKW<4>;

// Differentiable max-min: a probability and the input fact it comes from.
struct VTag {
  float v;
  uint32_t f;
};
// x keeps the smaller value, + the larger one; equal values keep the
// smaller fact number (order independent, so atomics and any + order agree)
__device__ __forceinline__ VTag vtag_pick(VTag a, VTag b, bool larger) {
  if (a.v != b.v) return (a.v > b.v) == larger ? a : b;
  return a.f <= b.f ? a : b;
}

enum SemiringKind : int { SR_BOOL = 0, SR_MAXMIN = 1, SR_MINPLUS = 2, SR_ADDMULT = 3, SR_DIFF_ADDMULT = 4, SR_TOPK = 5, SR_DIFF_TOPK = 6, SR_DIFF_MAXMIN = 7 };

// x for binary32 semirings (`sr` is uniform across the launch).
__device__ __forceinline__ float f_otimes(int sr, float a, float b) {
  switch (sr) {
    case SR_MAXMIN: return fminf(a, b);
    case SR_MINPLUS: return __fadd_rn(a, b);
    default: return __fmul_rn(a, b);
  }
}
// + for binary32 semirings; add-mult clamps at 1.
__device__ __forceinline__ float f_oplus(int sr, float a, float b) {
  switch (sr) {
    case SR_MAXMIN: return fmaxf(a, b);
    case SR_MINPLUS: return fminf(a, b);
    default: return fminf(1.0f, __fadd_rn(a, b));
  }
}

// Probability of a proof: product of its facts' probabilities in binary32,
// ascending fact id, starting from 1 (multiplications only: no contraction).
template <int W>
__device__ __forceinline__ float proof_prob(const uint64_t* bits, const float* __restrict__ q) {
  float acc = 1.0f;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    uint64_t x = bits[w];
    while (x) {
      const int i = __builtin_ctzll(x);
      acc = __fmul_rn(acc, q[w * 64 + i]);
      x &= x - 1;
    }
  }
  return acc;
}

// Proof sets as the unsigned integers they spell: a < b.
template <int W>
__device__ __forceinline__ bool bits_less(const uint64_t* a, const uint64_t* b) {
#pragma unroll
  for (int w = W - 1; w >= 0; --w)
    if (a[w] != b[w]) return a[w] < b[w];
  return false;
}
template <int W>
__device__ __forceinline__ bool bits_equal(const uint64_t* a, const uint64_t* b) {
#pragma unroll
  for (int w = 0; w < W; ++w)
    if (a[w] != b[w]) return false;
  return true;
}

// Ranking of proofs: higher probability first, then smaller set.
template <int W>
__device__ __forceinline__ bool proof_before(float pa, const uint64_t* ba, float pb, const uint64_t* bb) {
  return pa > pb || (pa == pb && bits_less<W>(ba, bb));
}

// Offer one proof to a best-k list (kept sorted, distinct sets).
template <int W>
__device__ __forceinline__ void topk_offer(TopKW<W>& t, int k, const uint64_t* b, float p) {
  for (uint32_t i = 0; i < t.cnt; ++i)
    if (bits_equal<W>(t.b + i * W, b)) return;
  int pos = (int)t.cnt;
  while (pos > 0 && proof_before<W>(p, b, t.p[pos - 1], t.b + (pos - 1) * W)) --pos;
  if (pos >= k) return;
  int last = (int)t.cnt < k ? (int)t.cnt : k - 1;
  for (int i = last; i > pos; --i) {
#pragma unroll
    for (int w = 0; w < W; ++w) t.b[i * W + w] = t.b[(i - 1) * W + w];
    t.p[i] = t.p[i - 1];
  }
#pragma unroll
  for (int w = 0; w < W; ++w) t.b[pos * W + w] = b[w];
  t.p[pos] = p;
  if ((int)t.cnt < k) ++t.cnt;
}

template <int W>
__device__ __forceinline__ TopKW<W> topk_empty() {
  TopKW<W> t;
  t.cnt = 0;
#pragma unroll
  for (int i = 0; i < 3 * W; ++i) t.b[i] = 0;
  t.p[0] = t.p[1] = t.p[2] = 0.0f;
  return t;
}

// a x b: the k best distinct unions of one proof of a with one of b.
template <int W>
__device__ __forceinline__ TopKW<W> topk_otimes(const TopKW<W>& a, const TopKW<W>& b, int k,
                                                const float* __restrict__ q) {
  TopKW<W> t = topk_empty<W>();
  for (uint32_t i = 0; i < a.cnt; ++i)
    for (uint32_t j = 0; j < b.cnt; ++j) {
      uint64_t u[W];
#pragma unroll
      for (int w = 0; w < W; ++w) u[w] = a.b[i * W + w] | b.b[j * W + w];
      topk_offer<W>(t, k, u, proof_prob<W>(u, q));
    }
  return t;
}

// a + b: the k best distinct proofs of the two lists.
template <int W>
__device__ __forceinline__ TopKW<W> topk_oplus(const TopKW<W>& a, const TopKW<W>& b, int k) {
  TopKW<W> t = a;
  for (uint32_t j = 0; j < b.cnt; ++j) topk_offer<W>(t, k, b.b + j * W, b.p[j]);
  return t;
}

template <int W>
__device__ __forceinline__ bool topk_same(const TopKW<W>& a, const TopKW<W>& b) {
  if (a.cnt != b.cnt) return false;
  for (uint32_t i = 0; i < a.cnt; ++i)
    if (!bits_equal<W>(a.b + i * W, b.b + i * W)) return false;
  return true;
}

}  // namespace dlfix
