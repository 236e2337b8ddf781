// Data-parallel primitives for gfx950: device-wide scan (reduce, scan the
// block partials, rescan), stable LSD radix sort whose in-tile ranks come
// from 64-lane ballots (one ballot per digit bit isolates the lanes holding
// the same digit, mbcnt ranks a lane among them), stream compaction, gather.
#include "dl_device.h"
#include "kernels.h"
#include "prof.h"

namespace dlfix {

// ------------------------------------------------------------------- scan
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;

size_t scan_scratch_words(size_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 2; }

__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const uint32_t* __restrict__ in, size_t n,
                                                       uint64_t* __restrict__ partial) {
  __shared__ uint64_t tmp[NWAVES];
  const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) s += in[base + i];
  s = wave_sum(s);
  if (lane_id() == 0) tmp[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int i = 0; i < NWAVES; ++i) t += tmp[i];
    partial[blockIdx.x] = t;
  }
}

// One block scans the partials (exclusive, in place), looping with a carry.
__global__ __launch_bounds__(BLOCK) void k_scan_partials(uint64_t* __restrict__ partial, size_t nb,
                                                         uint64_t* __restrict__ d_total, uint64_t* __restrict__ acc) {
  __shared__ uint64_t tmp[NWAVES];
  uint64_t carry = 0;
  for (size_t b0 = 0; b0 < nb; b0 += BLOCK) {
    size_t i = b0 + threadIdx.x;
    uint64_t v = i < nb ? partial[i] : 0;
    uint64_t tot;
    uint64_t ex = block_exclusive_scan(v, tmp, &tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    *d_total = carry;
    if (acc) *acc += carry;
  }
}

__global__ __launch_bounds__(BLOCK) void k_scan_down(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                     size_t n, const uint64_t* __restrict__ partial,
                                                     const uint64_t* __restrict__ d_total, int sentinel) {
  __shared__ uint64_t tmp[NWAVES];
  const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  uint64_t tot;
  uint64_t run = partial[blockIdx.x] + block_exclusive_scan(s, tmp, &tot);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = (uint32_t)run;
    run += v[i];
  }
  if (sentinel && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (uint32_t)*d_total;
}

// Whole scan in one workgroup when n <= SCAN_TILE (one launch instead of three).
__global__ __launch_bounds__(BLOCK) void k_scan_small(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                      size_t n, uint64_t* __restrict__ d_total, int sentinel,
                                                      uint64_t* __restrict__ acc) {
  __shared__ uint64_t tmp[NWAVES];
  const size_t base = (size_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  uint64_t tot;
  uint64_t run = block_exclusive_scan(s, tmp, &tot);
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = (uint32_t)run;
    run += v[i];
  }
  if (threadIdx.x == 0) {
    *d_total = tot;
    if (sentinel) out[n] = (uint32_t)tot;
    if (acc) *acc += tot;
  }
}

// Down-sweep that finds its block's carry itself: the sum of the partials of
// the blocks before it (nb small), so the partials need no scan launch; the
// last block publishes the total (and the sentinel, and the accumulation).
constexpr size_t SCAN_FUSED_MAX_BLOCKS = 2048;

__global__ __launch_bounds__(BLOCK) void k_scan_down_carry(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                           size_t n, const uint64_t* __restrict__ partial,
                                                           uint64_t* __restrict__ d_total, int sentinel,
                                                           uint64_t* __restrict__ acc) {
  __shared__ uint64_t tmp[NWAVES], s_pre[NWAVES];
  uint64_t pre = 0;
  for (size_t i = threadIdx.x; i < blockIdx.x; i += BLOCK) pre += partial[i];
  pre = wave_sum(pre);
  if (lane_id() == 0) s_pre[threadIdx.x / WAVE] = pre;
  const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  uint64_t tot;
  const uint64_t ex = block_exclusive_scan(s, tmp, &tot);  // its barriers also publish s_pre
  const uint64_t carry = s_pre[0] + s_pre[1] + s_pre[2] + s_pre[3];
  uint64_t run = carry + ex;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = (uint32_t)run;
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const uint64_t total = carry + tot;
    *d_total = total;
    if (sentinel) out[n] = (uint32_t)total;
    if (acc) *acc += total;
  }
}

__global__ void k_empty_scan(uint32_t* out, uint64_t* d_total, int sentinel) {
  *d_total = 0;
  if (sentinel) out[0] = 0;
}

void scan_u32(const uint32_t* in, uint32_t* out, size_t n, uint64_t* d_total, bool sentinel, uint64_t* scratch,
              hipStream_t st, uint64_t* acc) {
  if (n == 0) {
    k_empty_scan<<<1, 1, 0, st>>>(out, d_total, sentinel ? 1 : 0);
    return;
  }
  size_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  DL_PROF_BEGIN(4, st);
  if (nb == 1) {
    k_scan_small<<<1, BLOCK, 0, st>>>(in, out, n, d_total, sentinel ? 1 : 0, acc);
    DL_PROF_END(4, st, n * 8.0);
    return;
  }
  k_scan_reduce<<<nb, BLOCK, 0, st>>>(in, n, scratch);
  if (nb <= SCAN_FUSED_MAX_BLOCKS) {  // two launches instead of three
    k_scan_down_carry<<<nb, BLOCK, 0, st>>>(in, out, n, scratch, d_total, sentinel ? 1 : 0, acc);
    DL_PROF_END(4, st, n * 8.0);
    return;
  }
  k_scan_partials<<<1, BLOCK, 0, st>>>(scratch, nb, d_total, acc);
  k_scan_down<<<nb, BLOCK, 0, st>>>(in, out, n, scratch, d_total, sentinel ? 1 : 0);
  DL_PROF_END(4, st, n * 8.0);
}

// ------------------------------------------------------------- radix sort
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SORT_ITEMS = 8;  // per thread; a wave owns WAVE*SORT_ITEMS consecutive keys
constexpr int SORT_TILE = BLOCK * SORT_ITEMS;

size_t radix_scratch_words(size_t n) {
  size_t nb = (n + SORT_TILE - 1) / SORT_TILE;
  size_t hist = (size_t)RADIX * nb;
  return (hist + 1) / 2 + 2 + scan_scratch_words(hist) + 2;  // hist (u32) + total + scan partials
}

template <typename K>
__global__ __launch_bounds__(BLOCK) void k_radix_hist(const K* __restrict__ keys, size_t n, int shift,
                                                      uint32_t* __restrict__ hist, uint32_t nb) {
  __shared__ uint32_t h[NWAVES][RADIX];
  for (int i = threadIdx.x; i < NWAVES * RADIX; i += BLOCK) (&h[0][0])[i] = 0;
  __syncthreads();
  const int w = threadIdx.x / WAVE;
  const size_t base = (size_t)blockIdx.x * SORT_TILE;
#pragma unroll
  for (int i = 0; i < SORT_ITEMS; ++i) {
    size_t idx = base + (size_t)i * BLOCK + threadIdx.x;
    if (idx < n) atomicAdd(&h[w][(uint32_t)(keys[idx] >> shift) & (RADIX - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < RADIX; d += BLOCK) {
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < NWAVES; ++j) c += h[j][d];
    hist[(size_t)d * nb + blockIdx.x] = c;
  }
}

template <typename K, bool VALS>
__global__ __launch_bounds__(BLOCK) void k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                         K* __restrict__ kout, uint32_t* __restrict__ vout, size_t n,
                                                         int shift, int nbits, const uint32_t* __restrict__ offs,
                                                         uint32_t nb) {
  __shared__ uint32_t wcnt[NWAVES][RADIX];
  __shared__ uint32_t dstart[RADIX];
  __shared__ uint32_t gbase[RADIX];
  __shared__ uint32_t tmp[NWAVES];
  __shared__ K skeys[SORT_TILE];
  __shared__ uint32_t svals[VALS ? SORT_TILE : 1];
  for (int i = threadIdx.x; i < NWAVES * RADIX; i += BLOCK) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  const int w = threadIdx.x / WAVE;
  const int lane = lane_id();
  const size_t tile0 = (size_t)blockIdx.x * SORT_TILE;
  const size_t wbase = tile0 + (size_t)w * WAVE * SORT_ITEMS;
  K key[SORT_ITEMS];
  uint32_t val[SORT_ITEMS];
  uint32_t rank[SORT_ITEMS];
#pragma unroll
  for (int i = 0; i < SORT_ITEMS; ++i) {
    size_t idx = wbase + (size_t)i * WAVE + lane;
    bool valid = idx < n;
    key[i] = valid ? kin[idx] : (K)0;
    if (VALS) val[i] = valid ? vin[idx] : 0u;
    uint32_t d = (uint32_t)(key[i] >> shift) & (RADIX - 1);
    uint64_t m = ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      bool bit = (d >> b) & 1u;
      uint64_t bb = ballot(bit);
      m &= bit ? bb : ~bb;
    }
    // all lanes of this row with digit d: m; earlier rows are already counted
    uint32_t before = wcnt[w][d];
    uint32_t r = rank_below(m);
    rank[i] = before + r;
    if (valid && r == 0) wcnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  // per digit: prefix over the waves (in tile order) and the tile total
  uint32_t total = 0;
  {
    const int d = threadIdx.x;  // BLOCK == RADIX
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < NWAVES; ++j) {
      uint32_t t = wcnt[j][d];
      wcnt[j][d] = s;
      s += t;
    }
    uint32_t all;
    uint32_t ex = block_exclusive_scan(s, tmp, &all);
    dstart[d] = ex;
    gbase[d] = offs[(size_t)d * nb + blockIdx.x];
    total = all;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SORT_ITEMS; ++i) {
    size_t idx = wbase + (size_t)i * WAVE + lane;
    if (idx < n) {
      uint32_t d = (uint32_t)(key[i] >> shift) & (RADIX - 1);
      uint32_t p = dstart[d] + wcnt[w][d] + rank[i];
      skeys[p] = key[i];
      if (VALS) svals[p] = val[i];
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < total; i += BLOCK) {
    K kk = skeys[i];
    uint32_t d = (uint32_t)(kk >> shift) & (RADIX - 1);
    uint32_t o = gbase[d] + (i - dstart[d]);
    kout[o] = kk;
    if (VALS) vout[o] = svals[i];
  }
}

template <typename K>
void radix_sort(K** keys, uint32_t** vals, K** keys_alt, uint32_t** vals_alt, size_t n, int key_bits,
                uint64_t* scratch, hipStream_t st) {
  if (n <= 1 || key_bits <= 0) return;
  static_assert(BLOCK == RADIX, "one digit per thread in the scatter prefix step");
  const uint32_t nb = (uint32_t)((n + SORT_TILE - 1) / SORT_TILE);
  const size_t hn = (size_t)RADIX * nb;
  uint32_t* hist = reinterpret_cast<uint32_t*>(scratch);
  uint64_t* total = scratch + (hn + 1) / 2;
  uint64_t* sc = total + 2;
  const bool v = vals && *vals;
  for (int shift = 0; shift < key_bits; shift += RADIX_BITS) {
    int nbits = key_bits - shift < RADIX_BITS ? key_bits - shift : RADIX_BITS;
    DL_PROF_BEGIN(2, st);
    k_radix_hist<K><<<nb, BLOCK, 0, st>>>(*keys, n, shift, hist, nb);
    DL_PROF_END(2, st, (double)n * sizeof(K));
    scan_u32(hist, hist, hn, total, false, sc, st);
    DL_PROF_BEGIN(3, st);
    if (v)
      k_radix_scatter<K, true><<<nb, BLOCK, 0, st>>>(*keys, *vals, *keys_alt, *vals_alt, n, shift, nbits, hist, nb);
    else
      k_radix_scatter<K, false><<<nb, BLOCK, 0, st>>>(*keys, nullptr, *keys_alt, nullptr, n, shift, nbits, hist, nb);
    DL_PROF_END(3, st, 2.0 * n * (sizeof(K) + (v ? 4 : 0)));
    K* t = *keys;
    *keys = *keys_alt;
    *keys_alt = t;
    if (v) {
      uint32_t* tv = *vals;
      *vals = *vals_alt;
      *vals_alt = tv;
    }
  }
}

template void radix_sort<uint32_t>(uint32_t**, uint32_t**, uint32_t**, uint32_t**, size_t, int, uint64_t*, hipStream_t);
template void radix_sort<uint64_t>(uint64_t**, uint32_t**, uint64_t**, uint32_t**, size_t, int, uint64_t*, hipStream_t);

// ------------------------------------------------------------------ misc
__global__ void k_iota(uint32_t* out, size_t n, uint32_t start) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = start + (uint32_t)i;
}
__global__ void k_fill32(uint32_t* out, size_t n, uint32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = v;
}

static unsigned grid_for(size_t n) {
  size_t b = (n + BLOCK - 1) / BLOCK;
  return (unsigned)(b < 65536 ? (b ? b : 1) : 65536);
}

void iota_u32(uint32_t* out, size_t n, uint32_t start, hipStream_t st) {
  if (n) k_iota<<<grid_for(n), BLOCK, 0, st>>>(out, n, start);
}
void fill_u32(uint32_t* out, size_t n, uint32_t v, hipStream_t st) {
  if (n) k_fill32<<<grid_for(n), BLOCK, 0, st>>>(out, n, v);
}
void fill_f32(float* out, size_t n, float v, hipStream_t st) {
  uint32_t u;
  __builtin_memcpy(&u, &v, 4);
  fill_u32(reinterpret_cast<uint32_t*>(out), n, u, st);
}

template <typename T>
__global__ void k_gather(const T* __restrict__ in, const uint32_t* __restrict__ idx, T* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = in[idx[i]];
}

void gather(const void* in, const uint32_t* idx, void* out, size_t n, size_t bytes, hipStream_t st) {
  if (!n) return;
  if (bytes == 4)
    k_gather<uint32_t><<<grid_for(n), BLOCK, 0, st>>>((const uint32_t*)in, idx, (uint32_t*)out, n);
  else if (bytes == 8)
    k_gather<uint64_t><<<grid_for(n), BLOCK, 0, st>>>((const uint64_t*)in, idx, (uint64_t*)out, n);
  else if (bytes == sizeof(TopK))
    k_gather<TopK><<<grid_for(n), BLOCK, 0, st>>>((const TopK*)in, idx, (TopK*)out, n);
  else
    k_gather<TopK4><<<grid_for(n), BLOCK, 0, st>>>((const TopK4*)in, idx, (TopK4*)out, n);
}

__global__ void k_max(const uint32_t* __restrict__ in, size_t n, uint32_t* out) {
  uint32_t m = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    m = in[i] > m ? in[i] : m;
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    uint32_t t = __shfl_xor(m, d, WAVE);
    m = t > m ? t : m;
  }
  if (lane_id() == 0) atomicMax(out, m);
}

struct Cols4 {
  const uint32_t* c[4];
};

// Facts usually come grouped by sample: a wave whose active lanes share one
// sample reduces first and issues a single atomic.
__global__ void k_sample_max(Cols4 cols, int ncols, const uint32_t* __restrict__ sample, size_t n,
                             uint32_t* __restrict__ smax) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t n_pad = (n + WAVE - 1) / WAVE * WAVE;  // whole waves stay in the loop together
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n_pad; i += stride) {
    const bool act = i < n;
    uint32_t m = 0, s = 0;
    if (act) {
      for (int c = 0; c < ncols; ++c) m = cols.c[c][i] > m ? cols.c[c][i] : m;
      s = sample[i];
    }
    const uint64_t live = ballot(act);
    const int first = live ? __builtin_ctzll(live) : 0;
    const uint32_t s0 = __shfl(s, first, WAVE);
    if (ballot(act && s != s0) == 0ull) {  // one sample in the wave
      uint32_t w = m;
#pragma unroll
      for (int d = WAVE / 2; d > 0; d >>= 1) {
        const uint32_t o = __shfl_xor(w, d, WAVE);
        w = o > w ? o : w;
      }
      if (live && lane_id() == first) atomicMax(smax + s0, w);
    } else if (act) {
      atomicMax(smax + s, m);
    }
  }
}

void sample_max_u32(const uint32_t* const* cols, int ncols, const uint32_t* sample, size_t n, uint32_t* smax,
                    hipStream_t st) {
  if (!n) return;
  Cols4 c{{nullptr, nullptr, nullptr, nullptr}};
  for (int i = 0; i < ncols && i < 4; ++i) c.c[i] = cols[i];
  k_sample_max<<<grid_for(n) < 2048 ? grid_for(n) : 2048, BLOCK, 0, st>>>(c, ncols, sample, n, smax);
}

void max_u32(const uint32_t* in, size_t n, uint32_t* d_out, hipStream_t st) {
  if (n) k_max<<<grid_for(n) < 2048 ? grid_for(n) : 2048, BLOCK, 0, st>>>(in, n, d_out);
}

template <typename T>
__global__ void k_compact(const T* __restrict__ in, const uint32_t* __restrict__ flags,
                          const uint32_t* __restrict__ pos, size_t n, T* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (flags[i]) out[pos[i]] = in[i];
}

void compact(const void* in, const uint32_t* flags, const uint32_t* pos, size_t n, size_t bytes, void* out,
             hipStream_t st) {
  if (!n) return;
  if (bytes == 4)
    k_compact<uint32_t><<<grid_for(n), BLOCK, 0, st>>>((const uint32_t*)in, flags, pos, n, (uint32_t*)out);
  else if (bytes == 8)
    k_compact<uint64_t><<<grid_for(n), BLOCK, 0, st>>>((const uint64_t*)in, flags, pos, n, (uint64_t*)out);
  else if (bytes == sizeof(TopK))
    k_compact<TopK><<<grid_for(n), BLOCK, 0, st>>>((const TopK*)in, flags, pos, n, (TopK*)out);
  else
    k_compact<TopK4><<<grid_for(n), BLOCK, 0, st>>>((const TopK4*)in, flags, pos, n, (TopK4*)out);
}

__global__ void k_status_flags(const uint32_t* __restrict__ status, size_t n, uint32_t mask,
                               uint32_t* __restrict__ flags) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    flags[i] = (status[i] & mask) ? 1u : 0u;
}

void status_flags(const uint32_t* status, size_t n, uint32_t mask, uint32_t* flags, hipStream_t st) {
  if (n) k_status_flags<<<grid_for(n), BLOCK, 0, st>>>(status, n, mask, flags);
}

__global__ void k_range_flags(const uint32_t* __restrict__ ids, size_t n, uint32_t lo, uint32_t hi,
                              uint32_t* __restrict__ flags) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t v = ids[i];
    flags[i] = (v >= lo && v < hi) ? 1u : 0u;
  }
}

void range_flags(const uint32_t* ids, size_t n, uint32_t lo, uint32_t hi, uint32_t* flags, hipStream_t st) {
  if (n) k_range_flags<<<grid_for(n), BLOCK, 0, st>>>(ids, n, lo, hi, flags);
}

}  // namespace dlfix
