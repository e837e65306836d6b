// Device-wide exclusive scan and stable LSD radix sort of (u32 key, u32 value)
// pairs for gfx950.  Both serve the compaction and the two sorts of the
// separate-sorting scheme (Sec. 3.2 "Sorting", App. B.2): a 32-bit depth sort
// of the visible Gaussians, then a stable sort of the instances by tile.
//
// Radix pass = histogram kernel + scan of the digit-major histogram + scatter
// kernel.  The scatter ranks keys stably inside a workgroup with wave64
// ballots: the 64 lanes of a wave find the lanes sharing their digit with 8
// ballots, count the ones below them, and keep a running per-digit counter
// per wave in LDS; wave offsets are then prefixed in wave order.  The ranked
// block is staged in LDS in digit order and written out in coalesced runs.
#include "fgs_internal.h"

namespace fgs {

template <int MODE>
__device__ __forceinline__ uint32_t scan_load(const uint32_t* __restrict__ in,
                                              const uint32_t* __restrict__ idx, uint32_t count,
                                              uint32_t i) {
  if (MODE == SCAN_IDENTITY) return in[i];
  if (MODE == SCAN_NONZERO) return in[i] != 0u ? 1u : 0u;
  return i < count ? in[idx[i]] : 0u;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ in,
                                                        const uint32_t* __restrict__ idx,
                                                        const uint32_t* __restrict__ d_count,
                                                        uint32_t n, uint32_t* __restrict__ partials) {
  __shared__ uint32_t lds[kBlock / kWave];
  const uint32_t count = (MODE == SCAN_GATHER) ? min(*d_count, n) : n;
  const uint32_t base = blockIdx.x * kScanTile;
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t i = base + k * kBlock + threadIdx.x;
    if (i < n) sum += scan_load<MODE>(in, idx, count, i);
  }
  const uint32_t tot = block_reduce_sum(sum, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Items are processed in 16 coalesced rounds of 256; `partials` holds the
// scanned block offsets (NULL for a single-block scan, which then also writes
// the grand total).  out may alias in (each item is read before it is written
// by the same thread).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_scan_down(const uint32_t* in, const uint32_t* __restrict__ idx,
                                                      const uint32_t* __restrict__ d_count, uint32_t n,
                                                      const uint32_t* __restrict__ partials, uint32_t* out,
                                                      uint32_t* __restrict__ d_total) {
  __shared__ uint32_t lds[kBlock / kWave];
  const uint32_t count = (MODE == SCAN_GATHER) ? min(*d_count, n) : n;
  const uint32_t base = blockIdx.x * kScanTile;
  uint32_t carry = partials ? partials[blockIdx.x] : 0u;
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t i = base + k * kBlock + threadIdx.x;
    const uint32_t v = (i < n) ? scan_load<MODE>(in, idx, count, i) : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, lds, &tot);
    if (i < n) out[i] = carry + ex;
    carry += tot;
  }
  if (partials == nullptr && d_total != nullptr && threadIdx.x == 0) *d_total = carry;
}

static inline size_t round_words(size_t w) { return (w + 63) & ~size_t(63); }

size_t scan_scratch_words(uint64_t n) {
  const uint64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb <= 1) return 0;
  return round_words(nb) + scan_scratch_words(nb);
}

template <int MODE>
static hipError_t scan_impl(const uint32_t* in, const uint32_t* idx, const uint32_t* d_count,
                            uint32_t* out, uint32_t n, uint32_t* d_total, uint32_t* scratch,
                            hipStream_t s) {
  if (n == 0) {
    if (d_total) return hipMemsetAsync(d_total, 0, sizeof(uint32_t), s);
    return hipSuccess;
  }
  const uint32_t nb = ceil_div(n, kScanTile);
  if (nb == 1) {
    k_scan_down<MODE><<<1, kBlock, 0, s>>>(in, idx, d_count, n, nullptr, out, d_total);
    return hipGetLastError();
  }
  uint32_t* partials = scratch;
  k_scan_reduce<MODE><<<nb, kBlock, 0, s>>>(in, idx, d_count, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_impl<SCAN_IDENTITY>(partials, nullptr, nullptr, partials, nb, d_total,
                               scratch + round_words(nb), s);
  if (e != hipSuccess) return e;
  k_scan_down<MODE><<<nb, kBlock, 0, s>>>(in, idx, d_count, n, partials, out, nullptr);
  return hipGetLastError();
}

hipError_t scan_u32(ScanMode mode, const uint32_t* in, const uint32_t* idx, const uint32_t* d_count,
                    uint32_t* out, uint32_t n, uint32_t* d_total, uint32_t* scratch, hipStream_t s) {
  switch (mode) {
    case SCAN_IDENTITY: return scan_impl<SCAN_IDENTITY>(in, idx, d_count, out, n, d_total, scratch, s);
    case SCAN_NONZERO: return scan_impl<SCAN_NONZERO>(in, idx, d_count, out, n, d_total, scratch, s);
    default: return scan_impl<SCAN_GATHER>(in, idx, d_count, out, n, d_total, scratch, s);
  }
}

// ----------------------------------------------------------------------------
// Radix sort
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* __restrict__ keys, uint32_t n,
                                                       const uint32_t* __restrict__ d_count, int shift,
                                                       uint32_t* __restrict__ hist, uint32_t nb) {
  __shared__ uint32_t h[kRadix];
  static_assert(kRadix == kBlock, "one digit per thread");
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t count = d_count ? min(*d_count, n) : n;
  const uint32_t base = blockIdx.x * kScanTile;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t i = base + k * kBlock + threadIdx.x;
    if (i < count) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one radix pass.  Each workgroup ranks its 4096 keys stably
// (wave ballots + per-wave digit counters), places them in LDS in
// (digit, input order) order, and then writes them out so that consecutive
// threads store consecutive addresses of each digit's run.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in,
                                                          uint32_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out, uint32_t n,
                                                          const uint32_t* __restrict__ d_count, int shift,
                                                          const uint32_t* __restrict__ hist_scan,
                                                          uint32_t nb) {
  constexpr int kWaves = kBlock / kWave;
  __shared__ uint32_t wcnt[kWaves][kRadix];
  __shared__ uint32_t gdelta[kRadix];  // global start of the digit minus its block-local start (mod 2^32)
  __shared__ uint32_t lstart[kRadix];  // block-local start of each digit
  __shared__ uint32_t s_key[kScanTile];
  __shared__ uint32_t s_val[kScanTile];
  __shared__ uint32_t scan_lds[kBlock / kWave];
  const uint32_t count = d_count ? min(*d_count, n) : n;
  const uint32_t base = blockIdx.x * kScanTile;
  if (base >= count) return;  // uniform for the whole workgroup
  const uint32_t in_block = min((uint32_t)kScanTile, count - base);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
  const uint32_t gbase = hist_scan[(size_t)threadIdx.x * nb + blockIdx.x];
  __syncthreads();

  // Wave w owns items [base + w*1024, base + (w+1)*1024), visited 64 at a time
  // in index order, so (wave, step, lane) order is the input order.
  const uint32_t wbase = base + wave * (kWave * kScanItems);
  const uint64_t lanes_below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  volatile uint32_t* my_cnt = wcnt[wave];
  uint32_t key[kScanItems], val[kScanItems], rank[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t i = wbase + k * kWave + lane;
    const bool valid = i < count;
    key[k] = valid ? keys_in[i] : 0u;
    val[k] = valid ? vals_in[i] : 0u;
    const uint32_t d = (key[k] >> shift) & (kRadix - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lanes_below);
    uint32_t before = 0;
    if (valid) before = my_cnt[d];           // every lane reads before the leader writes
    if (valid && below == 0) my_cnt[d] = before + (uint32_t)__popcll(peers);
    rank[k] = before + below;
  }
  __syncthreads();
  {
    // thread t = digit t: prefix over waves, block-local digit start, global offset
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t t = wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = run;
      run += t;
    }
    uint32_t tot;
    const uint32_t ls = block_exclusive_scan(run, scan_lds, &tot);
    lstart[threadIdx.x] = ls;
    gdelta[threadIdx.x] = gbase - ls;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t i = wbase + k * kWave + lane;
    if (i < count) {
      const uint32_t d = (key[k] >> shift) & (kRadix - 1);
      const uint32_t lp = lstart[d] + wcnt[wave][d] + rank[k];
      s_key[lp] = key[k];
      s_val[lp] = val[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t j = k * kBlock + threadIdx.x;
    if (j < in_block) {
      const uint32_t kk = s_key[j];
      const uint32_t d = (kk >> shift) & (kRadix - 1);
      const uint32_t pos = gdelta[d] + j;  // = gbase[d] + (j - lstart[d])
      keys_out[pos] = kk;
      vals_out[pos] = s_val[j];
    }
  }
}

size_t radix_scratch_words(uint64_t n) {
  const uint64_t nb = (n + kScanTile - 1) / kScanTile;
  const uint64_t hist = (uint64_t)kRadix * nb;
  return round_words(hist) + scan_scratch_words(hist);
}

hipError_t radix_sort_pairs(uint32_t* keys[2], uint32_t* vals[2], uint32_t n, const uint32_t* d_count,
                            int begin_bit, int end_bit, uint32_t* scratch, int* final_buf,
                            hipStream_t s) {
  int cur = 0;
  if (n == 0 || end_bit <= begin_bit) {
    *final_buf = 0;
    return hipSuccess;
  }
  const uint32_t nb = ceil_div(n, kScanTile);
  uint32_t* hist = scratch;
  uint32_t* scan_tmp = scratch + round_words((size_t)kRadix * nb);
  for (int shift = begin_bit; shift < end_bit; shift += kRadixBits) {
    k_radix_hist<<<nb, kBlock, 0, s>>>(keys[cur], n, d_count, shift, hist, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_u32(SCAN_IDENTITY, hist, nullptr, nullptr, hist, (uint32_t)(kRadix * nb), nullptr, scan_tmp, s);
    if (e != hipSuccess) return e;
    k_radix_scatter<<<nb, kBlock, 0, s>>>(keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1], n, d_count,
                                          shift, hist, nb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  *final_buf = cur;
  return hipSuccess;
}

}  // namespace fgs
