// Device-wide exclusive scan and stable LSD radix sort of (u32 or u16 key,
// u32 value) pairs for gfx950.  Both serve the compaction and the two sorts of the
// separate-sorting scheme (Sec. 3.2 "Sorting", App. B.2): a 32-bit depth sort
// of the visible Gaussians, then a stable sort of the instances by tile.
//
// Radix pass = histogram kernel + scan of the digit-major histogram + scatter
// kernel.  The scatter ranks keys stably inside a workgroup with wave64
// ballots: the 64 lanes of a wave find the lanes sharing their digit with 8
// ballots, count the ones below them, and keep a running per-digit counter
// per wave in LDS; wave offsets are then prefixed in wave order.  The ranked
// block is staged in LDS in digit order and written out in coalesced runs.
#include <algorithm>

#include "fgs_internal.h"

namespace fgs {

// Fill of n 32-bit words with a value: used instead of hipMemsetAsync so that
// a captured graph holds only kernel nodes.  16-byte stores where aligned.
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, uint64_t n,
                                                    uint32_t* __restrict__ word, uint32_t word_v) {
  if (word != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *word = word_v;
  const uint64_t i4 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) * 4;
  if (i4 + 4 <= n && ((uintptr_t)p & 15u) == 0) {
    *reinterpret_cast<uint4*>(p + i4) = make_uint4(v, v, v, v);
  } else {
    for (uint64_t i = i4; i < i4 + 4 && i < n; ++i) p[i] = v;
  }
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s, uint32_t* word, uint32_t word_v) {
  if (n == 0 && word == nullptr) return hipSuccess;
  const uint64_t threads = std::max<uint64_t>((n + 3) / 4, 1);
  k_fill_u32<<<(uint32_t)((threads + kBlock - 1) / kBlock), kBlock, 0, s>>>(p, v, n, word, word_v);
  return hipGetLastError();
}

// p[0..n) = 0 unless the pair flag[0..2) reads {kAccumClean, tag}: every
// block checks the pair first, so a known-zero region costs one launch of a
// few blocks.  A fixed grid of at most kClearBlocks blocks strides over the
// region, 16 bytes per thread and step (p is 256-byte aligned).
constexpr uint32_t kClearBlocks = 2048;
__global__ __launch_bounds__(kBlock) void k_clear_unless(uint32_t* __restrict__ p, uint64_t n,
                                                         const uint32_t* __restrict__ flag, uint32_t tag) {
  if (flag[0] == kAccumClean && flag[1] == tag) return;  // uniform
  const uint64_t n4 = n / 4, stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride)
    reinterpret_cast<uint4*>(p)[i] = make_uint4(0u, 0u, 0u, 0u);
  for (uint64_t i = n4 * 4 + (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

hipError_t launch_clear_unless(uint32_t* p, uint64_t n, const uint32_t* flag, uint32_t tag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if ((uintptr_t)p % 16) return hipErrorInvalidValue;
  const uint64_t want = (n / 4 + kBlock - 1) / kBlock;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, kClearBlocks));
  k_clear_unless<<<grid, kBlock, 0, s>>>(p, n, flag, tag);
  return hipGetLastError();
}

// Flat exclusive scan: a thread owns 4 consecutive items (one 16-byte access),
// so a workgroup covers kFlatTile items with a single workgroup scan.  Up to
// kFlatDirect blocks, each block of the down-sweep adds up the partial sums
// of the blocks before it itself (no scan of the partials in between).
constexpr uint32_t kFlatItems = 4;
constexpr uint32_t kFlatTile = kBlock * kFlatItems;
constexpr uint32_t kFlatDirect = 2048;

__device__ __forceinline__ uint4 flat_load(const uint32_t* in, uint32_t i, uint32_t n) {
  if (i + kFlatItems <= n) return *reinterpret_cast<const uint4*>(in + i);
  uint4 v = make_uint4(0u, 0u, 0u, 0u);
  if (i < n) v.x = in[i];
  if (i + 1 < n) v.y = in[i + 1];
  if (i + 2 < n) v.z = in[i + 2];
  return v;
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ in, uint32_t n,
                                                        uint32_t* __restrict__ partials) {
  __shared__ uint32_t lds[kBlock / kWave];
  const uint4 v = flat_load(in, (blockIdx.x * kBlock + threadIdx.x) * kFlatItems, n);
  const uint32_t tot = block_reduce_sum(v.x + v.y + v.z + v.w, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// partials: NULL for a single block; else the blocks' sums (direct) or their
// scanned offsets.  The block holding the last item writes the grand total to
// d_total when it is given.  out may alias in (a thread reads its items before
// writing them, and no other thread reads them).
__global__ __launch_bounds__(kBlock) void k_scan_down(const uint32_t* in, uint32_t n,
                                                      const uint32_t* __restrict__ partials, int direct,
                                                      uint32_t* out, uint32_t* __restrict__ d_total) {
  __shared__ uint32_t lds[kBlock / kWave];
  uint32_t carry = 0;
  if (partials != nullptr && direct) {
    uint32_t part = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kBlock) part += partials[b];
    carry = block_reduce_sum(part, lds);
  } else if (partials != nullptr) {
    carry = partials[blockIdx.x];
  }
  const uint32_t i = (blockIdx.x * kBlock + threadIdx.x) * kFlatItems;
  const uint4 v = flat_load(in, i, n);
  const uint32_t s0 = v.x, s1 = s0 + v.y, s2 = s1 + v.z, s3 = s2 + v.w;
  uint32_t tot;
  const uint32_t base = carry + block_exclusive_scan(s3, lds, &tot);
  const uint4 r = make_uint4(base, base + s0, base + s1, base + s2);
  if (i + kFlatItems <= n) {
    *reinterpret_cast<uint4*>(out + i) = r;
  } else {
    if (i < n) out[i] = r.x;
    if (i + 1 < n) out[i + 1] = r.y;
    if (i + 2 < n) out[i + 2] = r.z;
  }
  if (d_total != nullptr && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *d_total = carry + tot;
}

static inline size_t round_words(size_t w) { return (w + 63) & ~size_t(63); }

size_t scan_scratch_words(uint64_t n) {
  const uint64_t nb = (n + kFlatTile - 1) / kFlatTile;
  if (nb <= 1) return 0;
  return round_words(nb) + (nb > kFlatDirect ? scan_scratch_words(nb) : 0);
}

hipError_t scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* d_total, uint32_t* scratch,
                    hipStream_t s) {
  if (n == 0) {
    if (d_total) return launch_fill_u32(d_total, 0u, 1, s);
    return hipSuccess;
  }
  if (((uintptr_t)in | (uintptr_t)out | (uintptr_t)scratch) % 16) return hipErrorInvalidValue;
  const uint32_t nb = ceil_div(n, kFlatTile);
  if (nb == 1) {
    k_scan_down<<<1, kBlock, 0, s>>>(in, n, nullptr, 0, out, d_total);
    return hipGetLastError();
  }
  uint32_t* partials = scratch;
  k_scan_reduce<<<nb, kBlock, 0, s>>>(in, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nb <= kFlatDirect) {
    k_scan_down<<<nb, kBlock, 0, s>>>(in, n, partials, 1, out, d_total);
    return hipGetLastError();
  }
  e = scan_u32(partials, partials, nb, d_total, scratch + round_words(nb), s);
  if (e != hipSuccess) return e;
  k_scan_down<<<nb, kBlock, 0, s>>>(in, n, partials, 0, out, nullptr);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Radix sort
//
// A pass over RB <= 8 key bits is three launches:
//   hist     per-block digit counts, digit-major: hist[d * nb + b]
//   colscan  one workgroup per digit: exclusive prefix of hist[d][*] over the
//            blocks, in place, and the digit total
//   scatter  digit starts from the 2^RB totals (scanned in LDS), then the
//            stable block-local ranking and the coalesced write-out
// The bits of a sort are split evenly over ceil(bits / 8) passes, so a 13-bit
// tile key takes 7 + 6 bits: fewer, longer runs per digit in each block.
// Keys are 32-bit, or 16-bit for tile ids that fit (half the key traffic);
// values are 32-bit.  A block sorts kBlock * ITEMS pairs.
// ----------------------------------------------------------------------------
// With d_range = {min, max} of all keys given, a pass whose digit and every
// bit above it are the same in both (so in every key) keeps the order: its
// histogram and scan do nothing and its scatter is a copy.
__device__ __forceinline__ bool pass_is_constant(const uint32_t* __restrict__ d_range, int shift) {
  return d_range != nullptr && ((d_range[0] ^ d_range[1]) >> shift) == 0u;
}

// The chunk of the pairs that workgroup blockIdx.x of a pass takes: the
// workgroups below the number of chunks holding pairs share those chunks out
// in one contiguous band per XCD (xcd_tile); the others, past the count, keep
// their own index (the histogram zeroes those columns, the scatter does
// nothing for them).
__device__ __forceinline__ uint32_t radix_chunk(uint32_t count, uint32_t tile) {
  const uint32_t used = (uint32_t)(((uint64_t)count + tile - 1) / tile);
  return blockIdx.x < used ? xcd_tile(blockIdx.x, used) : blockIdx.x;
}

// fourth word of a raw buffer descriptor on gfx9-family GPUs (32-bit data format)
constexpr int kBufferWord3 = 0x00020000;

template <typename KT>
struct alignas(16) KeyVec {  // one 16-byte load of consecutive keys
  static constexpr int V = 16 / (int)sizeof(KT);
  KT k[V];
};

template <int RB, typename KT, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_radix_hist(const KT* __restrict__ keys, uint32_t n,
                                                       const uint32_t* __restrict__ d_count, int shift,
                                                       const uint32_t* __restrict__ d_range,
                                                       uint32_t* __restrict__ hist, uint32_t nb,
                                                       uint32_t* __restrict__ final_word, uint32_t final_if_run) {
  constexpr int R = 1 << RB;
  constexpr int kWaves = kBlock / kWave;
  constexpr int V = KeyVec<KT>::V;
  static_assert(ITEMS % V == 0, "whole 16-byte loads per thread");
  if (pass_is_constant(d_range, shift)) return;
  // a pass that runs notes the buffer its scatter writes: the last one to run
  // leaves the buffer holding the result
  if (final_word != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *final_word = final_if_run;
  const uint32_t count = d_count ? min(*d_count, n) : n;
  const uint32_t used = (uint32_t)(((uint64_t)count + kBlock * ITEMS - 1) / (kBlock * ITEMS));
  if (blockIdx.x >= used) {
    // the chunks past the count (a grid sized by a capacity) have zero
    // columns: these workgroups zero the entries (d, used .. nb) together,
    // row by row, so that consecutive threads write consecutive words
    const uint32_t m = nb - used;
    const uint64_t idx = (uint64_t)(blockIdx.x - used) * kBlock + threadIdx.x;
    if (idx < (uint64_t)R * m) hist[(size_t)(idx / m) * nb + used + (uint32_t)(idx % m)] = 0u;
    return;  // uniform for the whole workgroup
  }
  // kSplit histograms per wave (lane l adds to histogram l mod kSplit), so
  // that fewer lanes of one instruction add to the same counter.  With few
  // digits the collisions cost most and the extra counters least (measured at
  // 3M: 2 for 128 digits, 4 for 64; 256 digits gain nothing).
  constexpr int kSplit = R >= 256 ? 1 : (R >= 128 ? 2 : 4);
  constexpr int kSub = kWaves * kSplit;
  __shared__ uint32_t h[kSub][R];
  for (int i = threadIdx.x; i < kSub * R; i += kBlock) (&h[0][0])[i] = 0;
  __syncthreads();
  const uint32_t blk = radix_chunk(count, (uint32_t)(kBlock * ITEMS));  // see k_radix_scatter
  const uint32_t base = blk * (uint32_t)(kBlock * ITEMS);
  uint32_t* hw = h[(threadIdx.x / kWave) * kSplit + (threadIdx.x & (kSplit - 1))];
#pragma unroll
  for (int k = 0; k < ITEMS / V; ++k) {
    const uint32_t i0 = base + (uint32_t)(k * kBlock + threadIdx.x) * V;
    if (i0 + V <= count) {
      const KeyVec<KT> kv = *reinterpret_cast<const KeyVec<KT>*>(keys + i0);  // 16-byte aligned: base is
#pragma unroll
      for (int j = 0; j < V; ++j) atomicAdd(&hw[(kv.k[j] >> shift) & (R - 1)], 1u);
    } else {
      for (int j = 0; j < V; ++j)
        if (i0 + j < count) atomicAdd(&hw[(keys[i0 + j] >> shift) & (R - 1)], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += kBlock) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kSub; ++w) t += h[w][d];
    hist[(size_t)d * nb + blk] = t;
  }
}

// Workgroup d: exclusive scan of hist[d][0..nb) in place; totals[d] = its sum.
__global__ __launch_bounds__(kBlock) void k_radix_colscan(uint32_t* __restrict__ hist, uint32_t nb,
                                                          uint32_t* __restrict__ totals,
                                                          const uint32_t* __restrict__ d_range, int shift) {
  __shared__ uint32_t lds[kBlock / kWave];
  if (pass_is_constant(d_range, shift)) return;
  uint32_t* col = hist + (size_t)blockIdx.x * nb;
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nb; b0 += kBlock) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t v = b < nb ? col[b] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, lds, &tot);
    if (b < nb) col[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Scatter of one pass.  Each workgroup ranks its kBlock * ITEMS keys stably
// (wave ballots over the RB digit bits + per-wave digit counters), places them
// in LDS in (digit, input order) order, and writes them out so that
// consecutive threads store consecutive addresses of each digit's run.  With
// keys_out == NULL (the last pass of a sort whose keys are not needed) only
// the values are written.
template <int RB, typename KT, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const KT* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in,
                                                          KT* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out, uint32_t n,
                                                          const uint32_t* __restrict__ d_count, int shift,
                                                          const uint32_t* __restrict__ d_range,
                                                          const uint32_t* __restrict__ hist_scan,
                                                          const uint32_t* __restrict__ totals, uint32_t nb) {
  constexpr int R = 1 << RB;
  constexpr int kWaves = kBlock / kWave;
  constexpr uint32_t kTile = kBlock * ITEMS;
  __shared__ uint32_t wcnt[kWaves][R];
  __shared__ uint32_t gdelta[R];  // global start of the digit minus its block-local start (mod 2^32)
  __shared__ KT s_key[kTile];
  __shared__ uint32_t s_val[kTile];
  __shared__ uint32_t scan_lds[kBlock / kWave];
  const uint32_t count = d_count ? min(*d_count, n) : n;
  // Chunk blk of the pairs: each XCD takes a contiguous band of the chunks
  // that hold pairs (workgroups are dealt to the XCDs in turn), so the runs
  // that consecutive chunks write for one digit, which meet inside cache
  // lines, are merged in one L2 instead of leaving partial lines from two.
  const uint32_t blk = radix_chunk(count, kTile);
  const uint32_t base = blk * kTile;
  if (base >= count) return;  // uniform for the whole workgroup
  const uint32_t in_block = min(kTile, count - base);
  // uniform: the pass keeps the order.  Constant passes come last (a digit
  // is constant when it and every higher bit agree in the smallest and the
  // largest key), so they are skipped and the result stays where the last
  // pass that ran put it (noted on the device by that pass's histogram).
  if (pass_is_constant(d_range, shift)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const bool digit_thread = threadIdx.x < R;
  // Wave w owns items [base + w*64*ITEMS, base + (w+1)*64*ITEMS), visited 64
  // at a time in index order, so (wave, step, lane) order is the input order.
  // The block's loads go out first, so that their latency overlaps the digit
  // starts' loads and the barrier below.
  const uint32_t wbase = base + wave * (kWave * ITEMS);
  const bool full = in_block == kTile;  // uniform: no bounds tests in the block
  uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
  if (full) {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      key[k] = (uint32_t)keys_in[wbase + k * kWave + lane];
      val[k] = vals_in[wbase + k * kWave + lane];
    }
  } else {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t i = wbase + k * kWave + lane;
      const bool valid = i < count;
      key[k] = valid ? (uint32_t)keys_in[i] : 0u;
      val[k] = valid ? vals_in[i] : 0u;
    }
  }
  if (digit_thread) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
  }
  // global start of this block's run of digit t: with per-digit scans, the
  // digit start (scan of the totals) + the blocks before this one; with a flat
  // scan of the digit-major histogram (totals == NULL), the entry itself
  uint32_t gbase = digit_thread ? hist_scan[(size_t)threadIdx.x * nb + blk] : 0u;
  if (totals) {  // uniform
    uint32_t tot;
    const uint32_t dstart = block_exclusive_scan(digit_thread ? totals[threadIdx.x] : 0u, scan_lds, &tot);
    gbase += digit_thread ? dstart : 0u;
  }
  __syncthreads();

  lds_volatile_u32* my_cnt = lds_volatile(wcnt[wave]);
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const bool valid = full || wbase + k * kWave + lane < count;
    const uint32_t d = (key[k] >> shift) & (R - 1);
    // lanes holding the same digit: the valid lanes minus those whose digit
    // differs in some bit, as two 32-bit halves
    const uint64_t v = full ? ~0ull : __ballot(valid);
    // lanes whose digit differs from this lane's in some bit
    uint32_t dlo = 0u, dhi = 0u;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      // the bit as 0 or all ones (sign-extended one-bit field); the lanes
      // whose bit b differs are the ballot XOR that mask, OR-ed into the
      // accumulator with one three-input bit operation per half
      const int x = __builtin_amdgcn_sbfe((int)d, b, 1);
      const uint64_t m = __ballot(x);
      dlo = __builtin_amdgcn_bitop3_b32(dlo, (uint32_t)m, (uint32_t)x, 0xF6);          // dlo | (m ^ x)
      dhi = __builtin_amdgcn_bitop3_b32(dhi, (uint32_t)(m >> 32), (uint32_t)x, 0xF6);  // dhi | (m ^ x)
    }
    const uint32_t plo = (uint32_t)v & ~dlo, phi = (uint32_t)(v >> 32) & ~dhi;
    // peers in lanes below this one, and in all
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
    uint32_t before = 0;
    if (valid) before = my_cnt[d];           // every lane reads before the leader writes
    if (valid && below == 0) my_cnt[d] = before + (uint32_t)(__popc(plo) + __popc(phi));
    rank[k] = before + below;
  }
  __syncthreads();
  {
    // thread t = digit t: prefix over waves, block-local digit start, global offset
    uint32_t run = 0;
    if (digit_thread) {
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t t = wcnt[w][threadIdx.x];
        wcnt[w][threadIdx.x] = run;
        run += t;
      }
    }
    uint32_t tot;
    const uint32_t ls = block_exclusive_scan(run, scan_lds, &tot);
    if (digit_thread) {
      gdelta[threadIdx.x] = gbase - ls;
      // wcnt[w][t] becomes the block-local slot of wave w's first key of digit t
#pragma unroll
      for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] += ls;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    if (full || wbase + k * kWave + lane < count) {
      const uint32_t d = (key[k] >> shift) & (R - 1);
      const uint32_t lp = wcnt[wave][d] + rank[k];
      s_key[lp] = (KT)key[k];
      s_val[lp] = val[k];
    }
  }
  __syncthreads();
  // scattered stores through buffer descriptors: a 32-bit byte offset per
  // store instead of a 64-bit address (a sort takes fewer than 2^30 pairs, so
  // every byte offset of 4-byte values fits)
  const __amdgpu_buffer_rsrc_t kout = __builtin_amdgcn_make_buffer_rsrc(keys_out, 0, -1, kBufferWord3);
  const __amdgpu_buffer_rsrc_t vout = __builtin_amdgcn_make_buffer_rsrc(vals_out, 0, -1, kBufferWord3);
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t j = k * kBlock + threadIdx.x;
    if (full || j < in_block) {
      const uint32_t kk = s_key[j];
      const uint32_t d = (kk >> shift) & (R - 1);
      const uint32_t pos = gdelta[d] + j;  // = gbase[d] + (j - block-local start of d)
      if (keys_out) {
        if (sizeof(KT) == 2)
          __builtin_amdgcn_raw_buffer_store_b16((uint16_t)kk, kout, (int)(pos * 2u), 0, 0);
        else
          __builtin_amdgcn_raw_buffer_store_b32(kk, kout, (int)(pos * 4u), 0, 0);
      }
      __builtin_amdgcn_raw_buffer_store_b32(s_val[j], vout, (int)(pos * 4u), 0, 0);
    }
  }
}

// Pairs per block of the sorts (kBlock times the items per thread): smaller
// blocks mean more histogram entries and shorter digit runs per block to
// write out, larger ones fewer waves per SIMD (more registers and LDS).
// The default shapes, and the large blocks (kSortItemsLarge per thread) a
// caller may choose for the sort of many pairs over wide digits.
template <typename KT>
struct SortShape;
template <>
struct SortShape<uint32_t> {
  static constexpr int kItems = kScanItems;
};
template <>
struct SortShape<uint16_t> {
  static constexpr int kItems = FGS_SORT16_ITEMS;
};

// Up to this many blocks a pass scans its histogram with one workgroup per
// digit (a few chunks each); beyond, one device-wide scan of the flat
// digit-major histogram, whose entry (d, b) is then the block's global start.
constexpr uint32_t kColscanMaxBlocks = 2048;

size_t radix_scratch_words(uint64_t n) {
  // the smallest block size of any sort bounds the number of blocks
  constexpr uint64_t tile = (uint64_t)kBlock * (SortShape<uint32_t>::kItems < SortShape<uint16_t>::kItems
                                                    ? SortShape<uint32_t>::kItems
                                                    : SortShape<uint16_t>::kItems);
  const uint64_t nb = (n + tile - 1) / tile;
  return round_words((uint64_t)kRadix * nb) + round_words(kRadix) + scan_scratch_words((uint64_t)kRadix * nb);
}

template <int RB, typename KT, int kItems>
static hipError_t radix_pass(const KT* keys_in, const uint32_t* vals_in, KT* keys_out, uint32_t* vals_out,
                             uint32_t n, const uint32_t* d_count, const uint32_t* d_range, int shift,
                             uint32_t* hist, uint32_t* totals, uint32_t* scan_scratch, uint32_t nb,
                             uint32_t* final_word, uint32_t final_if_run, hipStream_t s) {
  k_radix_hist<RB, KT, kItems><<<nb, kBlock, 0, s>>>(keys_in, n, d_count, shift, d_range, hist, nb, final_word,
                                                     final_if_run);
  const uint32_t* digit_totals = totals;
  if (nb > kColscanMaxBlocks) {
    const hipError_t e = scan_u32(hist, hist, (uint32_t)(nb << RB), nullptr, scan_scratch, s);
    if (e != hipSuccess) return e;
    digit_totals = nullptr;
  } else {
    k_radix_colscan<<<1u << RB, kBlock, 0, s>>>(hist, nb, totals, d_range, shift);
  }
  k_radix_scatter<RB, KT, kItems><<<nb, kBlock, 0, s>>>(keys_in, vals_in, keys_out, vals_out, n, d_count, shift,
                                                        d_range, hist, digit_totals, nb);
  return hipGetLastError();
}

template <typename KT, int kItems>
static hipError_t radix_sort_impl(KT* keys[2], uint32_t* vals[2], uint32_t n, const uint32_t* d_count,
                                  const uint32_t* d_range, int begin_bit, int end_bit, bool keep_keys,
                                  uint32_t* scratch, int* final_buf, uint32_t* final_word, hipStream_t s) {
  int cur = 0;
  if (n == 0 || end_bit <= begin_bit) {
    *final_buf = 0;
    return hipSuccess;
  }
  const uint32_t nb = ceil_div(n, (uint64_t)kBlock * kItems);
  uint32_t* hist = scratch;
  uint32_t* totals = scratch + round_words((size_t)kRadix * nb);
  uint32_t* scan_scratch = totals + round_words(kRadix);
  const int bits = end_bit - begin_bit;
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  int shift = begin_bit;
  for (int p = 0; p < passes; ++p) {
    // the remaining bits, split evenly over the remaining passes; with 16-bit
    // keys the narrower digit goes first (13 tile bits as 6 + 7: histograms
    // and scatters 276 instead of 289 us per step at 3M Gaussians), with
    // 32-bit keys last (the depth keys' top digit is nearly constant, and its
    // histogram gains from having fewer digits)
    const int left = end_bit - shift, rest = passes - p;
    const int rb = sizeof(KT) == 2 ? left / rest : (left + rest - 1) / rest;
    KT* kout = (p + 1 == passes && !keep_keys) ? nullptr : keys[cur ^ 1];
    const uint32_t fin = (uint32_t)(cur ^ 1);
    hipError_t e = hipSuccess;
#define FGS_RADIX_PASS(RB_)                                                                                     \
  e = radix_pass<RB_, KT, kItems>(keys[cur], vals[cur], kout, vals[cur ^ 1], n, d_count, d_range, shift, hist,    \
                                  totals, scan_scratch, nb, final_word, fin, s)
    switch (rb) {
      case 1: FGS_RADIX_PASS(1); break;
      case 2: FGS_RADIX_PASS(2); break;
      case 3: FGS_RADIX_PASS(3); break;
      case 4: FGS_RADIX_PASS(4); break;
      case 5: FGS_RADIX_PASS(5); break;
      case 6: FGS_RADIX_PASS(6); break;
      case 7: FGS_RADIX_PASS(7); break;
      default: FGS_RADIX_PASS(8); break;
    }
#undef FGS_RADIX_PASS
    if (e != hipSuccess) return e;
    shift += rb;
    cur ^= 1;
  }
  // with d_range, trailing passes whose digit every key shares are skipped on
  // the device: the buffer holding the result is then known there only
  *final_buf = d_range != nullptr ? -1 : cur;
  return hipSuccess;
}

hipError_t radix_sort_pairs(uint32_t* keys[2], uint32_t* vals[2], uint32_t n, const uint32_t* d_count,
                            int begin_bit, int end_bit, uint32_t* scratch, int* final_buf, hipStream_t s,
                            const uint32_t* d_range, bool keep_keys, uint32_t* final_word, bool large_blocks) {
  if ((uint64_t)n >= (uint64_t)kMaxSortPairs || (d_range != nullptr && final_word == nullptr))
    return hipErrorInvalidValue;
  if (large_blocks)
    return radix_sort_impl<uint32_t, kSortItemsLarge>(keys, vals, n, d_count, d_range, begin_bit, end_bit, keep_keys,
                                                      scratch, final_buf, final_word, s);
  return radix_sort_impl<uint32_t, SortShape<uint32_t>::kItems>(keys, vals, n, d_count, d_range, begin_bit, end_bit,
                                                                keep_keys, scratch, final_buf, final_word, s);
}

hipError_t radix_sort_pairs16(uint16_t* keys[2], uint32_t* vals[2], uint32_t n, const uint32_t* d_count,
                              int begin_bit, int end_bit, uint32_t* scratch, int* final_buf, hipStream_t s,
                              bool large_blocks) {
  if ((uint64_t)n >= (uint64_t)kMaxSortPairs) return hipErrorInvalidValue;
  if (large_blocks)
    return radix_sort_impl<uint16_t, kSortItemsLarge>(keys, vals, n, d_count, nullptr, begin_bit, end_bit, true,
                                                      scratch, final_buf, nullptr, s);
  return radix_sort_impl<uint16_t, SortShape<uint16_t>::kItems>(keys, vals, n, d_count, nullptr, begin_bit, end_bit,
                                                                true, scratch, final_buf, nullptr, s);
}

}  // namespace fgs
