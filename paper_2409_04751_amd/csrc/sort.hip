// Binning and sorting (Sec. 3.1 "Rendering": every Gaussian's bounding
// rectangle gives its tiles; the (tile, Gaussian) intersections are sorted by
// tile id and depth).
//
// Instead of one radix sort over 64-bit (tile << 32 | depth) keys, the order
// is built in two stable sorts: the visible Gaussians are sorted once by
// depth (32-bit keys, N items), duplicated into (tile, id) pairs in that order,
// and the pairs are then sorted stably by tile id alone (ceil(log2 tiles)
// bits).  A stable sort keeps the depth order inside every tile, so the
// result is the order of (tile, depth, id) with 16-20 fewer key bits moved
// per intersection.
//
// Radix passes are 8-bit LSD: a histogram kernel, an exclusive scan of the
// digit-major histogram table, and a stable scatter.  The scatter ranks keys
// inside a block with wave64 ballots (each lane learns which lanes share its
// digit from one ballot per key bit), keeps per-wave digit counters in LDS,
// and stages the block's keys in LDS in sorted order so the global writes go
// out as runs of consecutive addresses.
#include "fgs_internal.hpp"

namespace fgs {
namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kItemsPerWave = kItemsPerBlock / kWaves;  // 1024
constexpr int kIters = kItemsPerWave / 64;              // 16

__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline uint32_t popc_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---- block-wide exclusive scan of one u32 per thread ----------------------
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* smem /* kBlock + kWaves */, uint32_t& total) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave inclusive scan via shuffles
  uint32_t x = v;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == 63) smem[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t t = smem[w];
      smem[w] = run;
      run += t;
    }
    smem[kWaves] = run;
  }
  __syncthreads();
  total = smem[kWaves];
  const uint32_t r = smem[wave] + x - v;
  __syncthreads();
  return r;
}

// ---- device-wide exclusive scan: partial sums, scan of partials, apply -----
__global__ __launch_bounds__(kBlock) void scan_partials_kernel(const uint32_t* in, const uint32_t* gather,
                                                               uint32_t count, uint32_t* partials) {
  __shared__ uint32_t smem[kBlock + kWaves + 1];
  const uint32_t base = blockIdx.x * kItemsPerBlock;
  uint32_t sum = 0;
  for (int k = 0; k < kItemsPerThread; ++k) {
    const uint32_t idx = base + k * kBlock + threadIdx.x;
    if (idx < count) sum += gather ? in[gather[idx]] : in[idx];
  }
  uint32_t total;
  block_exclusive_scan(sum, smem, total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void scan_top_kernel(uint32_t* partials, uint32_t nparts, uint32_t* total_out) {
  __shared__ uint32_t smem[kBlock + kWaves + 1];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nparts; base += kBlock * kItemsPerThread) {
    // each thread scans kItemsPerThread consecutive entries
    uint32_t vals[kItemsPerThread];
    uint32_t sum = 0;
    for (int k = 0; k < kItemsPerThread; ++k) {
      const uint32_t idx = base + threadIdx.x * kItemsPerThread + k;
      vals[k] = idx < nparts ? partials[idx] : 0u;
      sum += vals[k];
    }
    uint32_t total;
    uint32_t off = block_exclusive_scan(sum, smem, total) + carry;
    for (int k = 0; k < kItemsPerThread; ++k) {
      const uint32_t idx = base + threadIdx.x * kItemsPerThread + k;
      if (idx < nparts) partials[idx] = off;
      off += vals[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kBlock) void scan_apply_kernel(const uint32_t* in, const uint32_t* gather, uint32_t* out,
                                                            uint32_t count, const uint32_t* partials) {
  __shared__ uint32_t smem[kBlock + kWaves + 1];
  // thread t owns items base + t*16 .. +15 (blocked), so the scan is one pass
  const uint32_t base = blockIdx.x * kItemsPerBlock + threadIdx.x * kItemsPerThread;
  uint32_t vals[kItemsPerThread];
  uint32_t sum = 0;
  for (int k = 0; k < kItemsPerThread; ++k) {
    const uint32_t idx = base + k;
    vals[k] = idx < count ? (gather ? in[gather[idx]] : in[idx]) : 0u;
    sum += vals[k];
  }
  uint32_t total;
  uint32_t off = block_exclusive_scan(sum, smem, total) + partials[blockIdx.x];
  for (int k = 0; k < kItemsPerThread; ++k) {
    const uint32_t idx = base + k;
    if (idx < count) out[idx] = off;
    off += vals[k];
  }
}

// ---- radix sort ------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const uint32_t* keys, uint32_t count, int shift, int bits,
                                                            uint32_t nblocks, uint32_t* hist) {
  __shared__ uint32_t h[kRadix];
  const uint32_t radix = 1u << bits, mask = radix - 1u;
  for (uint32_t d = threadIdx.x; d < radix; d += kBlock) h[d] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * kItemsPerBlock;
  for (int k = 0; k < kItemsPerThread; ++k) {
    const uint32_t idx = base + k * kBlock + threadIdx.x;
    if (idx < count) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < radix; d += kBlock) hist[d * nblocks + blockIdx.x] = h[d];
}

__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(const uint32_t* keys_in, const uint32_t* vals_in,
                                                               uint32_t* keys_out, uint32_t* vals_out, uint32_t count,
                                                               int shift, int bits, uint32_t nblocks,
                                                               const uint32_t* scanned_hist) {
  __shared__ uint32_t wave_count[kWaves][kRadix];
  __shared__ uint32_t local_start[kRadix];
  __shared__ uint32_t global_start[kRadix];
  __shared__ uint32_t stage_keys[kItemsPerBlock];
  __shared__ uint32_t stage_vals[kItemsPerBlock];
  __shared__ uint32_t smem[kBlock + kWaves + 1];

  const uint32_t radix = 1u << bits, mask = radix - 1u;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t d = threadIdx.x; d < kRadix; d += kBlock) {
    for (int w = 0; w < kWaves; ++w) wave_count[w][d] = 0;
  }
  __syncthreads();

  const uint32_t block_base = blockIdx.x * kItemsPerBlock;
  const uint32_t wave_base = block_base + wave * kItemsPerWave;
  uint32_t my_key[kIters], my_val[kIters], my_rank[kIters];
  for (int it = 0; it < kIters; ++it) {
    const uint32_t idx = wave_base + it * 64 + lane;
    const bool valid = idx < count;
    const uint32_t key = valid ? keys_in[idx] : 0u;
    const uint32_t val = valid ? vals_in[idx] : 0u;
    const uint32_t digit = (key >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const uint64_t bal = __ballot((digit >> b) & 1u);
      peers &= ((digit >> b) & 1u) ? bal : ~bal;
    }
    uint32_t rank = 0;
    if (valid) {
      const uint32_t before = wave_count[wave][digit];
      rank = before + popc_below(peers);
      // the highest peer lane publishes the new count
      const uint32_t last_lane = 63u - (uint32_t)__builtin_clzll(peers);
      if (lane == last_lane) wave_count[wave][digit] = before + (uint32_t)__builtin_popcountll(peers);
    }
    my_key[it] = key;
    my_val[it] = val;
    my_rank[it] = valid ? rank : 0xFFFFFFFFu;
  }
  __syncthreads();
  // per digit: exclusive prefix over waves, block count, local and global starts
  uint32_t block_count = 0;
  if (threadIdx.x < radix) {
    const uint32_t d = threadIdx.x;
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = wave_count[w][d];
      wave_count[w][d] = block_count;
      block_count += c;
    }
    global_start[d] = scanned_hist[d * nblocks + blockIdx.x];
  }
  uint32_t total;
  const uint32_t ls = block_exclusive_scan(block_count, smem, total);
  if (threadIdx.x < radix) local_start[threadIdx.x] = ls;
  __syncthreads();
  for (int it = 0; it < kIters; ++it) {
    if (my_rank[it] == 0xFFFFFFFFu) continue;
    const uint32_t digit = (my_key[it] >> shift) & mask;
    const uint32_t pos = local_start[digit] + wave_count[wave][digit] + my_rank[it];
    stage_keys[pos] = my_key[it];
    stage_vals[pos] = my_val[it];
  }
  __syncthreads();
  const uint32_t nvalid = count > block_base ? min((uint32_t)kItemsPerBlock, count - block_base) : 0u;
  for (uint32_t p = threadIdx.x; p < nvalid; p += kBlock) {
    const uint32_t key = stage_keys[p];
    const uint32_t digit = (key >> shift) & mask;
    const uint32_t dst = global_start[digit] + (p - local_start[digit]);
    keys_out[dst] = key;
    vals_out[dst] = stage_vals[p];
  }
}

// ---- duplication: one pair per (Gaussian, covered tile) --------------------
// Block b handles Gaussians [b*256, b*256+256) of the depth order and emits
// their pairs cooperatively: each output slot finds its Gaussian by binary
// search over the block's 256 offsets in LDS, so a Gaussian covering
// thousands of tiles does not serialise one thread.
__global__ __launch_bounds__(kBlock) void duplicate_kernel(const uint32_t* depth_order, const uint32_t* tiles,
                                                           const uint32_t* offsets, const uint2* rects, uint32_t n,
                                                           uint32_t tiles_x, uint32_t* out_keys, uint32_t* out_vals) {
  __shared__ uint32_t s_off[kBlock + 1];
  __shared__ uint32_t s_id[kBlock];
  __shared__ uint2 s_rect[kBlock];
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  uint32_t cnt = 0;
  if (j < n) {
    const uint32_t g = depth_order[j];
    cnt = tiles[g];
    s_off[threadIdx.x] = offsets[j];
    s_id[threadIdx.x] = g;
    s_rect[threadIdx.x] = cnt ? rects[g] : make_uint2(0, 0);
  } else {
    s_off[threadIdx.x] = 0;
    s_id[threadIdx.x] = 0;
    s_rect[threadIdx.x] = make_uint2(0, 0);
  }
  // end offset of the block = offset of its last valid item + its count
  __shared__ uint32_t s_end;
  const uint32_t last = min(n - blockIdx.x * kBlock, (uint32_t)kBlock) - 1;
  if (threadIdx.x == last) s_end = offsets[j] + cnt;
  __syncthreads();
  if (threadIdx.x > last) s_off[threadIdx.x] = s_end;
  if (threadIdx.x == 0) s_off[kBlock] = s_end;
  __syncthreads();
  const uint32_t start = s_off[0], end = s_end;
  for (uint32_t o = start + threadIdx.x; o < end; o += kBlock) {
    // largest k with s_off[k] <= o (items with zero count share offsets)
    int lo = 0, hi = kBlock;  // invariant s_off[lo] <= o < s_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_off[mid] <= o) lo = mid; else hi = mid;
    }
    const uint32_t local = o - s_off[lo];
    const uint2 r = s_rect[lo];
    const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16, x1 = r.y & 0xFFFFu;
    const uint32_t w = x1 - x0;
    const uint32_t ty = y0 + local / w, tx = x0 + local % w;
    out_keys[o] = ty * tiles_x + tx;
    out_vals[o] = s_id[lo];
  }
}

__global__ __launch_bounds__(kBlock) void ranges_kernel(const uint32_t* keys, uint32_t K, uint2* ranges) {
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= K) return;
  const uint32_t t = keys[j];
  if (j == 0 || keys[j - 1] != t) ranges[t].x = j;
  if (j == K - 1 || keys[j + 1] != t) ranges[t].y = j + 1;
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t* p, uint32_t v, uint32_t count) {
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < count) p[j] = v;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)ceil_div(count, kBlock)), dim3(kBlock), 0, s, p, v,
                     (uint32_t)count);
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* in, const uint32_t* gather, uint32_t* out, int64_t count, uint32_t* partials,
                       uint32_t* total, hipStream_t s) {
  if (count <= 0) return total ? launch_fill_u32(total, 0u, 1, s) : hipSuccess;
  const uint32_t nb = (uint32_t)ceil_div(count, kItemsPerBlock);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(nb), dim3(kBlock), 0, s, in, gather, (uint32_t)count, partials);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kBlock), 0, s, partials, nb, total);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(kBlock), 0, s, in, gather, out, (uint32_t)count, partials);
  return hipGetLastError();
}

int radix_passes(int bits) { return bits <= 0 ? 0 : (bits + kRadixBits - 1) / kRadixBits; }

hipError_t launch_radix_sort(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, int64_t count,
                             int bits, uint32_t* hist, uint32_t* partials, bool* result_in_b, hipStream_t s) {
  // The result buffer depends only on the number of passes, so callers can
  // locate it from the layout; with count == 0 there is nothing to read.
  const int passes = radix_passes(bits);
  *result_in_b = (passes % 2) == 1;
  if (count <= 0 || passes == 0) return hipSuccess;
  const uint32_t nb = (uint32_t)ceil_div(count, kItemsPerBlock);
  uint32_t *ki = keys_a, *vi = vals_a, *ko = keys_b, *vo = vals_b;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int remaining = bits - shift;
    const int pb = (remaining + (passes - p) - 1) / (passes - p);  // balanced digit widths
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nb), dim3(kBlock), 0, s, ki, (uint32_t)count, shift, pb, nb, hist);
    hipError_t e = launch_scan(hist, nullptr, hist, (int64_t)nb << pb, partials, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nb), dim3(kBlock), 0, s, ki, vi, ko, vo, (uint32_t)count, shift,
                       pb, nb, hist);
    shift += pb;
    uint32_t* t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  return hipGetLastError();
}

hipError_t launch_duplicate(const uint32_t* depth_order, const uint32_t* tiles, const uint32_t* offsets,
                            const uint2* rects, int64_t n, int32_t tiles_x, uint32_t* out_keys, uint32_t* out_vals,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s, depth_order, tiles,
                     offsets, rects, (uint32_t)n, (uint32_t)tiles_x, out_keys, out_vals);
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* sorted_keys, int64_t K, uint2* ranges, int32_t ntiles, hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * (int64_t)ntiles, s);
  if (e != hipSuccess || K <= 0) return e;
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)ceil_div(K, kBlock)), dim3(kBlock), 0, s, sorted_keys,
                     (uint32_t)K, ranges);
  return hipGetLastError();
}

}  // namespace fgs
