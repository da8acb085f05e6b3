// Binning and sorting (Sec. 3.1 "Rendering": every Gaussian's bounding
// rectangle gives its tiles; the (tile, Gaussian) intersections are sorted by
// tile id and depth).
//
// Instead of one radix sort over 64-bit (tile << 32 | depth) keys, the order
// is built in two stable sorts: the visible Gaussians, compacted in id order,
// are sorted once by depth (31 key bits over V items, carrying their id and
// tile rectangle so that every later pass streams instead of gathering),
// duplicated into (tile, id) pairs in that order, and the pairs are then
// sorted stably by tile id alone (ceil(log2 tiles) bits).  A stable sort
// keeps the depth order inside every tile, so the result is the order of
// (tile, depth, id) with 16-20 fewer key bits moved per intersection.
//
// Radix passes are 8-bit LSD: a histogram kernel, an exclusive scan of the
// digit-major histogram table, and a stable scatter.  The scatter ranks keys
// inside a block with wave64 ballots (each lane learns which lanes share its
// digit from one ballot per key bit), keeps per-wave digit counters in LDS,
// and stages the block's items in LDS in sorted order so the global writes go
// out as runs of consecutive addresses.  Item counts may live in device
// memory (the visible count): grids are sized for the host-side bound and
// blocks past the device count do nothing.
#include "fgs_internal.hpp"

namespace fgs {
namespace {

constexpr int kWaves = kBlock / 64;

__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline uint32_t popc_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ inline uint32_t item_count(const uint32_t* d_count, uint32_t max_count) {
  return d_count ? min(*d_count, max_count) : max_count;
}

// ---- block-wide exclusive scan of one u32 per thread ----------------------
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* smem /* kWaves + 1 */, uint32_t& total) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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

// ---- scan inputs -----------------------------------------------------------
struct ScanIn {
  const uint32_t* a;  // values, flags, or rect x0|y0 plane
  const uint32_t* b;  // rect x1|y1 plane (kScanRectArea)
};

template <int MODE>
__device__ inline uint32_t scan_value(const ScanIn& in, uint32_t idx) {
  if (MODE == kScanFlag) return in.a[idx] != 0u ? 1u : 0u;
  if (MODE == kScanRectArea) {
    const uint32_t a = in.a[idx], b = in.b[idx];
    return ((b & 0xFFFFu) - (a & 0xFFFFu)) * ((b >> 16) - (a >> 16));
  }
  return in.a[idx];
}

// ---- device-wide exclusive scan: partial sums, scan of partials, apply -----
template <int MODE>
__global__ __launch_bounds__(kBlock) void scan_partials_kernel(ScanIn in, const uint32_t* d_count, uint32_t max_count,
                                                               uint32_t* partials) {
  __shared__ uint32_t smem[kWaves + 1];
  const uint32_t count = item_count(d_count, max_count);
  const uint32_t base = blockIdx.x * kItemsPerBlock;
  uint32_t sum = 0;
  for (int k = 0; k < kItemsPerThread; ++k) {
    const uint32_t idx = base + k * kBlock + threadIdx.x;
    if (idx < count) sum += scan_value<MODE>(in, idx);
  }
  uint32_t total;
  block_exclusive_scan(sum, smem, total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ __launch_bounds__(kBlock) void scan_top_kernel(uint32_t* partials, uint32_t nparts, uint32_t* total_out) {
  __shared__ uint32_t smem[kWaves + 1];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nparts; base += kBlock * kItemsPerThread) {
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

template <int MODE>
__global__ __launch_bounds__(kBlock) void scan_apply_kernel(ScanIn in, uint32_t* out, const uint32_t* d_count,
                                                            uint32_t max_count, const uint32_t* partials) {
  __shared__ uint32_t smem[kWaves + 1];
  const uint32_t count = item_count(d_count, max_count);
  // thread t owns items base + t*16 .. +15 (blocked), so the scan is one pass
  const uint32_t base = blockIdx.x * kItemsPerBlock + threadIdx.x * kItemsPerThread;
  uint32_t vals[kItemsPerThread];
  uint32_t sum = 0;
  for (int k = 0; k < kItemsPerThread; ++k) {
    const uint32_t idx = base + k;
    vals[k] = idx < count ? scan_value<MODE>(in, idx) : 0u;
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
template <int P>
struct ValPtrs {
  uint32_t* p[P];
};

// IPT items per thread; one block covers kBlock * IPT consecutive items.
template <int IPT>
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const uint32_t* keys, const uint32_t* d_count,
                                                            uint32_t max_count, int shift, int bits, uint32_t nblocks,
                                                            uint32_t* hist) {
  __shared__ uint32_t h[kRadix];
  const uint32_t count = item_count(d_count, max_count);
  const uint32_t radix = 1u << bits, mask = radix - 1u;
  for (uint32_t d = threadIdx.x; d < radix; d += kBlock) h[d] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * (kBlock * IPT);
  for (int k = 0; k < IPT; ++k) {
    const uint32_t idx = base + k * kBlock + threadIdx.x;
    if (idx < count) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < radix; d += kBlock) hist[d * nblocks + blockIdx.x] = h[d];
}

// Stable scatter of one pass; P u32 payload words per key.
template <int P, int IPT>
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(const uint32_t* keys_in, ValPtrs<P> vin,
                                                               uint32_t* keys_out, ValPtrs<P> vout,
                                                               const uint32_t* d_count, uint32_t max_count, int shift,
                                                               int bits, uint32_t nblocks,
                                                               const uint32_t* scanned_hist) {
  constexpr int kItems = kBlock * IPT;
  constexpr int kPerWave = kItems / kWaves;
  constexpr int kIters = kPerWave / 64;
  __shared__ uint32_t wave_count[kWaves][kRadix];
  __shared__ uint32_t local_start[kRadix];
  __shared__ uint32_t global_start[kRadix];
  __shared__ uint32_t stage_keys[kItems];
  __shared__ uint32_t stage_vals[P][kItems];
  __shared__ uint32_t smem[kWaves + 1];

  const uint32_t count = item_count(d_count, max_count);
  const uint32_t block_base = blockIdx.x * kItems;
  if (block_base >= count) return;  // uniform per block
  const uint32_t radix = 1u << bits, mask = radix - 1u;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t d = threadIdx.x; d < kRadix; d += kBlock) {
    for (int w = 0; w < kWaves; ++w) wave_count[w][d] = 0;
  }
  __syncthreads();

  const uint32_t wave_base = block_base + wave * kPerWave;
  uint32_t my_key[kIters], my_rank[kIters], my_val[kIters][P];
  for (int it = 0; it < kIters; ++it) {
    const uint32_t idx = wave_base + it * 64 + lane;
    const bool valid = idx < count;
    const uint32_t key = valid ? keys_in[idx] : 0u;
    for (int q = 0; q < P; ++q) my_val[it][q] = valid ? vin.p[q][idx] : 0u;
    const uint32_t digit = (key >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const uint64_t bal = __ballot((digit >> b) & 1u);
      peers &= ((digit >> b) & 1u) ? bal : ~bal;
    }
    uint32_t rank = 0xFFFFFFFFu;
    if (valid) {
      const uint32_t before = wave_count[wave][digit];
      rank = before + popc_below(peers);
      // the highest peer lane publishes the new count
      const uint32_t last_lane = 63u - (uint32_t)__builtin_clzll(peers);
      if (lane == last_lane) wave_count[wave][digit] = before + (uint32_t)__builtin_popcountll(peers);
    }
    my_key[it] = key;
    my_rank[it] = rank;
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
    for (int q = 0; q < P; ++q) stage_vals[q][pos] = my_val[it][q];
  }
  __syncthreads();
  const uint32_t nvalid = min((uint32_t)kItems, count - block_base);
  for (uint32_t e = threadIdx.x; e < nvalid; e += kBlock) {
    const uint32_t key = stage_keys[e];
    const uint32_t digit = (key >> shift) & mask;
    const uint32_t dst = global_start[digit] + (e - local_start[digit]);
    keys_out[dst] = key;
    for (int q = 0; q < P; ++q) vout.p[q][dst] = stage_vals[q][e];
  }
}

// ---- compaction of the visible Gaussians (stable, id order) ----------------
__global__ __launch_bounds__(kBlock) void compact_kernel(const uint32_t* tiles, const uint32_t* depth_keys,
                                                         const uint2* rects, const uint32_t* pos, uint32_t n,
                                                         uint32_t* keys, uint32_t* ids, uint32_t* rx, uint32_t* ry) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n || tiles[i] == 0) return;
  const uint32_t p = pos[i];
  const uint2 r = rects[i];
  keys[p] = depth_keys[i];
  ids[p] = i;
  rx[p] = r.x;
  ry[p] = r.y;
}

// ---- duplication: one pair per (Gaussian, covered tile) --------------------
// Block b handles depth-ordered Gaussians [b*256, b*256+256) and emits their
// pairs cooperatively: each output slot finds its Gaussian by binary search
// over the block's 256 offsets in LDS, so a Gaussian covering thousands of
// tiles does not serialise one thread, and consecutive lanes write
// consecutive addresses.
__global__ __launch_bounds__(kBlock) void duplicate_kernel(const uint32_t* ids, const uint32_t* rx, const uint32_t* ry,
                                                           const uint32_t* offsets, const uint32_t* d_count,
                                                           uint32_t max_count, uint32_t tiles_x, uint32_t* out_keys,
                                                           uint32_t* out_vals) {
  __shared__ uint32_t s_off[kBlock + 1];
  __shared__ uint32_t s_id[kBlock];
  __shared__ uint32_t s_x0[kBlock], s_y0[kBlock], s_w[kBlock];
  __shared__ uint32_t s_end;
  const uint32_t count = item_count(d_count, max_count);
  const uint32_t first = blockIdx.x * kBlock;
  if (first >= count) return;  // uniform per block
  const uint32_t j = first + threadIdx.x;
  const uint32_t last = min(count - first, (uint32_t)kBlock) - 1;
  if (j < count) {
    const uint32_t a = rx[j], b = ry[j];
    const uint32_t x0 = a & 0xFFFFu, y0 = a >> 16, x1 = b & 0xFFFFu, y1 = b >> 16;
    s_off[threadIdx.x] = offsets[j];
    s_id[threadIdx.x] = ids[j];
    s_x0[threadIdx.x] = x0;
    s_y0[threadIdx.x] = y0;
    s_w[threadIdx.x] = x1 - x0;
    if (threadIdx.x == last) s_end = offsets[j] + (x1 - x0) * (y1 - y0);
  }
  __syncthreads();
  if (threadIdx.x > last) s_off[threadIdx.x] = s_end;
  if (threadIdx.x == 0) s_off[kBlock] = s_end;
  __syncthreads();
  const uint32_t start = s_off[0], end = s_end;
  for (uint32_t o = start + threadIdx.x; o < end; o += kBlock) {
    // largest k with s_off[k] <= o (every compacted Gaussian has >= 1 tile)
    int lo = 0, hi = kBlock;  // invariant s_off[lo] <= o < s_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_off[mid] <= o) lo = mid; else hi = mid;
    }
    const uint32_t local = o - s_off[lo];
    const uint32_t w = s_w[lo];
    const uint32_t row = local / w;
    const uint32_t ty = s_y0[lo] + row, tx = s_x0[lo] + (local - row * w);
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

template <int P, int IPT>
hipError_t radix_sort_impl(const RadixBuffers& B, const uint32_t* d_count, int64_t max_count, int bits,
                           uint32_t* hist, uint32_t* partials, hipStream_t s, int hist_id, int scatter_id) {
  const int passes = radix_passes(bits);
  const uint32_t nb = (uint32_t)ceil_div(max_count, (int64_t)kBlock * IPT);
  uint32_t* ki = B.keys_a;
  uint32_t* ko = B.keys_b;
  ValPtrs<P> vi, vo;
  for (int q = 0; q < P; ++q) {
    vi.p[q] = B.vals_a[q];
    vo.p[q] = B.vals_b[q];
  }
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int remaining = bits - shift;
    const int pb = (remaining + (passes - p) - 1) / (passes - p);  // balanced digit widths
    {
      ProfScope prof(s, hist_id);
      hipLaunchKernelGGL((radix_hist_kernel<IPT>), dim3(nb), dim3(kBlock), 0, s, ki, d_count, (uint32_t)max_count,
                         shift, pb, nb, hist);
    }
    hipError_t e = launch_scan(hist, nullptr, nullptr, (int64_t)nb << pb, kScanPlain, partials, nullptr, hist, s);
    if (e != hipSuccess) return e;
    {
      ProfScope prof(s, scatter_id);
      hipLaunchKernelGGL((radix_scatter_kernel<P, IPT>), dim3(nb), dim3(kBlock), 0, s, ki, vi, ko, vo, d_count,
                         (uint32_t)max_count, shift, pb, nb, hist);
    }
    shift += pb;
    uint32_t* t = ki;
    ki = ko;
    ko = t;
    const ValPtrs<P> tv = vi;
    vi = vo;
    vo = tv;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  ProfScope prof(s, kKFill);
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)ceil_div(count, kBlock)), dim3(kBlock), 0, s, p, v,
                     (uint32_t)count);
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* in_a, const uint32_t* in_b, const uint32_t* d_count, int64_t max_count,
                       int mode, uint32_t* partials, uint32_t* total, uint32_t* out, hipStream_t s) {
  if (max_count <= 0) return total ? launch_fill_u32(total, 0u, 1, s) : hipSuccess;
  const uint32_t nb = (uint32_t)ceil_div(max_count, kItemsPerBlock);
  const ScanIn in{in_a, in_b};
  ProfScope prof(s, kKScan);
  switch (mode) {
    case kScanFlag:
      hipLaunchKernelGGL(scan_partials_kernel<kScanFlag>, dim3(nb), dim3(kBlock), 0, s, in, d_count,
                         (uint32_t)max_count, partials);
      break;
    case kScanRectArea:
      hipLaunchKernelGGL(scan_partials_kernel<kScanRectArea>, dim3(nb), dim3(kBlock), 0, s, in, d_count,
                         (uint32_t)max_count, partials);
      break;
    default:
      hipLaunchKernelGGL(scan_partials_kernel<kScanPlain>, dim3(nb), dim3(kBlock), 0, s, in, d_count,
                         (uint32_t)max_count, partials);
  }
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kBlock), 0, s, partials, nb, total);
  switch (mode) {
    case kScanFlag:
      hipLaunchKernelGGL(scan_apply_kernel<kScanFlag>, dim3(nb), dim3(kBlock), 0, s, in, out, d_count,
                         (uint32_t)max_count, partials);
      break;
    case kScanRectArea:
      hipLaunchKernelGGL(scan_apply_kernel<kScanRectArea>, dim3(nb), dim3(kBlock), 0, s, in, out, d_count,
                         (uint32_t)max_count, partials);
      break;
    default:
      hipLaunchKernelGGL(scan_apply_kernel<kScanPlain>, dim3(nb), dim3(kBlock), 0, s, in, out, d_count,
                         (uint32_t)max_count, partials);
  }
  return hipGetLastError();
}

int radix_passes(int bits) { return bits <= 0 ? 0 : (bits + kRadixBits - 1) / kRadixBits; }

int64_t radix_blocks(int64_t max_count, int payload) {
  return ceil_div(max_count, (int64_t)kBlock * (payload == 1 ? kIptPayload1 : kIptPayload3));
}

hipError_t launch_radix_sort(const RadixBuffers& B, const uint32_t* d_count, int64_t max_count, int bits,
                             uint32_t* hist, uint32_t* partials, hipStream_t s, int hist_id, int scatter_id) {
  if (max_count <= 0 || radix_passes(bits) == 0) return hipSuccess;
  if (B.payload == 1)
    return radix_sort_impl<1, kIptPayload1>(B, d_count, max_count, bits, hist, partials, s, hist_id, scatter_id);
  return radix_sort_impl<3, kIptPayload3>(B, d_count, max_count, bits, hist, partials, s, hist_id, scatter_id);
}

hipError_t launch_compact(const uint32_t* tiles, const uint32_t* depth_keys, const uint2* rects, const uint32_t* pos,
                          int64_t n, uint32_t* keys, uint32_t* ids, uint32_t* rx, uint32_t* ry, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  ProfScope prof(s, kKCompact);
  hipLaunchKernelGGL(compact_kernel, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s, tiles, depth_keys, rects,
                     pos, (uint32_t)n, keys, ids, rx, ry);
  return hipGetLastError();
}

hipError_t launch_duplicate(const uint32_t* ids, const uint32_t* rx, const uint32_t* ry, const uint32_t* offsets,
                            const uint32_t* d_count, int64_t max_count, int32_t tiles_x, uint32_t* out_keys,
                            uint32_t* out_vals, hipStream_t s) {
  if (max_count <= 0) return hipSuccess;
  ProfScope prof(s, kKDuplicate);
  hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)ceil_div(max_count, kBlock)), dim3(kBlock), 0, s, ids, rx, ry,
                     offsets, d_count, (uint32_t)max_count, (uint32_t)tiles_x, out_keys, out_vals);
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* sorted_keys, int64_t K, uint2* ranges, int32_t ntiles, hipStream_t s) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * (int64_t)ntiles, s);
  if (e != hipSuccess || K <= 0) return e;
  ProfScope prof(s, kKRanges);
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)ceil_div(K, kBlock)), dim3(kBlock), 0, s, sorted_keys,
                     (uint32_t)K, ranges);
  return hipGetLastError();
}

}  // namespace fgs
