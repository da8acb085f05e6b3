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
// Radix passes are LSD with digits of up to 9 bits: a histogram kernel, an
// exclusive scan of the digit-major histogram table, and a stable scatter.
// The scatter ranks keys inside a block with one 64-bit lane mask per digit
// and wave in LDS (each lane sets its bit, reads the mask back and clears
// it), keeps per-wave digit counters in LDS, and stages the block's items in
// LDS in sorted order so the global writes go out as runs of consecutive
// addresses.  The tile sort's first pass runs inside the duplication.  Item
// counts may live in device memory (the visible count): grids are sized for
// the host-side bound and blocks past the device count do nothing.
#include "fgs_internal.hpp"
#include "reach.hpp"

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
  const uint32_t* b;  // rect x1|y1 plane (kScanRectArea), or the gathered values (kScanGather)
  uint32_t* aux;      // null, or the item holding each multiple of aux_block (launch_scan)
  uint32_t aux_block;
};

template <int MODE>
__device__ inline uint32_t scan_value(const ScanIn& in, uint32_t idx) {
  if (MODE == kScanFlag) return in.a[idx] != 0u ? 1u : 0u;
  if (MODE == kScanRectArea) {
    const uint32_t a = in.a[idx], b = in.b[idx];
    return ((b & 0xFFFFu) - (a & 0xFFFFu)) * ((b >> 16) - (a >> 16));
  }
  if (MODE == kScanGather) return in.b[in.a[idx]];
  if (MODE == kScanRows) return (in.b[idx] >> 16) - (in.a[idx] >> 16);
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

// Up to this many partials, each apply block sums the partials of the blocks
// before it itself (no separate scan of the partials); beyond it, a
// one-block scan of the partials runs in between.
constexpr uint32_t kMaxFusedPartials = 2048;

// Items idx .. idx+15 of the scan input (idx a multiple of 16).
template <int MODE>
__device__ inline void load16(const ScanIn& in, uint32_t idx, uint32_t count, uint32_t vals[16]) {
  if (idx + 16u <= count) {
    const uint4* a4 = reinterpret_cast<const uint4*>(in.a + idx);
    uint32_t av[16];
    for (int q = 0; q < 4; ++q) {
      const uint4 v = a4[q];
      av[4 * q] = v.x;
      av[4 * q + 1] = v.y;
      av[4 * q + 2] = v.z;
      av[4 * q + 3] = v.w;
    }
    if (MODE == kScanRows) {
      const uint4* b4 = reinterpret_cast<const uint4*>(in.b + idx);
      for (int q = 0; q < 4; ++q) {
        const uint4 v = b4[q];
        const uint32_t bv[4] = {v.x, v.y, v.z, v.w};
        for (int r = 0; r < 4; ++r) vals[4 * q + r] = (bv[r] >> 16) - (av[4 * q + r] >> 16);
      }
    } else if (MODE == kScanRectArea) {
      const uint4* b4 = reinterpret_cast<const uint4*>(in.b + idx);
      for (int q = 0; q < 4; ++q) {
        const uint4 v = b4[q];
        const uint32_t bv[4] = {v.x, v.y, v.z, v.w};
        for (int r = 0; r < 4; ++r) {
          const uint32_t aa = av[4 * q + r], bb = bv[r];
          vals[4 * q + r] = ((bb & 0xFFFFu) - (aa & 0xFFFFu)) * ((bb >> 16) - (aa >> 16));
        }
      }
    } else if (MODE == kScanGather) {
      for (int k = 0; k < 16; ++k) vals[k] = in.b[av[k]];
    } else {
      for (int k = 0; k < 16; ++k) vals[k] = MODE == kScanFlag ? (av[k] != 0u ? 1u : 0u) : av[k];
    }
  } else {
    for (int k = 0; k < 16; ++k) vals[k] = idx + k < count ? scan_value<MODE>(in, idx + k) : 0u;
  }
}

// FUSED: partials holds the block sums and each block adds up those before
// it; otherwise partials already holds their exclusive scan.  The last block
// writes the grand total (FUSED only).
// parts_per_block: partials holds that many sums per block of items (the
// producer's finer block sums), FUSED only.
template <int MODE, bool FUSED>
__global__ __launch_bounds__(kBlock) void scan_apply_kernel(ScanIn in, uint32_t* out, const uint32_t* d_count,
                                                            uint32_t max_count, const uint32_t* partials,
                                                            uint32_t* total_out, uint32_t parts_per_block = 1u) {
  static_assert(kItemsPerThread == 16, "load16");
  __shared__ uint32_t smem[kWaves + 1];
  const uint32_t count = item_count(d_count, max_count);
  uint32_t block_off;
  if (FUSED) {
    // four independent sums, so that a thread's loads are in flight together
    uint32_t a4[4] = {0u, 0u, 0u, 0u};
    const uint32_t before = blockIdx.x * parts_per_block;
    uint32_t b = threadIdx.x;
    for (; b + 3u * kBlock < before; b += 4u * kBlock) {
#pragma unroll
      for (int q = 0; q < 4; ++q) a4[q] += partials[b + (uint32_t)q * kBlock];
    }
    for (; b < before; b += kBlock) a4[0] += partials[b];
    const uint32_t acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    uint32_t tot;
    block_exclusive_scan(acc, smem, tot);
    block_off = tot;
  } else {
    block_off = partials[blockIdx.x];
  }
  // thread t owns items base + t*16 .. +15 (blocked), so the scan is one pass
  const uint32_t base = blockIdx.x * kItemsPerBlock + threadIdx.x * kItemsPerThread;
  uint32_t vals[kItemsPerThread];
  load16<MODE>(in, base, count, vals);
  uint32_t sum = 0;
  for (int k = 0; k < kItemsPerThread; ++k) sum += vals[k];
  uint32_t total;
  uint32_t off = block_exclusive_scan(sum, smem, total) + block_off;
  uint32_t res[kItemsPerThread];
  for (int k = 0; k < kItemsPerThread; ++k) {
    res[k] = off;
    off += vals[k];
  }
  if (in.aux) {
    // the item whose range [res, res + vals) holds a multiple of aux_block
    // starts that block of the consuming kernel
    const uint32_t ab = in.aux_block;
    for (int k = 0; k < kItemsPerThread; ++k) {
      if (base + k >= count) break;
      for (uint32_t b = (res[k] + ab - 1u) / ab; b * ab < res[k] + vals[k]; ++b) in.aux[b] = base + k;
    }
  }
  if (base + 16u <= count) {
    uint4* o4 = reinterpret_cast<uint4*>(out + base);
    for (int q = 0; q < 4; ++q) o4[q] = make_uint4(res[4 * q], res[4 * q + 1], res[4 * q + 2], res[4 * q + 3]);
  } else {
    for (int k = 0; k < kItemsPerThread; ++k)
      if (base + k < count) out[base + k] = res[k];
  }
  if (FUSED && total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_out = block_off + total;
}

// ---- radix sort ------------------------------------------------------------
template <int P>
struct ValPtrs {
  uint32_t* p[P];
};

// IPT items per thread; one block covers kBlock * IPT consecutive items.
// KT: the stored key type (uint16_t for tile ids that fit 16 bits).
template <int IPT, class KT = uint32_t>
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const KT* keys, const uint32_t* d_count,
                                                            uint32_t max_count, uint32_t key_bias, int shift, int bits,
                                                            uint32_t nblocks, uint32_t* hist) {
  __shared__ uint32_t h[kRadix];
  const uint32_t count = item_count(d_count, max_count);
  const uint32_t radix = 1u << bits, mask = radix - 1u;
  for (uint32_t d = threadIdx.x; d < radix; d += kBlock) h[d] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * (kBlock * IPT);
  uint32_t key[IPT];
  for (int k = 0; k < IPT; ++k) {  // all loads in flight before the first atomic
    const uint32_t idx = base + k * kBlock + threadIdx.x;
    key[k] = idx < count ? keys[idx] : 0xFFFFFFFFu;
  }
  for (int k = 0; k < IPT; ++k) {
    if (base + k * kBlock + threadIdx.x < count) atomicAdd(&h[((key[k] - key_bias) >> shift) & mask], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < radix; d += kBlock) hist[d * nblocks + blockIdx.x] = h[d];
}

// LDS of a block's stable scatter: 16-bit per-wave digit counters and one
// start table (local start while staging, then global minus local start
// while writing) keep a 9-bit digit at the occupancy of an 8-bit one; the
// staging planes hold the block's items in (digit, item) order.
// While the block ranks its items, each wave keeps one 64-bit lane mask per
// digit (match, [kWaves][1 << RB]); that table may share memory with the
// staging planes, which are not used until the ranking is done.
template <int RB>
struct ScatterLds {
  uint16_t (*wave_count)[1 << RB];  // [kWaves][1 << RB], zero on entry
  uint32_t* start;                  // [1 << RB]
  uint32_t* smem;                   // [kWaves + 1]
  uint64_t* match;                  // [kWaves][1 << RB], any content on entry
};

// Orders the LDS accesses of one wave's lanes before and after this point.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Ranks the items of one block by digit and writes them, stably, to
// scanned_hist[digit * nblocks + chunk] + their rank among the block's items
// of that digit.  Wave w holds items w * IPT * 64 + it * 64 + lane in
// my_key[it] / my_val[it]; items at or past nvalid are not written, nor
// are items whose place would be at or past out_limit (only a histogram
// that disagrees with the items could put them there).
// stage_keys / stage_vals[q] hold kBlock * IPT words each.
template <int P, int IPT, int RB, class KO = uint32_t>
__device__ inline void rank_stage_write(const uint32_t (&my_key)[IPT], const uint32_t (&my_val)[IPT][P],
                                        uint32_t nvalid, uint32_t key_bias, int shift, int bits, uint32_t nblocks,
                                        uint32_t chunk, const uint32_t* scanned_hist, const ScatterLds<RB>& L,
                                        uint32_t* stage_keys, uint32_t* const (&stage_vals)[P], KO* keys_out,
                                        const ValPtrs<P>& vout, uint32_t out_limit) {
  constexpr int kItems = kBlock * IPT;
  constexpr int kPerWave = kItems / kWaves;
  static_assert(kPerWave / 64 == IPT, "one item per lane and iteration");
  static_assert((1u << RB) <= 2 * kBlock, "two digits per thread");
  static_assert(kItems <= 65535, "per-wave counts and prefixes fit 16 bits");
  const uint32_t radix = 1u << bits, mask = radix - 1u;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint64_t* match = L.match + (size_t)wave * (1u << RB);
  for (uint32_t d = lane; d < radix; d += 64) match[d] = 0ull;
  const uint64_t lane_bit = 1ull << lane;
  uint32_t my_rank[IPT];
  for (int it = 0; it < IPT; ++it) {
    const uint32_t e = wave * kPerWave + it * 64 + lane;
    const bool valid = e < nvalid;
    const uint32_t digit = ((my_key[it] - key_bias) >> shift) & mask;
    // lanes with the same digit: each lane sets its bit in its digit's mask,
    // reads the mask back once every lane has set its bit, and clears it
    // once every lane has read it
    wave_sync();
    if (valid) __hip_atomic_fetch_or(&match[digit], lane_bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    wave_sync();
    const uint64_t peers = valid ? match[digit] : 0ull;
    wave_sync();
    if (valid) match[digit] = 0ull;
    uint32_t rank = 0xFFFFFFFFu;
    if (valid) {
      const uint32_t before = L.wave_count[wave][digit];
      rank = before + popc_below(peers);
      // the highest peer lane publishes the new count
      const uint32_t last_lane = 63u - (uint32_t)__builtin_clzll(peers);
      if (lane == last_lane) L.wave_count[wave][digit] = (uint16_t)(before + (uint32_t)__builtin_popcountll(peers));
    }
    my_rank[it] = rank;
  }
  __syncthreads();
  // per digit: exclusive prefix over waves, block count, local and global
  // starts; thread t owns digits 2t and 2t+1
  uint32_t dcount[2] = {0u, 0u}, gstart[2] = {0u, 0u};
  for (int q = 0; q < 2; ++q) {
    const uint32_t d = 2u * threadIdx.x + q;
    if (d < radix) {
      for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = L.wave_count[w][d];
        L.wave_count[w][d] = (uint16_t)dcount[q];
        dcount[q] += c;
      }
      gstart[q] = scanned_hist[d * nblocks + chunk];
    }
  }
  uint32_t total;
  const uint32_t ls = block_exclusive_scan(dcount[0] + dcount[1], L.smem, total);
  const uint32_t lstart[2] = {ls, ls + dcount[0]};
  for (int q = 0; q < 2; ++q)
    if (2u * threadIdx.x + q < radix) L.start[2u * threadIdx.x + q] = lstart[q];
  __syncthreads();
  for (int it = 0; it < IPT; ++it) {
    if (my_rank[it] == 0xFFFFFFFFu) continue;
    const uint32_t digit = ((my_key[it] - key_bias) >> shift) & mask;
    const uint32_t pos = L.start[digit] + L.wave_count[wave][digit] + my_rank[it];
    stage_keys[pos] = my_key[it];
    for (int q = 0; q < P; ++q) stage_vals[q][pos] = my_val[it][q];
  }
  __syncthreads();
  // item e of the staged block goes to global_start + (e - local_start)
  for (int q = 0; q < 2; ++q)
    if (2u * threadIdx.x + q < radix) L.start[2u * threadIdx.x + q] = gstart[q] - lstart[q];
  __syncthreads();
  for (uint32_t e = threadIdx.x; e < nvalid; e += kBlock) {
    const uint32_t key = stage_keys[e];
    const uint32_t digit = ((key - key_bias) >> shift) & mask;
    const uint32_t dst = L.start[digit] + e;
    if (dst >= out_limit) continue;
    keys_out[dst] = (KO)key;
    for (int q = 0; q < P; ++q) vout.p[q][dst] = stage_vals[q][e];
  }
}

// Stable scatter of one pass; P u32 payload words per key.
// RB: the widest digit this instantiation handles (its LDS tables are 1 << RB
// long, so narrow digits keep the footprint, and the occupancy, of their width)
// KT: the stored type of the input keys (the output keys are uint32_t).
template <int P, int IPT, int RB, class KT = uint32_t>
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(const KT* keys_in, ValPtrs<P> vin,
                                                               uint32_t* keys_out, ValPtrs<P> vout,
                                                               const uint32_t* d_count, uint32_t max_count,
                                                               uint32_t key_bias, int shift, int bits, uint32_t nblocks,
                                                               const uint32_t* scanned_hist) {
  constexpr int kItems = kBlock * IPT;
  constexpr int kPerWave = kItems / kWaves;
  constexpr uint32_t kR = 1u << RB;
  static_assert(kWaves * kR <= (1 + P) * kItems / 2, "the match tables fit in the staging planes");
  __shared__ uint16_t wave_count[kWaves][kR];
  __shared__ uint32_t start[kR];
  __shared__ uint64_t stage[(1 + P) * kItems / 2];  // keys, then the P value planes
  __shared__ uint32_t smem[kWaves + 1];

  const uint32_t count = item_count(d_count, max_count);
  const uint32_t chunk = xcd_chunk(blockIdx.x, nblocks);
  const uint32_t block_base = chunk * kItems;
  if (block_base >= count) return;  // uniform per block
  const uint32_t radix = 1u << bits;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  for (uint32_t d = threadIdx.x; d < radix; d += kBlock) {
    for (int w = 0; w < kWaves; ++w) wave_count[w][d] = 0;
  }
  __syncthreads();

  const uint32_t wave_base = block_base + wave * kPerWave;
  uint32_t my_key[IPT], my_val[IPT][P];
  // every load of the tile is issued before the first one is used
  for (int it = 0; it < IPT; ++it) {
    const uint32_t idx = wave_base + it * 64 + lane;
    const bool valid = idx < count;
    my_key[it] = valid ? (uint32_t)keys_in[idx] : 0u;
    for (int q = 0; q < P; ++q) my_val[it][q] = valid ? vin.p[q][idx] : 0u;
  }
  uint32_t* const stage_keys = reinterpret_cast<uint32_t*>(stage);
  uint32_t* sv[P];
  for (int q = 0; q < P; ++q) sv[q] = stage_keys + (size_t)(1 + q) * kItems;
  const ScatterLds<RB> L{wave_count, start, smem, stage};
  rank_stage_write<P, IPT, RB>(my_key, my_val, min((uint32_t)kItems, count - block_base), key_bias, shift, bits,
                               nblocks, chunk, scanned_hist, L, stage_keys, sv, keys_out, vout, count);
}

// ---- compaction of the visible Gaussians (stable, id order) ----------------
// Also reduces, per block, the tile counts (u64) and the depth-key range of
// the visible entries into block_stats[b] = (sum lo, sum hi, min, max); a
// single-block pass folds them afterwards (thousands of blocks on three
// addresses would serialise as global atomics).
__global__ __launch_bounds__(kBlock) void compact_kernel(const uint32_t* tiles, const uint32_t* depth_keys,
                                                         const uint2* rects, const uint32_t* rowrange, int tight,
                                                         const uint32_t* pos, uint32_t n, uint32_t* keys, uint32_t* ids,
                                                         uint32_t* rx, uint32_t* ry, uint4* block_stats) {
  __shared__ unsigned long long s_k, s_r;
  __shared__ uint32_t s_min, s_max;
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (threadIdx.x == 0) {
    s_k = s_r = 0;
    s_min = 0xFFFFFFFFu;
    s_max = 0u;
  }
  __syncthreads();
  const uint32_t nt = i < n ? tiles[i] : 0u;
  uint32_t kmin = 0xFFFFFFFFu, kmax = 0u, ksum = 0u, rsum = 0u;
  if (nt != 0) {
    const uint32_t p = pos[i];
    const uint2 r = rects[i];
    const uint32_t key = depth_keys[i];
    uint32_t ya = r.x >> 16, yb = r.y >> 16;
    if (tight) {  // the rows from the first to the last with a kept tile
      const uint32_t rr = rowrange[i];
      ya = rr & 0xFFFFu;
      yb = rr >> 16;
    }
    keys[p] = key;
    ids[p] = i;
    rx[p] = (r.x & 0xFFFFu) | (ya << 16);
    ry[p] = (r.y & 0xFFFFu) | (yb << 16);
    kmin = kmax = key;
    ksum = nt;
    rsum = yb - ya;
  }
  unsigned long long k64 = ksum, r64 = rsum;  // u32 per entry: block sums fit 64 bits
  for (int d = 32; d >= 1; d >>= 1) {
    k64 += __shfl_xor(k64, d, 64);
    r64 += __shfl_xor(r64, d, 64);
    kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, d, 64));
    kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, d, 64));
  }
  if ((threadIdx.x & 63) == 0 && k64 != 0) {
    atomicAdd(&s_k, k64);
    atomicAdd(&s_r, r64);
    atomicMin(&s_min, kmin);
    atomicMax(&s_max, kmax);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    block_stats[2 * blockIdx.x] = make_uint4((uint32_t)s_k, (uint32_t)(s_k >> 32), s_min, s_max);
    block_stats[2 * blockIdx.x + 1] = make_uint4((uint32_t)s_r, (uint32_t)(s_r >> 32), 0u, 0u);
  }
}

constexpr int kStatsThreads = 1024;
__global__ __launch_bounds__(kStatsThreads) void stats_reduce_kernel(const uint4* block_stats, uint32_t nblocks,
                                                                     uint32_t* counters) {
  __shared__ unsigned long long s_k, s_r;
  __shared__ uint32_t s_min, s_max;
  if (threadIdx.x == 0) {
    s_k = s_r = 0;
    s_min = 0xFFFFFFFFu;
    s_max = 0u;
  }
  __syncthreads();
  unsigned long long k64 = 0, r64 = 0;
  uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
  auto fold = [&](const uint4& st, const uint4& sr) {
    k64 += (unsigned long long)st.x | ((unsigned long long)st.y << 32);
    r64 += (unsigned long long)sr.x | ((unsigned long long)sr.y << 32);
    kmin = min(kmin, st.z);
    kmax = max(kmax, st.w);
  };
  uint32_t b = threadIdx.x;
  for (; b + 3u * kStatsThreads < nblocks; b += 4u * kStatsThreads) {  // four blocks' loads in flight
    uint4 st[4], sr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      st[q] = block_stats[2 * (b + (uint32_t)q * kStatsThreads)];
      sr[q] = block_stats[2 * (b + (uint32_t)q * kStatsThreads) + 1];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) fold(st[q], sr[q]);
  }
  for (; b < nblocks; b += kStatsThreads) fold(block_stats[2 * b], block_stats[2 * b + 1]);
  for (int d = 32; d >= 1; d >>= 1) {
    k64 += __shfl_xor(k64, d, 64);
    r64 += __shfl_xor(r64, d, 64);
    kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, d, 64));
    kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, d, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&s_k, k64);
    atomicAdd(&s_r, r64);
    atomicMin(&s_min, kmin);
    atomicMax(&s_max, kmax);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    counters[kCountK64] = (uint32_t)s_k;
    counters[kCountK64 + 1] = (uint32_t)(s_k >> 32);
    counters[kCountRows64] = (uint32_t)s_r;
    counters[kCountRows64 + 1] = (uint32_t)(s_r >> 32);
    counters[kCountKeyMin] = s_min;
    counters[kCountKeyMax] = s_max;
  }
}

// ---- duplication: one pair per (Gaussian, covered tile) --------------------
// Balanced by output: block b owns the kDupItems output slots from
// b * kDupItems on -- the items of radix block b of the tile sort's first
// pass -- whatever Gaussians they belong to, so the near, large splats at the
// front of the depth order do not pile up in a few blocks.  The duplication
// is fused with that first pass: a histogram kernel counts each block's
// first digits from the rows alone, a scan of those counts gives every
// block's starts, and the duplication block then generates its pairs in
// LDS, ranks them by the digit and writes them straight to their places
// after the pass.  The pairs in slot order never go through memory.

struct TileMap {
  int32_t count;                     // views
  uint32_t n;                        // Gaussians per view (ids are view * n + Gaussian)
  uint32_t tile_base[kMaxViews];
  uint32_t tiles_x[kMaxViews];
};

__device__ inline void view_of(const TileMap& m, uint32_t id, uint32_t& base, uint32_t& tx) {
  const uint32_t v = m.count > 1 ? id / m.n : 0u;
  base = m.tile_base[v];
  tx = m.tiles_x[v];
}

__device__ inline uint32_t pad_index(uint32_t e) { return e + (e >> 5); }  // one pad word per 32

// Rows to bin (see launch_rows): a block takes kRowsPerBlock consecutive
// rows, four per thread, strided so that the stores coalesce.  They belong
// to at most kRowsPerBlock entries (each entry has at least one row), whose
// row bases the block copies to LDS for short binary searches; the row scan
// recorded the block's first entry, so no search runs in memory.
__global__ __launch_bounds__(kBlock) void rows_kernel(const uint32_t* ids, const uint32_t* rx, const uint32_t* ry,
                                                      const uint32_t* row_base, const uint32_t* first_entry,
                                                      uint32_t V, uint32_t R,
                                                      const float4* splats, int tight, uint32_t* row_cnt,
                                                      uint32_t* row_g, uint32_t* row_yc, uint32_t* block_pairs) {
  __shared__ uint32_t s_base[kRowsPerBlock];
  __shared__ uint32_t s_first, s_count, s_sum;
  const uint32_t t0 = blockIdx.x * kRowsPerBlock;
  const uint32_t t1 = min(t0 + (uint32_t)kRowsPerBlock, R);
  if (threadIdx.x == 0) {
    // the entries of this block's rows: from the entry of its first row to,
    // at most, the entry of the next block's first row (recorded by the row
    // scan)
    const uint32_t first = first_entry[blockIdx.x];
    const uint32_t last = t1 < R ? first_entry[blockIdx.x + 1] : V - 1u;
    s_first = first;
    s_count = min(last - first + 1u, (uint32_t)kRowsPerBlock);
    s_sum = 0u;
  }
  __syncthreads();
  const uint32_t first = s_first, m = s_count;
  for (uint32_t k = threadIdx.x; k < m; k += kBlock) s_base[k] = row_base[first + k];
  __syncthreads();
  uint32_t kept = 0u;
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const uint32_t t = t0 + (uint32_t)q * kBlock + threadIdx.x;
    if (t >= t1) break;
    uint32_t lo = 0, hi = m;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_base[mid] <= t) lo = mid; else hi = mid;
    }
    const uint32_t j = first + lo;
    const uint32_t g = ids[j], a = rx[j], b = ry[j];
    const int x0 = (int)(a & 0xFFFFu), x1 = (int)(b & 0xFFFFu);
    const int y = (int)(a >> 16) + (int)(t - s_base[lo]);
    int c0 = x0, c1 = x1;
    if (tight) reach_row(splat_reach(splats[2 * (size_t)g], splats[2 * (size_t)g + 1]), y, x0, x1, c0, c1);
    row_cnt[t] = (uint32_t)(c1 - c0);
    row_g[t] = g;
    row_yc[t] = ((uint32_t)y << 16) | (uint32_t)c0;
    kept += (uint32_t)(c1 - c0);
  }
  // the block's pair count, which the row-count scan adds up instead of
  // reading the counts twice
  for (int d = 32; d >= 1; d >>= 1) kept += __shfl_xor(kept, d, 64);
  if ((threadIdx.x & 63u) == 0u) atomicAdd(&s_sum, kept);
  __syncthreads();
  if (threadIdx.x == 0) block_pairs[blockIdx.x] = s_sum;
}

// First digit of the tile sort (digit_bits low key bits) for the pairs of
// each duplication block, from the rows alone: the slots of one row hold
// consecutive tile keys, so a row's part of a block adds n >> digit_bits to
// every digit and one to each of the n mod radix digits from its first key's
// on (cyclically).  One wave per duplication block keeps a difference array
// over the digits in LDS; hist[d * nblocks + b] = block b's count of digit d.
constexpr int kDupHistRows = 4;  // rows each lane loads before it counts them
__global__ __launch_bounds__(kBlock) void dup_hist_kernel(const uint32_t* row_off, const uint32_t* row_g,
                                                          const uint32_t* row_yc, const uint32_t* first_row,
                                                          uint32_t R, uint32_t K, TileMap map, int digit_bits,
                                                          uint32_t nblocks, uint32_t* hist) {
  __shared__ uint32_t s_diff[kWaves][kRadix + 1];
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  const uint32_t db = blockIdx.x * kWaves + wave;  // this wave's duplication block
  if (db >= nblocks) return;  // uniform per wave; no block barrier below
  uint32_t* diff = s_diff[wave];
  const uint32_t radix = 1u << digit_bits, mask = radix - 1u;
  const uint32_t o_begin = db * kDupItems;
  const uint32_t o_end = min(o_begin + (uint32_t)kDupItems, K);
  for (uint32_t d = lane; d <= radix; d += 64) diff[d] = 0u;
  // the rows from the one holding the block's first slot to the one holding
  // the next block's first slot (the row-count scan recorded both)
  const uint32_t first = first_row[db];
  const uint32_t last = o_end < K ? first_row[db + 1] : R - 1u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t full = 0u;
  for (uint32_t r0 = first; r0 <= last; r0 += 64u * kDupHistRows) {
    uint32_t off[kDupHistRows], next[kDupHistRows], g[kDupHistRows], yc[kDupHistRows];
#pragma unroll
    for (int j = 0; j < kDupHistRows; ++j) {  // every load before the first use
      const uint32_t r = r0 + (uint32_t)j * 64u + lane;
      const bool in = r <= last;
      off[j] = in ? row_off[r] : 0u;
      next[j] = in ? (r + 1u < R ? row_off[r + 1u] : K) : 0u;
      g[j] = in ? row_g[r] : 0u;
      yc[j] = in ? row_yc[r] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kDupHistRows; ++j) {
      const uint32_t a = max(off[j], o_begin), e = min(next[j], o_end);
      if (e <= a) continue;  // past the block's rows, no kept tile, or none in this block
      uint32_t tbase, tiles_x;
      view_of(map, g[j], tbase, tiles_x);
      const uint32_t key0 = tbase + (yc[j] >> 16) * tiles_x + (yc[j] & 0xFFFFu) + (a - off[j]);
      const uint32_t n = e - a, rem = n & mask, d0 = key0 & mask;
      full += n >> digit_bits;
      if (rem != 0u) {  // digits d0 .. d0 + rem - 1, modulo radix (differences wrap as u32)
        atomicAdd(&diff[d0], 1u);
        if (d0 + rem <= radix) {
          atomicSub(&diff[d0 + rem], 1u);
        } else {
          atomicSub(&diff[radix], 1u);
          atomicAdd(&diff[0], 1u);
          atomicSub(&diff[d0 + rem - radix], 1u);
        }
      }
    }
  }
  for (int d = 32; d >= 1; d >>= 1) full += __shfl_xor(full, d, 64);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // lane l: digits l * per .. l * per + per - 1, per = ceil(radix / 64) <= 8
  const uint32_t per = (radix + 63u) / 64u;
  uint32_t v[8], sum = 0u;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t d = lane * per + (uint32_t)k;
    v[k] = ((uint32_t)k < per && d < radix) ? diff[d] : 0u;
    sum += v[k];
  }
  uint32_t incl = sum;
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= (uint32_t)d) incl += y;
  }
  uint32_t run = incl - sum + full;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t d = lane * per + (uint32_t)k;
    run += v[k];
    if ((uint32_t)k < per && d < radix) hist[d * nblocks + db] = run;
  }
}

// Pairs of one duplication block (logical block chunk = xcd_chunk of the
// hardware block, so that neighbouring blocks, whose output runs interleave
// after the pass, share an XCD's L2).  The block's rows (from the one
// holding its first slot to the one holding the next block's first slot)
// are dealt to the threads, kDupGenRows at a time per thread with every load
// issued first; a thread writes the slots of its rows that fall in the block
// into LDS, in slot order.  The waves then take the pairs in slot order and
// scatter them by the first digit as a radix block does.
constexpr int kDupGenRows = 4;
// KO: the stored key type of the output (uint16_t when a later pass reads
// the keys and the tile ids fit 16 bits).
template <int RB, class KO>
__global__ __launch_bounds__(kBlock) void dup_scatter_kernel(const uint32_t* row_off, const uint32_t* row_g,
                                                             const uint32_t* row_yc, const uint32_t* first_row,
                                                             uint32_t R, uint32_t K, TileMap map, int digit_bits,
                                                             uint32_t nblocks, const uint32_t* scanned_hist,
                                                             KO* out_keys, uint32_t* out_vals) {
  constexpr int kPerWave = kDupItems / kWaves;
  // pairs in slot order (keys, then ids; one pad word per 32), then the
  // scatter's match tables and staging planes
  constexpr int kPadded = kDupItems + kDupItems / 32;
  static_assert(kPadded % 2 == 0 && kWaves * (1 << RB) <= kPadded, "the match tables fit");
  __shared__ uint64_t s_kv[kPadded];
  uint32_t* const s_keys = reinterpret_cast<uint32_t*>(s_kv);
  uint32_t* const s_vals = s_keys + kPadded;
  __shared__ uint16_t wave_count[kWaves][1 << RB];
  __shared__ uint32_t start[1 << RB];
  __shared__ uint32_t smem[kWaves + 1];
  const uint32_t chunk = xcd_chunk(blockIdx.x, nblocks);
  const uint32_t o_begin = chunk * kDupItems;
  const uint32_t o_end = min(o_begin + (uint32_t)kDupItems, K);
  const uint32_t radix = 1u << digit_bits;
  for (uint32_t d = threadIdx.x; d < radix; d += kBlock)
    for (int w = 0; w < kWaves; ++w) wave_count[w][d] = 0;
  // the rows that hold this block's pairs run from the row of its first pair
  // to, at most, the row of the next block's first pair (the scan of the row
  // counts recorded both)
  const uint32_t first = first_row[chunk];
  const uint32_t last = o_end < K ? first_row[chunk + 1] : R - 1u;
  for (uint32_t r0 = first; r0 <= last; r0 += kBlock * kDupGenRows) {
    uint32_t off[kDupGenRows], next[kDupGenRows], g[kDupGenRows], yc[kDupGenRows];
#pragma unroll
    for (int j = 0; j < kDupGenRows; ++j) {
      const uint32_t r = r0 + (uint32_t)j * kBlock + threadIdx.x;
      const bool in = r <= last;
      off[j] = in ? row_off[r] : 0u;
      next[j] = in ? (r + 1u < R ? row_off[r + 1u] : K) : 0u;
      g[j] = in ? row_g[r] : 0u;
      yc[j] = in ? row_yc[r] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kDupGenRows; ++j) {
      const uint32_t a = max(off[j], o_begin), e = min(next[j], o_end);
      if (e <= a) continue;  // past the block's rows, no kept tile, or none in this block
      uint32_t tbase, tiles_x;
      view_of(map, g[j], tbase, tiles_x);
      const uint32_t key0 = tbase + (yc[j] >> 16) * tiles_x + (yc[j] & 0xFFFFu) - off[j];
      for (uint32_t o = a; o < e; ++o) {
        const uint32_t el = pad_index(o - o_begin);
        s_keys[el] = key0 + o;
        s_vals[el] = g[j];
      }
    }
  }
  __syncthreads();
  const uint32_t cnt = o_end - o_begin;
  const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t my_key[kDupIpt], my_val[kDupIpt][1];
  for (int it = 0; it < kDupIpt; ++it) {
    const uint32_t e = wave * kPerWave + it * 64 + lane;
    my_key[it] = e < cnt ? s_keys[pad_index(e)] : 0u;
    my_val[it][0] = e < cnt ? s_vals[pad_index(e)] : 0u;
  }
  __syncthreads();  // the match tables and staging planes reuse s_kv
  uint32_t* const sv[1] = {s_vals};
  const ScatterLds<RB> L{wave_count, start, smem, s_kv};
  ValPtrs<1> vout;
  vout.p[0] = out_vals;
  rank_stage_write<1, kDupIpt, RB, KO>(my_key, my_val, cnt, 0u, 0, digit_bits, nblocks, chunk, scanned_hist, L,
                                        s_keys, sv, out_keys, vout, K);
}

// ranges[t].x = first index whose key >= t (so ranges[t].y = ranges[t+1].x):
// one wave per boundary, a 64-ary search of the sorted keys.
__global__ __launch_bounds__(kBlock) void ranges_kernel(const uint32_t* keys, uint32_t K, uint32_t ntiles,
                                                        uint2* ranges) {
  const uint32_t t = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);  // boundary: first key >= t
  const uint32_t lane = threadIdx.x & 63u;
  if (t > ntiles) return;  // uniform per wave
  uint32_t lo = 0, hi = K;  // answer in [lo, hi]
  while (hi - lo > 0) {
    const uint32_t span = hi - lo;
    const uint32_t step = (span + 63u) / 64u;
    const uint32_t idx = lo + lane * step;
    const bool below = idx < hi && keys[idx] < t;  // probes are increasing in lane
    const uint64_t m = __ballot(below);
    const uint32_t nb = (uint32_t)__builtin_popcountll(m);  // probes below t form a prefix
    if (nb == 0) {
      hi = lo;
    } else {
      const uint32_t last_below = lo + (nb - 1) * step;
      lo = last_below + 1;
      hi = min(hi, last_below + step);
    }
  }
  if (lane == 0) {
    if (t < ntiles) ranges[t].x = lo;
    if (t > 0) ranges[t - 1].y = lo;
  }
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t* p, uint32_t v, uint32_t count) {
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < count) p[j] = v;
}

// 16 bytes per thread for a 16-byte aligned array; count4 groups of four
__global__ __launch_bounds__(kBlock) void fill_u32x4_kernel(uint4* p, uint32_t v, uint32_t count4) {
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < count4) p[j] = make_uint4(v, v, v, v);
}

// p[0 .. count) = 0 except p[at] = v
__global__ __launch_bounds__(kBlock) void fill_u32_but_one_kernel(uint32_t* p, uint32_t count, uint32_t at,
                                                                  uint32_t v) {
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j < count) p[j] = j == at ? v : 0u;
}

template <int P, int IPT>
hipError_t radix_sort_impl(const RadixBuffers& B, const uint32_t* d_count, int64_t max_count, int bits,
                           uint32_t* hist, uint32_t* partials, hipStream_t s, int hist_id, int scatter_id,
                           int first_pass, uint32_t key_bias) {
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
    if (p < first_pass) {  // done by the caller: the keys in *_a are in this pass's order
      shift += pb;
      continue;
    }
    // the first pass that runs may read 16-bit keys (the caller's, see
    // RadixBuffers::keys16); every pass writes 32-bit keys
    const bool k16 = P == 1 && B.keys16 && p == first_pass;
    {
      ProfScope prof(s, hist_id);
      if (k16)
        hipLaunchKernelGGL((radix_hist_kernel<IPT, uint16_t>), dim3(nb), dim3(kBlock), 0, s,
                           reinterpret_cast<const uint16_t*>(ki), d_count, (uint32_t)max_count, key_bias, shift, pb,
                           nb, hist);
      else
        hipLaunchKernelGGL((radix_hist_kernel<IPT>), dim3(nb), dim3(kBlock), 0, s, ki, d_count, (uint32_t)max_count,
                           key_bias, shift, pb, nb, hist);
    }
    hipError_t e = launch_scan(hist, nullptr, nullptr, (int64_t)nb << pb, kScanPlain, partials, nullptr, hist, s);
    if (e != hipSuccess) return e;
    {
      ProfScope prof(s, scatter_id);
      auto scatter32 = [&]() {
        if (pb <= 7)
          hipLaunchKernelGGL((radix_scatter_kernel<P, IPT, 7>), dim3(nb), dim3(kBlock), 0, s, ki, vi, ko, vo, d_count,
                             (uint32_t)max_count, key_bias, shift, pb, nb, hist);
        else if (pb == 8)
          hipLaunchKernelGGL((radix_scatter_kernel<P, IPT, 8>), dim3(nb), dim3(kBlock), 0, s, ki, vi, ko, vo, d_count,
                             (uint32_t)max_count, key_bias, shift, pb, nb, hist);
        else
          hipLaunchKernelGGL((radix_scatter_kernel<P, IPT, kRadixBits>), dim3(nb), dim3(kBlock), 0, s, ki, vi, ko,
                             vo, d_count, (uint32_t)max_count, key_bias, shift, pb, nb, hist);
      };
      if constexpr (P == 1) {
        const uint16_t* k16i = reinterpret_cast<const uint16_t*>(ki);
        if (k16 && pb <= 7)
          hipLaunchKernelGGL((radix_scatter_kernel<1, IPT, 7, uint16_t>), dim3(nb), dim3(kBlock), 0, s, k16i, vi, ko,
                             vo, d_count, (uint32_t)max_count, key_bias, shift, pb, nb, hist);
        else if (k16)  // 16-bit ids: the second of two passes has at most 8 bits
          hipLaunchKernelGGL((radix_scatter_kernel<1, IPT, 8, uint16_t>), dim3(nb), dim3(kBlock), 0, s, k16i, vi, ko,
                             vo, d_count, (uint32_t)max_count, key_bias, shift, pb, nb, hist);
        else
          scatter32();
      } else {
        scatter32();
      }
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

hipError_t launch_clear_but_one(uint32_t* p, int64_t count, int64_t at, uint32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  ProfScope prof(s, kKFill);
  hipLaunchKernelGGL(fill_u32_but_one_kernel, dim3((unsigned)ceil_div(count, kBlock)), dim3(kBlock), 0, s, p,
                     (uint32_t)count, (uint32_t)at, v);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  ProfScope prof(s, kKFill);
  const int64_t c4 = (reinterpret_cast<uintptr_t>(p) & 15u) == 0 ? count / 4 : 0;
  if (c4 > 0)
    hipLaunchKernelGGL(fill_u32x4_kernel, dim3((unsigned)ceil_div(c4, kBlock)), dim3(kBlock), 0, s,
                       reinterpret_cast<uint4*>(p), v, (uint32_t)c4);
  const int64_t rest = count - 4 * c4;
  if (rest > 0)
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)ceil_div(rest, kBlock)), dim3(kBlock), 0, s, p + 4 * c4, v,
                       (uint32_t)rest);
  return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* in_a, const uint32_t* in_b, const uint32_t* d_count, int64_t max_count,
                       int mode, uint32_t* partials, uint32_t* total, uint32_t* out, hipStream_t s, uint32_t* aux,
                       uint32_t aux_block) {
  if (max_count <= 0) return total ? launch_fill_u32(total, 0u, 1, s) : hipSuccess;
  if (aux && aux_block == 0) return hipErrorInvalidValue;
  const uint32_t nb = (uint32_t)ceil_div(max_count, kItemsPerBlock);
  const ScanIn in{in_a, in_b, aux, aux_block};
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
    case kScanGather:
      hipLaunchKernelGGL(scan_partials_kernel<kScanGather>, dim3(nb), dim3(kBlock), 0, s, in, d_count,
                         (uint32_t)max_count, partials);
      break;
    case kScanRows:
      hipLaunchKernelGGL(scan_partials_kernel<kScanRows>, dim3(nb), dim3(kBlock), 0, s, in, d_count,
                         (uint32_t)max_count, partials);
      break;
    case kScanPlain:
      hipLaunchKernelGGL(scan_partials_kernel<kScanPlain>, dim3(nb), dim3(kBlock), 0, s, in, d_count,
                         (uint32_t)max_count, partials);
      break;
    default:
      return hipErrorInvalidValue;
  }
  const bool fused = nb <= kMaxFusedPartials;
  if (!fused) hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kBlock), 0, s, partials, nb, total);
#define FGS_APPLY(M)                                                                                            \
  if (fused)                                                                                                     \
    hipLaunchKernelGGL((scan_apply_kernel<M, true>), dim3(nb), dim3(kBlock), 0, s, in, out, d_count,            \
                       (uint32_t)max_count, partials, total);                                                    \
  else                                                                                                           \
    hipLaunchKernelGGL((scan_apply_kernel<M, false>), dim3(nb), dim3(kBlock), 0, s, in, out, d_count,           \
                       (uint32_t)max_count, partials, total);
  switch (mode) {
    case kScanFlag: FGS_APPLY(kScanFlag) break;
    case kScanRectArea: FGS_APPLY(kScanRectArea) break;
    case kScanGather: FGS_APPLY(kScanGather) break;
    case kScanRows: FGS_APPLY(kScanRows) break;
    default: FGS_APPLY(kScanPlain) break;
  }
#undef FGS_APPLY
  return hipGetLastError();
}

hipError_t launch_scan_from_parts(const uint32_t* in_a, int mode, int64_t max_count, const uint32_t* parts,
                                  int64_t part_items, uint32_t* total, uint32_t* out, hipStream_t s, uint32_t* aux,
                                  uint32_t aux_block) {
  if (max_count <= 0) return total ? launch_fill_u32(total, 0u, 1, s) : hipSuccess;
  if (part_items <= 0 || kItemsPerBlock % part_items != 0 || ceil_div(max_count, part_items) > kMaxPartsScan ||
      (mode != kScanFlag && mode != kScanPlain) || (aux && aux_block == 0))
    return hipErrorInvalidValue;
  const uint32_t nb = (uint32_t)ceil_div(max_count, kItemsPerBlock);
  const uint32_t per = (uint32_t)(kItemsPerBlock / part_items);
  const ScanIn in{in_a, nullptr, aux, aux_block};
  ProfScope prof(s, kKScan);
  if (mode == kScanFlag)
    hipLaunchKernelGGL((scan_apply_kernel<kScanFlag, true>), dim3(nb), dim3(kBlock), 0, s, in, out, nullptr,
                       (uint32_t)max_count, parts, total, per);
  else
    hipLaunchKernelGGL((scan_apply_kernel<kScanPlain, true>), dim3(nb), dim3(kBlock), 0, s, in, out, nullptr,
                       (uint32_t)max_count, parts, total, per);
  return hipGetLastError();
}

int radix_passes(int bits) { return bits <= 0 ? 0 : (bits + kRadixBits - 1) / kRadixBits; }

int64_t radix_blocks(int64_t max_count, int payload) {
  return ceil_div(max_count, (int64_t)kBlock * (payload == 1 ? kIptPayload1 : kIptPayload3));
}

hipError_t launch_radix_sort(const RadixBuffers& B, const uint32_t* d_count, int64_t max_count, int bits,
                             uint32_t* hist, uint32_t* partials, hipStream_t s, int hist_id, int scatter_id,
                             int first_pass, uint32_t key_bias) {
  if (max_count <= 0 || radix_passes(bits) <= first_pass) return hipSuccess;
  if (B.payload == 1)
    return radix_sort_impl<1, kIptPayload1>(B, d_count, max_count, bits, hist, partials, s, hist_id, scatter_id,
                                            first_pass, key_bias);
  return radix_sort_impl<3, kIptPayload3>(B, d_count, max_count, bits, hist, partials, s, hist_id, scatter_id,
                                          first_pass, key_bias);
}

hipError_t launch_compact(const uint32_t* tiles, const uint32_t* depth_keys, const uint2* rects,
                          const uint32_t* rowrange, bool tight, const uint32_t* pos, int64_t n, uint32_t* keys,
                          uint32_t* ids, uint32_t* rx, uint32_t* ry, uint32_t* counters, uint4* block_stats,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  ProfScope prof(s, kKCompact);
  const unsigned blocks = (unsigned)ceil_div(n, kBlock);
  hipLaunchKernelGGL(compact_kernel, dim3(blocks), dim3(kBlock), 0, s, tiles, depth_keys, rects, rowrange, tight ? 1 : 0,
                     pos, (uint32_t)n, keys, ids, rx, ry, block_stats);
  hipLaunchKernelGGL(stats_reduce_kernel, dim3(1), dim3(kStatsThreads), 0, s, block_stats, blocks, counters);
  return hipGetLastError();
}

hipError_t launch_rows(const uint32_t* ids, const uint32_t* rx, const uint32_t* ry, const uint32_t* row_base,
                       const uint32_t* first_entry, int64_t V, int64_t R, const float4* splats, bool tight,
                       uint32_t* row_cnt, uint32_t* row_g, uint32_t* row_yc, uint32_t* block_pairs, hipStream_t s) {
  if (V <= 0 || R <= 0) return hipSuccess;
  ProfScope prof(s, kKRows);
  hipLaunchKernelGGL(rows_kernel, dim3((unsigned)ceil_div(R, kRowsPerBlock)), dim3(kBlock), 0, s, ids, rx, ry, row_base,
                     first_entry,
                     (uint32_t)V, (uint32_t)R, splats, tight ? 1 : 0, row_cnt, row_g, row_yc, block_pairs);
  return hipGetLastError();
}

bool tile_keys16(int tile_bits) { return radix_passes(tile_bits) == 2 && tile_bits <= 16; }

hipError_t launch_duplicate_sorted(const uint32_t* row_off, const uint32_t* row_g, const uint32_t* row_yc,
                                   const uint32_t* first_row, int64_t R, int64_t K, const ViewBatch& b, int64_t n,
                                   int tile_bits, uint32_t* hist, uint32_t* partials, uint32_t* out_keys,
                                   uint32_t* out_vals, hipStream_t s) {
  if (R <= 0 || K <= 0) return hipSuccess;
  const int passes = radix_passes(tile_bits);
  const int first_bits = passes > 0 ? (tile_bits + passes - 1) / passes : 0;  // as launch_radix_sort
  const uint32_t nb = (uint32_t)ceil_div(K, kDupItems);
  TileMap map;
  map.count = b.count;
  map.n = (uint32_t)n;
  for (int v = 0; v < kMaxViews; ++v) {
    map.tile_base[v] = v < b.count ? b.v[v].tile_base : 0u;
    map.tiles_x[v] = v < b.count ? (uint32_t)b.v[v].tiles_x : 1u;
  }
  {
    ProfScope prof(s, kKDupHist);
    hipLaunchKernelGGL(dup_hist_kernel, dim3((unsigned)ceil_div(nb, kWaves)), dim3(kBlock), 0, s, row_off, row_g,
                       row_yc, first_row, (uint32_t)R, (uint32_t)K, map, first_bits, nb, hist);
  }
  hipError_t e = launch_scan(hist, nullptr, nullptr, (int64_t)nb << first_bits, kScanPlain, partials, nullptr, hist, s);
  if (e != hipSuccess) return e;
  ProfScope prof(s, kKDuplicate);
  uint16_t* const out16 = reinterpret_cast<uint16_t*>(out_keys);
  const bool k16 = tile_keys16(tile_bits);
#define FGS_DUP(RB)                                                                                             \
  if (k16)                                                                                                       \
    hipLaunchKernelGGL((dup_scatter_kernel<RB, uint16_t>), dim3(nb), dim3(kBlock), 0, s, row_off, row_g, row_yc, \
                       first_row, (uint32_t)R, (uint32_t)K, map, first_bits, nb, hist, out16, out_vals);        \
  else                                                                                                           \
    hipLaunchKernelGGL((dup_scatter_kernel<RB, uint32_t>), dim3(nb), dim3(kBlock), 0, s, row_off, row_g, row_yc, \
                       first_row, (uint32_t)R, (uint32_t)K, map, first_bits, nb, hist, out_keys, out_vals);
  if (first_bits <= 7) {
    FGS_DUP(7)
  } else if (first_bits == 8) {
    FGS_DUP(8)
  } else {
    FGS_DUP(kRadixBits)
  }
#undef FGS_DUP
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* sorted_keys, int64_t K, uint2* ranges, int32_t ntiles, hipStream_t s) {
  if (K <= 0) return launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * (int64_t)ntiles, s);
  const int waves_per_block = kBlock / 64;
  ProfScope prof(s, kKRanges);
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)ceil_div((int64_t)ntiles + 1, waves_per_block)), dim3(kBlock), 0, s,
                     sorted_keys, (uint32_t)K, (uint32_t)ntiles, ranges);
  return hipGetLastError();
}

}  // namespace fgs
