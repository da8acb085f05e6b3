// Deterministic reduction of the blend backward's per-Gaussian 2D gradients.
//
// The default backward adds each tile's nine sums for a Gaussian (dL/d of the
// projected mean, the conic, the opacity and the colour; Sec. 4.2, the part
// shared with vanilla splatting) to the Gaussian's accumulators with float
// atomics, so the result depends on the order in which tiles finish.  Here
// each Gaussian g owns a run of tiles[g] slots (gauss_off = exclusive scan of
// the tile counts), the blend backward stores the sums of its entry in tile t
// at the slot of t's rank among g's tiles (tile order), and each Gaussian's
// run is added by sixteen lanes (or a whole wave for long runs) in an order
// fixed by the run's length.  The same
// inputs give the same bits on every run; the values differ from the atomic
// order only by the reassociation of the float additions.
#include <algorithm>

#include "fgs_internal.hpp"

namespace fgs {
namespace {

// grad2d[slot(g)][c] = the sum of g's run (tiles[g] slots from gauss_off[g]),
// sixteen lanes per Gaussian (a quarter wave, one row of the DPP
// exchanges), in an order fixed by the run's length: a run of up to
// kLongRun slots is read by its own sixteen lanes, lane j adding slots j,
// j + 16, ... in order (their loads coalesce), then the sixteen partial sums
// are added by a fixed butterfly; a longer run (the largest splats reach
// thousands of tiles) is read by the whole wave, lane l taking slots l,
// l + 64, ..., then a fixed 64-lane butterfly.  In both butterflies every
// lane ends with the same total (each step adds the same two values in both
// partner lanes).
constexpr uint32_t kGroup = 16;
constexpr uint32_t kLongRun = 256;

__global__ __launch_bounds__(kBlock) void seg_reduce_kernel(const uint32_t* tiles, const uint32_t* gauss_off,
                                                           const float* part, uint32_t n, float* grad2d) {
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t g = t / kGroup, sub = t % kGroup, lane = threadIdx.x & 63u;
  const bool live = g < n;
  const uint32_t cnt = live ? tiles[g] : 0u, beg = live ? gauss_off[g] : 0u;
  const bool long_run = cnt > kLongRun;
  float acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = 0.0f;
  if (!long_run)
    for (uint32_t k = beg + sub; k < beg + cnt; k += kGroup) {
      const float* p = part + (size_t)k * 9;
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[c] += p[c];
    }
#pragma unroll
  for (int c = 0; c < 9; ++c)
#pragma unroll
    for (int d = 8; d >= 1; d >>= 1) acc[c] += __shfl_xor(acc[c], d, 64);
  // long runs, one at a time, by the whole wave (the group's lanes all hold
  // the run: take its first lane's)
  uint64_t m = __ballot(long_run && sub == 0u);
  while (m != 0ull) {  // wave-uniform
    const uint32_t l = (uint32_t)__builtin_ctzll(m);
    m &= m - 1ull;
    const uint32_t b = (uint32_t)__shfl((int)beg, (int)l, 64), e = b + (uint32_t)__shfl((int)cnt, (int)l, 64);
    float v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = 0.0f;
    for (uint32_t k = b + lane; k < e; k += 64) {
      const float* p = part + (size_t)k * 9;
#pragma unroll
      for (int c = 0; c < 9; ++c) v[c] += p[c];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) v[c] += __shfl_xor(v[c], d, 64);
      if ((lane & ~(kGroup - 1u)) == l) acc[c] = v[c];
    }
  }
  if (live && sub < 9u) {
    float mine = acc[0];
#pragma unroll
    for (int c = 1; c < 9; ++c)
      if (sub == (uint32_t)c) mine = acc[c];
    grad2d[(size_t)grad_slot(g) * 9 + sub] = mine;
  }
}

struct DetLayout {
  size_t part, off, partials, bytes;
};

DetLayout det_layout(int64_t n, int64_t kcap) {
  const int64_t nn = n > 0 ? n : 1, kk = kcap > 0 ? kcap : 1;
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  DetLayout d;
  size_t off = 0;  // part first: the blend backward writes it at the scratch's start
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += up(bytes);
    return at;
  };
  d.part = take((size_t)kk * 9 * 4);
  d.off = take((size_t)nn * 4);
  d.partials = take((size_t)(ceil_div(nn, kItemsPerBlock) + 1) * 4);
  d.bytes = off;
  return d;
}

}  // namespace

size_t det_workspace_bytes(int64_t n, int64_t k_capacity) { return det_layout(n, k_capacity).bytes; }

uint32_t* det_gauss_off(char* dws, int64_t n, int64_t K) {
  return reinterpret_cast<uint32_t*>(dws + det_layout(n, K).off);
}

hipError_t launch_grad_offsets(const uint32_t* tiles, int64_t n, int64_t K, char* dws, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const DetLayout d = det_layout(n, K);
  return launch_scan(tiles, nullptr, nullptr, n, kScanPlain, reinterpret_cast<uint32_t*>(dws + d.partials), nullptr,
                     reinterpret_cast<uint32_t*>(dws + d.off), s);
}

hipError_t launch_grad_segreduce(const uint32_t* tiles, int64_t n, int64_t K, char* dws, float* grad2d,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n * (int64_t)kGroup > 0xFFFFFFFFll) return hipErrorInvalidValue;  // thread index in 32 bits
  const DetLayout d = det_layout(n, K);
  ProfScope prof(s, kKSegReduce);
  hipLaunchKernelGGL(seg_reduce_kernel, dim3((unsigned)ceil_div(n * (int64_t)kGroup, kBlock)), dim3(kBlock), 0, s,
                     tiles,
                     reinterpret_cast<const uint32_t*>(dws + d.off), reinterpret_cast<const float*>(dws + d.part),
                     (uint32_t)n, grad2d);
  return hipGetLastError();
}

}  // namespace fgs
