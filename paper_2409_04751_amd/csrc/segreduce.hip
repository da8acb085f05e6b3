// Deterministic reduction of the blend backward's per-Gaussian 2D gradients.
//
// The default backward adds each tile's nine sums for a Gaussian (dL/d of the
// projected mean, the conic, the opacity and the colour; Sec. 4.2, the part
// shared with vanilla splatting) to the Gaussian's accumulators with float
// atomics, so the result depends on the order in which tiles finish.  Here
// the blend backward stores the nine sums of every list entry instead
// (part[e][9], e the entry's position in the tile-sorted list), and this file
// adds them up per Gaussian in a fixed order: the entries are stably sorted by
// Gaussian id (so each Gaussian's entries form one run, in list order), and
// one wave per Gaussian sums its run in an order fixed by the run's length.  The same inputs give
// the same bits on every run; the values differ from the atomic order only by
// the reassociation of the float additions.
#include <algorithm>

#include "fgs_internal.hpp"

namespace fgs {
namespace {

__global__ __launch_bounds__(kBlock) void iota_kernel(uint32_t* p, uint32_t count) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = i;
}

// seg[k] = [first, one past last) position of key k's run in the sorted keys;
// keys without a run keep the (0, 0) the caller stored.
__global__ __launch_bounds__(kBlock) void seg_bounds_kernel(const uint32_t* keys, uint32_t count, uint32_t nkeys,
                                                           uint2* seg) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const uint32_t k = keys[i];
  if (k >= nkeys) return;
  if (i == 0 || keys[i - 1] != k) seg[k].x = i;
  if (i + 1 == count || keys[i + 1] != k) seg[k].y = i + 1;
}

// grad2d[slot(g)][c] = the sum of part[pos][c] over g's run, one wave per
// Gaussian (runs reach thousands of entries for the largest splats, so a
// thread per Gaussian would serialise their loads): lane l adds entries
// l, l + 64, ... in order, then the lanes are added by a fixed butterfly.
// Both orders depend on the run's length only, so the sum is the same on
// every call (every lane ends with the same total: each butterfly step adds
// the same two values in both partner lanes).
constexpr int kReduceWaves = kBlock / 64;

__global__ __launch_bounds__(kBlock) void seg_reduce_kernel(const uint2* seg, const uint32_t* pos, const float* part,
                                                           uint32_t n, float* grad2d) {
  const uint32_t g = blockIdx.x * kReduceWaves + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  if (g >= n) return;  // wave-uniform
  const uint2 r = seg[g];
  float acc[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) acc[c] = 0.0f;
  for (uint32_t k = r.x + lane; k < r.y; k += 64) {
    const float* p = part + (size_t)pos[k] * 9;
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] += p[c];
  }
  float mine = 0.0f;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    float v = acc[c];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == (uint32_t)c) mine = v;
  }
  if (lane < 9u) grad2d[(size_t)grad_slot(g) * 9 + lane] = mine;
}

struct DetLayout {
  size_t part, keys_a, keys_b, vals_a, vals_b, seg, hist, partials, bytes;
};

DetLayout det_layout(int64_t n, int64_t kcap) {
  const int64_t nn = n > 0 ? n : 1, kk = kcap > 0 ? kcap : 1;
  const int64_t nb = radix_blocks(kk, 1);
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  DetLayout d;
  size_t off = 0;  // part first: the blend backward writes it at the scratch's start
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += up(bytes);
    return at;
  };
  d.part = take((size_t)kk * 9 * 4);
  d.keys_a = take((size_t)kk * 4);
  d.keys_b = take((size_t)kk * 4);
  d.vals_a = take((size_t)kk * 4);
  d.vals_b = take((size_t)kk * 4);
  d.seg = take((size_t)nn * 8);
  d.hist = take((size_t)nb * kRadix * 4);
  d.partials = take((size_t)(ceil_div(std::max<int64_t>(kk, nb * kRadix), kItemsPerBlock) + 1) * 4);
  d.bytes = off;
  return d;
}

}  // namespace

size_t det_workspace_bytes(int64_t n, int64_t k_capacity) { return det_layout(n, k_capacity).bytes; }

hipError_t launch_grad_segreduce(const uint32_t* ids, int64_t K, int64_t n, int key_bits, char* dws, size_t dws_bytes,
                                 float* grad2d, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const DetLayout d = det_layout(n, K);
  if (dws_bytes < d.bytes) return hipErrorInvalidValue;
  auto U = [&](size_t off) { return reinterpret_cast<uint32_t*>(dws + off); };
  uint2* seg = reinterpret_cast<uint2*>(dws + d.seg);
  hipError_t e = launch_fill_u32(U(d.seg), 0u, 2 * n, s);
  if (e != hipSuccess) return e;
  const uint32_t* keys = U(d.keys_a);
  const uint32_t* pos = U(d.vals_a);
  if (K > 0) {
    e = hipMemcpyAsync(U(d.keys_a), ids, (size_t)K * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    {
      ProfScope prof(s, kKSegReduce);
      hipLaunchKernelGGL(iota_kernel, dim3((unsigned)ceil_div(K, kBlock)), dim3(kBlock), 0, s, U(d.vals_a),
                         (uint32_t)K);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // stable: each Gaussian's entries keep their list order
    RadixBuffers B{1, U(d.keys_a), U(d.keys_b), {U(d.vals_a), nullptr, nullptr}, {U(d.vals_b), nullptr, nullptr}};
    e = launch_radix_sort(B, nullptr, K, key_bits, U(d.hist), U(d.partials), s, kKSegReduce, kKSegReduce);
    if (e != hipSuccess) return e;
    if (radix_passes(key_bits) % 2 == 1) {
      keys = U(d.keys_b);
      pos = U(d.vals_b);
    }
    ProfScope prof(s, kKSegReduce);
    hipLaunchKernelGGL(seg_bounds_kernel, dim3((unsigned)ceil_div(K, kBlock)), dim3(kBlock), 0, s, keys, (uint32_t)K,
                       (uint32_t)n, seg);
  }
  {
    ProfScope prof(s, kKSegReduce);
    hipLaunchKernelGGL(seg_reduce_kernel, dim3((unsigned)ceil_div(n, kReduceWaves)), dim3(kBlock), 0, s, seg, pos,
                       reinterpret_cast<const float*>(dws + d.part), (uint32_t)n, grad2d);
  }
  return hipGetLastError();
}

}  // namespace fgs
