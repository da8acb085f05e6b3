// Spatial order of a resident scene: Gaussians sorted by the Morton code of
// their mean, and a gather that applies such an order to parameter planes.
//
// A view culls whole regions of space (the cone behind a fisheye, what falls
// outside the image), so in an order where neighbours in space are
// neighbours in memory the culled Gaussians come in long runs: the forward
// skips their SH coefficients line by line instead of fetching every line
// for its few visible members, and the Gaussians of one tile list sit closer
// together.  The order is a permutation of the scene: images and gradients
// are the same up to the order of depth ties, which the sort breaks by id.
#include <algorithm>

#include "fgs_internal.hpp"

namespace fgs {
namespace {

// Float bits mapped to uint32 so that unsigned order is float order.
__device__ inline uint32_t ordered_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float from_ordered_bits(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// box[0..2] min, box[3..5] max of the finite means (ordered bits; the caller
// sets min to all ones and max to zero first).
__global__ __launch_bounds__(kBlock) void bounds_kernel(const float* means, uint32_t n, uint32_t* box) {
  __shared__ uint32_t s[6];
  if (threadIdx.x < 6) s[threadIdx.x] = threadIdx.x < 3 ? 0xFFFFFFFFu : 0u;
  __syncthreads();
  uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const float x[3] = {means[i], means[n + i], means[2 * (size_t)n + i]};
    if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) continue;
    for (int a = 0; a < 3; ++a) {
      const uint32_t b = ordered_bits(x[a]);
      lo[a] = min(lo[a], b);
      hi[a] = max(hi[a], b);
    }
  }
  for (int a = 0; a < 3; ++a) {
    for (int d = 32; d >= 1; d >>= 1) {
      lo[a] = min(lo[a], (uint32_t)__shfl_xor((int)lo[a], d, 64));
      hi[a] = max(hi[a], (uint32_t)__shfl_xor((int)hi[a], d, 64));
    }
  }
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) {
      atomicMin(&s[a], lo[a]);
      atomicMax(&s[3 + a], hi[a]);
    }
  __syncthreads();
  if (threadIdx.x < 3) atomicMin(&box[threadIdx.x], s[threadIdx.x]);
  else if (threadIdx.x < 6) atomicMax(&box[threadIdx.x], s[threadIdx.x]);
}

__device__ inline uint32_t spread10(uint32_t v) {  // bits b0..b9 to b0, b3, ..., b27
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// 30-bit Morton code of each mean on a 1024^3 grid over the box; a
// non-finite mean gets the largest code.  ids[i] = i.
__global__ __launch_bounds__(kBlock) void morton_kernel(const float* means, uint32_t n, const uint32_t* box,
                                                        uint32_t* codes, uint32_t* ids) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float x[3] = {means[i], means[n + i], means[2 * (size_t)n + i]};
  uint32_t code = (1u << 30) - 1u;
  if (isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2])) {
    code = 0;
    for (int a = 0; a < 3; ++a) {
      const float lo = from_ordered_bits(box[a]), hi = from_ordered_bits(box[3 + a]);
      const float ext = hi - lo;
      const float u = ext > 0.0f ? (x[a] - lo) / ext : 0.0f;
      const uint32_t q = (uint32_t)fminf(fmaxf(u * 1024.0f, 0.0f), 1023.0f);
      code |= spread10(q) << (2 - a);
    }
  }
  codes[i] = code;
  ids[i] = i;
}

// out[p][j] = in[p][order[j]] for planes p of length n.
__global__ __launch_bounds__(kBlock) void gather_planes_kernel(const float* in, float* out, uint32_t planes,
                                                               uint32_t n, const uint32_t* order) {
  const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  const uint32_t src = order[j];
  for (uint32_t p = 0; p < planes; ++p) out[(size_t)p * n + j] = in[(size_t)p * n + src];
}

}  // namespace

size_t spatial_order_workspace(int64_t n) {
  const int64_t nn = n > 0 ? n : 1;
  const int64_t nb = radix_blocks(nn, 1);
  const size_t a = 256;
  auto up = [&](size_t x) { return (x + a - 1) / a * a; };
  return up(6 * 4) + 3 * up((size_t)nn * 4) + up((size_t)nb * kRadix * 4) +
         up((size_t)(ceil_div(std::max<int64_t>(nn, nb * kRadix), kItemsPerBlock) + 1) * 4);
}

hipError_t launch_spatial_order(const float* means, int64_t n, uint32_t* order, char* ws, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = radix_blocks(n, 1);
  const size_t a = 256;
  auto up = [&](size_t x) { return (x + a - 1) / a * a; };
  uint32_t* box = reinterpret_cast<uint32_t*>(ws);
  size_t off = up(6 * 4);
  uint32_t* codes_a = reinterpret_cast<uint32_t*>(ws + off);
  off += up((size_t)n * 4);
  uint32_t* codes_b = reinterpret_cast<uint32_t*>(ws + off);
  off += up((size_t)n * 4);
  uint32_t* ids_b = reinterpret_cast<uint32_t*>(ws + off);
  off += up((size_t)n * 4);
  uint32_t* hist = reinterpret_cast<uint32_t*>(ws + off);
  off += up((size_t)nb * kRadix * 4);
  uint32_t* partials = reinterpret_cast<uint32_t*>(ws + off);
  // box: min slots all ones, max slots zero
  hipError_t e = launch_fill_u32(box, 0xFFFFFFFFu, 3, s);
  if (e == hipSuccess) e = launch_fill_u32(box + 3, 0u, 3, s);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)ceil_div(n, kBlock);
  {
    ProfScope prof(s, kKOrder);
    hipLaunchKernelGGL(bounds_kernel, dim3(std::min(blocks, 1024u)), dim3(kBlock), 0, s, means, (uint32_t)n, box);
    hipLaunchKernelGGL(morton_kernel, dim3(blocks), dim3(kBlock), 0, s, means, (uint32_t)n, box, codes_a, order);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // 30 key bits in an even number of passes, so the sorted ids end in `order`
  if (radix_passes(30) % 2 != 0) return hipErrorInvalidValue;
  RadixBuffers B{1, codes_a, codes_b, {order, nullptr, nullptr}, {ids_b, nullptr, nullptr}};
  return launch_radix_sort(B, nullptr, n, 30, hist, partials, s, kKOrder, kKOrder);
}

hipError_t launch_gather_planes(const float* in, float* out, int64_t planes, int64_t n, const uint32_t* order,
                                hipStream_t s) {
  if (n <= 0 || planes <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_planes_kernel, dim3((unsigned)ceil_div(n, kBlock)), dim3(kBlock), 0, s, in, out,
                     (uint32_t)planes, (uint32_t)n, order);
  return hipGetLastError();
}

}  // namespace fgs
