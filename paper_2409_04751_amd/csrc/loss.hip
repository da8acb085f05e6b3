// L1 photometric loss of a rendered image against a target and its
// gradient, for the training step: L = mean over the 3 H W values of
// |C - C_target| (the L1 term of the 3DGS objective the paper trains with,
// Sec. 5.1), dL/dC = sign(C - C_target) dL/dL_out / count.
//
// The loss is a two-stage sum (fixed grid of per-block partial sums in
// double, then one block adding them in order), so it is bit-deterministic.
// The gradient is one streaming pass: both images in with 128-bit loads, the
// gradient out.
#include <algorithm>
#include <mutex>

#include "fgs_internal.hpp"

namespace fgs {
namespace {

constexpr int kL1Blocks = FGS_L1_PARTIALS;

__device__ inline double block_sum_f64(double v, double* sh) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kBlock / 64; ++k) s += sh[k];
  return s;
}

__global__ __launch_bounds__(kBlock) void l1_partials_kernel(const float* img, const float* tgt, uint32_t count,
                                                             double* partials) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  const uint32_t n4 = count / 4u;
  const float4* a4 = reinterpret_cast<const float4*>(img);
  const float4* b4 = reinterpret_cast<const float4*>(tgt);
  for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n4; j += gridDim.x * kBlock) {
    const float4 a = a4[j], b = b4[j];
    acc += (double)(fabsf(a.x - b.x) + fabsf(a.y - b.y)) + (double)(fabsf(a.z - b.z) + fabsf(a.w - b.w));
  }
  // the tail past the last whole float4 (count not a multiple of 4)
  if (blockIdx.x == 0 && threadIdx.x < count - 4u * n4) {
    const uint32_t j = 4u * n4 + threadIdx.x;
    acc += (double)fabsf(img[j] - tgt[j]);
  }
  const double s = block_sum_f64(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void l1_finish_kernel(const double* partials, uint32_t count, float* loss) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int k = threadIdx.x; k < kL1Blocks; k += kBlock) acc += partials[k];
  const double s = block_sum_f64(acc, sh);
  if (threadIdx.x == 0) *loss = (float)(s / (double)count);
}

// sign(a - b) as torch's abs backward takes it: 0 where a == b
__device__ inline float l1_sign(float a, float b) {
  const float d = a - b;
  return d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
}

__global__ __launch_bounds__(kBlock) void l1_grad_kernel(const float* img, const float* tgt, uint32_t count,
                                                         const float* dl, float* out) {
  // the mean's backward: the upstream gradient over the element count
  // (exact in double for any count, rounded once to float), then times the
  // sign (exact)
  const float w = (float)((double)dl[0] / (double)count);
  const uint32_t n4 = count / 4u;
  const float4* a4 = reinterpret_cast<const float4*>(img);
  const float4* b4 = reinterpret_cast<const float4*>(tgt);
  float4* o4 = reinterpret_cast<float4*>(out);
  for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < n4; j += gridDim.x * kBlock) {
    const float4 a = a4[j], b = b4[j];
    o4[j] = make_float4(w * l1_sign(a.x, b.x), w * l1_sign(a.y, b.y), w * l1_sign(a.z, b.z), w * l1_sign(a.w, b.w));
  }
  if (blockIdx.x == 0 && threadIdx.x < count - 4u * n4) {
    const uint32_t j = 4u * n4 + threadIdx.x;
    out[j] = w * l1_sign(img[j], tgt[j]);
  }
}

// Partial sums of fgs_l1_loss_noalloc: a file-scope device array, one copy per
// GPU for the life of the process (the entry point allocates nothing).  Host
// code never passes this name to a kernel: on the host it only stands for the
// symbol, whose device address hipGetSymbolAddress returns per device.
__device__ __align__(256) double scratch[kL1Blocks];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t l1_static_partials(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_l1_loss(const float* image, const float* target, int64_t count, double* partials, float* loss,
                          hipStream_t s) {
  ProfScope prof(s, kKLoss);
  hipLaunchKernelGGL(l1_partials_kernel, dim3(kL1Blocks), dim3(kBlock), 0, s, image, target, (uint32_t)count,
                     partials);
  hipLaunchKernelGGL(l1_finish_kernel, dim3(1), dim3(kBlock), 0, s, partials, (uint32_t)count, loss);
  return hipGetLastError();
}

hipError_t launch_l1_grad(const float* image, const float* target, int64_t count, const float* dl, float* out,
                          hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(ceil_div(count / 4 + 1, kBlock), 4096);
  ProfScope prof(s, kKLoss);
  hipLaunchKernelGGL(l1_grad_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, image, target, (uint32_t)count, dl,
                     out);
  return hipGetLastError();
}

}  // namespace fgs
