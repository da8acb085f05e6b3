// Internal declarations shared by the HIP translation units of libfgs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fgs.h"

namespace fgs {

constexpr int kTile = 16;          // 16x16 pixel tiles (Sec. 3.1 "Rendering")
constexpr int kBlock = 256;        // threads per block = pixels per tile
constexpr int kItemsPerThread = 16;
constexpr int kItemsPerBlock = kBlock * kItemsPerThread;  // radix sort / scan tile
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// Counters slots in the workspace.
enum Counter { kCountK = 0, kCountVisible = 1, kCountFlags = 2 };

// Workspace layout (host computation, shared by the API and the launchers).
struct Layout {
  int64_t n = 0;
  int32_t width = 0, height = 0, tiles_x = 0, tiles_y = 0;
  int64_t kcap = 0;
  size_t bytes = 0;
  size_t splats, depth_keys, tiles, rects, radii;
  size_t dkeys_a, dvals_a, dkeys_b, dvals_b;
  size_t offsets, grad2d, ranges, pixel_T, pixel_last, counters;
  size_t hist, partials;
  size_t tkeys_a, tvals_a, tkeys_b, tvals_b;
  int tile_bits = 0, tile_passes = 0;
  size_t tile_keys_final, tile_ids_final;
};

Layout make_layout(int64_t n, int32_t width, int32_t height, int64_t kcap);
// Largest kcap whose layout fits in `bytes`; kcap < 0 if even kcap = 0 does not fit.
Layout fit_layout(int64_t n, int32_t width, int32_t height, size_t bytes);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device-side views of the per-view inputs.
struct ViewParams {
  double R[9];
  double t[3];
  double fx, fy, cx, cy;
  double near_dist, theta_max;
  int32_t width, height, tiles_x, tiles_y;
  float bg[3];
};

// ---- launchers (each returns hipSuccess or the first HIP error) ----------

// Preprocess: writes splats, depth_keys, tiles, rects, radii, and seeds the
// depth sort with (key, id) in dkeys_a / dvals_a.
hipError_t launch_preprocess(const fgs_gaussians& g, const ViewParams& v, char* ws, const Layout& L,
                             hipStream_t s);

// Exclusive scan of `count` u32 values.  If `gather` is non-null the i-th
// input is in[gather[i]].  Writes total to *total (device) if non-null.
hipError_t launch_scan(const uint32_t* in, const uint32_t* gather, uint32_t* out, int64_t count,
                       uint32_t* partials, uint32_t* total, hipStream_t s);

// Stable LSD radix sort of (key, val) u32 pairs on bits [0, bits).  Buffers
// a (input) and b (scratch); returns in *result_in_b whether the sorted data
// ended in b.
hipError_t launch_radix_sort(uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b,
                             int64_t count, int bits, uint32_t* hist, uint32_t* partials, bool* result_in_b,
                             hipStream_t s);
int radix_passes(int bits);

// One (tile, id) pair per covered tile, Gaussians taken in depth order.
hipError_t launch_duplicate(const uint32_t* depth_order, const uint32_t* tiles, const uint32_t* offsets,
                            const uint2* rects, int64_t n, int32_t tiles_x, uint32_t* out_keys,
                            uint32_t* out_vals, hipStream_t s);

hipError_t launch_ranges(const uint32_t* sorted_keys, int64_t K, uint2* ranges, int32_t ntiles, hipStream_t s);

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s);

hipError_t launch_blend_forward(const ViewParams& v, const uint2* ranges, const uint32_t* ids,
                                const float4* splats, float* out, float* pixel_T, uint32_t* pixel_last,
                                bool save, hipStream_t s);

hipError_t launch_blend_backward(const ViewParams& v, const uint2* ranges, const uint32_t* ids,
                                 const float4* splats, const float* dL_dimg, const float* pixel_T,
                                 const uint32_t* pixel_last, const uint32_t* counters, float* grad2d, int64_t n,
                                 hipStream_t s);

hipError_t launch_preprocess_backward(const fgs_gaussians& g, const ViewParams& v, const char* ws,
                                      const Layout& L, const fgs_grads& out, hipStream_t s);

}  // namespace fgs
