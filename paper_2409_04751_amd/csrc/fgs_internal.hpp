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
constexpr int kRadixBits = 9;  // widest digit: a 17-bit batch tile id still sorts in 2 passes
constexpr int kRadix = 1 << kRadixBits;
constexpr int kIptPayload1 = 12;  // radix items per thread with one payload word
constexpr int kIptPayload3 = 8;   // ... with three payload words (LDS staging size)

// The hardware hands the blocks of a launch to the 8 XCDs round-robin (block
// b to XCD b % 8), and every XCD has an L2 of its own.  xcd_chunk maps a
// hardware block to a logical block such that each XCD gets one contiguous
// range of logical blocks; neighbouring logical blocks (adjacent output runs
// of a radix scatter, adjacent tiles that gather the same splats) then meet
// in one L2 instead of eight.  A bijection on [0, nb) for any nb.
constexpr uint32_t kXcds = 8;
__device__ inline uint32_t xcd_chunk(uint32_t b, uint32_t nb) {
  const uint32_t x = b % kXcds, k = b / kXcds;
  const uint32_t q = nb / kXcds, r = nb % kXcds;
  return x * q + (x < r ? x : r) + k;
}

// Slot of Gaussian g in the per-Gaussian gradient sums ([slot][9] floats):
// ids are permuted inside each aligned group of 64 (g * 9 mod 64), so
// Gaussians with adjacent ids -- neighbours in space when a scene is stored
// in spatial order -- accumulate into cache lines about 2.5 lines apart, while
// the 64 Gaussians of a wave still read one contiguous 2304-byte block.
__host__ __device__ inline uint32_t grad_slot(uint32_t g) { return (g & ~63u) | ((g * 9u) & 63u); }
// u32 words of the gradient sums for n Gaussians (whole groups of 64)
inline int64_t grad_words(int64_t n) { return (n + 63) / 64 * 64 * 9; }

// What a device-wide scan reads.
enum ScanMode {
  kScanPlain = 0,     // in_a[i]
  kScanFlag = 1,      // in_a[i] != 0
  kScanRectArea = 2,  // tile count of the rect (in_a[i] = x0 | y0 << 16, in_b[i] = x1 | y1 << 16)
  kScanGather = 3,    // in_b[in_a[i]]
  kScanRows = 4,      // row count of the rect (in_a[i] = x0 | y0 << 16, in_b[i] = x1 | y1 << 16)
};

// Output slots (pairs) per duplication block (the duplication is also the
// tile sort's first radix pass, with blocks of its own size), rows per
// rows-kernel block.
constexpr int kDupIpt = 8;
constexpr int kDupItems = kBlock * kDupIpt;
constexpr int kRowsPerThread = 4;
constexpr int kRowsPerBlock = kBlock * kRowsPerThread;

// Key / payload planes of a radix sort: input in *_a, scratch in *_b.
struct RadixBuffers {
  int payload;  // 1 or 3
  uint32_t* keys_a;
  uint32_t* keys_b;
  uint32_t* vals_a[3];
  uint32_t* vals_b[3];
  // payload 1: keys_a holds uint16_t keys for the first pass that runs (the
  // duplication's output, tile_keys16); every pass writes uint32_t keys
  bool keys16 = false;
};

// Kernels known to the event profiler (fgs_profile_*).
enum KernelId {
  kKPreprocess = 0,
  kKCompact,
  kKDepthHist,
  kKDepthScatter,
  kKScan,
  kKDuplicate,
  kKTileHist,
  kKTileScatter,
  kKRanges,
  kKFill,
  kKBlendForward,
  kKBlendBackward,
  kKPreprocessBackward,
  kKColor,
  kKRows,
  kKLoss,
  kKOrder,
  kKSegReduce,
  kKDupHist,
  kKNumKernels
};
const char* kernel_name(int id);

// Records a start event on construction and a stop event on destruction
// (no-op unless profiling is enabled).
class ProfScope {
 public:
  ProfScope(hipStream_t s, int id);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  hipStream_t s_;
  int slot_;
};

constexpr int kMaxViews = FGS_MAX_BATCH;

// Counters slots in the workspace (uint32).
// Device counters at the start of the workspace (u32 slots).  K64 is a u64
// at slots 14-15 (8-byte aligned).
enum Counter {
  kCountK = 0,
  kCountVisible = 1,
  kCountFlags = 2,
  kCountViewK = 3,
  kCountKeyMin = 3 + kMaxViews,  // smallest depth key of a visible entry
  kCountKeyMax = 4 + kMaxViews,  // largest
  kCountK64 = 14,                // sum of the visible entries' tile counts
  kCountRows64 = 16,             // sum of the visible entries' row ranges (rows to bin)
  kNumCounters = 18
};
static_assert(kCountKeyMax < kCountK64, "counter slots overlap");

// Workspace layout (host computation, shared by the API and the launchers).
// Per-(view, Gaussian) arrays have n * nviews entries, view-major; the
// per-tile and per-pixel arrays concatenate the views.
struct Layout {
  int64_t n = 0;
  int32_t nviews = 1;
  int64_t nv = 0;  // n * nviews
  int32_t width = 0, height = 0, tiles_x = 0, tiles_y = 0;  // view 0
  int64_t total_tiles = 0, total_pixels = 0;
  int64_t kcap = 0;
  size_t bytes = 0;
  size_t splats, colors, depth_keys, tiles, rects, radii;
  size_t colorjac;  // single view: float4 [n][3], d rgb / d view direction per channel + clamp mask
  size_t dkeys_a, dvals_a, dkeys_b, dvals_b, drx_a, dry_a, drx_b, dry_b;
  size_t offsets, grad2d, ranges, pixel_T, pixel_last, counters;
  size_t row_off;  // [kcap]: per binned row its kept-tile count, then their exclusive scan
  size_t rowrange;  // tight binning, [entry]: first | (last + 1) << 16 of the rows with a kept tile
  size_t block_first;  // [kcap / kRowsPerBlock + 2]: per rows-kernel block its first entry, then per
                       // duplication block its first row
  // the rows' Gaussian and (y << 16 | first column) live in tvals_b / tkeys_b
  // until the tile sort needs them
  size_t hist, partials, block_tiles;
  size_t block_kept;  // one view: [ceil(n / 256)] entries each preprocess block kept
  size_t block_pairs;  // [kcap / kRowsPerBlock + 1]: pairs of each rows-kernel block
  size_t tkeys_a, tvals_a, tkeys_b, tvals_b;
  int tile_bits = 0, tile_passes = 0;
  size_t tile_keys_final, tile_ids_final;
};

Layout make_layout(int64_t n, int32_t nviews, const int32_t* widths, const int32_t* heights, int64_t kcap);
// Largest kcap whose layout fits in `bytes`; kcap < 0 if even kcap = 0 does not fit.
Layout fit_layout(int64_t n, int32_t nviews, const int32_t* widths, const int32_t* heights, size_t bytes);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device-side views of the per-view inputs.
struct ViewParams {
  double R[9];
  double t[3];
  double campos[3];  // -R^T t
  double fx, fy, cx, cy;
  double near_dist, theta_max;
  int32_t model;
  int32_t width, height, tiles_x, tiles_y;
  uint32_t tile_base;   // first global tile id of the view
  uint32_t pixel_base;  // first pixel of the view in the per-pixel arrays
  float bg[3];
};

// Up to kMaxViews views rendered by one set of launches (passed by value).
struct ViewBatch {
  int32_t count;
  ViewParams v[kMaxViews];
};

struct BatchOut {
  float* rgb[kMaxViews];  // [3][H_v][W_v] per view
};

// ---- launchers (each returns hipSuccess or the first HIP error) ----------

// Preprocess: writes splats, depth_keys, tiles, rects, radii (and, for one
// view, each block's kept count).  Also clears the device counters, storing
// `flags` in their flags slot.
hipError_t launch_preprocess(const fgs_gaussians& g, const ViewBatch& b, bool tight, uint32_t flags, char* ws,
                             const Layout& L, hipStream_t s);

// Exclusive scan of u32 values read as `mode` says; the item count is
// *d_count if d_count is non-null (device), capped by max_count (host).
// Writes the total to *total (device) if non-null.  out may alias in_a.
// With aux (device, [total / aux_block + 1]) the scan also records, for every
// multiple m * aux_block below the total, the item i whose range
// [out[i], out[i] + value[i]) holds it: aux[m] = i.  A kernel that takes
// aux_block consecutive units of the scanned ranges per block finds its first
// item there instead of searching the offsets.
hipError_t launch_scan(const uint32_t* in_a, const uint32_t* in_b, const uint32_t* d_count, int64_t max_count,
                       int mode, uint32_t* partials, uint32_t* total, uint32_t* out, hipStream_t s,
                       uint32_t* aux = nullptr, uint32_t aux_block = 0);
// The same exclusive scan (mode kScanFlag or kScanPlain, max_count items,
// aux as launch_scan) when the producer already left the sum of every
// part_items consecutive items in parts (part_items divides kItemsPerBlock):
// one launch instead of two.  Returns hipErrorInvalidValue (nothing
// launched) beyond kMaxPartsScan parts.
constexpr int64_t kMaxPartsScan = 16384;
hipError_t launch_scan_from_parts(const uint32_t* in_a, int mode, int64_t max_count, const uint32_t* parts,
                                  int64_t part_items, uint32_t* total, uint32_t* out, hipStream_t s,
                                  uint32_t* aux = nullptr, uint32_t aux_block = 0);

// Stable LSD radix sort of u32 keys with B.payload u32 value planes on key
// bits [0, bits), same item-count convention as launch_scan.  Passes before
// first_pass are taken as done (the keys in *_a are in their order); the
// result is in the *_a buffers after an even number of the remaining passes,
// else in *_b.
// Digits are taken from key - key_bias (every key must be >= key_bias); the
// keys themselves are moved unchanged.
hipError_t launch_radix_sort(const RadixBuffers& B, const uint32_t* d_count, int64_t max_count, int bits,
                             uint32_t* hist, uint32_t* partials, hipStream_t s, int hist_id, int scatter_id,
                             int first_pass = 0, uint32_t key_bias = 0);
int radix_passes(int bits);
int64_t radix_blocks(int64_t max_count, int payload);

// Visible Gaussians (tiles > 0) in id order: key, id and row-range planes
// at position pos[i] (exclusive scan of the visibility flags).  The planes
// hold the rect's columns and the rows to bin: with tight binning those
// from the first to the last row with a kept tile (rowrange, from the
// preprocess), else all rows of the rect.  Also stores the visible entries'
// total tile count in counters[kCountK64] (u64), their total row count in
// counters[kCountRows64] (u64) and their depth-key range in
// counters[kCountKeyMin / kCountKeyMax], through block_stats (two uint4 per
// 256 entries, scratch).
hipError_t launch_compact(const uint32_t* tiles, const uint32_t* depth_keys, const uint2* rects,
                          const uint32_t* rowrange, bool tight, const uint32_t* pos, int64_t n, uint32_t* keys,
                          uint32_t* ids, uint32_t* rx, uint32_t* ry, uint32_t* counters, uint4* block_stats,
                          hipStream_t s);

// Rows to bin, one thread each: row t of depth-ordered entry j (row_base[j]
// = exclusive scan of its row-range heights) gets its kept columns
// [c0, c1) -- with tight binning from reach_row on the splat record, else the
// whole rect row -- as row_cnt[t] = c1 - c0, row_g[t] = Gaussian (entry) id,
// row_yc[t] = y << 16 | c0.
// first_entry[b]: the entry that holds row b * kRowsPerBlock (the row scan's aux)
// block_pairs[b]: the kept tiles of the rows of block b (kRowsPerBlock rows).
hipError_t launch_rows(const uint32_t* ids, const uint32_t* rx, const uint32_t* ry, const uint32_t* row_base,
                       const uint32_t* first_entry, int64_t V, int64_t R, const float4* splats, bool tight,
                       uint32_t* row_cnt, uint32_t* row_g, uint32_t* row_yc, uint32_t* block_pairs, hipStream_t s);

// Whether the duplication leaves its keys as uint16_t for the tile sort's
// second pass: two passes (the first one fused) over ids that fit 16 bits.
bool tile_keys16(int tile_bits);

// One (tile, id) pair per kept tile of each row, at the row's offset
// row_off[t] (exclusive scan of the counts) in depth order, K pairs in
// total, put through the first pass of the tile sort (the tile_bits-bit
// sort launch_radix_sort would do, first digit) on the way: the pairs land
// in out_keys / out_vals in that pass's order.  Ids are view-major (view * n
// + Gaussian); the pair's key is the view's tile_base plus the tile index
// inside the view (uint16_t keys if tile_keys16(tile_bits)).  hist and
// partials are the radix sort's scratch.
// first_row[b]: the row that holds pair b * kDupItems (the row-count scan's aux)
hipError_t launch_duplicate_sorted(const uint32_t* row_off, const uint32_t* row_g, const uint32_t* row_yc,
                                   const uint32_t* first_row, int64_t R, int64_t K, const ViewBatch& b, int64_t n,
                                   int tile_bits, uint32_t* hist, uint32_t* partials, uint32_t* out_keys,
                                   uint32_t* out_vals, hipStream_t s);

hipError_t launch_ranges(const uint32_t* sorted_keys, int64_t K, uint2* ranges, int32_t ntiles, hipStream_t s);

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s);

// p[0 .. count) = 0 except p[at] = v, in one launch
hipError_t launch_clear_but_one(uint32_t* p, int64_t count, int64_t at, uint32_t v, hipStream_t s);

hipError_t launch_blend_forward(const ViewBatch& b, int64_t total_tiles, const uint2* ranges, const uint32_t* ids,
                                const float4* splats, const float4* colors, const BatchOut& out, float* pixel_T,
                                uint32_t* pixel_last, bool save, hipStream_t s);

// Deterministic mode of the blend backward: each list entry's nine sums are
// stored at part[gauss_off[g] + rank][9] (rank = the entry's tile among the
// tiles g was binned to, in tile order), so each Gaussian's sums form one
// run in tile order.  rects / rowrange as the forward's preprocess left them.
struct DetStore {
  float* part;
  const uint2* rects;
  const uint32_t* rowrange;
  const uint32_t* gauss_off;
};

// grad2d: [grad_slot(g)][9] per-Gaussian sums (dL/d mu_p xy, conic A B C, opacity, rgb),
// grad_words(n) zeroed words, to which each (Gaussian, tile) adds its sums
// with float atomics; with det not null the sums are stored as DetStore says
// (entries the backward does not reach keep what the caller stored: zeros)
// and grad2d is not touched.
hipError_t launch_blend_backward(const ViewParams& v, const uint2* ranges, const uint32_t* ids,
                                 const float4* splats, const float4* colors, const float* dL_dimg,
                                 const float* pixel_T,
                                 const uint32_t* pixel_last, const uint32_t* counters, float* grad2d,
                                 const DetStore* det, int64_t n, hipStream_t s);

// Deterministic reduction, in det_workspace_bytes(n, K) bytes of scratch whose
// first 36 K bytes are the part[K][9] array:
//   launch_grad_offsets: gauss_off = exclusive scan of the tile counts (the
//     start of each Gaussian's run), before the blend backward;
//   launch_grad_segreduce: grad2d[grad_slot(g)][9] = the sum of g's run
//     (tiles[g] entries) in an order fixed by its length (written, every g < n).
size_t det_workspace_bytes(int64_t n, int64_t k_capacity);
uint32_t* det_gauss_off(char* dws, int64_t n, int64_t K);
hipError_t launch_grad_offsets(const uint32_t* tiles, int64_t n, int64_t K, char* dws, hipStream_t s);
hipError_t launch_grad_segreduce(const uint32_t* tiles, int64_t n, int64_t K, char* dws, float* grad2d,
                                 hipStream_t s);

hipError_t launch_preprocess_backward(const fgs_gaussians& g, const ViewParams& v, const char* ws,
                                      const Layout& L, const fgs_grads& out, hipStream_t s);

// L1 loss of an image against a target (FGS_L1_PARTIALS block partials, then
// the mean into *loss) and its gradient sign(image - target) * dl[0] / count.
hipError_t launch_l1_loss(const float* image, const float* target, int64_t count, double* partials, float* loss,
                          hipStream_t s);
hipError_t launch_l1_grad(const float* image, const float* target, int64_t count, const float* dl, float* out,
                          hipStream_t s);
// Spatial order of a scene (Morton code of the means, ties by id): the
// permutation into `order` (device [n]), scratch `ws` of
// spatial_order_workspace(n) bytes; and the gather of parameter planes by it.
size_t spatial_order_workspace(int64_t n);
hipError_t launch_spatial_order(const float* means, int64_t n, uint32_t* order, char* ws, hipStream_t s);
hipError_t launch_gather_planes(const float* in, float* out, int64_t planes, int64_t n, const uint32_t* order,
                                hipStream_t s);

// Device address, on the current device, of the library's own array of
// FGS_L1_PARTIALS doubles (looked up once per device and kept).
hipError_t l1_static_partials(double** out);

}  // namespace fgs
