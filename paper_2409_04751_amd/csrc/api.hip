// C ABI of libfgs: argument checks, workspace layout and the launch order of
// the forward and backward passes.  All device memory comes from the caller.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "fgs_internal.hpp"

namespace fgs {
namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(FGS_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int bits_for(int64_t values) {  // bits needed to represent 0 .. values-1
  int b = 0;
  while (((int64_t)1 << b) < values) ++b;
  return b;
}

int tiles_of(int32_t px) { return (px + kTile - 1) / kTile; }

}  // namespace

Layout make_layout(int64_t n, int32_t nviews, const int32_t* widths, const int32_t* heights, int64_t kcap) {
  Layout L;
  L.n = n;
  L.nviews = nviews;
  L.width = widths[0];
  L.height = heights[0];
  L.tiles_x = tiles_of(widths[0]);
  L.tiles_y = tiles_of(heights[0]);
  L.kcap = kcap;
  for (int v = 0; v < nviews; ++v) {
    L.total_tiles += (int64_t)tiles_of(widths[v]) * tiles_of(heights[v]);
    L.total_pixels += (int64_t)widths[v] * heights[v];
  }
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const size_t nv = nn * (size_t)nviews;
  L.nv = (int64_t)n * nviews;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + (bytes > 0 ? bytes : 1));
    return o;
  };
  L.counters = take(kNumCounters * sizeof(uint32_t));
  L.splats = take(nv * 2 * sizeof(float4));
  L.colors = take(nv * sizeof(float4));
  L.depth_keys = take(nv * 4);
  L.tiles = take(nv * 4);
  L.rects = take(nv * 8);
  L.radii = take(nv * 4);
  L.dkeys_a = take(nv * 4);
  L.dvals_a = take(nv * 4);
  L.drx_a = take(nv * 4);
  L.dry_a = take(nv * 4);
  L.dkeys_b = take(nv * 4);
  L.dvals_b = take(nv * 4);
  L.offsets = take(nv * 4);
  L.grad2d = take((size_t)grad_words((int64_t)nn) * 4);
  L.ranges = take((size_t)L.total_tiles * 8);
  L.pixel_T = take((size_t)L.total_pixels * 4);
  L.pixel_last = take((size_t)L.total_pixels * 4);
  L.block_tiles = take((size_t)ceil_div((int64_t)nn, kBlock) * nviews * 4);
  const int64_t kk = kcap > 0 ? kcap : 1;
  const int64_t nb_max = std::max({radix_blocks((int64_t)nv, 3), radix_blocks(kk, 1), ceil_div(kk, kDupItems)});
  // radix histograms; before the depth sort also the compaction's per-block
  // stats (one uint4 per 256 entries)
  L.hist = take(std::max((size_t)nb_max * kRadix * 4, (size_t)ceil_div((int64_t)nv, kBlock) * 32));
  const int64_t scan_items = std::max<int64_t>({(int64_t)nv, kk, nb_max * kRadix});
  L.partials = take((size_t)(ceil_div(scan_items, kItemsPerBlock) + 1) * 4);
  L.tkeys_a = take((size_t)kk * 4);
  L.tvals_a = take((size_t)kk * 4);
  L.tkeys_b = take((size_t)kk * 4);
  L.tvals_b = take((size_t)kk * 4);
  L.colorjac = take(nn * 3 * sizeof(float4));
  L.row_off = take((size_t)kk * 4);
  L.rowrange = take(nv * 4);
  L.block_first = take((size_t)(kk / std::min(kRowsPerBlock, kDupItems) + 2) * 4);
  // the depth sort's second rect planes last: where the gradient accumulators
  // sit relative to the splat records changes the blend backward's atomics
  // (a sweep of offsets at the benchmark view: 0.198 to 0.257 ms), and this
  // order keeps them at a measured good offset there
  L.drx_b = take(nv * 4);
  L.dry_b = take(nv * 4);
  // last: these move no other array
  L.block_kept = take((size_t)ceil_div((int64_t)nn, kBlock) * 4);
  L.block_pairs = take((size_t)(kk / kRowsPerBlock + 1) * 4);
  L.bytes = off;
  L.tile_bits = bits_for(L.total_tiles);
  L.tile_passes = radix_passes(L.tile_bits);
  // the duplication does the first pass into *_a (also with no key bits),
  // each later pass swaps the planes
  const bool in_b = (std::max(L.tile_passes, 1) - 1) % 2 == 1;
  L.tile_keys_final = in_b ? L.tkeys_b : L.tkeys_a;
  L.tile_ids_final = in_b ? L.tvals_b : L.tvals_a;
  return L;
}

Layout fit_layout(int64_t n, int32_t nviews, const int32_t* widths, const int32_t* heights, size_t bytes) {
  Layout L0 = make_layout(n, nviews, widths, heights, 0);
  if (L0.bytes > bytes) {
    L0.kcap = -1;
    return L0;
  }
  // largest kcap with make_layout(kcap).bytes <= bytes (monotone in kcap)
  int64_t lo = 0, hi = std::min<int64_t>((int64_t)(bytes / 16) + 1, 0x7FFFFFFF);
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (make_layout(n, nviews, widths, heights, mid).bytes <= bytes) lo = mid; else hi = mid;
  }
  return make_layout(n, nviews, widths, heights, lo);
}

}  // namespace fgs

using namespace fgs;

namespace {

int check_gaussians(const fgs_gaussians* g) {
  if (!g) return fail(FGS_ERR_ARG, "null gaussians");
  if (g->n < 0) return fail(FGS_ERR_ARG, "n < 0");
  if (g->n > 0x7FFFFFFF) return fail(FGS_ERR_OVERFLOW, "more than 2^31-1 Gaussians");
  if (g->sh_degree < 0 || g->sh_degree > 3) return fail(FGS_ERR_ARG, "sh_degree must be 0..3");
  if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh))
    return fail(FGS_ERR_ARG, "null parameter array");
  return FGS_OK;
}

int check_view(const fgs_pose* pose, const fgs_camera* cam, const float* bg) {
  if (!pose || !cam || !bg) return fail(FGS_ERR_ARG, "null pose, camera or bg");
  if (cam->width <= 0 || cam->height <= 0) return fail(FGS_ERR_ARG, "image size must be positive");
  if ((int64_t)cam->width * cam->height > ((int64_t)1 << 31)) return fail(FGS_ERR_ARG, "image too large");
  if (tiles_of(cam->width) > 0xFFFF || tiles_of(cam->height) > 0xFFFF)
    return fail(FGS_ERR_ARG, "more than 65535 tiles along one axis");
  if (cam->model < FGS_MODEL_EQUIDISTANT || cam->model > FGS_MODEL_STEREOGRAPHIC)
    return fail(FGS_ERR_ARG, "unsupported camera model");
  if (!(cam->fx > 0) || !(cam->fy > 0) || !std::isfinite(cam->fx) || !std::isfinite(cam->fy) ||
      !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
    return fail(FGS_ERR_ARG, "focal lengths must be positive and the principal point finite");
  const bool half = cam->model == FGS_MODEL_PINHOLE || cam->model == FGS_MODEL_ORTHOGRAPHIC ||
                    cam->model == FGS_MODEL_PANORAMA;
  if (!(cam->theta_max > 0) || !(cam->theta_max < (half ? 0.5 : 1.0) * 3.14159265358979323846))
    return fail(FGS_ERR_ARG, half ? "theta_max must be in (0, pi/2) for this camera model"
                                  : "theta_max must be in (0, pi)");
  if (!(cam->near_dist >= 0) || !std::isfinite(cam->near_dist)) return fail(FGS_ERR_ARG, "near_dist must be >= 0");
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(pose->R[k])) return fail(FGS_ERR_ARG, "non-finite pose");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(pose->t[k]) || !std::isfinite(bg[k])) return fail(FGS_ERR_ARG, "non-finite pose or bg");
  return FGS_OK;
}

ViewParams make_view(const fgs_pose* pose, const fgs_camera* cam, const float* bg, uint32_t tile_base,
                     uint32_t pixel_base) {
  ViewParams v;
  for (int k = 0; k < 9; ++k) v.R[k] = pose->R[k];
  for (int k = 0; k < 3; ++k) v.t[k] = pose->t[k];
  for (int c = 0; c < 3; ++c) v.campos[c] = -(v.R[0 * 3 + c] * v.t[0] + v.R[1 * 3 + c] * v.t[1] + v.R[2 * 3 + c] * v.t[2]);
  v.fx = cam->fx;
  v.fy = cam->fy;
  v.cx = cam->cx;
  v.cy = cam->cy;
  v.near_dist = cam->near_dist;
  v.theta_max = cam->theta_max;
  v.model = cam->model;
  v.width = cam->width;
  v.height = cam->height;
  v.tiles_x = tiles_of(cam->width);
  v.tiles_y = tiles_of(cam->height);
  v.tile_base = tile_base;
  v.pixel_base = pixel_base;
  for (int k = 0; k < 3; ++k) v.bg[k] = bg[k];
  return v;
}

void export_layout(const Layout& L, fgs_layout* out) {
  std::memset(out, 0, sizeof(*out));
  out->n = L.n;
  out->width = L.width;
  out->height = L.height;
  out->tiles_x = L.tiles_x;
  out->tiles_y = L.tiles_y;
  out->k_capacity = L.kcap;
  out->bytes = L.bytes;
  out->splats = L.splats;
  out->colors = L.colors;
  out->depth_keys = L.depth_keys;
  out->tiles = L.tiles;
  out->rects = L.rects;
  out->radii = L.radii;
  out->depth_order = L.dvals_a;
  out->offsets = L.offsets;
  out->tile_keys = L.tile_keys_final;
  out->tile_ids = L.tile_ids_final;
  out->ranges = L.ranges;
  out->grad2d = L.grad2d;
  out->pixel_T = L.pixel_T;
  out->pixel_last = L.pixel_last;
  out->counters = L.counters;
}

// The forward's one read-back: the counters go to a small pinned host
// buffer (one per host thread, allocated on first use and kept), and the
// host polls the stream until they have arrived rather than sleeping in a
// stream synchronisation, so the launches that depend on them follow with
// less delay.  After a few seconds of polling it falls back to a plain
// synchronisation, which also reports any error of the stream.
hipError_t read_counters(const uint32_t* counters, uint32_t* out, hipStream_t s) {
  thread_local uint32_t* pinned = nullptr;
  if (!pinned) {
    void* p = nullptr;
    const hipError_t e = hipHostMalloc(&p, kNumCounters * sizeof(uint32_t), hipHostMallocDefault);
    if (e != hipSuccess) return e;
    pinned = static_cast<uint32_t*>(p);
  }
  hipError_t e = hipMemcpyAsync(pinned, counters, kNumCounters * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  const auto t0 = std::chrono::steady_clock::now();
  while ((e = hipStreamQuery(s)) == hipErrorNotReady) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      e = hipStreamSynchronize(s);
      break;
    }
  }
  if (e != hipSuccess) return e;
  std::memcpy(out, pinned, kNumCounters * sizeof(uint32_t));
  return hipSuccess;
}

#define HIP_TRY(expr, where)                          \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// Shared forward of 1..kMaxViews views: preprocess of every (view, Gaussian),
// visibility scan and compaction (which also sum K and R and find the
// depth-key range), the one read-back of those counts, depth sort, row
// numbering, rows, row-count scan, duplication, tile sort, ranges and one
// blend launch over the tiles of all views.
int forward_impl(const fgs_gaussians* g, int32_t nviews, const fgs_pose* poses, const fgs_camera* cams,
                 const float* bgs, uint32_t flags, void* workspace, size_t workspace_bytes, float* const* out_rgb,
                 int64_t* k_views, int64_t* k_total, hipStream_t s) {
  int32_t widths[kMaxViews], heights[kMaxViews];
  for (int v = 0; v < nviews; ++v) {
    widths[v] = cams[v].width;
    heights[v] = cams[v].height;
  }
  const Layout L = fit_layout(g->n, nviews, widths, heights, workspace_bytes);
  if (L.kcap < 0) {
    if (k_total) *k_total = -1;
    return fail(FGS_ERR_WORKSPACE, "workspace smaller than the fixed part of the layout");
  }
  char* ws = static_cast<char*>(workspace);
  auto U = [&](size_t off) { return reinterpret_cast<uint32_t*>(ws + off); };
  ViewBatch b;
  b.count = nviews;
  uint32_t tile_base = 0, pixel_base = 0;
  BatchOut out;
  for (int v = 0; v < kMaxViews; ++v) out.rgb[v] = nullptr;
  for (int v = 0; v < nviews; ++v) {
    b.v[v] = make_view(&poses[v], &cams[v], &bgs[3 * v], tile_base, pixel_base);
    tile_base += (uint32_t)(b.v[v].tiles_x * b.v[v].tiles_y);
    pixel_base += (uint32_t)(cams[v].width * cams[v].height);
    out.rgb[v] = out_rgb[v];
  }
  const int64_t n = g->n, nv = L.nv;
  uint32_t* counters = U(L.counters);
  uint32_t* partials = U(L.partials);
  uint32_t* hist = U(L.hist);

  const bool tight = (flags & FGS_RECT_BINNING) == 0;
  HIP_TRY(launch_preprocess(*g, b, tight, flags, ws, L, s), "preprocess");  // also clears the counters
  // stable compaction of the visible (view, Gaussian) entries; offsets holds
  // their positions until the tile-count scan reuses it.  The compaction
  // also sums K and finds the depth-key range, so one read-back gives every
  // later stage its exact size.
  if (nviews == 1 && ceil_div(n, kBlock) <= kMaxPartsScan)  // the preprocess counted each block's kept entries
    HIP_TRY(launch_scan_from_parts(U(L.tiles), kScanFlag, nv, U(L.block_kept), kBlock, counters + kCountVisible,
                                   U(L.offsets), s),
            "visibility scan");
  else
    HIP_TRY(launch_scan(U(L.tiles), nullptr, nullptr, nv, kScanFlag, partials, counters + kCountVisible,
                        U(L.offsets), s),
            "visibility scan");
  HIP_TRY(launch_compact(U(L.tiles), U(L.depth_keys), reinterpret_cast<const uint2*>(ws + L.rects),
                         U(L.rowrange), tight, U(L.offsets), nv, U(L.dkeys_b),
                         U(L.dvals_b), U(L.drx_b), U(L.dry_b), counters, reinterpret_cast<uint4*>(hist), s),
          "compact");
  uint32_t host_counters[kNumCounters];
  HIP_TRY(read_counters(counters, host_counters, s), "read counts");
  const int64_t V = host_counters[kCountVisible];
  uint64_t K64;
  std::memcpy(&K64, &host_counters[kCountK64], sizeof(K64));
  if (k_total) *k_total = K64 > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)K64;
  if (k_views)  // one view: its count is the total (the per-view sums run for batches only)
    for (int v = 0; v < nviews; ++v) k_views[v] = nviews == 1 ? (int64_t)K64 : (int64_t)host_counters[kCountViewK + v];
  if (K64 > 0x7FFFFFFFull) return fail(FGS_ERR_OVERFLOW, "more than 2^31-1 intersections");
  const int64_t K = (int64_t)K64;
  // the rows to bin share the intersection capacity (they are fewer with
  // tight binning unless most rows keep no tile; never more with rect binning)
  uint64_t R64;
  std::memcpy(&R64, &host_counters[kCountRows64], sizeof(R64));
  if (R64 > 0x7FFFFFFFull) return fail(FGS_ERR_OVERFLOW, "more than 2^31-1 rows to bin");
  const int64_t R = (int64_t)R64;
  if (K > L.kcap || R > L.kcap) {
    const int64_t need = std::max(K, R);
    if (k_total) *k_total = need;
    if (k_views && nviews == 1) k_views[0] = need;
    char msg[160];
    std::snprintf(msg, sizeof(msg), "workspace holds %lld intersections, %lld needed", (long long)L.kcap,
                  (long long)need);
    return fail(FGS_ERR_WORKSPACE, msg);
  }
  // depth sort of the V visible entries carrying (id, rect); digits over
  // key - min key, so only the bits in which the visible depths differ are
  // sorted (26 of 31 for depths 0.2-12 m: 3 passes).  Views may interleave here: the tile
  // sort below separates them again and keeps each view's depth order.
  const uint32_t kmin = host_counters[kCountKeyMin], kmax = host_counters[kCountKeyMax];
  const int depth_bits = V > 1 ? bits_for((int64_t)(kmax - kmin) + 1) : 0;
  // the compaction filled the *_b planes, so the usual odd number of passes
  // (3) leaves the order in the *_a planes, where the layout's depth_order
  // points; after an even number the id plane is copied there
  RadixBuffers DB{3, U(L.dkeys_b), U(L.dkeys_a), {U(L.dvals_b), U(L.drx_b), U(L.dry_b)},
                  {U(L.dvals_a), U(L.drx_a), U(L.dry_a)}};
  HIP_TRY(launch_radix_sort(DB, nullptr, V, depth_bits, hist, partials, s, kKDepthHist, kKDepthScatter, 0, kmin),
          "depth sort");
  const bool odd = radix_passes(depth_bits) % 2 == 1;
  uint32_t* d_ids = odd ? U(L.dvals_a) : U(L.dvals_b);
  uint32_t* d_rx = odd ? U(L.drx_a) : U(L.drx_b);
  uint32_t* d_ry = odd ? U(L.dry_a) : U(L.dry_b);
  if (!odd && V > 0)
    HIP_TRY(hipMemcpyAsync(U(L.dvals_a), d_ids, (size_t)V * 4, hipMemcpyDeviceToDevice, s), "depth order");
  // binning by rows: the depth-ordered entries' rows to bin (offsets = the
  // exclusive scan of their row ranges), each row's kept columns, the rows'
  // pair offsets (exclusive scan of their counts; total K), then the pairs.
  // The rows' Gaussian ids and (y, first column) sit in the tile sort's
  // second buffers, which the sort first writes after the duplication.
  uint32_t* row_g = U(L.tvals_b);
  uint32_t* row_yc = U(L.tkeys_b);
  HIP_TRY(launch_scan(d_rx, d_ry, nullptr, V, kScanRows, partials, nullptr, U(L.offsets), s, U(L.block_first),
                      kRowsPerBlock),
          "row scan");
  HIP_TRY(launch_rows(d_ids, d_rx, d_ry, U(L.offsets), U(L.block_first), V, R,
                      reinterpret_cast<const float4*>(ws + L.splats), tight, U(L.row_off), row_g, row_yc,
                      U(L.block_pairs), s),
          "rows");
  if (ceil_div(R, kRowsPerBlock) <= kMaxPartsScan)  // the rows kernel summed each block's counts
    HIP_TRY(launch_scan_from_parts(U(L.row_off), kScanPlain, R, U(L.block_pairs), kRowsPerBlock, counters + kCountK,
                                   U(L.row_off), s, U(L.block_first), kDupItems),
            "row count scan");
  else
    HIP_TRY(launch_scan(U(L.row_off), nullptr, nullptr, R, kScanPlain, partials, counters + kCountK, U(L.row_off), s,
                        U(L.block_first), kDupItems),
            "row count scan");
  // the pairs come out of the duplication in the order of the tile sort's
  // first pass (into *_a: the rows still sit in *_b); the sort does the rest
  HIP_TRY(launch_duplicate_sorted(U(L.row_off), row_g, row_yc, U(L.block_first), R, K, b, n, L.tile_bits, hist,
                                  partials, U(L.tkeys_a), U(L.tvals_a), s),
          "duplicate");
  RadixBuffers TB{1, U(L.tkeys_a), U(L.tkeys_b), {U(L.tvals_a), nullptr, nullptr}, {U(L.tvals_b), nullptr, nullptr},
                  tile_keys16(L.tile_bits)};
  HIP_TRY(launch_radix_sort(TB, nullptr, K, L.tile_bits, hist, partials, s, kKTileHist, kKTileScatter, 1),
          "tile sort");
  uint2* ranges = reinterpret_cast<uint2*>(ws + L.ranges);
  HIP_TRY(launch_ranges(U(L.tile_keys_final), K, ranges, (int32_t)L.total_tiles, s), "ranges");
  HIP_TRY(launch_blend_forward(b, L.total_tiles, ranges, U(L.tile_ids_final),
                               reinterpret_cast<const float4*>(ws + L.splats),
                               reinterpret_cast<const float4*>(ws + L.colors), out,
                               reinterpret_cast<float*>(ws + L.pixel_T), U(L.pixel_last),
                               (flags & FGS_SAVE_PIXEL_STATE) != 0, s),
          "blend forward");
  return FGS_OK;
}

}  // namespace

extern "C" {

const char* fgs_version(void) { return "fgs 0.2 gfx950"; }

const char* fgs_last_error(void) { return g_last_error.c_str(); }

int fgs_workspace_bytes(int64_t n, int32_t width, int32_t height, int64_t k_capacity, size_t* bytes) {
  if (!bytes || n < 0 || width <= 0 || height <= 0 || k_capacity < 0) return fail(FGS_ERR_ARG, "bad argument");
  if (n > 0x7FFFFFFF || k_capacity > 0x7FFFFFFF) return fail(FGS_ERR_OVERFLOW, "size beyond 2^31-1");
  *bytes = make_layout(n, 1, &width, &height, k_capacity).bytes;
  return FGS_OK;
}

int fgs_workspace_layout(int64_t n, int32_t width, int32_t height, size_t bytes, fgs_layout* out) {
  if (!out || n < 0 || width <= 0 || height <= 0) return fail(FGS_ERR_ARG, "bad argument");
  const Layout L = fit_layout(n, 1, &width, &height, bytes);
  if (L.kcap < 0) return fail(FGS_ERR_WORKSPACE, "workspace smaller than the fixed part of the layout");
  export_layout(L, out);
  return FGS_OK;
}

int fgs_batch_workspace_bytes(int64_t n, int32_t nviews, const fgs_camera* cams, int64_t k_capacity,
                              size_t* bytes) {
  if (!bytes || !cams || n < 0 || nviews < 1 || nviews > kMaxViews || k_capacity < 0)
    return fail(FGS_ERR_ARG, "bad argument");
  if ((int64_t)n * nviews > 0x7FFFFFFF || k_capacity > 0x7FFFFFFF) return fail(FGS_ERR_OVERFLOW, "size beyond 2^31-1");
  int32_t w[kMaxViews], h[kMaxViews];
  for (int v = 0; v < nviews; ++v) {
    if (cams[v].width <= 0 || cams[v].height <= 0) return fail(FGS_ERR_ARG, "image size must be positive");
    w[v] = cams[v].width;
    h[v] = cams[v].height;
  }
  *bytes = make_layout(n, nviews, w, h, k_capacity).bytes;
  return FGS_OK;
}

int fgs_render_forward(const fgs_gaussians* g, const fgs_pose* pose, const fgs_camera* cam, const float bg[3],
                       uint32_t flags, void* workspace, size_t workspace_bytes, float* out_rgb, int64_t* k_out,
                       void* stream) {
  int rc = check_gaussians(g);
  if (rc == FGS_OK) rc = check_view(pose, cam, bg);
  if (rc != FGS_OK) return rc;
  if (!workspace || !out_rgb) return fail(FGS_ERR_ARG, "null workspace or output");
  if (flags & ~(FGS_SAVE_PIXEL_STATE | FGS_RECT_BINNING)) return fail(FGS_ERR_ARG, "unknown flags");
  float* outs[1] = {out_rgb};
  return forward_impl(g, 1, pose, cam, bg, flags, workspace, workspace_bytes, outs, nullptr, k_out,
                      reinterpret_cast<hipStream_t>(stream));
}

int fgs_render_forward_batch(const fgs_gaussians* g, int32_t nviews, const fgs_pose* poses, const fgs_camera* cams,
                             const float* bgs, void* workspace, size_t workspace_bytes, float* const* out_rgb,
                             int64_t* k_views, int64_t* k_total, void* stream) {
  int rc = check_gaussians(g);
  if (rc != FGS_OK) return rc;
  if (nviews < 1 || nviews > kMaxViews) return fail(FGS_ERR_ARG, "nviews must be 1..FGS_MAX_BATCH");
  if (!poses || !cams || !bgs || !out_rgb || !workspace) return fail(FGS_ERR_ARG, "null argument");
  if ((int64_t)g->n * nviews > 0x7FFFFFFF) return fail(FGS_ERR_OVERFLOW, "n * nviews beyond 2^31-1");
  int64_t tiles = 0;
  for (int v = 0; v < nviews; ++v) {
    rc = check_view(&poses[v], &cams[v], &bgs[3 * v]);
    if (rc != FGS_OK) return rc;
    if (!out_rgb[v]) return fail(FGS_ERR_ARG, "null output image");
    tiles += (int64_t)tiles_of(cams[v].width) * tiles_of(cams[v].height);
  }
  if (tiles > 0x7FFFFFFF) return fail(FGS_ERR_OVERFLOW, "too many tiles in the batch");
  return forward_impl(g, nviews, poses, cams, bgs, 0u, workspace, workspace_bytes, out_rgb, k_views, k_total,
                      reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

// Backward of one view; with det_ws the 2D gradients go through the
// deterministic per-entry store and segmented reduction instead of atomics.
int backward_impl(const fgs_gaussians* g, const fgs_pose* pose, const fgs_camera* cam, const float bg[3],
                  void* workspace, size_t workspace_bytes, const float* dL_drgb, const fgs_grads* grads,
                  void* det_ws, size_t det_bytes, bool det, void* stream) {
  int rc = check_gaussians(g);
  if (rc == FGS_OK) rc = check_view(pose, cam, bg);
  if (rc != FGS_OK) return rc;
  if (!workspace || !dL_drgb || !grads) return fail(FGS_ERR_ARG, "null workspace, dL_drgb or grads");
  if (g->n > 0 && (!grads->means || !grads->scales || !grads->quats || !grads->opacities || !grads->sh))
    return fail(FGS_ERR_ARG, "null gradient array");
  if (det && !det_ws) return fail(FGS_ERR_ARG, "null deterministic workspace");
  const Layout L = fit_layout(g->n, 1, &cam->width, &cam->height, workspace_bytes);
  if (L.kcap < 0) return fail(FGS_ERR_WORKSPACE, "workspace smaller than the fixed part of the layout");
  if (g->n == 0) return FGS_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const ViewParams v = make_view(pose, cam, bg, 0u, 0u);
  float* grad2d = reinterpret_cast<float*>(ws + L.grad2d);
  const uint32_t* ids = reinterpret_cast<const uint32_t*>(ws + L.tile_ids_final);
  DetStore store{};
  int64_t K = 0;
  if (det) {
    // the forward's K, read back once: it sizes the per-entry sums
    uint32_t host_counters[kNumCounters];
    HIP_TRY(read_counters(reinterpret_cast<uint32_t*>(ws + L.counters), host_counters, s), "read counts");
    uint64_t K64;
    std::memcpy(&K64, &host_counters[kCountK64], sizeof(K64));
    if (K64 > (uint64_t)L.kcap) return fail(FGS_ERR_WORKSPACE, "workspace holds no forward state of this view");
    K = (int64_t)K64;
    if (det_bytes < det_workspace_bytes(g->n, K)) {
      char msg[160];
      std::snprintf(msg, sizeof(msg), "deterministic workspace of %zu bytes, %zu needed for %lld intersections",
                    det_bytes, det_workspace_bytes(g->n, K), (long long)K);
      return fail(FGS_ERR_WORKSPACE, msg);
    }
    char* dws = static_cast<char*>(det_ws);
    store.part = reinterpret_cast<float*>(dws);
    store.rects = reinterpret_cast<const uint2*>(ws + L.rects);
    store.rowrange = reinterpret_cast<const uint32_t*>(ws + L.rowrange);
    store.gauss_off = det_gauss_off(dws, g->n, K);
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(store.part), 0u, 9 * K, s), "clear per-entry sums");
    HIP_TRY(launch_grad_offsets(reinterpret_cast<const uint32_t*>(ws + L.tiles), g->n, K, dws, s),
            "per-Gaussian runs");
  } else {
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u, grad_words(g->n), s), "clear grad2d");
  }
  HIP_TRY(launch_blend_backward(v, reinterpret_cast<const uint2*>(ws + L.ranges), ids,
                                reinterpret_cast<const float4*>(ws + L.splats),
                                reinterpret_cast<const float4*>(ws + L.colors), dL_drgb,
                                reinterpret_cast<const float*>(ws + L.pixel_T),
                                reinterpret_cast<const uint32_t*>(ws + L.pixel_last),
                                reinterpret_cast<const uint32_t*>(ws + L.counters), grad2d, det ? &store : nullptr,
                                g->n, s),
          "blend backward");
  if (det)
    HIP_TRY(launch_grad_segreduce(reinterpret_cast<const uint32_t*>(ws + L.tiles), g->n, K, static_cast<char*>(det_ws),
                                  grad2d, s),
            "deterministic reduction");
  HIP_TRY(launch_preprocess_backward(*g, v, ws, L, *grads, s), "preprocess backward");
  return FGS_OK;
}

}  // namespace

extern "C" {

int fgs_render_backward(const fgs_gaussians* g, const fgs_pose* pose, const fgs_camera* cam, const float bg[3],
                        void* workspace, size_t workspace_bytes, const float* dL_drgb, const fgs_grads* grads,
                        void* stream) {
  return backward_impl(g, pose, cam, bg, workspace, workspace_bytes, dL_drgb, grads, nullptr, 0, false, stream);
}

int fgs_deterministic_workspace_bytes(int64_t n, int64_t k_capacity, size_t* bytes) {
  if (!bytes || n < 0 || k_capacity < 0) return fail(FGS_ERR_ARG, "fgs_deterministic_workspace_bytes: bad argument");
  if (n > 0x7FFFFFFF || k_capacity > 0x7FFFFFFF) return fail(FGS_ERR_OVERFLOW, "size beyond 2^31-1");
  *bytes = det_workspace_bytes(n, k_capacity);
  return FGS_OK;
}

int fgs_render_backward_deterministic(const fgs_gaussians* g, const fgs_pose* pose, const fgs_camera* cam,
                                      const float bg[3], void* workspace, size_t workspace_bytes,
                                      const float* dL_drgb, const fgs_grads* grads, void* det_workspace,
                                      size_t det_workspace_bytes, void* stream) {
  return backward_impl(g, pose, cam, bg, workspace, workspace_bytes, dL_drgb, grads, det_workspace,
                       det_workspace_bytes, true, stream);
}

}  // extern "C"

namespace {
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
}  // namespace

extern "C" int fgs_l1_loss(const float* image, const float* target, int64_t count, double* partials, float* loss,
                           void* stream) {
  if (!image || !target || !partials || !loss || count <= 0) return fail(FGS_ERR_ARG, "fgs_l1_loss: bad argument");
  if (count > 0x7FFFFFFFll) return fail(FGS_ERR_OVERFLOW, "fgs_l1_loss: more than 2^31 - 1 values");
  if (!aligned16(image) || !aligned16(target)) return fail(FGS_ERR_ARG, "fgs_l1_loss: images must be 16-byte aligned");
  const hipError_t e = launch_l1_loss(image, target, count, partials, loss, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? FGS_OK : hip_fail(e, "fgs_l1_loss");
}

extern "C" int fgs_l1_loss_backward(const float* image, const float* target, int64_t count, const float* dL_dloss,
                                    float* dL_dimage, void* stream) {
  if (!image || !target || !dL_dloss || !dL_dimage || count <= 0)
    return fail(FGS_ERR_ARG, "fgs_l1_loss_backward: bad argument");
  if (count > 0x7FFFFFFFll) return fail(FGS_ERR_OVERFLOW, "fgs_l1_loss_backward: more than 2^31 - 1 values");
  if (!aligned16(image) || !aligned16(target) || !aligned16(dL_dimage))
    return fail(FGS_ERR_ARG, "fgs_l1_loss_backward: images must be 16-byte aligned");
  const hipError_t e =
      launch_l1_grad(image, target, count, dL_dloss, dL_dimage, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? FGS_OK : hip_fail(e, "fgs_l1_loss_backward");
}

extern "C" int fgs_l1_loss_noalloc(const float* image, const float* target, int64_t count, float* loss,
                                   void* stream) {
  if (!image || !target || !loss || count <= 0) return fail(FGS_ERR_ARG, "fgs_l1_loss_noalloc: bad argument");
  if (count > 0x7FFFFFFFll)
    return fail(FGS_ERR_OVERFLOW, "fgs_l1_loss_noalloc: more than 2^31 - 1 values (the largest count it takes)");
  if (!aligned16(image) || !aligned16(target))
    return fail(FGS_ERR_ARG, "fgs_l1_loss_noalloc: images must be 16-byte aligned");
  double* partials = nullptr;
  hipError_t e = l1_static_partials(&partials);
  if (e != hipSuccess) return hip_fail(e, "fgs_l1_loss_noalloc: device address of the partials array");
  e = launch_l1_loss(image, target, count, partials, loss, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? FGS_OK : hip_fail(e, "fgs_l1_loss_noalloc");
}

extern "C" int fgs_spatial_order_workspace_bytes(int64_t n, size_t* bytes) {
  if (!bytes || n < 0) return fail(FGS_ERR_ARG, "fgs_spatial_order_workspace_bytes: bad argument");
  if (n > 0x7FFFFFFF) return fail(FGS_ERR_OVERFLOW, "fgs_spatial_order_workspace_bytes: more than 2^31-1 Gaussians");
  *bytes = spatial_order_workspace(n);
  return FGS_OK;
}

extern "C" int fgs_spatial_order(const float* means, int64_t n, uint32_t* order, void* workspace,
                                 size_t workspace_bytes, void* stream) {
  if (n < 0 || (n > 0 && (!means || !order || !workspace))) return fail(FGS_ERR_ARG, "fgs_spatial_order: bad argument");
  if (n > 0x7FFFFFFF) return fail(FGS_ERR_OVERFLOW, "fgs_spatial_order: more than 2^31-1 Gaussians");
  if (workspace_bytes < spatial_order_workspace(n))
    return fail(FGS_ERR_WORKSPACE, "fgs_spatial_order: workspace smaller than fgs_spatial_order_workspace_bytes");
  const hipError_t e =
      launch_spatial_order(means, n, order, static_cast<char*>(workspace), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? FGS_OK : hip_fail(e, "fgs_spatial_order");
}

extern "C" int fgs_gather_planes(const float* in, float* out, int64_t planes, int64_t n, const uint32_t* order,
                                 void* stream) {
  if (n < 0 || planes < 0 || (n > 0 && planes > 0 && (!in || !out || !order)))
    return fail(FGS_ERR_ARG, "fgs_gather_planes: bad argument");
  if (in == out && n > 0 && planes > 0) return fail(FGS_ERR_ARG, "fgs_gather_planes: in and out must differ");
  if (n > 0x7FFFFFFF) return fail(FGS_ERR_OVERFLOW, "fgs_gather_planes: more than 2^31-1 Gaussians");
  const hipError_t e = launch_gather_planes(in, out, planes, n, order, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? FGS_OK : hip_fail(e, "fgs_gather_planes");
}
