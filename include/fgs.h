/*
 * fgs.h - C ABI of the MI355X fisheye Gaussian-splatting rasterizer.
 *
 * The library renders 3D Gaussians (Fisheye-GS, arXiv 2409.04751) through
 * the equidistant fisheye model r = f theta (Sec. 3.2) with the tile-based
 * pipeline the paper keeps from 3DGS (Sec. 4.1): a per-Gaussian preprocess,
 * tile binning, a sort by (tile, depth) and front-to-back alpha blending
 * (Eq. 3), plus the backward pass whose projection gradients the paper
 * derives (Sec. 4.2, 4.3).
 *
 * Conventions shared by every entry point
 *   - Every array argument is DEVICE memory owned by the caller; the library
 *     never allocates, frees or retains it.  Structs and bg[3] are HOST memory
 *     read during the call only.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Work is enqueued on it; calls return before it finishes except
 *     where stated (the forward calls wait once, to read their counts back).
 *   - Parameter layout is structure-of-arrays float32, plane-major:
 *       means [3][n], scales [3][n] (activated, > 0), quats [4][n] (w,x,y,z;
 *       any non-zero norm, normalised inside), opacities [n] (activated, in
 *       (0,1)), sh [S][n] with S = 3 (sh_degree+1)^2 and plane k*3+c holding
 *       real-SH basis function k (index l(l+1)+m, Condon-Shortley phase) for
 *       colour channel c.
 *   - Images are planar float32 [3][height][width]; pixel (x, y) has its
 *     centre at image coordinate (x, y).
 *   - Return value: FGS_OK (0) or a negative FGS_ERR_* code; the message of
 *     the last failure on the calling thread is available from
 *     fgs_last_error().  No C++ exception crosses this boundary.
 *   - n = 0, or every Gaussian culled, is not an error: the image is bg.
 *     Gaussians with a non-finite mean, scale, quaternion, opacity or colour,
 *     or a zero quaternion, are culled.
 */
#ifndef FGS_H
#define FGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGS_OK 0
#define FGS_ERR_ARG (-1)       /* null pointer, bad size, unsupported model or degree */
#define FGS_ERR_WORKSPACE (-2) /* workspace too small; *k_out holds the intersections needed */
#define FGS_ERR_HIP (-3)       /* HIP runtime error; text in fgs_last_error() */
#define FGS_ERR_OVERFLOW (-4)  /* more than 2^31 - 1 intersections or Gaussians */

/* Camera models (fgs_camera.model).  Radial models place a point at
 * incidence theta = atan2(|(x_c, y_c)|, z_c) on its azimuth's ray at
 * distance f r(theta) from (c_x, c_y); Sec. 3.2 lists the four fisheye
 * projections, and the pinhole is the textbook r = tan theta.  The panorama
 * is the equirectangular projection of Sec. 5.3 (paragraph "Extension to Other
 * Cameras Models"): x_p = c_x + f_x atan2(x_c, z_c),
 * y_p = c_y + f_y atan2(y_c, |(x_c, z_c)|); the paper's image of width w and
 * height h has f_x = w / (2 pi), f_y = h / pi, c = (w/2, h/2).  Splats are
 * not wrapped across the panorama's left/right seam. */
#define FGS_MODEL_EQUIDISTANT 0   /* r = theta (Sec. 3.2) */
#define FGS_MODEL_PINHOLE 1       /* r = tan theta */
#define FGS_MODEL_PANORAMA 2      /* equirectangular (Sec. 5.3) */
#define FGS_MODEL_EQUISOLID 3     /* r = 2 sin(theta / 2) */
#define FGS_MODEL_ORTHOGRAPHIC 4  /* r = sin theta */
#define FGS_MODEL_STEREOGRAPHIC 5 /* r = 2 tan(theta / 2) */

#define FGS_MAX_BATCH 8 /* views per fgs_render_forward_batch call */

/* Forward flags */
#define FGS_SAVE_PIXEL_STATE 1u /* also store per-pixel final transmittance and
                                   contributor count; the backward then reads
                                   them instead of recomputing them */
#define FGS_RECT_BINNING 2u     /* bin each Gaussian to every tile of its
                                   3-sigma rectangle (the vanilla 3DGS lists)
                                   instead of only the tiles its alpha >= 1/255
                                   ellipse can reach (the default); images and
                                   gradients are the same either way */

/* Intrinsics of one view (Sec. 3.2: f_x, f_y, c_x, c_y).  Gaussians are culled
 * when |mu_c| <= near_dist or when the model's cull angle exceeds theta_max
 * (radians): for radial models the incidence angle theta, with theta_max < pi
 * (< pi/2 for the pinhole and orthographic models), since the splat of a
 * Gaussian near the rear axis is unbounded; for the panorama the absolute
 * latitude, with theta_max < pi/2, since its J is unbounded at the poles. */
typedef struct fgs_camera {
  int32_t width, height;
  double fx, fy, cx, cy;
  int32_t model;
  double near_dist;
  double theta_max;
} fgs_camera;

/* View transform x_c = W x + b (Sec. 3.1 "Transformation"), W row-major. */
typedef struct fgs_pose {
  double R[9];
  double t[3];
} fgs_pose;

/* Gaussian parameters (Eq. 1; Sigma = R S S^T R^T), device SoA planes. */
typedef struct fgs_gaussians {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacities;
  const float* sh;
  int64_t n;
  int32_t sh_degree; /* 0..3 */
} fgs_gaussians;

/* Gradient outputs, same layouts as fgs_gaussians.  With accumulate = 0
 * every element is WRITTEN (culled Gaussians get 0); with accumulate = 1 the
 * view's gradient is ADDED to the values already there (culled Gaussians
 * keep them), so the views of a training step share one set of buffers.
 * means2d, if not NULL, receives (or accumulates) dL/dmu_p as [2][n]
 * (pixel units). */
typedef struct fgs_grads {
  float* means;
  float* scales;
  float* quats;
  float* opacities;
  float* sh;
  float* means2d;
  int32_t accumulate;
} fgs_grads;

/* Byte offsets of the arrays inside a workspace, for inspection.  All
 * offsets are from the workspace base and 256-byte aligned. */
typedef struct fgs_layout {
  int64_t n;
  int32_t width, height, tiles_x, tiles_y;
  int64_t k_capacity;  /* intersections the workspace can hold */
  size_t bytes;        /* bytes the layout uses (<= workspace size) */
  size_t splats;       /* float4 [n][2]: (mu_x hi, mu_y hi, mu_x lo, mu_y lo),
                          (-A/2 log2 e, B/A, -(C - B^2/A)/2 log2 e, log2(1/(255 o))) */
  size_t colors;       /* float4 [n]: (o, r, g, b) */
  size_t depth_keys;   /* uint32 [n]: float bits of |mu_c|, 0xFFFFFFFF if culled */
  size_t tiles;        /* uint32 [n]: tiles touched (0 if culled) */
  size_t rects;        /* uint32 [n][2]: x0 | y0 << 16, x1 | y1 << 16 (half-open) */
  size_t radii;        /* int32 [n]: screen radius ceil(3 sqrt(lambda_max)), 0 if culled */
  size_t depth_order;  /* uint32 [n]: Gaussian ids sorted by (depth, id), culled last */
  size_t offsets;      /* uint32 [n]: exclusive scan, in depth order, of the tile rows each
                          visible Gaussian is binned over */
  size_t tile_keys;    /* uint32 [K]: sorted tile id per intersection */
  size_t tile_ids;     /* uint32 [K]: Gaussian id per sorted intersection */
  size_t ranges;       /* uint32 [tiles][2]: [start, end) of each tile's run */
  size_t grad2d;       /* float [slot][9]: backward scratch, per Gaussian dL/d mu_p xy, conic A B C,
                          opacity, rgb; Gaussian g at slot (g & ~63) | (9 g & 63) (a permutation
                          inside each group of 64), n rounded up to a multiple of 64 slots */
  size_t pixel_T;      /* float [H][W]: final transmittance (FGS_SAVE_PIXEL_STATE) */
  size_t pixel_last;   /* uint32 [H][W]: 1 + list index of the last blended Gaussian */
  size_t counters;     /* uint32 [18]: [0] K, [1] visible count, [2] forward flags, [3..10] K per view,
                          [11] / [12] smallest / largest depth key of a visible entry,
                          [14..15] K as a uint64, [16..17] tile rows binned as a uint64 */
} fgs_layout;

/* Library version string (static storage). */
const char* fgs_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* fgs_last_error(void);

/* Bytes of workspace a forward + backward of one view needs for n Gaussians,
 * a width x height image and up to k_capacity intersections. */
int fgs_workspace_bytes(int64_t n, int32_t width, int32_t height, int64_t k_capacity, size_t* bytes);

/* Layout of a workspace of `bytes` bytes (host-only computation). */
int fgs_workspace_layout(int64_t n, int32_t width, int32_t height, size_t bytes, fgs_layout* out);

/*
 * Forward render of one view: preprocess (cull, project mu by the
 * equidistant model, Sigma_p = J W Sigma W^T J^T, conic, 3-sigma radius, tile
 * rectangle, SH colour, depth |mu_c|), sort the visible Gaussians by depth,
 * emit one (tile, id) pair per covered tile, sort the pairs stably by tile,
 * find each tile's run and blend every pixel front to back (Eq. 3):
 *   alpha = min(0.99, o exp(q)), skipped if alpha < 1/255, stop before the
 *   Gaussian that would take T below 1e-4, C = sum c alpha T + T_final bg.
 *
 * workspace / workspace_bytes: device scratch, kept by the caller until the
 *   matching fgs_render_backward; its layout is fgs_workspace_layout().
 * out_rgb: device [3][H][W].
 * k_out: host, may be NULL; receives the number of intersections K.
 * flags: 0 or FGS_SAVE_PIXEL_STATE.
 * Waits for `stream` once, after the compaction, to read V, K and the depth
 * range: the counts are copied to a small pinned host buffer (one per calling
 * thread, allocated on its first call and kept for the life of the process)
 * and the stream is polled until they have arrived.  If K
 * exceeds the workspace's capacity it returns FGS_ERR_WORKSPACE with *k_out
 * = K and out_rgb untouched; the caller grows the workspace
 * (fgs_workspace_bytes(n, w, h, K, ...)) and calls again.
 */
int fgs_render_forward(const fgs_gaussians* g, const fgs_pose* pose, const fgs_camera* cam, const float bg[3],
                       uint32_t flags, void* workspace, size_t workspace_bytes, float* out_rgb, int64_t* k_out,
                       void* stream);

/*
 * Bytes of workspace fgs_render_forward_batch needs for nviews views (host
 * cams[nviews]: only width and height are read) and up to k_capacity
 * intersections in total.
 */
int fgs_batch_workspace_bytes(int64_t n, int32_t nviews, const fgs_camera* cams, int64_t k_capacity, size_t* bytes);

/*
 * Forward render of 1..FGS_MAX_BATCH views of one resident scene in one set of
 * launches (serving): one preprocess launch walks the Gaussians once and
 * projects each into every view, so each Gaussian's parameters are read
 * from HBM once per batch; the visible (view, Gaussian) entries share one
 * depth sort, their (tile, id) pairs use view-major tile ids and share one
 * tile sort, and one blend launch covers the tiles of all views.  Views
 * may differ in pose, resolution, focal length and field of view.
 *
 * poses, cams: host [nviews]; bgs: host [nviews][3]; out_rgb: host array of
 * nviews device pointers, view v's image [3][H_v][W_v].  k_views (host
 * [nviews]) and k_total (host) may be NULL; they receive the intersections
 * per view and in total, also when FGS_ERR_WORKSPACE is returned, so a
 * server can split the batch.  Waits for `stream` once, like
 * fgs_render_forward.  The workspace is the batch layout
 * (fgs_batch_workspace_bytes), not usable by fgs_render_backward.
 */
int fgs_render_forward_batch(const fgs_gaussians* g, int32_t nviews, const fgs_pose* poses, const fgs_camera* cams,
                             const float* bgs, void* workspace, size_t workspace_bytes, float* const* out_rgb,
                             int64_t* k_views, int64_t* k_total, void* stream);

/*
 * Backward of the same view.  Inputs must be those of the preceding
 * fgs_render_forward on this workspace.  dL_drgb: device [3][H][W].
 * Blend backward walks each pixel's contributors last to first, recovering
 * T_i = T_{i+1} / (1 - alpha_i) from the final transmittance (recomputed by a
 * front-to-back sweep unless the forward saved it), reduces per-Gaussian
 * gradients within each tile, adds them up over each block of four
 * neighbouring tiles in LDS and then to global accumulators; the
 * preprocess backward then applies the chain of Sec. 4.2-4.3 (J_phi and
 * dJ/dmu_c) and the covariance / SH derivatives.  Overwrites the
 * workspace's grad2d scratch.  Gradients are deterministic up to the order of
 * float atomic additions (fgs_render_backward_deterministic fixes that order).
 */
int fgs_render_backward(const fgs_gaussians* g, const fgs_pose* pose, const fgs_camera* cam, const float bg[3],
                        void* workspace, size_t workspace_bytes, const float* dL_drgb, const fgs_grads* grads,
                        void* stream);

/*
 * Bytes of scratch fgs_render_backward_deterministic needs for n Gaussians
 * and up to k_capacity intersections (the K the view's forward reported):
 * 36 bytes per intersection for the per-entry sums, 4 per Gaussian for the
 * start of its run, and a scan's partial sums.
 */
int fgs_deterministic_workspace_bytes(int64_t n, int64_t k_capacity, size_t* bytes);

/*
 * fgs_render_backward with a run-to-run deterministic result.  Each Gaussian
 * owns a run of as many slots as tiles it was binned to (an exclusive scan of
 * the tile counts).  The blend backward stores each list entry's nine
 * 2D-gradient sums (the reverse pass of Eq. 3 as in Sec. 4.2) in the slot of
 * the entry's tile among its Gaussian's tiles, in tile order, instead of
 * adding them to per-Gaussian accumulators with float atomics; one wave per
 * Gaussian then adds its run in an order fixed by the run's length (strided
 * partial sums, then a fixed butterfly).  The same inputs give bit-identical
 * gradients on every call; they differ from fgs_render_backward's only by the
 * order of the float additions.
 * det_workspace: device, caller-owned, at least
 *   fgs_deterministic_workspace_bytes(n, K) bytes for the forward's K (its
 *   contents on entry do not matter; it holds nothing afterwards).
 * Reads K back from the workspace once (one wait for `stream`); returns
 * FGS_ERR_WORKSPACE, with the bytes needed in fgs_last_error(), if
 * det_workspace is smaller.  Every other argument as fgs_render_backward.
 */
int fgs_render_backward_deterministic(const fgs_gaussians* g, const fgs_pose* pose, const fgs_camera* cam,
                                      const float bg[3], void* workspace, size_t workspace_bytes,
                                      const float* dL_drgb, const fgs_grads* grads, void* det_workspace,
                                      size_t det_workspace_bytes, void* stream);

/*
 * L1 photometric loss of a rendered image against a target, the L1 term of
 * the 3DGS objective the paper trains with (Sec. 5.1):
 *   L = (1 / count) sum_j |image_j - target_j|,
 *   dL/dimage_j = sign(image_j - target_j) * dL_dloss[0] / count
 * (sign 0 where the two are equal; the quotient dL_dloss[0] / count is
 * taken in double and rounded to float, then multiplied by the sign).
 *
 * fgs_l1_loss: image, target device float32 [count] (any layout, the same
 * for both), 16-byte aligned; partials device scratch of FGS_L1_PARTIALS
 * doubles (caller-owned, overwritten); loss device float32 scalar, written
 * as the mean.  The sum runs in double over a fixed grid, so the loss is
 * bit-deterministic.
 * fgs_l1_loss_backward: dL_dloss device float32 scalar (the upstream
 * gradient); dL_dimage device float32 [count], 16-byte aligned, overwritten.
 * Both only enqueue work on the stream.  FGS_ERR_ARG for a null pointer,
 * count <= 0 or a misaligned image; FGS_ERR_OVERFLOW past 2^31 - 1 values.
 */
#define FGS_L1_PARTIALS 1024
int fgs_l1_loss(const float* image, const float* target, int64_t count, double* partials, float* loss, void* stream);
int fgs_l1_loss_backward(const float* image, const float* target, int64_t count, const float* dL_dloss,
                         float* dL_dimage, void* stream);

/*
 * fgs_l1_loss without the partials argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid allocation): the FGS_L1_PARTIALS
 * partial sums live in an array the library holds on every GPU it runs on
 * (8 KiB each, kept until the process ends), found on the first call on each
 * device.  It allocates nothing and calls no allocating routine; every
 * partial is written before it is read, so nothing needs clearing.  Same
 * kernels, same result bit for bit, same errors as fgs_l1_loss; count is at
 * most 2^31 - 1 (FGS_ERR_OVERFLOW beyond).  Calls that overlap on one GPU
 * (two streams, or two host threads) share that array and race: serialise
 * them.
 */
int fgs_l1_loss_noalloc(const float* image, const float* target, int64_t count, float* loss, void* stream);

/*
 * Spatial order of a scene, for storing a resident scene once (not part of
 * the per-view path).  The paper's rasterizer reads each Gaussian's
 * parameters, SH coefficients included, from structure-of-arrays planes; a
 * view culls whole regions (behind the fisheye, outside the image), and with
 * the Gaussians in random order every cache line of every plane still holds
 * some visible Gaussian.  Sorting the scene by the Morton code of its means
 * (a 1024^3 grid over their bounding box) puts culled Gaussians in long runs
 * whose lines the preprocess then skips.
 *
 * fgs_spatial_order: means device [3][n]; order device uint32 [n] receives
 * the permutation (order[j] = the Gaussian at position j), ties and
 * non-finite means (sorted last) in id order; workspace device scratch of
 * fgs_spatial_order_workspace_bytes(n) bytes.  Enqueues work only.
 * fgs_gather_planes: out[p][j] = in[p][order[j]] for `planes` planes of
 * length n (device, in != out): apply the order to every parameter array.
 * Images and gradients of the reordered scene equal the original's (the
 * gradients reordered the same way) up to depth ties, broken by the new ids.
 */
int fgs_spatial_order_workspace_bytes(int64_t n, size_t* bytes);
int fgs_spatial_order(const float* means, int64_t n, uint32_t* order, void* workspace, size_t workspace_bytes,
                      void* stream);
int fgs_gather_planes(const float* in, float* out, int64_t planes, int64_t n, const uint32_t* order, void* stream);

/*
 * Per-kernel timing with HIP events, for benchmarks and tracing.  While
 * enabled, every kernel launch of the library is bracketed by two events
 * recorded on the stream it is launched on; fgs_profile_read waits for the
 * recorded events and returns the accumulated milliseconds and launch count
 * per kernel.  Turning recording on clears earlier data.  Process-wide, not
 * meant for concurrent calls from several threads.
 */
#define FGS_PROF_MAX_KERNELS 32
typedef struct fgs_profile {
  int32_t count;                                /* kernels listed */
  const char* names[FGS_PROF_MAX_KERNELS];      /* static strings */
  int64_t launches[FGS_PROF_MAX_KERNELS];
  double total_ms[FGS_PROF_MAX_KERNELS];
} fgs_profile;

int fgs_profile_enable(int32_t on);
int fgs_profile_read(fgs_profile* out);

#ifdef __cplusplus
}
#endif

#endif /* FGS_H */
