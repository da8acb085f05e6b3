// Per-Gaussian preprocess (forward) and its backward.
//
// Forward, one thread per Gaussian, in the order of the 3DGS preprocess the
// paper modifies (Sec. 4.1; only the projection changes, Sec. 4.2-4.3):
// cull (non-finite, |mu_c| <= near, theta > theta_max), project the mean by
// the equidistant model (Sec. 3.2) or another camera model, Sigma = R S S^T R^T (Eq. 1), T = J W,
// Sigma_p = T Sigma T^T (Eq. 2) plus a 0.3 px^2 low-pass dilation, conic,
// radius = ceil(3 sqrt(lambda_max)), tile rectangle, SH colour, depth key.
//
// Loads are structure-of-arrays, so every load instruction of a wave is one
// contiguous 256-byte segment per plane.
#include "fgs_internal.hpp"
#include "fisheye.hpp"
#include "reach.hpp"

namespace fgs {
namespace {

constexpr double kLog2e = 1.4426950408889634;
constexpr double kDilation = 0.3;
constexpr double kMaxRadius = 1073741824.0;  // 2^30: keeps the radius an int; the rect is clamped anyway

struct PreArgs {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  uint32_t n;
  int sh_degree;
  // outputs, entry view * n + i
  float4* splats;  // [entry][2]: position, conic
  float4* colors;  // [entry]: opacity, rgb
  float4* colorjac;  // one view only, [i][3]: d rgb / d dir (9 floats, row per channel), clamp mask; or null
  uint32_t* depth_keys;
  uint32_t* tiles;
  uint2* rects;
  int32_t* radii;
  uint32_t* block_tiles;  // [view][block] tiles touched (multi-view only)
  int tight;              // count only the tiles the alpha >= 1/255 ellipse reaches
  uint32_t* rowrange;     // tight: [entry] first | (last + 1) << 16 of the rows with a kept tile
  uint32_t* block_kept;   // one view: [block] entries the block kept (tile count > 0 after the colour)
  uint32_t* counters;     // cleared by the first block, with the flags stored (no launch of its own)
  uint32_t flags;
  ViewBatch batch;
};

// The forward's device counters start at zero, the flags slot holding the
// call's flags; the first kernel of the forward writes them.
__device__ inline void clear_counters(const PreArgs& a) {
  if (blockIdx.x == 0 && threadIdx.x < (uint32_t)kNumCounters)
    a.counters[threadIdx.x] = threadIdx.x == (uint32_t)kCountFlags ? a.flags : 0u;
}

struct Geometry {
  double pc[3];
  FisheyePoint P;   // equidistant model
  OtherPoint O;     // the other models
  double mu[2];
  double Rq[9];  // rotation of the normalised quaternion
  double qn[4], qnorm;
  double s[3];
  double Sig[6];  // xx xy xz yy yz zz
  double T[6];    // J W
  double J[6];
  double Sp[3];   // dilated 2D covariance: xx xy yy
  double det;
  double conic[3];
};

// Which camera models a kernel instantiation handles: only the equidistant
// one, only the others, or any (a batch that mixes them).  Keeping the
// equidistant path alone in its own instantiation keeps its register count.
enum ModelClass { kMcEquidistant = 0, kMcOther = 1, kMcAny = 2 };

__host__ inline int model_class_of(const ViewBatch& b) {
  bool eq = false, other = false;
  for (int k = 0; k < b.count; ++k) (b.v[k].model == kModelEquidistant ? eq : other) = true;
  return eq && other ? kMcAny : (other ? kMcOther : kMcEquidistant);
}

// Returns false if culled.  Shared by forward and backward so both take the
// same decisions on the same inputs.
template <int MC>
__device__ inline bool compute_geometry(const float* means, const float* scales, const float* quats,
                                        const float* opac, uint32_t i, uint32_t n, const ViewParams& v,
                                        bool need_m, Geometry& G) {
  const float mf[3] = {means[i], means[n + i], means[2 * n + i]};
  const float sf[3] = {scales[i], scales[n + i], scales[2 * n + i]};
  const float qf[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
  const float o = opac[i];
  bool finite = isfinite(o);
  for (int a = 0; a < 3; ++a) finite = finite && isfinite(mf[a]) && isfinite(sf[a]);
  for (int a = 0; a < 4; ++a) finite = finite && isfinite(qf[a]);
  if (!finite) return false;
  double q2 = 0.0;
  for (int a = 0; a < 4; ++a) q2 += (double)qf[a] * (double)qf[a];
  if (!(q2 > 0.0)) return false;
  // mu_c = W mu + b, rows summed left to right
  for (int r = 0; r < 3; ++r)
    G.pc[r] = ((v.R[r * 3 + 0] * (double)mf[0] + v.R[r * 3 + 1] * (double)mf[1]) + v.R[r * 3 + 2] * (double)mf[2]) +
              v.t[r];
  const double x = G.pc[0], y = G.pc[1], z = G.pc[2];
  const double dist = sqrt((x * x + y * y) + z * z);
  if (!(dist > v.near_dist)) return false;
  if (MC == kMcEquidistant || (MC == kMcAny && v.model == kModelEquidistant)) {
    G.P.x = x;
    G.P.y = y;
    G.P.z = z;
    fisheye_terms(G.P, need_m);
    if (!(G.P.theta <= v.theta_max)) return false;
    if (G.P.lz > 0.0) {
      const double t = G.P.theta / G.P.lz;
      G.mu[0] = v.cx + v.fx * t * x;
      G.mu[1] = v.cy + v.fy * t * y;
    } else {
      G.mu[0] = v.cx;
      G.mu[1] = v.cy;
    }
    fisheye_jacobian(G.P, v.fx, v.fy, G.J);
  } else {
    G.O.x = x;
    G.O.y = y;
    G.O.z = z;
    if (!other_project(v.model, G.O, v.theta_max, v.fx, v.fy, v.cx, v.cy, need_m, G.mu, G.J)) return false;
  }
  // Sigma = M M^T, M = R S
  G.qnorm = sqrt(q2);
  const double iq = 1.0 / G.qnorm;
  for (int a = 0; a < 4; ++a) G.qn[a] = (double)qf[a] * iq;
  quat_to_rot(G.qn, G.Rq);
  for (int a = 0; a < 3; ++a) G.s[a] = (double)sf[a];
  double M[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[r * 3 + c] = G.Rq[r * 3 + c] * G.s[c];
  G.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  G.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  G.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  G.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  G.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  G.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      G.T[r * 3 + c] = G.J[r * 3 + 0] * v.R[0 * 3 + c] + G.J[r * 3 + 1] * v.R[1 * 3 + c] + G.J[r * 3 + 2] * v.R[2 * 3 + c];
  // Sigma_p = T Sigma T^T
  double TS[6];
  for (int r = 0; r < 2; ++r) {
    const double* t = &G.T[r * 3];
    TS[r * 3 + 0] = t[0] * G.Sig[0] + t[1] * G.Sig[1] + t[2] * G.Sig[2];
    TS[r * 3 + 1] = t[0] * G.Sig[1] + t[1] * G.Sig[3] + t[2] * G.Sig[4];
    TS[r * 3 + 2] = t[0] * G.Sig[2] + t[1] * G.Sig[4] + t[2] * G.Sig[5];
  }
  G.Sp[0] = TS[0] * G.T[0] + TS[1] * G.T[1] + TS[2] * G.T[2] + kDilation;
  G.Sp[1] = TS[0] * G.T[3] + TS[1] * G.T[4] + TS[2] * G.T[5];
  G.Sp[2] = TS[3] * G.T[3] + TS[4] * G.T[4] + TS[5] * G.T[5] + kDilation;
  G.det = G.Sp[0] * G.Sp[2] - G.Sp[1] * G.Sp[1];
  if (!(G.det > 0.0)) return false;
  const double idet = 1.0 / G.det;
  G.conic[0] = G.Sp[2] * idet;
  G.conic[1] = -G.Sp[1] * idet;
  G.conic[2] = G.Sp[0] * idet;
  return true;
}

// The 3 (DEG+1)^2 SH coefficients of Gaussian i, plane k*3+c, into registers.
template <int DEG>
__device__ inline void load_sh(const float* __restrict__ sh, uint32_t i, uint32_t n, float c[48]) {
  constexpr int nc = 3 * (DEG + 1) * (DEG + 1);
#pragma unroll
  for (int k = 0; k < nc; ++k) c[k] = sh[(size_t)k * n + i];
}

// Colour from SH in float: rgb_c = sum_k c[k*3+c] Y_k(dir) + 0.5 (the
// caller clamps at 0).
template <int DEG>
__device__ inline void sh_color(const float c[48], const float dir[3], float rgb[3], float Y[16]) {
  constexpr int nb = (DEG + 1) * (DEG + 1);
  sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
  float acc[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
  for (int k = 0; k < nb; ++k)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) acc[ch] += c[k * 3 + ch] * Y[k];
  for (int ch = 0; ch < 3; ++ch) rgb[ch] = acc[ch];
}

__device__ inline void view_dir(const float* means, uint32_t i, uint32_t n, const double campos[3], float dir[3],
                                double vdir[3], double& vlen) {
  for (int a = 0; a < 3; ++a) vdir[a] = (double)means[a * n + i] - campos[a];
  vlen = sqrt(vdir[0] * vdir[0] + vdir[1] * vdir[1] + vdir[2] * vdir[2]);
  const double il = 1.0 / vlen;
  for (int a = 0; a < 3; ++a) dir[a] = (float)(vdir[a] * il);
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// block_tiles[v * nblocks + b] -> out[v]: one block per view.
__global__ __launch_bounds__(kBlock) void view_sums_kernel(const uint32_t* block_tiles, uint32_t nblocks,
                                                           uint32_t* out) {
  __shared__ uint32_t s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  uint32_t acc = 0;
  for (uint32_t b = threadIdx.x; b < nblocks; b += kBlock) acc += block_tiles[(size_t)blockIdx.x * nblocks + b];
  acc = wave_sum_u32(acc);
  if ((threadIdx.x & 63) == 0) atomicAdd(&s_sum, acc);
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = s_sum;
}

// Tiles that reach_row keeps over the tile rows [y0, y0 + nr) of each
// lane's splat, and the first and last of those rows with a kept tile, for a
// whole wave: the wave's (lane, row) pairs are dealt out 64 at a time, so a
// lane with a tall rect (the large splats) does not hold up the other 63.
// Every lane of the wave takes part; lanes without rows pass nr = 0.  The
// per-row evaluation is reach_row on the owner's own values, so the counts
// equal the per-lane loop's (and the duplication's) exactly.
struct RowCountLds {
  uint32_t count[64], first[64], end[64];  // per lane of the wave
};

// Orders the LDS accesses of one wave's lanes: what a lane wrote before it
// is visible to every lane of the wave after it (the wave executes in lock
// step; the fences keep the compiler from reordering or forwarding).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint32_t wave_bcast_u32(uint32_t v, uint32_t src) { return (uint32_t)__shfl((int)v, (int)src, 64); }
__device__ inline float wave_bcast_f32(float v, uint32_t src) { return __shfl(v, (int)src, 64); }

__device__ inline void wave_count_rows(const SplatReach& rr, uint32_t nr, uint32_t x0, uint32_t x1, uint32_t y0,
                                       RowCountLds& L, uint32_t& area, uint32_t& ya, uint32_t& yb) {
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t incl = nr;  // inclusive prefix sum of nr over the wave
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = (uint32_t)__shfl_up((int)incl, d, 64);
    if (lane >= (uint32_t)d) incl += t;
  }
  const uint32_t excl = incl - nr;
  const uint32_t total = __builtin_amdgcn_readfirstlane(wave_bcast_u32(incl, 63u));
  L.count[lane] = 0u;
  L.first[lane] = 0xFFFFFFFFu;
  L.end[lane] = 0u;
  wave_sync();
  const float kind = (float)rr.kind;
  for (uint32_t base = 0; base < total; base += 64u) {
    // owner of pair base + lane: the last lane whose pairs start at or
    // before it (the exclusive prefixes do not decrease over the lanes, and
    // a later lane without rows starts past it)
    const uint32_t item = base + lane;
    uint32_t own = 0;
    for (uint32_t step = 32; step >= 1; step >>= 1) {
      const uint32_t probe = own + step;
      if (wave_bcast_u32(excl, probe) <= item) own = probe;
    }
    SplatReach ro;
    ro.mx = wave_bcast_f32(rr.mx, own);
    ro.my = wave_bcast_f32(rr.my, own);
    ro.Pa = wave_bcast_f32(rr.Pa, own);
    ro.da = wave_bcast_f32(rr.da, own);
    ro.beta = wave_bcast_f32(rr.beta, own);
    ro.ry = wave_bcast_f32(rr.ry, own);
    ro.ds = wave_bcast_f32(rr.ds, own);
    ro.kind = (int)wave_bcast_f32(kind, own);
    const uint32_t ox0 = wave_bcast_u32(x0, own), ox1 = wave_bcast_u32(x1, own);
    const uint32_t oy0 = wave_bcast_u32(y0, own), oexcl = wave_bcast_u32(excl, own);
    if (item < total) {
      const uint32_t ty = oy0 + (item - oexcl);
      int c0, c1;
      reach_row(ro, (int)ty, (int)ox0, (int)ox1, c0, c1);
      if (c1 > c0) {
        atomicAdd(&L.count[own], (uint32_t)(c1 - c0));
        atomicMin(&L.first[own], ty);
        atomicMax(&L.end[own], ty + 1u);
      }
    }
  }
  wave_sync();
  area = L.count[lane];
  ya = L.first[lane];
  yb = L.end[lane];
}

// Geometry of entry e = (view vi, Gaussian i): cull, project, conic, radius,
// tile rect, depth key.  A culled entry writes only its tile count (0) and an
// all-ones depth key.  Returns the tile count.  Every lane of the wave calls
// it (the tight tile count is shared across the wave); lanes past the last
// Gaussian pass active = false and write nothing.
template <int MC>
__device__ inline uint32_t entry_geometry(const PreArgs& a, uint32_t vi, uint32_t i, size_t e, bool active,
                                          RowCountLds& L) {
  const uint32_t n = a.n;
  const ViewParams& vp = a.batch.v[vi];
  bool keep = false;
  uint32_t x0 = 0, y0 = 0, x1 = 0, y1 = 0, area = 0;
  float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0;
  double rad = 0.0, dist = 0.0;
  if (active) {
    Geometry G;
    if (compute_geometry<MC>(a.means, a.scales, a.quats, a.opac, i, n, vp, false, G)) {
      const double mid = 0.5 * (G.Sp[0] + G.Sp[2]);
      const double lam = mid + sqrt(fmax(0.1, mid * mid - G.det));
      rad = ceil(3.0 * sqrt(lam));
      if (rad > kMaxRadius) rad = kMaxRadius;
      const double gx = vp.tiles_x, gy = vp.tiles_y;
      const double vx0 = floor((G.mu[0] - rad) / kTile), vy0 = floor((G.mu[1] - rad) / kTile);
      const double vx1 = floor((G.mu[0] + rad + (kTile - 1)) / kTile),
                   vy1 = floor((G.mu[1] + rad + (kTile - 1)) / kTile);
      x0 = (uint32_t)fmin(fmax(vx0, 0.0), gx);
      y0 = (uint32_t)fmin(fmax(vy0, 0.0), gy);
      x1 = (uint32_t)fmin(fmax(vx1, 0.0), gx);
      y1 = (uint32_t)fmin(fmax(vy1, 0.0), gy);
      area = (x1 - x0) * (y1 - y0);
      if (area != 0) {
        keep = true;
        const float o = a.opac[i];
        const double A = G.conic[0], B = G.conic[1], iA = 1.0 / A;
        const float hx = (float)G.mu[0], hy = (float)G.mu[1];
        s0 = make_float4(hx, hy, (float)(G.mu[0] - (double)hx), (float)(G.mu[1] - (double)hy));
        // D = C - B^2 / A = 1 / (det' A), det' the determinant of Sigma'.
        // The alpha cut-off log2(1 / (255 o)) of the float product 255 o is
        // taken in double and rounded once, like the other record values.
        s1 = make_float4((float)(-0.5 * kLog2e * A), (float)(B * iA), (float)(-0.5 * kLog2e / (G.det * A)),
                         (float)(-log2((double)(255.0f * o))));
        dist = sqrt((G.pc[0] * G.pc[0] + G.pc[1] * G.pc[1]) + G.pc[2] * G.pc[2]);
      }
    }
  }
  if (a.tight) {  // the tiles of the rect the splat's pixels can lie in
    SplatReach rr;
    if (keep) {
      rr = splat_reach(s0, s1);
    } else {
      rr.mx = rr.my = rr.Pa = rr.da = rr.beta = rr.ry = rr.ds = 0.0f;
      rr.kind = 0;
    }
    uint32_t ya = 0, yb = 0;
    wave_count_rows(rr, keep ? y1 - y0 : 0u, x0, x1, y0, L, area, ya, yb);
    if (keep && area == 0) keep = false;
    if (keep) a.rowrange[e] = ya | (yb << 16);
  }
  if (!active) return 0;
  uint32_t key = 0xFFFFFFFFu, ntiles = 0;
  if (keep) {
    a.splats[2 * e + 0] = s0;
    a.splats[2 * e + 1] = s1;
    a.rects[e] = make_uint2(x0 | (y0 << 16), x1 | (y1 << 16));
    a.radii[e] = (int32_t)rad;
    key = __float_as_uint((float)dist);
    ntiles = area;
  }
  a.depth_keys[e] = key;
  a.tiles[e] = ntiles;
  return ntiles;
}

// SH colour of a kept entry, coefficients c already loaded.  An entry whose
// colour is not finite is culled here, before the scans read the tile
// counts.  Returns the entry's tile count afterwards.
template <int DEG>
__device__ inline uint32_t entry_color(const PreArgs& a, uint32_t vi, uint32_t i, size_t e, const float c[48],
                                       uint32_t ntiles) {
  float dir[3], Y[16], rgb[3];
  double vd[3], vlen;
  view_dir(a.means, i, a.n, a.batch.v[vi].campos, dir, vd, vlen);
  sh_color<DEG>(c, dir, rgb, Y);
  if (isfinite(rgb[0]) && isfinite(rgb[1]) && isfinite(rgb[2])) {
    a.colors[e] = make_float4(a.opac[i], fmaxf(rgb[0], 0.0f), fmaxf(rgb[1], 0.0f), fmaxf(rgb[2], 0.0f));
    if (a.colorjac) {
      // what the backward needs of the SH: per channel the gradient of the
      // colour in the view direction (sum_k c_k grad Y_k) and whether the
      // channel was clamped at 0, so that it need not read the coefficients
      float D[3][3];
      sh_grad_dir3<DEG>(dir[0], dir[1], dir[2], c, D);
      const uint32_t mask = (rgb[0] < 0.0f ? 1u : 0u) | (rgb[1] < 0.0f ? 2u : 0u) | (rgb[2] < 0.0f ? 4u : 0u);
      a.colorjac[3 * e + 0] = make_float4(D[0][0], D[0][1], D[0][2], D[1][0]);
      a.colorjac[3 * e + 1] = make_float4(D[1][1], D[1][2], D[2][0], D[2][1]);
      a.colorjac[3 * e + 2] = make_float4(D[2][2], __uint_as_float(mask), 0.0f, 0.0f);
    }
    return ntiles;
  }
  a.tiles[e] = 0;
  a.depth_keys[e] = 0xFFFFFFFFu;
  return 0;
}

// One view: geometry and colour in one thread (the coefficients are read
// only for the Gaussians the view keeps).
template <int DEG, int MC>
__global__ __launch_bounds__(kBlock) void preprocess_fused_kernel(PreArgs a) {
  __shared__ RowCountLds rows_lds[kBlock / 64];
  clear_counters(a);
  __shared__ uint32_t s_kept;
  if (threadIdx.x == 0) s_kept = 0u;
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  uint32_t ntiles = entry_geometry<MC>(a, 0u, i, i, i < a.n, rows_lds[threadIdx.x >> 6]);
  if (ntiles != 0) {
    float c[48];
    load_sh<DEG>(a.sh, i, a.n, c);
    ntiles = entry_color<DEG>(a, 0u, i, i, c, ntiles);
  }
  // the block's count of kept entries: the compaction's scan adds these up
  // instead of counting the tile counts again
  const uint64_t kept = __ballot(ntiles != 0);
  __syncthreads();
  if ((threadIdx.x & 63u) == 0u && kept != 0ull) atomicAdd(&s_kept, (uint32_t)__builtin_popcountll(kept));
  __syncthreads();
  if (threadIdx.x == 0) a.block_kept[blockIdx.x] = s_kept;
}

// Batches: the geometry and the colour run as two kernels over a grid of
// nviews x blocks-per-view blocks (one thread per entry; a thread looping
// over the views needed over 200 VGPRs once the compiler hoisted the
// view-invariant work).  The xcd_chunk order puts the views of one Gaussian
// block on one XCD at about the same time, so the parameters come from HBM
// once per batch and from that XCD's L2 for the other views.
__device__ inline void entry_of_block(uint32_t nviews, uint32_t& vi, uint32_t& i) {
  const uint32_t logical = xcd_chunk(blockIdx.x, gridDim.x);
  vi = logical % nviews;
  i = (logical / nviews) * kBlock + threadIdx.x;
}

template <int MC>
__global__ __launch_bounds__(kBlock) void preprocess_kernel(PreArgs a) {
  __shared__ RowCountLds rows_lds[kBlock / 64];
  clear_counters(a);
  uint32_t vi, i;
  entry_of_block((uint32_t)a.batch.count, vi, i);
  entry_geometry<MC>(a, vi, i, (size_t)vi * a.n + i, i < a.n, rows_lds[threadIdx.x >> 6]);
}

// Also leaves each block's tile total in block_tiles[view][block] (a plain
// store per block, summed per view afterwards: no contended atomics).
template <int DEG>
__global__ __launch_bounds__(kBlock) void color_kernel(PreArgs a) {
  uint32_t vi, i;
  entry_of_block((uint32_t)a.batch.count, vi, i);
  const uint32_t n = a.n;
  const size_t e = (size_t)vi * n + i;
  const bool in_range = i < n;
  uint32_t ntiles = in_range ? a.tiles[e] : 0u;
  // the coefficients are loaded without waiting for the visibility (a wave
  // with any visible lane fetches all of their lines)
  float c[48];
  if (in_range) load_sh<DEG>(a.sh, i, n, c);
  if (ntiles != 0) ntiles = entry_color<DEG>(a, vi, i, e, c, ntiles);
  __shared__ uint32_t s_sum;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  const uint32_t wsum = wave_sum_u32(ntiles);
  if ((threadIdx.x & 63) == 0) atomicAdd(&s_sum, wsum);
  __syncthreads();
  // thread 0 holds the block's first Gaussian, so i / kBlock is the block of the view
  if (threadIdx.x == 0) a.block_tiles[(size_t)vi * (gridDim.x / a.batch.count) + i / kBlock] = s_sum;
}

// ---------------------------------------------------------------------------
// Backward.  Inputs per Gaussian: the blend's accumulated dL/d(mu_p, conic A B
// C, opacity, rgb).  Chain (Sec. 4.2, 4.3):
//   dL/dSigma' = -Q G Q,  dL/dT = 2 dL/dSigma' T Sigma,
//   dL/dSigma = T^T dL/dSigma' T,  dL/dJ = dL/dT W^T,
//   dL/dmu_c = J^T dL/dmu_p + sum_ij dL/dJ_ij dJ_ij/dmu_c,
//   dL/dmu = W^T dL/dmu_c + colour term;  Sigma -> (s, q) through M = R S.
// ---------------------------------------------------------------------------
struct PreBwdArgs {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  uint32_t n;
  int sh_degree;
  ViewParams v;
  const uint32_t* tiles;
  const float* grad2d;  // [grad_slot(i)][9]
  const float4* colorjac;  // [n][3], from the forward
  float* g_means;
  float* g_scales;
  float* g_quats;
  float* g_opac;
  float* g_sh;
  float* g_means2d;
  int accumulate;  // add to the gradient buffers instead of writing them
};

// Colour part of the backward for Gaussian i: dL/dSH and the term of dL/dmu
// that flows through the view direction of the SH evaluation (written to
// g_means; the geometry part adds its own term).  It streams the 4S bytes of
// gradient out without reading the coefficients.
template <int DEG>
__device__ inline void sh_backward_body(const PreBwdArgs& a, uint32_t i) {
  const uint32_t n = a.n;
  constexpr int nb = (DEG + 1) * (DEG + 1);
  // one path for every lane (culled lanes compute and select zeros), so each
  // plane is written by one full-wave store.  The SH coefficients are not
  // read: the forward left, per channel, the colour's gradient in the view
  // direction and the clamp mask.  Adding to earlier views' gradients, a
  // culled Gaussian has nothing to add and touches nothing.
  const bool vis = a.tiles[i] != 0;
  if (a.accumulate && !vis) return;
  const float* g2 = a.grad2d + 9 * (size_t)grad_slot(i);
  const float grgb[3] = {g2[6], g2[7], g2[8]};
  float4 J0 = make_float4(0.f, 0.f, 0.f, 0.f), J1 = J0, J2 = J0;
  if (vis) {
    J0 = a.colorjac[3 * (size_t)i + 0];
    J1 = a.colorjac[3 * (size_t)i + 1];
    J2 = a.colorjac[3 * (size_t)i + 2];
  }
  const uint32_t mask = __float_as_uint(J2.y);
  float dir[3], Y[16];
  double vd[3], vlen;
  view_dir(a.means, i, n, a.v.campos, dir, vd, vlen);
  sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
  float gcol[3];
  for (int ch = 0; ch < 3; ++ch) gcol[ch] = (vis && !((mask >> ch) & 1u)) ? grgb[ch] : 0.0f;
  if (a.accumulate) {
#pragma unroll
    for (int k = 0; k < nb; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) a.g_sh[(size_t)(k * 3 + ch) * n + i] += Y[k] * gcol[ch];
  } else {
#pragma unroll
    for (int k = 0; k < nb; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) a.g_sh[(size_t)(k * 3 + ch) * n + i] = Y[k] * gcol[ch];
  }
  double gm[3] = {0.0, 0.0, 0.0};
  if constexpr (DEG > 0) {
    // sum over channels of dL/drgb_c times the colour's gradient in the direction
    const float gd[3] = {gcol[0] * J0.x + gcol[1] * J0.w + gcol[2] * J1.z,
                         gcol[0] * J0.y + gcol[1] * J1.x + gcol[2] * J1.w,
                         gcol[0] * J0.z + gcol[1] * J1.y + gcol[2] * J2.x};
    // d dir / d v = (I - dir dir^T) / |v|
    const double dd = (double)dir[0] * gd[0] + (double)dir[1] * gd[1] + (double)dir[2] * gd[2];
    for (int e = 0; e < 3; ++e) gm[e] = ((double)gd[e] - (double)dir[e] * dd) / vlen;
  }
  if (!a.accumulate)
    for (int ch = 0; ch < 3; ++ch) a.g_means[ch * n + i] = vis ? (float)gm[ch] : 0.0f;
  else if (vis && DEG > 0)
    for (int ch = 0; ch < 3; ++ch) a.g_means[ch * n + i] += (float)gm[ch];
}

// Geometry part of the backward (Sec. 4.3) for Gaussian i: from
// dL/d(mu_p, conic, opacity) to dL/d(mu, s, q, o) through the fisheye
// Jacobian, in fp64.  Runs after the colour part and adds to the direction
// term it left in g_means.
template <int MC>
__device__ inline void geometry_backward_body(const PreBwdArgs& a, uint32_t i) {
  const uint32_t n = a.n;
  Geometry G;
  const bool visible =
      a.tiles[i] != 0 && compute_geometry<MC>(a.means, a.scales, a.quats, a.opac, i, n, a.v, true, G);
  if (!visible) {
    if (a.accumulate) return;
    for (int c = 0; c < 3; ++c) { a.g_means[c * n + i] = 0.0f; a.g_scales[c * n + i] = 0.0f; }
    for (int c = 0; c < 4; ++c) a.g_quats[c * n + i] = 0.0f;
    a.g_opac[i] = 0.0f;
    if (a.g_means2d) { a.g_means2d[i] = 0.0f; a.g_means2d[n + i] = 0.0f; }
    return;
  }
  // written, or added to what earlier views left (the SH kernel has already
  // put this view's view-direction term into g_means either way); a written
  // buffer is never read, it may hold anything
  const bool acc = a.accumulate != 0;
  auto put = [acc](float* p, float v) { *p = acc ? *p + v : v; };
  const float* g2 = a.grad2d + 9 * (size_t)grad_slot(i);
  const double gmu[2] = {g2[0], g2[1]};
  const double gA = g2[2], gB = g2[3], gC = g2[4];
  const float go = g2[5];
  // H = dL/dSigma' = -Q Gs Q with Gs = [[gA, gB/2], [gB/2, gC]]
  const double Q00 = G.conic[0], Q01 = G.conic[1], Q11 = G.conic[2];
  const double G00 = gA, G01 = 0.5 * gB, G11 = gC;
  const double QG00 = Q00 * G00 + Q01 * G01, QG01 = Q00 * G01 + Q01 * G11;
  const double QG10 = Q01 * G00 + Q11 * G01, QG11 = Q01 * G01 + Q11 * G11;
  const double H00 = -(QG00 * Q00 + QG01 * Q01);
  const double H01 = -(QG00 * Q01 + QG01 * Q11);
  const double H11 = -(QG10 * Q01 + QG11 * Q11);
  // dL/dT = 2 H T Sigma
  double HT[6];
  for (int c = 0; c < 3; ++c) {
    HT[0 * 3 + c] = H00 * G.T[0 * 3 + c] + H01 * G.T[1 * 3 + c];
    HT[1 * 3 + c] = H01 * G.T[0 * 3 + c] + H11 * G.T[1 * 3 + c];
  }
  const double* S = G.Sig;
  double dT[6];
  for (int r = 0; r < 2; ++r) {
    const double* h = &HT[r * 3];
    dT[r * 3 + 0] = 2.0 * (h[0] * S[0] + h[1] * S[1] + h[2] * S[2]);
    dT[r * 3 + 1] = 2.0 * (h[0] * S[1] + h[1] * S[3] + h[2] * S[4]);
    dT[r * 3 + 2] = 2.0 * (h[0] * S[2] + h[1] * S[4] + h[2] * S[5]);
  }
  // dL/dSigma = T^T H T (full symmetric 3x3)
  double dS[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) dS[r * 3 + c] = G.T[0 * 3 + r] * HT[0 * 3 + c] + G.T[1 * 3 + r] * HT[1 * 3 + c];
  // dL/dJ = dL/dT W^T
  double dJ[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c)
      dJ[r * 3 + c] = dT[r * 3 + 0] * a.v.R[c * 3 + 0] + dT[r * 3 + 1] * a.v.R[c * 3 + 1] + dT[r * 3 + 2] * a.v.R[c * 3 + 2];
  // dL/dmu_c
  double gpc[3];
  for (int c = 0; c < 3; ++c) gpc[c] = G.J[0 * 3 + c] * gmu[0] + G.J[1 * 3 + c] * gmu[1];
  if (MC == kMcEquidistant)
    fisheye_jacobian_vjp(G.P, a.v.fx, a.v.fy, dJ, gpc);
  else
    other_jacobian_vjp(a.v.model, G.O, a.v.fx, a.v.fy, dJ, gpc);
  double gm[3];
  for (int c = 0; c < 3; ++c)
    gm[c] = a.v.R[0 * 3 + c] * gpc[0] + a.v.R[1 * 3 + c] * gpc[1] + a.v.R[2 * 3 + c] * gpc[2];
  for (int c = 0; c < 3; ++c) a.g_means[c * n + i] = (float)(gm[c] + (double)a.g_means[c * n + i]);
  // Sigma = M M^T, M = R S: dL/dM = 2 dS M.  The rotation, the normalised
  // quaternion and the scales are formed again from the inputs, as
  // compute_geometry formed them (the same operations, so the same values):
  // the registers of G's copies are then free through the chain above, which
  // keeps the kernel at four waves per SIMD.
  double Rq[9], qn[4], sc[3];
  double qnorm;
  {
    const float qf[4] = {a.quats[i], a.quats[n + i], a.quats[2 * n + i], a.quats[3 * n + i]};
    double q2 = 0.0;
    for (int k = 0; k < 4; ++k) q2 += (double)qf[k] * (double)qf[k];
    qnorm = sqrt(q2);
    const double iq = 1.0 / qnorm;
    for (int k = 0; k < 4; ++k) qn[k] = (double)qf[k] * iq;
    quat_to_rot(qn, Rq);
    for (int k = 0; k < 3; ++k) sc[k] = (double)a.scales[k * n + i];
  }
  double M[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[r * 3 + c] = Rq[r * 3 + c] * sc[c];
  double dM[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      dM[r * 3 + c] = 2.0 * (dS[r * 3 + 0] * M[0 * 3 + c] + dS[r * 3 + 1] * M[1 * 3 + c] + dS[r * 3 + 2] * M[2 * 3 + c]);
  for (int c = 0; c < 3; ++c)
    put(&a.g_scales[c * n + i], (float)(dM[0 * 3 + c] * Rq[0 * 3 + c] + dM[1 * 3 + c] * Rq[1 * 3 + c] +
                                        dM[2 * 3 + c] * Rq[2 * 3 + c]));
  double dR[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) dR[r * 3 + c] = dM[r * 3 + c] * sc[c];
  const double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  double gq[4];
  gq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  gq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                 2.0 * x * dR[8]);
  gq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                 2.0 * y * dR[8]);
  gq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] + y * dR[5] + x * dR[6] +
                 y * dR[7]);
  // through the normalisation q / |q|
  const double qd = qn[0] * gq[0] + qn[1] * gq[1] + qn[2] * gq[2] + qn[3] * gq[3];
  for (int c = 0; c < 4; ++c) put(&a.g_quats[c * n + i], (float)((gq[c] - qn[c] * qd) / qnorm));
  put(&a.g_opac[i], go);
  if (a.g_means2d) {
    put(&a.g_means2d[i], (float)gmu[0]);
    put(&a.g_means2d[n + i], (float)gmu[1]);
  }
}

// The two parts of the backward in one launch, one thread per Gaussian: the
// colour part streams the SH gradients out while the fp64 geometry of the
// same wave waits on its dependent loads, and both read the Gaussian's
// gradient slot and tile count once.  The geometry part adds to the view-
// direction term the colour part left in g_means (same thread, program order).
template <int DEG, int MC>
__global__ __launch_bounds__(kBlock) void backward_fused_kernel(PreBwdArgs a) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  sh_backward_body<DEG>(a, i);
  geometry_backward_body<MC>(a, i);
}

}  // namespace

hipError_t launch_preprocess(const fgs_gaussians& g, const ViewBatch& b, bool tight, uint32_t flags, char* ws,
                             const Layout& L, hipStream_t s) {
  uint32_t* const counters = reinterpret_cast<uint32_t*>(ws + L.counters);
  if (g.n == 0) return launch_clear_but_one(counters, kNumCounters, kCountFlags, flags, s);
  PreArgs a;
  a.counters = counters;
  a.flags = flags;
  a.block_kept = reinterpret_cast<uint32_t*>(ws + L.block_kept);
  a.means = g.means;
  a.scales = g.scales;
  a.quats = g.quats;
  a.opac = g.opacities;
  a.sh = g.sh;
  a.n = (uint32_t)g.n;
  a.sh_degree = g.sh_degree;
  a.batch = b;
  a.tight = tight ? 1 : 0;
  a.rowrange = reinterpret_cast<uint32_t*>(ws + L.rowrange);
  a.block_tiles = reinterpret_cast<uint32_t*>(ws + L.block_tiles);
  a.splats = reinterpret_cast<float4*>(ws + L.splats);
  a.colors = reinterpret_cast<float4*>(ws + L.colors);
  a.colorjac = b.count == 1 ? reinterpret_cast<float4*>(ws + L.colorjac) : nullptr;
  a.depth_keys = reinterpret_cast<uint32_t*>(ws + L.depth_keys);
  a.tiles = reinterpret_cast<uint32_t*>(ws + L.tiles);
  a.rects = reinterpret_cast<uint2*>(ws + L.rects);
  a.radii = reinterpret_cast<int32_t*>(ws + L.radii);
  const unsigned blocks = (unsigned)ceil_div(g.n, kBlock);
  const bool multi = b.count > 1;
  const int mc = model_class_of(b);
  if (!multi) {
    ProfScope prof(s, kKPreprocess);
#define FGS_PRE_LAUNCH(D)                                                                          \
  if (mc == kMcEquidistant)                                                                        \
    hipLaunchKernelGGL((preprocess_fused_kernel<D, kMcEquidistant>), dim3(blocks), dim3(kBlock), 0, s, a); \
  else                                                                                             \
    hipLaunchKernelGGL((preprocess_fused_kernel<D, kMcOther>), dim3(blocks), dim3(kBlock), 0, s, a);
    switch (g.sh_degree) {
      case 0: FGS_PRE_LAUNCH(0) break;
      case 1: FGS_PRE_LAUNCH(1) break;
      case 2: FGS_PRE_LAUNCH(2) break;
      default: FGS_PRE_LAUNCH(3) break;
    }
#undef FGS_PRE_LAUNCH
    return hipGetLastError();
  }
  const dim3 grid(blocks * (unsigned)b.count);
  {
    ProfScope prof(s, kKPreprocess);
    if (mc == kMcEquidistant)
      hipLaunchKernelGGL(preprocess_kernel<kMcEquidistant>, grid, dim3(kBlock), 0, s, a);
    else if (mc == kMcOther)
      hipLaunchKernelGGL(preprocess_kernel<kMcOther>, grid, dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL(preprocess_kernel<kMcAny>, grid, dim3(kBlock), 0, s, a);
  }
  ProfScope prof(s, kKColor);
#define FGS_PRE_LAUNCH(D) hipLaunchKernelGGL((color_kernel<D>), grid, dim3(kBlock), 0, s, a);
  switch (g.sh_degree) {
    case 0: FGS_PRE_LAUNCH(0) break;
    case 1: FGS_PRE_LAUNCH(1) break;
    case 2: FGS_PRE_LAUNCH(2) break;
    default: FGS_PRE_LAUNCH(3) break;
  }
#undef FGS_PRE_LAUNCH
  {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(view_sums_kernel, dim3(b.count), dim3(kBlock), 0, s, a.block_tiles, blocks,
                       reinterpret_cast<uint32_t*>(ws + L.counters) + kCountViewK);
  }
  return hipGetLastError();
}

hipError_t launch_preprocess_backward(const fgs_gaussians& g, const ViewParams& v, const char* ws,
                                      const Layout& L, const fgs_grads& out, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  PreBwdArgs a;
  a.means = g.means;
  a.scales = g.scales;
  a.quats = g.quats;
  a.opac = g.opacities;
  a.sh = g.sh;
  a.n = (uint32_t)g.n;
  a.sh_degree = g.sh_degree;
  a.v = v;
  a.tiles = reinterpret_cast<const uint32_t*>(ws + L.tiles);
  a.grad2d = reinterpret_cast<const float*>(ws + L.grad2d);
  a.colorjac = reinterpret_cast<const float4*>(ws + L.colorjac);
  a.g_means = out.means;
  a.g_scales = out.scales;
  a.g_quats = out.quats;
  a.g_opac = out.opacities;
  a.g_sh = out.sh;
  a.g_means2d = out.means2d;
  a.accumulate = out.accumulate ? 1 : 0;
  const unsigned blocks = (unsigned)ceil_div(g.n, kBlock);
  ProfScope prof(s, kKPreprocessBackward);
#define FGS_BWD(D)                                                                                            \
  if (v.model == kModelEquidistant)                                                                           \
    hipLaunchKernelGGL((backward_fused_kernel<D, kMcEquidistant>), dim3(blocks), dim3(kBlock), 0, s, a);     \
  else                                                                                                        \
    hipLaunchKernelGGL((backward_fused_kernel<D, kMcOther>), dim3(blocks), dim3(kBlock), 0, s, a);
  switch (g.sh_degree) {
    case 0: FGS_BWD(0) break;
    case 1: FGS_BWD(1) break;
    case 2: FGS_BWD(2) break;
    default: FGS_BWD(3) break;
  }
#undef FGS_BWD
  return hipGetLastError();
}

}  // namespace fgs
