// Front-to-back alpha blending of each 16x16 tile (Eq. 3) and its reverse-
// order backward.
//
// One block of 256 threads per tile, one thread per pixel.  The four wave64s
// of a block each own an 8x8 quadrant, so a small splat touches few waves and
// the backward can skip whole waves.  The tile's sorted list is consumed in
// batches of 256 Gaussians whose 2D records are staged in LDS once and then
// read by all 256 pixels (broadcast reads, no bank conflicts).
//
// Per (pixel, Gaussian) the exponent is evaluated as
//   q = -(A t^2 + D dy^2) / 2,  t = dx + (B/A) dy,  D = C - B^2/A,
// a sum of two non-negative terms, which avoids the cancellation of
// A dx^2 + 2 B dx dy + C dy^2 for thin splats; the record stores A and D
// pre-scaled by -log2(e)/2 so that e^q is one v_exp_f32.  The mean is stored
// as a float hi + lo pair and converted to tile-relative coordinates once per
// staged Gaussian, so dx, dy carry no rounding of |mu_p| ~ 10^3 px.
//
// Decisions (Eq. 3 plus the 3DGS cut-offs): skip when alpha < 1/255
// (equivalently q2 < log2(1/(255 o))), alpha = min(0.99, o e^q), stop before
// the Gaussian that would take T below 1e-4.
#include "fgs_internal.hpp"

namespace fgs {
namespace {

constexpr float kTmin = 1e-4f;
constexpr float kAlphaMax = 0.99f;
constexpr float kNegTwoLn2 = -1.3862943611198906f;  // converts the log2-scaled A, D back to natural units

struct BlendArgs {
  const uint2* ranges;
  const uint32_t* ids;
  const float4* splats;
  const float4* colors;
  float* pixel_T;
  uint32_t* pixel_last;
  int save;
  BatchOut out;
  ViewBatch batch;
};

// Pixel of this thread inside its tile: wave w owns quadrant (w & 1, w >> 1).
__device__ inline void pixel_of_thread(int& i, int& j) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  i = (w & 1) * 8 + (l & 7);
  j = (w >> 1) * 8 + (l >> 3);
}

struct Staged {
  float4 a;  // mx, my (tile-relative), A', beta
  float4 b;  // D', q2min, o, r
  float2 c;  // g, b
};

__device__ inline void stage_splat(const float4* splats, const float4* colors, uint32_t g, float x0, float y0,
                                   float4& a, float4& b, float2& c) {
  const float4 p = splats[2 * (size_t)g + 0];
  const float4 q = splats[2 * (size_t)g + 1];
  const float4 r = colors[g];
  a = make_float4((p.x - x0) + p.z, (p.y - y0) + p.w, q.x, q.y);
  b = make_float4(q.z, q.w, r.x, r.y);
  c = make_float2(r.z, r.w);
}

// log2-scaled exponent at tile-relative pixel (fi, fj).
__device__ inline float exponent2(const float4& a, const float4& b, float fi, float fj, float& dx, float& dy,
                                  float& t) {
  dx = a.x - fi;
  dy = a.y - fj;
  t = __builtin_fmaf(a.w, dy, dx);
  return __builtin_fmaf(a.z * t, t, (b.x * dy) * dy);
}

// Quadrants of the tile (wave w owns the 8x8 pixel block (w & 1, w >> 1))
// that can hold a pixel at which the splat is not skipped.  Such a pixel has
// |A'| t^2 + |D'| dy^2 <= P = -q2min with t = dx + beta dy: an ellipse with
// half extents ry = sqrt(P / |D'|) in y and rx = sqrt(P (1/|A'| + beta^2/|D'|))
// in x.  The box is widened by 1% + 1/16 px, so the float evaluation of the
// per-pixel test cannot pass outside it; a non-finite extent, or P so small
// that the per-pixel terms could underflow, keeps every quadrant, and P < 0
// (opacity below 1/255) keeps none, as the per-pixel test would.  Lists of
// the entries per quadrant let each wave skip splats that cannot reach its
// 64 pixels; the tile lists themselves are unchanged.
__device__ inline uint32_t quadrant_mask(const float4& a, const float4& b) {
  const float P = -b.y;
  if (!(P > 1e-6f)) return P >= 0.0f ? 0xFu : 0u;
  // t = dx + beta dy loses ~1e-7 (1 + |beta|) px to rounding: past |beta| =
  // 1e3 that could approach the margin, so such slivers keep every quadrant
  if (!(fabsf(a.w) <= 1e3f)) return 0xFu;
  const float iA = 1.0f / fabsf(a.z), iD = 1.0f / fabsf(b.x);
  constexpr float kBig = 1e30f;
  float ry = sqrtf(P * iD), rx = sqrtf(P * __builtin_fmaf(a.w * a.w, iD, iA));
  ry = ry <= kBig ? __builtin_fmaf(ry, 1.01f, 0.0625f) : kBig;
  rx = rx <= kBig ? __builtin_fmaf(rx, 1.01f, 0.0625f) : kBig;
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float qx0 = (float)((q & 1) * 8), qy0 = (float)((q >> 1) * 8);
    if (a.x + rx >= qx0 && a.x - rx <= qx0 + 7.0f && a.y + ry >= qy0 && a.y - ry <= qy0 + 7.0f) m |= 1u << q;
  }
  return m;
}

// Per-quadrant lists of the staged entries, in entry order.
struct QuadLists {
  uint8_t idx[4][kBlock];
  uint32_t wcount[4][4];  // [staging wave][quadrant]
};

__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Called by all threads after thread t staged entry t with quadrant mask m
// (0 for no entry); returns the length of the calling wave's list.  Contains
// the barriers that publish the staged records too.
__device__ inline int build_quad_lists(uint32_t m, QuadLists& Q) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint64_t bal[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) bal[q] = __ballot((m >> q) & 1u);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) Q.wcount[wave][q] = (uint32_t)__builtin_popcountll(bal[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if ((m >> q) & 1u) {
      uint32_t off = 0;
      for (uint32_t w = 0; w < wave; ++w) off += Q.wcount[w][q];
      Q.idx[q][off + lanes_below(bal[q])] = (uint8_t)threadIdx.x;
    }
  }
  const int n = (int)(Q.wcount[0][wave] + Q.wcount[1][wave] + Q.wcount[2][wave] + Q.wcount[3][wave]);
  __syncthreads();
  return n;
}

// One block per tile of every view of the batch (tiles are numbered view by
// view; the view of a block is found from the views' first tile ids).
__global__ __launch_bounds__(kBlock) void blend_forward_kernel(BlendArgs a) {
  __shared__ float4 sa[kBlock];
  __shared__ float4 sb[kBlock];
  __shared__ float2 sc[kBlock];
  __shared__ QuadLists Q;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t gtile = xcd_chunk(blockIdx.x, gridDim.x);
  int vi = 0;
  while (vi + 1 < a.batch.count && gtile >= a.batch.v[vi + 1].tile_base) ++vi;
  const ViewParams& vp = a.batch.v[vi];
  const int tile = (int)(gtile - vp.tile_base);
  const int tx = tile % vp.tiles_x, ty = tile / vp.tiles_x;
  int i, j;
  pixel_of_thread(i, j);
  const int px = tx * kTile + i, py = ty * kTile + j;
  const bool inside = px < vp.width && py < vp.height;
  const float fi = (float)i, fj = (float)j;
  const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
  const uint2 r = a.ranges[gtile];
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  uint32_t last = 0;
  bool done = !inside;
  for (uint32_t base = r.x; base < r.y; base += kBlock) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t k = base + threadIdx.x;
    uint32_t m = 0;
    if (k < r.y) {
      float4 ta, tb;
      float2 tc;
      stage_splat(a.splats, a.colors, a.ids[k], x0, y0, ta, tb, tc);
      sa[threadIdx.x] = ta;
      sb[threadIdx.x] = tb;
      sc[threadIdx.x] = tc;
      m = quadrant_mask(ta, tb);
    }
    const int cnt = build_quad_lists(m, Q);
    if (!done) {
      for (int jj = 0; jj < cnt; ++jj) {
        const int e = __builtin_amdgcn_readfirstlane(Q.idx[wave][jj]);
        const float4 ga = sa[e], gb = sb[e];
        float dx, dy, t;
        const float q2 = exponent2(ga, gb, fi, fj, dx, dy, t);
        if (!(q2 >= gb.y)) continue;
        const float alpha = fminf(kAlphaMax, gb.z * __builtin_amdgcn_exp2f(q2));
        const float tn = T * (1.0f - alpha);
        if (tn < kTmin) {
          done = true;
          break;
        }
        const float2 gc = sc[e];
        const float w = alpha * T;
        C0 = __builtin_fmaf(gb.w, w, C0);
        C1 = __builtin_fmaf(gc.x, w, C1);
        C2 = __builtin_fmaf(gc.y, w, C2);
        T = tn;
        last = base - r.x + (uint32_t)e + 1u;
      }
    }
  }
  if (inside) {
    const size_t hw = (size_t)vp.width * vp.height, p = (size_t)py * vp.width + px;
    float* out = a.out.rgb[vi];
    out[p] = __builtin_fmaf(T, vp.bg[0], C0);
    out[hw + p] = __builtin_fmaf(T, vp.bg[1], C1);
    out[2 * hw + p] = __builtin_fmaf(T, vp.bg[2], C2);
    if (a.save) {
      a.pixel_T[vp.pixel_base + p] = T;
      a.pixel_last[vp.pixel_base + p] = last;
    }
  }
}

// ---------------------------------------------------------------------------
struct BlendBwdArgs {
  const uint2* ranges;
  const uint32_t* ids;
  const float4* splats;
  const float4* colors;
  int32_t width, height, tiles_x;
  float bg[3];
  const float* dL;
  const float* pixel_T;
  const uint32_t* pixel_last;
  const uint32_t* counters;
  float* grad2d;  // [9][n]
  uint32_t n;
};

// DPP lane exchange inside each 16-lane row (all patterns are permutations,
// so every lane has a valid source).
template <int CTRL>
__device__ inline float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppRowMirror = 0x140;      // lane i <- lane 15 - i   (partner differs in bit 3)
constexpr int kDppRowHalfMirror = 0x141;  // lane i <- lane 7 - i    (same bit 3, differs in bit 2)
constexpr int kDppQuadXor2 = 0x4E;        // quad_perm [2,3,0,1]     (differs in bit 1 only)
constexpr int kDppQuadXor1 = 0xB1;        // quad_perm [1,0,3,2]     (differs in bit 0 only)

// Reduce-scatter of 9 per-lane values over the 16 lanes of each row by
// recursive halving: at each step a lane keeps half of its value slots and
// adds its partner's copy of them.  Afterwards the lane with row position
// (b3 b2 b1 b0) holds the row sum of value (b3 ? 5 : 0) + (b2 ? 3 : 0) +
// (b1 ? 2 : 0) + b0; positions outside kRowValid hold padding.
constexpr uint32_t kRowValid = 0x1737u;  // positions 0,1,2,4,5,8,9,10,12 -> values 0..8

__device__ inline float row_reduce_scatter9(const float v[9], bool b3, bool b2, bool b1, bool b0) {
  float K[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const float lo = v[s], hi = (s + 5 < 9) ? v[s + 5] : 0.0f;
    const float keep = b3 ? hi : lo, send = b3 ? lo : hi;
    K[s] = keep + dpp<kDppRowMirror>(send);
  }
  float L[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const float lo = K[s], hi = (s + 3 < 5) ? K[s + 3] : 0.0f;
    const float keep = b2 ? hi : lo, send = b2 ? lo : hi;
    L[s] = keep + dpp<kDppRowHalfMirror>(send);
  }
  float M[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const float lo = L[s], hi = (s + 2 < 3) ? L[s + 2] : 0.0f;
    const float keep = b1 ? hi : lo, send = b1 ? lo : hi;
    M[s] = keep + dpp<kDppQuadXor2>(send);
  }
  const float keep = b0 ? M[1] : M[0], send = b0 ? M[0] : M[1];
  return keep + dpp<kDppQuadXor1>(send);
}

__global__ __launch_bounds__(kBlock) void blend_backward_kernel(BlendBwdArgs a) {
  __shared__ float4 sa[kBlock];
  __shared__ float4 sb[kBlock];
  __shared__ float4 sc[kBlock];  // g, b, and the conic's A, D in natural units
  __shared__ uint32_t sid[kBlock];
  __shared__ float acc[9][kBlock];
  __shared__ uint32_t s_maxlast;
  __shared__ QuadLists Q;
  const uint32_t wave = threadIdx.x >> 6;
  const int tile = (int)xcd_chunk(blockIdx.x, gridDim.x);
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  int i, j;
  pixel_of_thread(i, j);
  const int px = tx * kTile + i, py = ty * kTile + j;
  const bool inside = px < a.width && py < a.height;
  const float fi = (float)i, fj = (float)j;
  const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
  const uint2 r = a.ranges[tile];
  const size_t hw = (size_t)a.width * a.height, p = (size_t)py * a.width + px;
  const bool saved = (a.counters[kCountFlags] & FGS_SAVE_PIXEL_STATE) != 0;

  // ---- final transmittance and last contributor of each pixel ----
  float T = 1.0f;
  uint32_t last = 0;
  if (saved) {
    if (inside) {
      T = a.pixel_T[p];
      last = a.pixel_last[p];
    }
  } else {
    // front-to-back re-sweep with the forward's arithmetic (no colour)
    bool done = !inside;
    for (uint32_t base = r.x; base < r.y; base += kBlock) {
      if (__syncthreads_count(!done) == 0) break;
      const uint32_t k = base + threadIdx.x;
      uint32_t m = 0;
      if (k < r.y) {
        float4 ta, tb;
        float2 tc;
        stage_splat(a.splats, a.colors, a.ids[k], x0, y0, ta, tb, tc);
        sa[threadIdx.x] = ta;
        sb[threadIdx.x] = tb;
        m = quadrant_mask(ta, tb);
      }
      const int cnt = build_quad_lists(m, Q);
      if (!done) {
        for (int jj = 0; jj < cnt; ++jj) {
          const int e = __builtin_amdgcn_readfirstlane(Q.idx[wave][jj]);
          const float4 ga = sa[e], gb = sb[e];
          float dx, dy, t;
          const float q2 = exponent2(ga, gb, fi, fj, dx, dy, t);
          if (!(q2 >= gb.y)) continue;
          const float alpha = fminf(kAlphaMax, gb.z * __builtin_amdgcn_exp2f(q2));
          const float tn = T * (1.0f - alpha);
          if (tn < kTmin) {
            done = true;
            break;
          }
          T = tn;
          last = base - r.x + (uint32_t)e + 1u;
        }
      }
    }
  }
  if (threadIdx.x == 0) s_maxlast = 0;
  __syncthreads();
  atomicMax(&s_maxlast, last);
  uint32_t wlast = last;  // this wave's largest last contributor
  for (int d = 32; d >= 1; d >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, d, 64));
  wlast = __builtin_amdgcn_readfirstlane(wlast);
  __syncthreads();
  const uint32_t maxlast = s_maxlast;

  // ---- reverse sweep ----
  float G0 = 0.0f, G1 = 0.0f, G2 = 0.0f;
  if (inside) {
    G0 = a.dL[p];
    G1 = a.dL[hw + p];
    G2 = a.dL[2 * hw + p];
  }
  float B0 = a.bg[0], B1 = a.bg[1], B2 = a.bg[2];  // colour behind the current Gaussian
  float Tc = T;
  // this lane's slot in the row reduce-scatter
  const uint32_t rpos = threadIdx.x & 15u;
  const bool rb3 = (rpos >> 3) & 1u, rb2 = (rpos >> 2) & 1u, rb1 = (rpos >> 1) & 1u, rb0 = rpos & 1u;
  const int rval = (rb3 ? 5 : 0) + (rb2 ? 3 : 0) + (rb1 ? 2 : 0) + (rb0 ? 1 : 0);
  const bool rvalid = (kRowValid >> rpos) & 1u;
  for (int end = (int)maxlast; end > 0; end -= kBlock) {
    const int beg = max(end - kBlock, 0);
    __syncthreads();
    uint32_t m = 0;
    if (beg + (int)threadIdx.x < end) {
      const uint32_t g = a.ids[r.x + beg + threadIdx.x];
      sid[threadIdx.x] = g;
      float4 ta, tb;
      float2 tc;
      stage_splat(a.splats, a.colors, g, x0, y0, ta, tb, tc);
      sa[threadIdx.x] = ta;
      sb[threadIdx.x] = tb;
      sc[threadIdx.x] = make_float4(tc.x, tc.y, kNegTwoLn2 * ta.z, kNegTwoLn2 * tb.x);
      m = quadrant_mask(ta, tb);
    }
    for (int k = 0; k < 9; ++k) acc[k][threadIdx.x] = 0.0f;
    const int cnt = build_quad_lists(m, Q);
    for (int jj = cnt - 1; jj >= 0; --jj) {
      const int idx = __builtin_amdgcn_readfirstlane(Q.idx[wave][jj]);
      const int e = beg + idx;
      if ((uint32_t)e >= wlast) continue;  // past every pixel of this wave
      const float4 ga = sa[idx], gb = sb[idx];
      float dx, dy, t;
      const float q2 = exponent2(ga, gb, fi, fj, dx, dy, t);
      const bool pass = (uint32_t)e < last && q2 >= gb.y;
      if (__ballot(pass) == 0ull) continue;  // wave-uniform
      // one path for every lane: a lane the splat does not reach gets
      // alpha = 0, which leaves Tc and the colour behind unchanged and
      // zeroes its gradient terms, so the DPP exchange needs no branches
      const float4 gc = sc[idx];  // g, b, A, D (natural scale)
      const float eq = __builtin_amdgcn_exp2f(q2);
      const float raw = gb.z * eq;
      const float alpha = pass ? fminf(kAlphaMax, raw) : 0.0f;
      const float om = 1.0f - alpha;
      const float Ti = pass ? Tc * __builtin_amdgcn_rcpf(om) : Tc;
      const float w = alpha * Ti;
      float v[9];
      v[6] = w * G0;
      v[7] = w * G1;
      v[8] = w * G2;
      const float dLda = Ti * ((gb.w - B0) * G0 + (gc.x - B1) * G1 + (gc.y - B2) * G2);
      B0 = alpha * gb.w + om * B0;
      B1 = alpha * gc.x + om * B1;
      B2 = alpha * gc.y + om * B2;
      Tc = Ti;
      const bool live = pass && raw < kAlphaMax;  // the clamp passes no gradient
      const float dLdq = live ? dLda * alpha : 0.0f;
      v[5] = live ? dLda * eq : 0.0f;
      const float At = gc.z * t;
      v[0] = -dLdq * At;
      v[1] = -dLdq * (ga.w * At + gc.w * dy);
      const float h = -0.5f * dLdq, hdx = h * dx;
      v[2] = hdx * dx;
      v[3] = (hdx + hdx) * dy;
      v[4] = (h * dy) * dy;
      // wave-uniform: every lane takes part in the DPP exchanges
      const float part = row_reduce_scatter9(v, rb3, rb2, rb1, rb0);
      if (rvalid) atomicAdd(&acc[rval][idx], part);
    }
    __syncthreads();
    if ((int)threadIdx.x < end - beg) {
      const uint32_t g = sid[threadIdx.x];
      for (int k = 0; k < 9; ++k) {
        const float val = acc[k][threadIdx.x];
        if (val != 0.0f) atomicAdd(&a.grad2d[(size_t)k * a.n + g], val);
      }
    }
  }
}

}  // namespace

hipError_t launch_blend_forward(const ViewBatch& b, int64_t total_tiles, const uint2* ranges, const uint32_t* ids,
                                const float4* splats, const float4* colors, const BatchOut& out, float* pixel_T,
                                uint32_t* pixel_last,
                                bool save, hipStream_t s) {
  if (total_tiles <= 0) return hipSuccess;
  BlendArgs a;
  a.ranges = ranges;
  a.ids = ids;
  a.splats = splats;
  a.colors = colors;
  a.pixel_T = pixel_T;
  a.pixel_last = pixel_last;
  a.save = save ? 1 : 0;
  a.out = out;
  a.batch = b;
  ProfScope prof(s, kKBlendForward);
  hipLaunchKernelGGL(blend_forward_kernel, dim3((unsigned)total_tiles), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_blend_backward(const ViewParams& v, const uint2* ranges, const uint32_t* ids, const float4* splats,
                                 const float4* colors,
                                 const float* dL_dimg, const float* pixel_T, const uint32_t* pixel_last,
                                 const uint32_t* counters, float* grad2d, int64_t n, hipStream_t s) {
  BlendBwdArgs a;
  a.ranges = ranges;
  a.ids = ids;
  a.splats = splats;
  a.colors = colors;
  a.width = v.width;
  a.height = v.height;
  a.tiles_x = v.tiles_x;
  for (int c = 0; c < 3; ++c) a.bg[c] = v.bg[c];
  a.dL = dL_dimg;
  a.pixel_T = pixel_T;
  a.pixel_last = pixel_last;
  a.counters = counters;
  a.grad2d = grad2d;
  a.n = (uint32_t)n;
  const unsigned tiles = (unsigned)v.tiles_x * (unsigned)v.tiles_y;
  ProfScope prof(s, kKBlendBackward);
  hipLaunchKernelGGL(blend_backward_kernel, dim3(tiles), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace fgs
