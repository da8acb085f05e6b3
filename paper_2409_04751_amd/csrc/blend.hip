// Front-to-back alpha blending of each 16x16 tile (Eq. 3) and its reverse-
// order backward.
//
// One block of 128 threads per tile: two wave64s, each owning a 16x8 half,
// two pixels per lane.  The tile's sorted list is consumed in batches of 128
// Gaussians whose 2D records are staged in LDS once and then read by all
// pixels (broadcast reads, no bank conflicts); per batch each half gets the
// list of splats that can reach it, so a wave skips the others.
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
#include <algorithm>
#include <type_traits>

#include "fgs_internal.hpp"
#include "reach.hpp"

namespace fgs {
namespace {

constexpr float kTmin = 1e-4f;
constexpr float kAlphaMax = 0.99f;

struct BlendArgs {
  uint32_t total_tiles;
  const uint2* ranges;
  const uint32_t* ids;
  const float4* splats;
  const float4* colors;
  float* pixel_T;
  uint32_t* pixel_last;  // written only by the forward that saves the pixel state
  BatchOut out;
  ViewBatch batch;
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

// Front-to-back step of one pixel, branch-free: a pixel that is done, or that
// the splat does not reach (alpha < 1/255), or that the splat would take
// below the transmittance floor (which makes it done) adds w = 0 and keeps
// T and last, exactly as if it had been skipped.  The blend backward's
// re-sweep runs the same arithmetic, so T and last agree bit for bit.
// kLast: also track last (a forward that does not save it skips that).
template <bool kColorAcc, bool kLast = true>
__device__ inline void front_step(float fi, float fj, const float4& ga, const float4& gb, const float2& gc,
                                  uint32_t index, bool& done, float& T, uint32_t& last, float& C0, float& C1,
                                  float& C2) {
  float dx, dy, t;
  const float q2 = exponent2(ga, gb, fi, fj, dx, dy, t);
  const float alpha = fminf(kAlphaMax, gb.z * __builtin_amdgcn_exp2f(q2));
  const float tn = T * (1.0f - alpha);
  const bool pass = !done && q2 >= gb.y;
  const bool stop = tn < kTmin;
  const bool blend = pass && !stop;
  done = done || (pass && stop);
  if (kColorAcc) {
    const float w = blend ? alpha * T : 0.0f;
    C0 = __builtin_fmaf(gb.w, w, C0);
    C1 = __builtin_fmaf(gc.x, w, C1);
    C2 = __builtin_fmaf(gc.y, w, C2);
  }
  T = blend ? tn : T;
  if (kLast) last = blend ? index + 1u : last;
}

// The forward runs ONE wave per tile of every view of the batch (tiles are
// numbered view by view; the view of a wave is found from the views' first
// tile ids), each lane owning four pixels: column l & 15, rows (l >> 4) + 4k.
// A wave stages 64 entries of its tile's list at a time (one per lane) in an
// LDS region of its own, so there is no block barrier: a wave barrier makes
// the staged records visible to its lanes.  The four pixels per lane are four
// independent dependency chains per entry.
constexpr int kFwdWaves = 4;  // tiles (waves) per block
constexpr int kFwdThreads = 64 * kFwdWaves;
constexpr int kFwdChunk = 64;

struct FwdStage {
  float4 sa[kFwdChunk];
  float4 sb[kFwdChunk];
  float2 sc[kFwdChunk];
};

// What a lane wrote to its wave's LDS before the call is visible to every
// lane of the wave after it, and reads issued before it complete first.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SAVE: the per-pixel final transmittance and last contributor are stored
// (only then is the last contributor tracked).
template <bool SAVE>
__device__ inline void forward_tile(const BlendArgs& a, FwdStage& S, uint32_t gtile, uint32_t lane) {
  int vi = 0;
  while (vi + 1 < a.batch.count && gtile >= a.batch.v[vi + 1].tile_base) ++vi;
  const ViewParams& vp = a.batch.v[vi];
  const int tile = (int)(gtile - vp.tile_base);
  const int tx = tile % vp.tiles_x, ty = tile / vp.tiles_x;
  const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
  const uint2 r = a.ranges[gtile];
  const float fi = (float)(lane & 15u);
  const int px = tx * kTile + (int)(lane & 15u);
  bool inside[4], done[4];
  float fj[4], T[4], C0[4], C1[4], C2[4];
  uint32_t last[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = (int)(lane >> 4) + 4 * q;
    fj[q] = (float)j;
    inside[q] = px < vp.width && ty * kTile + j < vp.height;
    done[q] = !inside[q];
    T[q] = 1.0f;
    C0[q] = C1[q] = C2[q] = 0.0f;
    last[q] = 0;
  }
  for (uint32_t base = r.x; base < r.y; base += kFwdChunk) {
    if (__ballot(!(done[0] && done[1] && done[2] && done[3])) == 0ull) break;
    const uint32_t k = base + lane;
    if (k < r.y) {
      float4 ta, tb;
      float2 tc;
      stage_splat(a.splats, a.colors, a.ids[k], x0, y0, ta, tb, tc);
      S.sa[lane] = ta;
      S.sb[lane] = tb;
      S.sc[lane] = tc;
    }
    wave_lds_sync();
    const int cnt = (int)min((uint32_t)kFwdChunk, r.y - base);
    const uint32_t first = base - r.x;
    float4 na = S.sa[0], nb = S.sb[0];
    float2 nc = S.sc[0];
    for (int e = 0; e < cnt; ++e) {
      const float4 ga = na, gb = nb;
      const float2 gc = nc;
      if (e + 1 < cnt) {
        na = S.sa[e + 1];
        nb = S.sb[e + 1];
        nc = S.sc[e + 1];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        front_step<true, SAVE>(fi, fj[q], ga, gb, gc, first + (uint32_t)e, done[q], T[q], last[q], C0[q], C1[q],
                               C2[q]);
      if (__ballot(!(done[0] && done[1] && done[2] && done[3])) == 0ull) break;
    }
    wave_lds_sync();  // this chunk's reads complete before the next staging overwrites it
  }
  const size_t hw = (size_t)vp.width * vp.height;
  float* out = a.out.rgb[vi];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!inside[q]) continue;
    const size_t p = (size_t)(ty * kTile + (int)(lane >> 4) + 4 * q) * vp.width + px;
    out[p] = __builtin_fmaf(T[q], vp.bg[0], C0[q]);
    out[hw + p] = __builtin_fmaf(T[q], vp.bg[1], C1[q]);
    out[2 * hw + p] = __builtin_fmaf(T[q], vp.bg[2], C2[q]);
    if (SAVE) {
      a.pixel_T[vp.pixel_base + p] = T[q];
      a.pixel_last[vp.pixel_base + p] = last[q];
    }
  }
}

template <bool SAVE>
__global__ __launch_bounds__(kFwdThreads) void blend_forward_kernel(BlendArgs a) {
  __shared__ FwdStage stage[kFwdWaves];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  FwdStage& S = stage[wave];
  // consecutive tiles in one block, neighbouring blocks on one XCD (tiles
  // that gather the same splats share an L2)
  const uint32_t gtile = xcd_chunk(blockIdx.x, gridDim.x) * kFwdWaves + wave;
  if (gtile < a.total_tiles) forward_tile<SAVE>(a, S, gtile, lane);
}


// ---------------------------------------------------------------------------
struct BlendBwdArgs {
  const uint2* ranges;
  const uint32_t* ids;
  const float4* splats;
  const float4* colors;
  int32_t width, height, tiles_x, tiles_y;
  float bg[3];
  const float* dL;
  const float* pixel_T;
  const uint32_t* pixel_last;
  const uint32_t* counters;
  float* grad2d;  // [grad_slot(g)][9]
  // deterministic mode: the nine sums of each list entry are stored at
  // part[gauss_off[g] + rank][9], rank = the entry's tile among g's tiles in
  // tile order (its position in g's run of the duplication), recomputed from
  // g's rect, rows to bin and splat record as the binning counted them
  float* part;
  const uint2* rects;
  const uint32_t* rowrange;
  const float4* raw_splats;  // the records as stored (splats, unshifted)
  const uint32_t* gauss_off;
  uint32_t n;
};

// Position of tile (tx, ty) among the tiles Gaussian g was binned to, in
// tile order: the kept columns of g's rows above ty, then the columns of row
// ty before tx.  Rows and columns are those the binning took: the whole rect
// with FGS_RECT_BINNING, else the rows from rowrange with reach_row's
// columns on the float record (the same routine, so the same counts).
__device__ inline uint32_t tile_rank(const BlendBwdArgs& a, uint32_t g, int tx, int ty, bool rect) {
  const uint2 rc = a.rects[g];
  const int x0 = (int)(rc.x & 0xFFFFu), x1 = (int)(rc.y & 0xFFFFu);
  if (rect) return (uint32_t)((ty - (int)(rc.x >> 16)) * (x1 - x0) + (tx - x0));
  const int y0 = (int)(a.rowrange[g] & 0xFFFFu);
  const SplatReach R = splat_reach(a.raw_splats[2 * (size_t)g], a.raw_splats[2 * (size_t)g + 1]);
  uint32_t rank = 0;
  int c0, c1;
  for (int y = y0; y < ty; ++y) {
    reach_row(R, y, x0, x1, c0, c1);
    rank += (uint32_t)(c1 - c0);
  }
  reach_row(R, ty, x0, x1, c0, c1);
  return rank + (uint32_t)(tx - c0);
}

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

// State of one pixel in the backward.
struct BwdPixel {
  float fj;            // tile-relative row (the column is the lane's)
  bool inside;
  float T;             // final transmittance, then transmittance in front of the current splat
  uint32_t last;       // 1 + list index of its last blended splat
  float G0, G1, G2;    // dL/dC
  float B0, B1, B2;    // colour behind the current splat
};

// Reverse step for one pixel: recovers the transmittance in front of the
// splat, adds the pixel's colour and opacity gradient terms to v[5..8],
// updates the colour behind, and returns dL/dq (q the natural-log exponent)
// for the mean and conic terms, which the caller accumulates as moments.  One
// path for every lane: a pixel the splat does not reach takes alpha = 0,
// which leaves its transmittance and colour-behind exactly unchanged and adds
// zeros, so the lane exchanges need no branches.
__device__ inline float reverse_step(BwdPixel& px, bool pass, float q2, const float4& gb, const float2& gc,
                                     float v[9]) {
  const float eq = __builtin_amdgcn_exp2f(q2);
  const float raw = gb.z * eq;
  const float alpha = pass ? fminf(kAlphaMax, raw) : 0.0f;
  const float Ti = pass ? px.T * __builtin_amdgcn_rcpf(1.0f - alpha) : px.T;
  const float w = alpha * Ti;
  v[6] = __builtin_fmaf(w, px.G0, v[6]);
  v[7] = __builtin_fmaf(w, px.G1, v[7]);
  v[8] = __builtin_fmaf(w, px.G2, v[8]);
  // colour minus colour behind, for dL/dalpha and for the update behind
  const float d0 = gb.w - px.B0, d1 = gc.x - px.B1, d2 = gc.y - px.B2;
  const float dLda = Ti * __builtin_fmaf(d0, px.G0, __builtin_fmaf(d1, px.G1, d2 * px.G2));
  px.B0 = __builtin_fmaf(alpha, d0, px.B0);
  px.B1 = __builtin_fmaf(alpha, d1, px.B1);
  px.B2 = __builtin_fmaf(alpha, d2, px.B2);
  px.T = Ti;
  const float dl = (pass && raw < kAlphaMax) ? dLda : 0.0f;  // the clamp passes no gradient
  v[5] = __builtin_fmaf(dl, eq, v[5]);
  return dl * alpha;
}

// Sum over the 64 lanes of a wave, on every lane, with the two gfx950 lane
// swaps (halves, then neighbouring 16-lane rows): no LDS round trip.
__device__ inline float wave_rows_sum(float x) {
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  const float y = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(y), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// The mean and conic terms from the moments of g = dL/dq over the pixels.
// With q = -(A t^2 + D dy^2) / 2 (natural log), t = dx + beta dy, and the
// record's A' = -A/(2 ln2), D' = -D/(2 ln2): dq/dmu_x = -A t = 2 ln2 A' t,
// dq/dmu_y = -(beta A t + D dy) = 2 ln2 (beta A' t + D' dy), dq/dA = -dx^2/2,
// dq/dB = -dx dy (B enters q twice), dq/dC = -dy^2/2.  Per lane and entry the
// moments sum_g g t, sum g dy, sum g dx^2, sum g dx dy, sum g dy^2 over the
// lane's four pixels share dx (one column); v[0] and v[1] take the record's
// factors, the constants below are applied once per entry.
__constant__ const float kGradScale[9] = {1.3862943611198906f, 1.3862943611198906f, -0.5f, -1.0f, -0.5f,
                                          1.0f, 1.0f, 1.0f, 1.0f};

// The backward runs ONE wave per tile, each lane owning four pixels of the
// tile: column l & 15, rows (l >> 4) + 4k, k = 0..3.  A wave shares nothing
// with the other waves of its block (its LDS is its own), so there is no
// block barrier anywhere: a wave stages 64 entries of its tile's list at a
// time (one per lane), makes them visible to its own lanes with a wave
// barrier, and walks them; the four pixels per lane are four independent
// dependency chains per entry.  Per entry the wave's 9 gradient sums are
// reduced in registers (a DPP reduce-scatter inside each 16-lane row, then
// the four rows added with two lane exchanges) and added to the global
// accumulators by the 9 lanes holding them: no LDS accumulators and no
// flush phase.
constexpr int kBwdWaves = 4;              // tiles (waves) per block
constexpr int kBwdThreads = 64 * kBwdWaves;
constexpr int kBwdChunk = 64;             // entries staged per step

struct BwdStage {
  float4 sa[kBwdChunk];
  float4 sb[kBwdChunk];
  float2 sc[kBwdChunk];
  uint32_t sid[kBwdChunk];
  uint32_t sslot[kBwdChunk];  // the entry's slot in the block's table (kNoSlot: none)
};

// The block's four waves blend four neighbouring tiles, whose lists share
// most of their Gaussians.  Device-scope float atomics are performed past the
// per-XCD L2s, on the memory side, so each (Gaussian, tile) adding its nine
// sums to the global accumulators costs a memory-side atomic request; the
// block instead adds them into an LDS table keyed by Gaussian (open
// addressing, linear probing, LDS atomics) and adds each Gaussian's totals to
// the accumulators once, after its four tiles are done.  An entry that finds
// no free slot within kTableProbes adds directly, as before, and so does a
// wave whose pixels blend more than kTableListMax entries (unsaturated
// tiles): its Gaussians would only crowd the table.
constexpr int kTableBits = 8;
constexpr uint32_t kTableSize = 1u << kTableBits;
constexpr int kTableProbes = 8;
constexpr uint32_t kTableListMax = 128;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

struct GradTable {
  uint32_t key[kTableSize];
  float val[kTableSize][9];
  uint32_t used;  // slots taken; past three quarters new Gaussians add directly
};
struct NoTable {};

// Slot of Gaussian g in the table, inserting it if absent (one lane per call).
// Long unsaturated lists (thousands of entries per block) would fill the
// table and make every entry probe in vain, so once three quarters of the
// slots are taken a Gaussian not yet in the table is not inserted (the count
// is read without ordering: it only decides between two correct paths).
__device__ inline uint32_t table_slot(GradTable& T, uint32_t g) {
  const uint32_t h = (g * 2654435761u) >> (32 - kTableBits);
  const bool full = __hip_atomic_load(&T.used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >=
                    kTableSize / 4 * 3;
  for (int p = 0; p < kTableProbes; ++p) {
    const uint32_t s = (h + (uint32_t)p) & (kTableSize - 1u);
    if (full) {
      const uint32_t k = __hip_atomic_load(&T.key[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (k == g) return s;
      if (k == kEmptyKey) return kNoSlot;
      continue;
    }
    const uint32_t old = atomicCAS(&T.key[s], kEmptyKey, g);
    if (old == kEmptyKey) {
      atomicAdd(&T.used, 1u);
      return s;
    }
    if (old == g) return s;
  }
  return kNoSlot;
}


__device__ inline uint32_t wave_max_u32(uint32_t v) {
  for (int d = 32; d >= 1; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, 64));
  return __builtin_amdgcn_readfirstlane(v);
}

// STORE: the nine sums of each entry are stored at part[entry] (the
// deterministic mode) instead of added to the Gaussian's accumulators
template <bool STORE, class Table>
__device__ inline void backward_tile(const BlendBwdArgs& a, BwdStage& S, Table& T, uint32_t tile, uint32_t lane) {
  const int tx = (int)(tile % (uint32_t)a.tiles_x), ty = (int)(tile / (uint32_t)a.tiles_x);
  const float x0 = (float)(tx * kTile), y0 = (float)(ty * kTile);
  const uint2 r = a.ranges[tile];
  const size_t hw = (size_t)a.width * a.height;
  const bool saved = (a.counters[kCountFlags] & FGS_SAVE_PIXEL_STATE) != 0;
  const bool rect = (a.counters[kCountFlags] & FGS_RECT_BINNING) != 0;
  const float fi = (float)(lane & 15u);
  const int px = tx * kTile + (int)(lane & 15u);
  BwdPixel P[4];
  size_t pidx[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int j = (int)(lane >> 4) + 4 * k;
    const int py = ty * kTile + j;
    P[k].fj = (float)j;
    P[k].inside = px < a.width && py < a.height;
    pidx[k] = P[k].inside ? (size_t)py * a.width + px : 0;
    P[k].T = 1.0f;
    P[k].last = 0;
  }

  // ---- final transmittance and last contributor of each pixel ----
  if (saved) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (P[k].inside) {
        P[k].T = a.pixel_T[pidx[k]];
        P[k].last = a.pixel_last[pidx[k]];
      }
  } else {
    bool done[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) done[k] = !P[k].inside;
    float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;  // unused: the re-sweep accumulates no colour
    for (uint32_t base = r.x; base < r.y; base += kBwdChunk) {
      if (__ballot(!(done[0] && done[1] && done[2] && done[3])) == 0ull) break;
      const uint32_t k = base + lane;
      if (k < r.y) {
        float4 ta, tb;
        float2 tc;
        stage_splat(a.splats, a.colors, a.ids[k], x0, y0, ta, tb, tc);
        S.sa[lane] = ta;
        S.sb[lane] = tb;
      }
      wave_lds_sync();
      const int cnt = (int)min((uint32_t)kBwdChunk, r.y - base);
      const uint32_t first = base - r.x;
      float4 na = S.sa[0], nb = S.sb[0];
      for (int e = 0; e < cnt; ++e) {
        const float4 ga = na, gb = nb;
        if (e + 1 < cnt) {
          na = S.sa[e + 1];
          nb = S.sb[e + 1];
        }
        const float2 gc = make_float2(0.0f, 0.0f);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          front_step<false>(fi, P[q].fj, ga, gb, gc, first + (uint32_t)e, done[q], P[q].T, P[q].last, c0, c1, c2);
        if (__ballot(!(done[0] && done[1] && done[2] && done[3])) == 0ull) break;
      }
      wave_lds_sync();  // this chunk's reads complete before the next staging overwrites it
    }
  }
  const uint32_t maxlast = wave_max_u32(max(max(P[0].last, P[1].last), max(P[2].last, P[3].last)));
  [[maybe_unused]] const bool use_table = maxlast <= kTableListMax;

  // ---- reverse sweep ----
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    P[k].G0 = P[k].G1 = P[k].G2 = 0.0f;
    if (P[k].inside) {
      P[k].G0 = a.dL[pidx[k]];
      P[k].G1 = a.dL[hw + pidx[k]];
      P[k].G2 = a.dL[2 * hw + pidx[k]];
    }
    P[k].B0 = a.bg[0];
    P[k].B1 = a.bg[1];
    P[k].B2 = a.bg[2];
  }
  // this lane's slot in the row reduce-scatter; lanes of the first row hold
  // the wave's totals after the rows are added
  const uint32_t rpos = lane & 15u;
  const bool rb3 = (rpos >> 3) & 1u, rb2 = (rpos >> 2) & 1u, rb1 = (rpos >> 1) & 1u, rb0 = rpos & 1u;
  const int rval = (rb3 ? 5 : 0) + (rb2 ? 3 : 0) + (rb1 ? 2 : 0) + (rb0 ? 1 : 0);
  const bool writer = lane < 16u && ((kRowValid >> rpos) & 1u);
  const float wscale = writer ? kGradScale[rval] : 0.0f;
  // a Gaussian's nine sums are adjacent ([slot][9]), so the nine writer
  // lanes' atomics go to one or two cache lines
  float* const gout = a.grad2d + (writer ? rval : 0);
  for (int end = (int)maxlast; end > 0; end -= kBwdChunk) {
    const int beg = max(end - kBwdChunk, 0);
    if (beg + (int)lane < end) {
      const uint32_t g = a.ids[r.x + beg + lane];
      float4 ta, tb;
      float2 tc;
      stage_splat(a.splats, a.colors, g, x0, y0, ta, tb, tc);
      S.sa[lane] = ta;
      S.sb[lane] = tb;
      S.sc[lane] = tc;
      if constexpr (STORE) {  // where this entry's sums go (sid is not needed for atomics)
        S.sid[lane] = a.gauss_off[g] + tile_rank(a, g, tx, ty, rect);
      } else {
        S.sid[lane] = g;
        S.sslot[lane] = use_table ? table_slot(T, g) : kNoSlot;
      }
    }
    wave_lds_sync();
    const int cnt = end - beg;
    // the records are read where they are used: no registers held for the
    // next entry, which keeps six waves per SIMD (the other waves hide the
    // LDS latency)
    for (int idx = cnt - 1; idx >= 0; --idx) {
      const float4 ga = S.sa[idx], gb = S.sb[idx];
      const float2 gc = S.sc[idx];
      const uint32_t e = (uint32_t)(beg + idx);
      // the exponent as the forward forms it (bit for bit); dx is shared by
      // the lane's four pixels, which lie in one column
      const float dx = ga.x - fi;
      float q2[4], dy[4];
      bool pass[4];
      bool any = false;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        dy[k] = ga.y - P[k].fj;
        const float t = __builtin_fmaf(ga.w, dy[k], dx);
        q2[k] = __builtin_fmaf(ga.z * t, t, (gb.x * dy[k]) * dy[k]);
        pass[k] = e < P[k].last && q2[k] >= gb.y;
        any = any || pass[k];
      }
      if (__ballot(any) == 0ull) continue;  // wave-uniform
      float v[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = 0.0f;
      float gs = 0.0f, gy = 0.0f, gyy = 0.0f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float g = reverse_step(P[k], pass[k], q2[k], gb, gc, v);
        const float gdy = g * dy[k];
        gs += g;
        gy += gdy;
        gyy = __builtin_fmaf(gdy, dy[k], gyy);
      }
      const float gt = __builtin_fmaf(ga.w, gy, dx * gs);  // sum g t
      v[0] = ga.z * gt;
      v[1] = __builtin_fmaf(ga.w, v[0], gb.x * gy);
      v[2] = (dx * dx) * gs;
      v[3] = dx * gy;
      v[4] = gyy;
      // wave-uniform: every lane takes part in the exchanges
      const float part = wave_rows_sum(row_reduce_scatter9(v, rb3, rb2, rb1, rb0));
      if (writer) {
        const float val = part * wscale;
        if constexpr (STORE) {
          a.part[(size_t)S.sid[idx] * 9 + rval] = val;
        } else if (val != 0.0f) {
          const uint32_t ts = S.sslot[idx];
          if (ts != kNoSlot)
            atomicAdd(&T.val[ts][rval], val);
          else
            atomicAdd(&gout[(size_t)grad_slot(S.sid[idx]) * 9], val);
        }
      }
    }
    wave_lds_sync();
  }
}

// Five waves per SIMD with the table (its 92 registers then need no spills;
// six would spill 14), six in the deterministic mode.
template <bool STORE>
__global__ __launch_bounds__(kBwdThreads) __attribute__((amdgpu_waves_per_eu(STORE ? 6 : 5))) void blend_backward_kernel(BlendBwdArgs a) {
  __shared__ BwdStage stage[kBwdWaves];
  using Table = std::conditional_t<STORE, NoTable, GradTable>;
  __shared__ Table table;
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  BwdStage& S = stage[wave];
  if constexpr (!STORE) {
    for (uint32_t i = threadIdx.x; i < kTableSize; i += kBwdThreads) table.key[i] = kEmptyKey;
    if (threadIdx.x == 0) table.used = 0;
    float* v = &table.val[0][0];
    for (uint32_t i = threadIdx.x; i < kTableSize * 9; i += kBwdThreads) v[i] = 0.0f;
    __syncthreads();
  }
  const uint32_t tile = xcd_chunk(blockIdx.x, gridDim.x) * kBwdWaves + wave;
  if (tile < (uint32_t)a.tiles_x * (uint32_t)a.tiles_y) backward_tile<STORE>(a, S, table, tile, lane);
  if constexpr (!STORE) {
    // each used slot's nine totals: lanes 16 k .. 16 k + 8 of a wave take
    // slot 4 w + k + 16 j, so one atomic instruction covers four Gaussians'
    // 36-byte blocks
    __syncthreads();
    const uint32_t c = lane & 15u;
    for (uint32_t sl = (threadIdx.x >> 4); sl < kTableSize; sl += kBwdThreads / 16) {
      const uint32_t g = table.key[sl];
      if (g == kEmptyKey || c >= 9u) continue;
      const float v = table.val[sl][c];
      if (v != 0.0f) atomicAdd(&a.grad2d[(size_t)grad_slot(g) * 9 + c], v);
    }
  }
}

}  // namespace

hipError_t launch_blend_forward(const ViewBatch& b, int64_t total_tiles, const uint2* ranges, const uint32_t* ids,
                                const float4* splats, const float4* colors, const BatchOut& out, float* pixel_T,
                                uint32_t* pixel_last, bool save, hipStream_t s) {
  if (total_tiles <= 0) return hipSuccess;
  BlendArgs a;
  a.ranges = ranges;
  a.ids = ids;
  a.splats = splats;
  a.colors = colors;
  a.pixel_T = pixel_T;
  a.pixel_last = pixel_last;
  a.out = out;
  a.batch = b;
  a.total_tiles = (uint32_t)total_tiles;
  ProfScope prof(s, kKBlendForward);
  const dim3 grid((unsigned)ceil_div(total_tiles, kFwdWaves));
  if (save)
    hipLaunchKernelGGL(blend_forward_kernel<true>, grid, dim3(kFwdThreads), 0, s, a);
  else
    hipLaunchKernelGGL(blend_forward_kernel<false>, grid, dim3(kFwdThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_blend_backward(const ViewParams& v, const uint2* ranges, const uint32_t* ids, const float4* splats,
                                 const float4* colors,
                                 const float* dL_dimg, const float* pixel_T, const uint32_t* pixel_last,
                                 const uint32_t* counters, float* grad2d, const DetStore* det, int64_t n,
                                 hipStream_t s) {
  BlendBwdArgs a;
  a.ranges = ranges;
  a.ids = ids;
  a.splats = splats;
  a.colors = colors;
  a.width = v.width;
  a.height = v.height;
  a.tiles_x = v.tiles_x;
  a.tiles_y = v.tiles_y;
  for (int c = 0; c < 3; ++c) a.bg[c] = v.bg[c];
  a.dL = dL_dimg;
  a.pixel_T = pixel_T;
  a.pixel_last = pixel_last;
  a.counters = counters;
  a.grad2d = grad2d;
  a.part = det ? det->part : nullptr;
  a.rects = det ? det->rects : nullptr;
  a.rowrange = det ? det->rowrange : nullptr;
  a.raw_splats = splats;
  a.gauss_off = det ? det->gauss_off : nullptr;
  a.n = (uint32_t)n;
  const int64_t tiles = (int64_t)v.tiles_x * v.tiles_y;
  ProfScope prof(s, kKBlendBackward);
  if (det)
    hipLaunchKernelGGL(blend_backward_kernel<true>, dim3((unsigned)ceil_div(tiles, kBwdWaves)), dim3(kBwdThreads), 0,
                       s, a);
  else
    hipLaunchKernelGGL(blend_backward_kernel<false>, dim3((unsigned)ceil_div(tiles, kBwdWaves)), dim3(kBwdThreads), 0,
                       s, a);
  return hipGetLastError();
}

}  // namespace fgs
