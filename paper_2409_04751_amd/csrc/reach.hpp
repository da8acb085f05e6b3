// Tiles of a splat's 3-sigma rect that its alpha >= 1/255 pixels can lie in.
//
// The blend skips a splat at a pixel when alpha < 1/255 (Eq. 3 with the 3DGS
// cut-off), i.e. outside the ellipse |A'| t^2 + |D'| dy^2 <= P of its record,
// t = dx + beta dy, dx = mx - px, dy = my - py, P = -q2min (log2 units).  A
// tile none of whose pixels lies in the ellipse carries nothing, so the tile
// lists keep only the tiles the ellipse -- grown to P * 1.0201 (radius + 1%)
// and padded by 1/8 px, so that the float per-pixel test can never pass
// outside them -- reaches.  Per row of tiles those form one interval of
// columns: the ellipse's x-extent over the row's dy-range, whose extremes
// px = mx + beta dy +/- s(dy), s(dy) = sqrt((P - |D'| dy^2) / |A'|) (concave /
// convex in dy) peak at dy = +/- beta sqrt(|A'| P / (|D'| (|D'| + beta^2 |A'|))),
// clamped to the row.
//
// Everything is evaluated in float from the stored record, so the count in
// the preprocess and the walk in the duplication take the same decisions, and
// each step is one correctly rounded operation (no contraction: the library
// is built with -ffp-contract=off), in this order:
//   P = -q2min, a = |A'|, d = |D'|; kind 0 if !(P >= 0); kind 2 if P <= 1e-6,
//   !(|beta| <= 1e3), !(a > 0) or !(d > 0);
//   Pg = P * 1.0201, ia = 1 / a, Pa = Pg * ia, da = d * ia,
//   ry = sqrt(Pg * (1 / d)), ds = beta * sqrt((a * Pg) * (1 / (d * fma(beta * beta, a, d))));
//   kind 2 if any of ry, |ds|, Pa, da is above 1e30 or not finite, else 1.
// Per row (reach_row): dlo, dhi, the clamped peaks, s = sqrt(max(0, Pa - (da * y) * y)),
// the x extremes and the columns, as written there.
#pragma once

#include <hip/hip_runtime.h>

namespace fgs {

constexpr float kReachGrow = 1.0201f;  // P factor: radius + 1%
constexpr float kReachPad = 0.125f;    // px

struct SplatReach {
  float mx, my;   // mean, pixels
  float Pa, da;   // P / |A'| and |D'| / |A'|: s(dy)^2 = Pa - da dy^2
  float beta, ry, ds;
  int kind;       // 0: no tile, 1: per-row intervals, 2: the whole rect
};

// Correctly rounded square root and reciprocal (IEEE binary32, the HIP
// defaults for sqrtf and /): with the plain correctly rounded +, *, fma,
// floor and ceil below, every decision is a fixed function of the float
// record, one that any IEEE float evaluation of the same steps reproduces bit
// for bit.
__device__ inline float reach_sqrt(float x) { return sqrtf(x); }
__device__ inline float reach_rcp(float x) { return 1.0f / x; }

// s0 = (mu_x hi, mu_y hi, mu_x lo, mu_y lo), s1 = (A', beta, D', q2min).
__device__ inline SplatReach splat_reach(const float4& s0, const float4& s1) {
  SplatReach r;
  r.mx = s0.x + s0.z;
  r.my = s0.y + s0.w;
  r.beta = s1.y;
  r.Pa = r.da = r.ry = r.ds = 0.0f;
  const float a = fabsf(s1.x), d = fabsf(s1.z), P = -s1.w;
  if (!(P >= 0.0f)) {  // opacity below 1/255: no pixel is ever blended
    r.kind = 0;
    return r;
  }
  r.kind = 2;  // conventions shared with the blend's culling box
  if (P <= 1e-6f || !(fabsf(r.beta) <= 1e3f) || !(a > 0.0f) || !(d > 0.0f)) return r;
  const float Pg = P * kReachGrow, ia = reach_rcp(a);
  r.Pa = Pg * ia;
  r.da = d * ia;
  r.ry = reach_sqrt(Pg * reach_rcp(d));
  r.ds = r.beta * reach_sqrt(a * Pg * reach_rcp(d * __builtin_fmaf(r.beta * r.beta, a, d)));
  if (!(r.ry <= 1e30f) || !(fabsf(r.ds) <= 1e30f) || !(r.Pa <= 1e30f) || !(r.da <= 1e30f)) return r;
  r.kind = 1;
  return r;
}

// Packed as two float4 (kind as a float) for the duplication.
__device__ inline void pack_reach(const SplatReach& r, float4& p0, float4& p1) {
  p0 = make_float4(r.mx, r.my, r.Pa, r.da);
  p1 = make_float4(r.beta, r.ry, r.ds, (float)r.kind);
}
__device__ inline SplatReach unpack_reach(const float4& p0, const float4& p1) {
  SplatReach r;
  r.mx = p0.x;
  r.my = p0.y;
  r.Pa = p0.z;
  r.da = p0.w;
  r.beta = p1.x;
  r.ry = p1.y;
  r.ds = p1.z;
  r.kind = (int)p1.w;
  return r;
}

// Columns [c0, c1) of tile row ty, within the rect columns [x0, x1).
__device__ inline void reach_row(const SplatReach& r, int ty, int x0, int x1, int& c0, int& c1) {
  c0 = c1 = x0;
  if (r.kind != 1) {
    if (r.kind == 2) c1 = x1;
    return;
  }
  const float dlo = fmaxf(r.my - (float)(16 * ty + 15) - kReachPad, -r.ry);
  const float dhi = fminf(r.my - (float)(16 * ty) + kReachPad, r.ry);
  if (!(dlo <= dhi)) return;
  const float da = fminf(fmaxf(r.ds, dlo), dhi), db = fminf(fmaxf(-r.ds, dlo), dhi);
  const float sa = reach_sqrt(fmaxf(0.0f, r.Pa - r.da * da * da));
  const float sb = reach_sqrt(fmaxf(0.0f, r.Pa - r.da * db * db));
  const float xhi = r.mx + r.beta * da + sa + kReachPad, xlo = r.mx + r.beta * db - sb - kReachPad;
  if (!(xhi >= xlo)) {  // not finite: keep the row
    c1 = x1;
    return;
  }
  // tile column tx holds pixel centres [16 tx, 16 tx + 15]; clamp before the
  // conversion to int
  const float fx0 = (float)x0, fx1 = (float)x1;
  const int lo = (int)fminf(fmaxf(ceilf((xlo - 15.0f) * (1.0f / 16.0f)), fx0), fx1);
  const int hi = (int)fminf(fmaxf(floorf(xhi * (1.0f / 16.0f)) + 1.0f, fx0), fx1);
  if (hi > lo) {
    c0 = lo;
    c1 = hi;
  }
}

}  // namespace fgs
