// Device math for the equidistant fisheye projection (Fisheye-GS, Sec. 3.2,
// 4.2, 4.3), the 3D covariance (Eq. 1) and the SH colour.
//
// Geometry runs in double precision: the per-Gaussian stage is bound by the
// 236 B of parameters it reads, so fp64 costs little, and the integer
// decisions taken from it (radius, tile rectangle, depth key) then agree
// with any other careful evaluation except at exact ties.
//
// The Jacobian is written through two scalars of the camera-space point
// p = (x, y, z), l_z = |(x, y)|, l_2 = |p|^2, theta = atan2(l_z, z):
//   h = (z l_z / l_2 - theta) / l_z^3        (the paper's S7 / (l_2^2 l_z^5))
//   m = (3 h + 2 z / l_2^2) / l_z^2           (the paper's -S8 / (l_2^2 l_z^5))
// so that J_phi (Sec. 4.2, f multiplying each whole entry) is
//   [[fx (z/l_2 - y^2 h), fx x y h, -fx x / l_2],
//    [fy x y h, fy (z/l_2 - x^2 h), -fy y / l_2]]
// and, since dh/dx = -x m, dh/dy = -y m, dh/dz = 2 / l_2^2, the entries of
// dJ/dp (Sec. 4.3) are S1 = x(3h - x^2 m), S2 = y(h - x^2 m),
// S3 = x(h - y^2 m), S4 = y(3h - y^2 m) plus the S5, S6 terms.  Near the
// optical axis h and m are 0/0; there they come from their Taylor series in
// u = l_z / z, which also removes the cancellation of the closed forms.
#pragma once

#include <hip/hip_runtime.h>

namespace fgs {

constexpr double kSeriesU = 0.05;

// h z^3 = sum_{k>=1} (-1)^k 2k/(2k+1) u^(2k-2)
// m z^5 = sum_{k>=2} (-1)^(k+1) 4k(k-1)/(2k+1) u^(2k-4)
__device__ inline double h_z3_series(double u2) {
  double s = -16.0 / 17.0;
  s = s * u2 + 14.0 / 15.0;
  s = s * u2 - 12.0 / 13.0;
  s = s * u2 + 10.0 / 11.0;
  s = s * u2 - 8.0 / 9.0;
  s = s * u2 + 6.0 / 7.0;
  s = s * u2 - 4.0 / 5.0;
  s = s * u2 + 2.0 / 3.0;
  return -s;
}
__device__ inline double m_z5_series(double u2) {
  double s = 288.0 / 19.0;
  s = s * u2 - 224.0 / 17.0;
  s = s * u2 + 168.0 / 15.0;
  s = s * u2 - 120.0 / 13.0;
  s = s * u2 + 80.0 / 11.0;
  s = s * u2 - 48.0 / 9.0;
  s = s * u2 + 24.0 / 7.0;
  s = s * u2 - 8.0 / 5.0;
  return s;
}

struct FisheyePoint {
  double x, y, z, lz2, lz, l2, theta;
  double h, m;
};

__device__ inline void fisheye_terms(FisheyePoint& P, bool need_m) {
  const double x = P.x, y = P.y, z = P.z;
  P.lz2 = x * x + y * y;
  P.lz = sqrt(P.lz2);
  P.l2 = P.lz2 + z * z;
  P.theta = atan2(P.lz, z);
  if (z > 0.0 && P.lz < kSeriesU * z) {
    const double u = P.lz / z;
    const double u2 = u * u;
    const double z3 = z * z * z;
    P.h = h_z3_series(u2) / z3;
    P.m = need_m ? m_z5_series(u2) / (z3 * z * z) : 0.0;
  } else {
    P.h = (z * P.lz / P.l2 - P.theta) / (P.lz2 * P.lz);
    P.m = need_m ? (3.0 * P.h + 2.0 * z / (P.l2 * P.l2)) / P.lz2 : 0.0;
  }
}

// J_phi, row-major 2x3.
__device__ inline void fisheye_jacobian(const FisheyePoint& P, double fx, double fy, double J[6]) {
  const double x = P.x, y = P.y, z = P.z, h = P.h, il2 = 1.0 / P.l2;
  J[0] = fx * (z * il2 - y * y * h);
  J[1] = fx * x * y * h;
  J[2] = -fx * x * il2;
  J[3] = fy * x * y * h;
  J[4] = fy * (z * il2 - x * x * h);
  J[5] = -fy * y * il2;
}

// g[k] += sum_ij G[i][j] dJ_ij / dp_k   (G = dL/dJ, row-major 2x3)
__device__ inline void fisheye_jacobian_vjp(const FisheyePoint& P, double fx, double fy, const double G[6],
                                            double g[3]) {
  const double x = P.x, y = P.y, z = P.z, h = P.h, m = P.m;
  const double il22 = 1.0 / (P.l2 * P.l2);
  const double S1 = x * (3.0 * h - x * x * m);
  const double S2 = y * (h - x * x * m);
  const double S3 = x * (h - y * y * m);
  const double S4 = y * (3.0 * h - y * y * m);
  const double S5 = (x * x - y * y - z * z) * il22;
  const double S6 = (y * y - x * x - z * z) * il22;
  const double xy2 = 2.0 * x * y * il22, xz2 = 2.0 * x * z * il22, yz2 = 2.0 * y * z * il22;
  const double a0 = fx * G[0], a1 = fx * G[1], a2 = fx * G[2];
  const double b0 = fy * G[3], b1 = fy * G[4], b2 = fy * G[5];
  g[0] += a0 * S1 + a1 * S2 + a2 * S5 + b0 * S2 + b1 * S3 + b2 * xy2;
  g[1] += a0 * S2 + a1 * S3 + a2 * xy2 + b0 * S3 + b1 * S4 + b2 * S6;
  g[2] += a0 * S5 + a1 * xy2 + a2 * xz2 + b0 * xy2 + b1 * S6 + b2 * yz2;
}

// ---- other camera models --------------------------------------------------
//
// Radial models (pinhole r = tan theta and the equisolid-angle, orthographic
// and stereographic fisheyes that Sec. 3.2 lists) put a point at
// mu_p = c + f r(theta) (x, y) / l_z.  Written through three scalars of
// (theta, d = |p|),
//   a = cos(theta) r'(theta) / d,   e = r'(theta) / d^2,
//   h = H(theta) / d^3,  H = (sin cos r' - r) / sin^3,
// J_phi has the same shape as the equidistant one:
//   [[fx (a - y^2 h), fx x y h, -fx x e], [fy x y h, fy (a - x^2 h), -fy y e]].
// For these four models H, H' / sin(theta) and r'' / sin(theta) have closed
// forms without cancellation, and nothing divides by l_z, so the optical
// axis needs no special case.  The backward differentiates a, e and h
// through theta and d: with F~ = (dF/dtheta) / l_z,
//   grad F = F~ (z / d^2) (x, y, 0) - F~ (0, 0, l_z^2 / d^2) + (dF/dd) p / d.
//
// The panorama (Sec. 5.3) maps longitude atan2(x, z) and latitude
// atan2(y, rho), rho = |(x, z)|, linearly: mu_p = c + (fx lon, fy lat).  Its
// J rows are fx grad lon and fy grad lat; the backward takes the Hessians of
// lon and lat against the two rows of dL/dJ.
enum CameraModel : int32_t {
  kModelEquidistant = 0,
  kModelPinhole = 1,
  kModelPanorama = 2,
  kModelEquisolid = 3,
  kModelOrthographic = 4,
  kModelStereographic = 5,
};

struct OtherPoint {
  double x, y, z, lz2, l2, d;
  double angle;         // incidence theta (radial) or |latitude| (panorama), for the cull
  double a, e, h;       // radial J scalars
  double at, et, ht;    // radial: dF/dtheta / l_z of a, e, h
  double rho2, rho;     // panorama
};

// r, r', r''/sin, H and H'/sin of a radial model at incidence th.
__device__ inline void radial_functions(int model, double th, double& r, double& r1, double& R2, double& H,
                                        double& Hp) {
  if (model == kModelPinhole) {
    const double c = cos(th);
    r = tan(th);
    r1 = 1.0 / (c * c);
    R2 = 2.0 * r1 / c;
    H = 0.0;
    Hp = 0.0;
  } else if (model == kModelEquisolid) {
    const double c = cos(0.5 * th), c2 = c * c, c3 = c2 * c;
    r = 2.0 * sin(0.5 * th);
    r1 = c;
    R2 = -0.25 / c;
    H = -(1.0 + 2.0 * c2) / (4.0 * c3);
    Hp = -(3.0 + 2.0 * c2) / (16.0 * c3 * c2);
  } else if (model == kModelOrthographic) {
    r = sin(th);
    r1 = cos(th);
    R2 = -1.0;
    H = -1.0;
    Hp = 0.0;
  } else {  // stereographic
    const double c = cos(0.5 * th), ic2 = 1.0 / (c * c);
    r = 2.0 * tan(0.5 * th);
    r1 = ic2;
    R2 = 0.5 * ic2 * ic2;
    H = -R2;
    Hp = -R2 * ic2;
  }
}

// Fills P (x, y, z set) and, if the point survives the cull angle, mu and J.
__device__ inline bool other_project(int model, OtherPoint& P, double angle_max, double fx, double fy, double cx,
                                     double cy, bool need_vjp, double mu[2], double J[6]) {
  const double x = P.x, y = P.y, z = P.z;
  if (model == kModelPanorama) {
    P.rho2 = x * x + z * z;
    P.rho = sqrt(P.rho2);
    P.l2 = P.rho2 + y * y;
    const double lat = atan2(y, P.rho);
    P.angle = fabs(lat);
    if (!(P.angle <= angle_max)) return false;
    mu[0] = cx + fx * atan2(x, z);
    mu[1] = cy + fy * lat;
    const double ir2 = 1.0 / P.rho2, k = fy / (P.rho * P.l2);
    J[0] = fx * z * ir2;
    J[1] = 0.0;
    J[2] = -fx * x * ir2;
    J[3] = -k * x * y;
    J[4] = k * P.rho2;
    J[5] = -k * y * z;
    return true;
  }
  P.lz2 = x * x + y * y;
  P.l2 = P.lz2 + z * z;
  P.d = sqrt(P.l2);
  const double lz = sqrt(P.lz2);
  const double th = atan2(lz, z);
  P.angle = th;
  if (!(th <= angle_max)) return false;
  double r, r1, R2, H, Hp;
  radial_functions(model, th, r, r1, R2, H, Hp);
  const double ct = z / P.d;
  P.a = ct * r1 / P.d;
  P.e = r1 / P.l2;
  P.h = H / (P.d * P.l2);
  if (need_vjp) {
    P.at = (ct * R2 - r1) / P.l2;
    P.et = R2 / (P.d * P.l2);
    P.ht = Hp / (P.l2 * P.l2);
  }
  if (lz > 0.0) {
    mu[0] = cx + fx * r * x / lz;
    mu[1] = cy + fy * r * y / lz;
  } else {
    mu[0] = cx;
    mu[1] = cy;
  }
  J[0] = fx * (P.a - y * y * P.h);
  J[1] = fx * x * y * P.h;
  J[2] = -fx * x * P.e;
  J[3] = fy * x * y * P.h;
  J[4] = fy * (P.a - x * x * P.h);
  J[5] = -fy * y * P.e;
  return true;
}

// g[k] += sum_ij G[i][j] dJ_ij / dp_k for the models of other_project.
__device__ inline void other_jacobian_vjp(int model, const OtherPoint& P, double fx, double fy, const double G[6],
                                          double g[3]) {
  const double x = P.x, y = P.y, z = P.z;
  if (model == kModelPanorama) {
    // row 0: fx grad lon, grad lon = (z, 0, -x) / rho^2
    const double ir2 = 1.0 / P.rho2, u = G[0] * z - G[2] * x;
    g[0] += fx * (-G[2] * ir2 - 2.0 * x * u * ir2 * ir2);
    g[2] += fx * (G[0] * ir2 - 2.0 * z * u * ir2 * ir2);
    // row 1: fy grad lat, grad lat = (rho e_y - y grad rho) / d^2
    const double rho = P.rho, ir = 1.0 / rho, s = G[3] * x + G[5] * z;
    const double N = rho * G[4] - y * s * ir;
    const double ir3 = ir * ir * ir, il2 = 1.0 / P.l2;
    const double dN0 = G[4] * x * ir - y * (G[3] * ir - s * x * ir3);
    const double dN1 = -s * ir;
    const double dN2 = G[4] * z * ir - y * (G[5] * ir - s * z * ir3);
    const double q = 2.0 * N * il2 * il2;
    g[0] += fy * (dN0 * il2 - q * x);
    g[1] += fy * (dN1 * il2 - q * y);
    g[2] += fy * (dN2 * il2 - q * z);
    return;
  }
  const double a0 = fx * G[0], a1 = fx * G[1], a2 = fx * G[2];
  const double b0 = fy * G[3], b1 = fy * G[4], b2 = fy * G[5];
  const double cA = a0 + b1;
  const double m = a1 + b0;
  const double cH = -a0 * y * y + m * x * y - b1 * x * x;
  const double cE = -a2 * x - b2 * y;
  const double S = cA * P.at + cH * P.ht + cE * P.et;
  const double il2 = 1.0 / P.l2;
  const double Q = -(cA * P.a + 3.0 * cH * P.h + 2.0 * cE * P.e) * il2;
  const double Szl = S * z * il2;
  g[0] += Szl * x + Q * x + m * y * P.h - 2.0 * b1 * x * P.h - a2 * P.e;
  g[1] += Szl * y + Q * y + m * x * P.h - 2.0 * a0 * y * P.h - b2 * P.e;
  g[2] += -S * P.lz2 * il2 + Q * z;
}

// Rotation of the normalised quaternion (w, x, y, z), row-major.
__device__ inline void quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// Real SH basis, Condon-Shortley phase, index l(l+1)+m.  Constants are
// sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the factors of the Cartesian
// polynomials; e.g. 0.4886 = sqrt(3/(4 pi)), 1.0925 = sqrt(15/(4 pi)).
constexpr float kY00 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kY1 = 0.4886025119029199f;     // sqrt(3/(4 pi))
constexpr float kY2a = 1.0925484305920792f;    // sqrt(15/(4 pi))
constexpr float kY2b = 0.31539156525252005f;   // sqrt(5/(16 pi))
constexpr float kY2c = 0.5462742152960396f;    // sqrt(15/(16 pi))
constexpr float kY3a = 0.5900435899266435f;    // sqrt(35/(32 pi))
constexpr float kY3b = 2.890611442640554f;     // sqrt(105/(4 pi))
constexpr float kY3c = 0.4570457994644658f;    // sqrt(21/(32 pi))
constexpr float kY3d = 0.3731763325901154f;    // sqrt(7/(16 pi))
constexpr float kY3e = 1.445305721320277f;     // sqrt(105/(16 pi))

template <int DEG>
__device__ inline void sh_basis(float x, float y, float z, float Y[16]) {
  Y[0] = kY00;
  if constexpr (DEG >= 1) {
    Y[1] = -kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = -kY1 * x;
  }
  if constexpr (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kY2a * x * y;
    Y[5] = -kY2a * y * z;
    Y[6] = kY2b * (2.0f * zz - xx - yy);
    Y[7] = -kY2a * x * z;
    Y[8] = kY2c * (xx - yy);
  }
  if constexpr (DEG >= 3) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[9] = -kY3a * y * (3.0f * xx - yy);
    Y[10] = kY3b * x * y * z;
    Y[11] = -kY3c * y * (4.0f * zz - xx - yy);
    Y[12] = kY3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    Y[13] = -kY3c * x * (4.0f * zz - xx - yy);
    Y[14] = kY3e * z * (xx - yy);
    Y[15] = -kY3a * x * (xx - 3.0f * yy);
  }
}

// g = sum_k w[k] grad Y_k at (x, y, z), each Y_k read as a polynomial in R^3
// (only its tangential part matters once multiplied by d dir / d v).
template <int DEG>
__device__ inline void sh_grad_dir(float x, float y, float z, const float w[16], float g[3]) {
  g[0] = g[1] = g[2] = 0.0f;
  if constexpr (DEG >= 1) {
    g[1] -= kY1 * w[1];
    g[2] += kY1 * w[2];
    g[0] -= kY1 * w[3];
  }
  if constexpr (DEG >= 2) {
    g[0] += kY2a * y * w[4];
    g[1] += kY2a * x * w[4];
    g[1] -= kY2a * z * w[5];
    g[2] -= kY2a * y * w[5];
    g[0] -= 2.0f * kY2b * x * w[6];
    g[1] -= 2.0f * kY2b * y * w[6];
    g[2] += 4.0f * kY2b * z * w[6];
    g[0] -= kY2a * z * w[7];
    g[2] -= kY2a * x * w[7];
    g[0] += 2.0f * kY2c * x * w[8];
    g[1] -= 2.0f * kY2c * y * w[8];
  }
  if constexpr (DEG >= 3) {
    const float xx = x * x, yy = y * y, zz = z * z;
    g[0] -= 6.0f * kY3a * x * y * w[9];
    g[1] -= 3.0f * kY3a * (xx - yy) * w[9];
    g[0] += kY3b * y * z * w[10];
    g[1] += kY3b * x * z * w[10];
    g[2] += kY3b * x * y * w[10];
    g[0] += 2.0f * kY3c * x * y * w[11];
    g[1] -= kY3c * (4.0f * zz - xx - 3.0f * yy) * w[11];
    g[2] -= 8.0f * kY3c * y * z * w[11];
    g[0] -= 6.0f * kY3d * x * z * w[12];
    g[1] -= 6.0f * kY3d * y * z * w[12];
    g[2] += kY3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12];
    g[0] -= kY3c * (4.0f * zz - 3.0f * xx - yy) * w[13];
    g[1] += 2.0f * kY3c * x * y * w[13];
    g[2] -= 8.0f * kY3c * x * z * w[13];
    g[0] += 2.0f * kY3e * x * z * w[14];
    g[1] -= 2.0f * kY3e * y * z * w[14];
    g[2] += kY3e * (xx - yy) * w[14];
    g[0] -= 3.0f * kY3a * (xx - yy) * w[15];
    g[1] += 6.0f * kY3a * x * y * w[15];
  }
}

// D[ch] = sum_k c[k*3+ch] grad Y_k at (x, y, z) for the three channels at
// once (the gradient of each channel's colour in the view direction, each
// Y_k read as a polynomial in R^3), the monomials shared.
template <int DEG>
__device__ inline void sh_grad_dir3(float x, float y, float z, const float c[48], float D[3][3]) {
  for (int ch = 0; ch < 3; ++ch) D[ch][0] = D[ch][1] = D[ch][2] = 0.0f;
  auto add = [&](int k, int a, float v) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) D[ch][a] += v * c[k * 3 + ch];
  };
  if constexpr (DEG >= 1) {
    add(1, 1, -kY1);
    add(2, 2, kY1);
    add(3, 0, -kY1);
  }
  if constexpr (DEG >= 2) {
    add(4, 0, kY2a * y);
    add(4, 1, kY2a * x);
    add(5, 1, -kY2a * z);
    add(5, 2, -kY2a * y);
    add(6, 0, -2.0f * kY2b * x);
    add(6, 1, -2.0f * kY2b * y);
    add(6, 2, 4.0f * kY2b * z);
    add(7, 0, -kY2a * z);
    add(7, 2, -kY2a * x);
    add(8, 0, 2.0f * kY2c * x);
    add(8, 1, -2.0f * kY2c * y);
  }
  if constexpr (DEG >= 3) {
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, xz = x * z, yz = y * z;
    add(9, 0, -6.0f * kY3a * xy);
    add(9, 1, -3.0f * kY3a * (xx - yy));
    add(10, 0, kY3b * yz);
    add(10, 1, kY3b * xz);
    add(10, 2, kY3b * xy);
    add(11, 0, 2.0f * kY3c * xy);
    add(11, 1, -kY3c * (4.0f * zz - xx - 3.0f * yy));
    add(11, 2, -8.0f * kY3c * yz);
    add(12, 0, -6.0f * kY3d * xz);
    add(12, 1, -6.0f * kY3d * yz);
    add(12, 2, kY3d * (6.0f * zz - 3.0f * xx - 3.0f * yy));
    add(13, 0, -kY3c * (4.0f * zz - 3.0f * xx - yy));
    add(13, 1, 2.0f * kY3c * xy);
    add(13, 2, -8.0f * kY3c * xz);
    add(14, 0, 2.0f * kY3e * xz);
    add(14, 1, -2.0f * kY3e * yz);
    add(14, 2, kY3e * (xx - yy));
    add(15, 0, -3.0f * kY3a * (xx - yy));
    add(15, 1, 6.0f * kY3a * xy);
  }
}

}  // namespace fgs
