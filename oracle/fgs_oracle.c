/*
 * CPU oracle for the fisheye Gaussian-splatting rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  The parity tests, the smoke check and the CPU
 * baseline of the benchmark call this file; the rendering library never
 * includes, links or calls it, and it includes nothing from the library.
 *
 * Plain, slow, obviously correct: double precision throughout, one loop per
 * step of the method in the order the paper gives them, OpenMP only over
 * independent Gaussians / tiles.
 *
 * Paper: Fisheye-GS (arXiv 2409.04751).
 *   Eq. 1 and Sec. 3.1 "Definition"   3D Gaussian, Sigma = R S S^T R^T
 *   Eq. 2 and Sec. 3.1 "Transformation"  mu_c = W mu + b, Sigma_p = J W Sigma W^T J^T
 *   Eq. 3 and Sec. 3.1 "Rendering"    front-to-back alpha blending, 16x16 tiles,
 *                                      sort by tile id then depth
 *   Sec. 3.2, Eq. 4 onward            equidistant model r_d = f theta, pixel coords
 *   Sec. 4.2                          J_phi (printed with the f factor missing on the
 *                                      theta terms; read as f times the whole entry)
 *   Sec. 4.3                          dJ/dx_c, dJ/dy_c, dJ/dz_c via S1..S8 (entry
 *                                      [0][2] of dJ/dy_c printed with f_y; read as f_x)
 *   Sec. 3.2 (model list), Sec. 5.3   other camera models: the equisolid-angle,
 *                                      orthographic and stereographic fisheyes Sec. 3.2
 *                                      names, the pinhole, and the panorama projection of
 *                                      Sec. 5.3, paragraph "Extension to Other Cameras Models"; their
 *                                      J and dJ are the first and second derivatives of
 *                                      the projection, taken by forward-mode
 *                                      differentiation (the paper prints only the
 *                                      panorama's J)
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   theta = atan2(l_z, z_c) (the printed arctan(l_z/z_c) only covers z_c > 0);
 *   near cull on the Euclidean distance |mu_c| <= near, rear cull theta > theta_max;
 *   depth key = |mu_c| as float32; 0.3 px^2 low-pass dilation of Sigma_p;
 *   lambda_max = mid + sqrt(max(0.1, mid^2 - det)); radius = ceil(3 sqrt(lambda_max));
 *   rect = clamp(floor((mu -/+ r (+15)) / 16)); alpha = min(0.99, o e^q),
 *   skipped when q > 0 or alpha < 1/255; blending stops before a Gaussian whose
 *   T (1 - alpha) would fall below 1e-4; background added as T_final * bg;
 *   real SH basis with Condon-Shortley phase, rgb = max(0, sum + 0.5);
 *   quaternion (w, x, y, z) normalised inside; near-axis J and dJ through the
 *   series of their closed forms (the closed forms are 0/0 on the axis).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TILE 16
#define ND 7 /* dual-number directions: scales (3) + quaternion (4), or mean (3) */

typedef struct {
  int32_t width, height;
  double fx, fy, cx, cy;
  double near_dist, theta_max;
  int32_t model;
} orc_camera;

/* Camera models.  Radial models put a point at incidence theta on the ray of
 * its azimuth at distance f r(theta) from the principal point:
 *   equidistant r = theta (Sec. 3.2), pinhole r = tan theta,
 *   equisolid angle r = 2 sin(theta / 2), orthographic r = sin theta,
 *   stereographic r = 2 tan(theta / 2)  (the fisheye models Sec. 3.2 lists).
 * The panorama (Sec. 5.3) maps longitude atan2(x_c, z_c) and latitude
 * atan2(y_c, |(x_c, z_c)|) linearly to x and y. */
enum { MODEL_EQUIDISTANT = 0, MODEL_PINHOLE = 1, MODEL_PANORAMA = 2, MODEL_EQUISOLID = 3, MODEL_ORTHOGRAPHIC = 4,
       MODEL_STEREOGRAPHIC = 5 };

/* ------------------------------------------------------------------------ */
/* Forward-mode dual numbers, used for the parts of the backward that the     */
/* paper takes from vanilla 3DGS (Sigma -> scale/rotation, SH colour -> mean). */
/* ------------------------------------------------------------------------ */
typedef struct { double v, d[ND]; } dual;

static dual d_const(double v) { dual r; r.v = v; for (int k = 0; k < ND; ++k) r.d[k] = 0; return r; }
static dual d_var(double v, int k) { dual r = d_const(v); r.d[k] = 1.0; return r; }
static dual d_add(dual a, dual b) { dual r; r.v = a.v + b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
static dual d_sub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
static dual d_mul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
static dual d_scale(dual a, double s) { dual r; r.v = a.v * s; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * s; return r; }
static dual d_div(dual a, dual b) {
  dual r; r.v = a.v / b.v;
  for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
static dual d_sqrt(dual a) {
  dual r; r.v = sqrt(a.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Equidistant projection phi (Sec. 3.2) and its Jacobian (Sec. 4.2, 4.3).     */
/* ------------------------------------------------------------------------ */

/* mu_p = (c_x + f_x theta x_c / l_z, c_y + f_y theta y_c / l_z). */
void orc_project(const double p[3], double fx, double fy, double cx, double cy, double out[2]) {
  double x = p[0], y = p[1], z = p[2];
  double lz = sqrt(x * x + y * y);
  double theta = atan2(lz, z);
  if (lz > 0) {
    out[0] = cx + fx * theta * x / lz;
    out[1] = cy + fy * theta * y / lz;
  } else { /* on the optical axis the limit is the principal point */
    out[0] = cx;
    out[1] = cy;
  }
}

/* Near-axis series (z > 0, u = l_z / z small).  With
 *   h = S7 / (l_2^2 l_z^5) = (z l_z / l_2 - theta) / l_z^3,
 *   m = -S8 / (l_2^2 l_z^5) = (3 h + 2 z / l_2^2) / l_z^2,
 * expanding u/(1+u^2) - atan(u) and 1/(1+u^2)^2 term by term gives
 *   h z^3 = sum_{k>=1} (-1)^k 2k/(2k+1) u^(2k-2)
 *   m z^5 = sum_{k>=2} (-1)^(k+1) 4k(k-1)/(2k+1) u^(2k-4).                  */
static double h_series(double u) {
  double s = 0, p = 1, u2 = u * u;
  for (int k = 1; k <= 10; ++k) {
    double c = (k % 2 ? -1.0 : 1.0) * (2.0 * k) / (2.0 * k + 1.0);
    s += c * p;
    p *= u2;
  }
  return s;
}
static double m_series(double u) {
  double s = 0, p = 1, u2 = u * u;
  for (int k = 2; k <= 11; ++k) {
    double c = (k % 2 ? 1.0 : -1.0) * 4.0 * k * (k - 1.0) / (2.0 * k + 1.0);
    s += c * p;
    p *= u2;
  }
  return s;
}
#define SERIES_U 1e-2

/* J_phi, row-major 2x3 (Sec. 4.2, with f multiplying the whole entry). */
void orc_jacobian(const double p[3], double fx, double fy, double J[6]) {
  double x = p[0], y = p[1], z = p[2];
  double lz2 = x * x + y * y, l2 = lz2 + z * z, lz = sqrt(lz2);
  double theta = atan2(lz, z);
  if (z > 0 && lz < SERIES_U * z) {
    double h = h_series(lz / z) / (z * z * z);
    J[0] = fx * (z / l2 - y * y * h);
    J[1] = fx * x * y * h;
    J[2] = -fx * x / l2;
    J[3] = fy * x * y * h;
    J[4] = fy * (z / l2 - x * x * h);
    J[5] = -fy * y / l2;
    return;
  }
  double lz3 = lz2 * lz;
  J[0] = fx * (x * x * z / (lz2 * l2) + y * y * theta / lz3);
  J[1] = fx * x * y * (z / (lz2 * l2) - theta / lz3);
  J[2] = -fx * x / l2;
  J[3] = fy * x * y * (z / (lz2 * l2) - theta / lz3);
  J[4] = fy * (y * y * z / (lz2 * l2) + x * x * theta / lz3);
  J[5] = -fy * y / l2;
}

/* dJ/dx_c, dJ/dy_c, dJ/dz_c (Sec. 4.3).  Output dJ[c*6 + r*3 + k] =
 * d J[r][k] / d(coordinate c).  The four S1..S4 entries share the
 * denominator D = l_2^2 l_z^5. */
void orc_jacobian_grad(const double p[3], double fx, double fy, double dJ[18]) {
  double x = p[0], y = p[1], z = p[2];
  double lz2 = x * x + y * y, l2 = lz2 + z * z, lz = sqrt(lz2);
  double theta = atan2(lz, z);
  double l22 = l2 * l2;
  double S1, S2, S3, S4; /* already divided by D */
  if (z > 0 && lz < SERIES_U * z) {
    double u = lz / z;
    double h = h_series(u) / (z * z * z);
    double m = m_series(u) / (z * z * z * z * z);
    S1 = x * (3 * h - x * x * m);
    S2 = y * (h - x * x * m);
    S3 = x * (h - y * y * m);
    S4 = y * (3 * h - y * y * m);
  } else {
    double lz3 = lz2 * lz, lz5 = lz3 * lz2;
    double S7 = -l22 * lz2 * theta + l2 * lz3 * z;
    double S8 = 3 * l22 * theta - 3 * l2 * lz * z - 2 * lz3 * z;
    double D = l22 * lz5;
    S1 = x * (3 * S7 + x * x * S8) / D;
    S2 = y * (S7 + x * x * S8) / D;
    S3 = x * (S7 + y * y * S8) / D;
    S4 = y * (3 * S7 + y * y * S8) / D;
  }
  double S5 = x * x - y * y - z * z;
  double S6 = y * y - x * x - z * z;
  /* d/dx_c */
  dJ[0] = fx * S1;  dJ[1] = fx * S2;  dJ[2] = fx * S5 / l22;
  dJ[3] = fy * S2;  dJ[4] = fy * S3;  dJ[5] = 2 * fy * x * y / l22;
  /* d/dy_c */
  dJ[6] = fx * S2;  dJ[7] = fx * S3;  dJ[8] = 2 * fx * x * y / l22;
  dJ[9] = fy * S3;  dJ[10] = fy * S4; dJ[11] = fy * S6 / l22;
  /* d/dz_c */
  dJ[12] = fx * S5 / l22;          dJ[13] = 2 * fx * x * y / l22; dJ[14] = 2 * fx * x * z / l22;
  dJ[15] = 2 * fy * x * y / l22;   dJ[16] = fy * S6 / l22;        dJ[17] = 2 * fy * y * z / l22;
}

/* ------------------------------------------------------------------------ */
/* Other camera models: projection, J = d mu_p / d mu_c and dJ / d mu_c as    */
/* the value, gradient and Hessian of each pixel coordinate, carried through  */
/* the projection's formula by second-order forward-mode differentiation:     */
/* for a value v with gradient g and Hessian H in (x_c, y_c, z_c),            */
/*   (a b)'' = a'' b + a' b'^T + b' a'^T + a b'',                               */
/*   f(a)'' = f'(a) a'' + f''(a) a' a'^T.                                       */
/* ------------------------------------------------------------------------ */
typedef struct { double v, g[3], h[9]; } hd;

static hd hd_const(double v) { hd r; memset(&r, 0, sizeof r); r.v = v; return r; }
static hd hd_var(double v, int k) { hd r = hd_const(v); r.g[k] = 1.0; return r; }
static hd hd_add(hd a, hd b) {
  hd r; r.v = a.v + b.v;
  for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] + b.g[k];
  for (int k = 0; k < 9; ++k) r.h[k] = a.h[k] + b.h[k];
  return r;
}
static hd hd_scale(hd a, double s) {
  hd r; r.v = a.v * s;
  for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * s;
  for (int k = 0; k < 9; ++k) r.h[k] = a.h[k] * s;
  return r;
}
static hd hd_mul(hd a, hd b) {
  hd r; r.v = a.v * b.v;
  for (int k = 0; k < 3; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      r.h[i * 3 + j] = a.h[i * 3 + j] * b.v + a.g[i] * b.g[j] + b.g[i] * a.g[j] + a.v * b.h[i * 3 + j];
  return r;
}
/* f(a) given f(a.v), f'(a.v), f''(a.v) */
static hd hd_chain(hd a, double f0, double f1, double f2) {
  hd r; r.v = f0;
  for (int k = 0; k < 3; ++k) r.g[k] = f1 * a.g[k];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.h[i * 3 + j] = f1 * a.h[i * 3 + j] + f2 * a.g[i] * a.g[j];
  return r;
}
static hd hd_recip(hd a) { return hd_chain(a, 1.0 / a.v, -1.0 / (a.v * a.v), 2.0 / (a.v * a.v * a.v)); }
static hd hd_sqrt(hd a) {
  double s = sqrt(a.v);
  return hd_chain(a, s, 0.5 / s, -0.25 / (s * a.v));
}
static hd hd_sin(hd a) { return hd_chain(a, sin(a.v), cos(a.v), -sin(a.v)); }
static hd hd_tan(hd a) {
  double t = tan(a.v), sec2 = 1.0 + t * t;
  return hd_chain(a, t, sec2, 2.0 * sec2 * t);
}
/* atan2(a, b): partials b / s and -a / s with s = a^2 + b^2; second partials
 * -2ab / s^2 (aa), 2ab / s^2 (bb), (a^2 - b^2) / s^2 (ab). */
static hd hd_atan2(hd a, hd b) {
  double s = a.v * a.v + b.v * b.v, s2 = s * s;
  double fa = b.v / s, fb = -a.v / s;
  double faa = -2.0 * a.v * b.v / s2, fbb = 2.0 * a.v * b.v / s2, fab = (a.v * a.v - b.v * b.v) / s2;
  hd r; r.v = atan2(a.v, b.v);
  for (int k = 0; k < 3; ++k) r.g[k] = fa * a.g[k] + fb * b.g[k];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      r.h[i * 3 + j] = fa * a.h[i * 3 + j] + fb * b.h[i * 3 + j] + faa * a.g[i] * a.g[j] + fbb * b.g[i] * b.g[j] +
                       fab * (a.g[i] * b.g[j] + b.g[i] * a.g[j]);
  return r;
}

/* The pixel coordinates of a camera-space point as hd values. */
static void project_hd(int model, const double p[3], double fx, double fy, double cx, double cy, hd out[2]) {
  hd x = hd_var(p[0], 0), y = hd_var(p[1], 1), z = hd_var(p[2], 2);
  if (model == MODEL_PANORAMA) {
    hd rho = hd_sqrt(hd_add(hd_mul(x, x), hd_mul(z, z)));
    out[0] = hd_add(hd_const(cx), hd_scale(hd_atan2(x, z), fx));
    out[1] = hd_add(hd_const(cy), hd_scale(hd_atan2(y, rho), fy));
    return;
  }
  hd lz = hd_sqrt(hd_add(hd_mul(x, x), hd_mul(y, y)));
  hd th = hd_atan2(lz, z), r;
  switch (model) {
    case MODEL_PINHOLE: r = hd_tan(th); break;
    case MODEL_EQUISOLID: r = hd_scale(hd_sin(hd_scale(th, 0.5)), 2.0); break;
    case MODEL_ORTHOGRAPHIC: r = hd_sin(th); break;
    case MODEL_STEREOGRAPHIC: r = hd_scale(hd_tan(hd_scale(th, 0.5)), 2.0); break;
    default: r = th; break;
  }
  hd k = hd_mul(r, hd_recip(lz)); /* r(theta) / l_z */
  out[0] = hd_add(hd_const(cx), hd_scale(hd_mul(k, x), fx));
  out[1] = hd_add(hd_const(cy), hd_scale(hd_mul(k, y), fy));
}

/* The angle each model culls on: the incidence theta for radial models, the
 * absolute latitude for the panorama (its poles are where J is unbounded). */
double orc_cull_angle(int model, const double p[3]) {
  if (model == MODEL_PANORAMA) return fabs(atan2(p[1], sqrt(p[0] * p[0] + p[2] * p[2])));
  return atan2(sqrt(p[0] * p[0] + p[1] * p[1]), p[2]);
}

/* Model dispatch: the equidistant model keeps the paper's closed forms
 * (Sec. 3.2, 4.2, 4.3); the others use the hd derivatives.  Radial models
 * other than the equidistant are not evaluated exactly on the optical axis
 * (l_z = 0), where the hd chain divides by zero. */
void orc_project_model(int model, const double p[3], double fx, double fy, double cx, double cy, double out[2]) {
  if (model == MODEL_EQUIDISTANT) { orc_project(p, fx, fy, cx, cy, out); return; }
  hd m[2];
  project_hd(model, p, fx, fy, cx, cy, m);
  out[0] = m[0].v;
  out[1] = m[1].v;
}
void orc_jacobian_model(int model, const double p[3], double fx, double fy, double J[6]) {
  if (model == MODEL_EQUIDISTANT) { orc_jacobian(p, fx, fy, J); return; }
  hd m[2];
  project_hd(model, p, fx, fy, 0.0, 0.0, m);
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) J[r * 3 + k] = m[r].g[k];
}
void orc_jacobian_grad_model(int model, const double p[3], double fx, double fy, double dJ[18]) {
  if (model == MODEL_EQUIDISTANT) { orc_jacobian_grad(p, fx, fy, dJ); return; }
  hd m[2];
  project_hd(model, p, fx, fy, 0.0, 0.0, m);
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k) dJ[c * 6 + r * 3 + k] = m[r].h[k * 3 + c];
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, degree <= 3, by the associated-Legendre          */
/* recurrence (Condon-Shortley phase).  Index k = l (l + 1) + m.              */
/*   Y_l0  = N_l^0 P_l(z)                                                      */
/*   Y_lm  = sqrt2 N_l^m Pt_l^m(z) Re((x + i y)^m)     m > 0                   */
/*   Y_l-m = sqrt2 N_l^m Pt_l^m(z) Im((x + i y)^m)     m > 0                   */
/* with Pt_l^m = P_l^m / (1 - z^2)^(m/2), N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). */
/* ------------------------------------------------------------------------ */
static double factorial(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

static void sh_basis_dual(int degree, dual x, dual y, dual z, dual Y[16]) {
  dual Pt[4][4]; /* Pt[l][m] */
  for (int m = 0; m <= degree; ++m) {
    double dfact = 1; /* (2m-1)!! */
    for (int i = 2 * m - 1; i > 1; i -= 2) dfact *= i;
    Pt[m][m] = d_const((m % 2 ? -1.0 : 1.0) * dfact);
    if (m + 1 <= degree) Pt[m + 1][m] = d_scale(d_mul(z, Pt[m][m]), 2.0 * m + 1.0);
    for (int l = m + 2; l <= degree; ++l)
      Pt[l][m] = d_scale(d_sub(d_scale(d_mul(z, Pt[l - 1][m]), 2.0 * l - 1.0),
                               d_scale(Pt[l - 2][m], l + m - 1.0)),
                         1.0 / (l - m));
  }
  dual cm[4], sm[4];
  cm[0] = d_const(1.0);
  sm[0] = d_const(0.0);
  for (int m = 1; m <= degree; ++m) {
    cm[m] = d_sub(d_mul(x, cm[m - 1]), d_mul(y, sm[m - 1]));
    sm[m] = d_add(d_mul(x, sm[m - 1]), d_mul(y, cm[m - 1]));
  }
  for (int l = 0; l <= degree; ++l) {
    for (int m = 0; m <= l; ++m) {
      double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
      if (m == 0) {
        Y[l * (l + 1)] = d_scale(Pt[l][0], N);
      } else {
        Y[l * (l + 1) + m] = d_scale(d_mul(Pt[l][m], cm[m]), sqrt(2.0) * N);
        Y[l * (l + 1) - m] = d_scale(d_mul(Pt[l][m], sm[m]), sqrt(2.0) * N);
      }
    }
  }
}

void orc_sh_basis(int degree, const double dir[3], double out[16]) {
  dual Y[16];
  sh_basis_dual(degree, d_const(dir[0]), d_const(dir[1]), d_const(dir[2]), Y);
  int nb = (degree + 1) * (degree + 1);
  for (int k = 0; k < nb; ++k) out[k] = Y[k].v;
}

/* rgb_c = max(0, sum_k sh[k*3+c] Y_k(dir) + 0.5), dir = (mu - cam)/|mu - cam|.
 * Derivatives (if wanted) are with respect to mu, in d[0..2]. */
static void sh_color(int degree, const double mu[3], const double cam[3], const double* sh, int64_t n,
                     int64_t i, dual rgb[3], double Yv[16]) {
  dual v[3];
  for (int a = 0; a < 3; ++a) v[a] = d_sub(d_var(mu[a], a), d_const(cam[a]));
  dual len = d_sqrt(d_add(d_add(d_mul(v[0], v[0]), d_mul(v[1], v[1])), d_mul(v[2], v[2])));
  dual dir[3];
  for (int a = 0; a < 3; ++a) dir[a] = d_div(v[a], len);
  dual Y[16];
  sh_basis_dual(degree, dir[0], dir[1], dir[2], Y);
  int nb = (degree + 1) * (degree + 1);
  for (int c = 0; c < 3; ++c) {
    dual s = d_const(0.5);
    for (int k = 0; k < nb; ++k) s = d_add(s, d_scale(Y[k], sh[(int64_t)(k * 3 + c) * n + i]));
    rgb[c] = s;
  }
  for (int k = 0; k < nb; ++k) Yv[k] = Y[k].v;
}

/* ------------------------------------------------------------------------ */
/* 3D covariance (Eq. 1): Sigma = R S S^T R^T, R from the normalised           */
/* quaternion (w, x, y, z).  Dual directions 0..2 = scale, 3..6 = quaternion. */
/* ------------------------------------------------------------------------ */
static void cov3d_dual(const double s[3], const double q[4], dual Sig[9]) {
  dual sd[3], qd[4];
  for (int a = 0; a < 3; ++a) sd[a] = d_var(s[a], a);
  for (int a = 0; a < 4; ++a) qd[a] = d_var(q[a], 3 + a);
  dual qn2 = d_const(0);
  for (int a = 0; a < 4; ++a) qn2 = d_add(qn2, d_mul(qd[a], qd[a]));
  dual qn = d_sqrt(qn2);
  dual w = d_div(qd[0], qn), x = d_div(qd[1], qn), y = d_div(qd[2], qn), z = d_div(qd[3], qn);
  dual one = d_const(1.0);
  dual R[9];
  R[0] = d_sub(one, d_scale(d_add(d_mul(y, y), d_mul(z, z)), 2));
  R[1] = d_scale(d_sub(d_mul(x, y), d_mul(w, z)), 2);
  R[2] = d_scale(d_add(d_mul(x, z), d_mul(w, y)), 2);
  R[3] = d_scale(d_add(d_mul(x, y), d_mul(w, z)), 2);
  R[4] = d_sub(one, d_scale(d_add(d_mul(x, x), d_mul(z, z)), 2));
  R[5] = d_scale(d_sub(d_mul(y, z), d_mul(w, x)), 2);
  R[6] = d_scale(d_sub(d_mul(x, z), d_mul(w, y)), 2);
  R[7] = d_scale(d_add(d_mul(y, z), d_mul(w, x)), 2);
  R[8] = d_sub(one, d_scale(d_add(d_mul(x, x), d_mul(y, y)), 2));
  dual M[9]; /* M = R S */
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[r * 3 + c] = d_mul(R[r * 3 + c], sd[c]);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      dual acc = d_const(0);
      for (int k = 0; k < 3; ++k) acc = d_add(acc, d_mul(M[r * 3 + k], M[c * 3 + k]));
      Sig[r * 3 + c] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Preprocess: one Gaussian at a time, in the order of the paper's            */
/* commented PreprocessCUDA algorithm (frustum test, project, cov3D, cov2D,   */
/* det test, eigenvalues, radius, rect, colour, depth).                       */
/* ------------------------------------------------------------------------ */
typedef struct {
  double pc[3];
  double theta;
  double mu_p[2];
  double J[6];
  double T[6];
  double Sig[9];
  double Sp[4]; /* dilated 2D covariance */
  double conic[3];
} geom;

/* Returns 0 if culled. */
static int geometry(int64_t i, int64_t n, const double* means, const double* scales, const double* quats,
                    const double* opac, const double* Rw, const double* tw, const orc_camera* cam, geom* g,
                    dual Sig[9]) {
  double mf[3] = {means[i], means[n + i], means[2 * n + i]};
  double sf[3] = {scales[i], scales[n + i], scales[2 * n + i]};
  double qf[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
  for (int a = 0; a < 3; ++a) if (!isfinite(mf[a]) || !isfinite(sf[a])) return 0;
  for (int a = 0; a < 4; ++a) if (!isfinite(qf[a])) return 0;
  if (!isfinite(opac[i])) return 0;
  double q2 = 0;
  for (int a = 0; a < 4; ++a) q2 += qf[a] * qf[a];
  if (!(q2 > 0)) return 0;
  /* mu_c = W mu + b (Eq. 2), each row summed left to right. */
  for (int r = 0; r < 3; ++r)
    g->pc[r] = ((Rw[r * 3 + 0] * mf[0] + Rw[r * 3 + 1] * mf[1]) + Rw[r * 3 + 2] * mf[2]) + tw[r];
  double dist = sqrt((g->pc[0] * g->pc[0] + g->pc[1] * g->pc[1]) + g->pc[2] * g->pc[2]);
  if (!(dist > cam->near_dist)) return 0;
  g->theta = orc_cull_angle(cam->model, g->pc);
  if (!(g->theta <= cam->theta_max)) return 0;
  orc_project_model(cam->model, g->pc, cam->fx, cam->fy, cam->cx, cam->cy, g->mu_p);
  double s[3] = {sf[0], sf[1], sf[2]}, q[4] = {qf[0], qf[1], qf[2], qf[3]};
  cov3d_dual(s, q, Sig);
  for (int k = 0; k < 9; ++k) g->Sig[k] = Sig[k].v;
  orc_jacobian_model(cam->model, g->pc, cam->fx, cam->fy, g->J);
  /* T = J W */
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += g->J[r * 3 + k] * Rw[k * 3 + c];
      g->T[r * 3 + c] = acc;
    }
  /* Sigma_p = T Sigma T^T, plus the 0.3 px^2 low-pass dilation */
  double TS[6];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += g->T[r * 3 + k] * g->Sig[k * 3 + c];
      TS[r * 3 + c] = acc;
    }
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += TS[r * 3 + k] * g->T[c * 3 + k];
      g->Sp[r * 2 + c] = acc;
    }
  g->Sp[0] += 0.3;
  g->Sp[3] += 0.3;
  double det = g->Sp[0] * g->Sp[3] - g->Sp[1] * g->Sp[2];
  if (!(det > 0)) return 0;
  g->conic[0] = g->Sp[3] / det;
  g->conic[1] = -g->Sp[1] / det;
  g->conic[2] = g->Sp[0] / det;
  return 1;
}

static double tie_dist(double v) { return fabs(v - nearbyint(v)); }

/*
 * Outputs (arrays of length n unless stated):
 *   visible u8, mu_p [n][2], conic [n][3] (A, B, C with q = -(A dx^2 + C dy^2)/2 - B dx dy),
 *   rgb [n][3], clamped u8 (bit c = channel c clamped at 0), radius i32,
 *   rect [n][4] (x0, y0, x1, y1, tile units, half-open), depth f32 (|mu_c|),
 *   tiles u32, tie u8 (1 = radius or rect decision within 1e-9 of a boundary),
 *   cov2d [n][3] (the dilated 2D covariance Sigma': xx, xy, yy).
 */
void orc_preprocess(int64_t n, const double* means, const double* scales, const double* quats, const double* opac,
                    const double* sh, int sh_degree, const double* Rw, const double* tw, const orc_camera* cam,
                    uint8_t* visible, double* mu_p, double* conic, double* rgb, uint8_t* clamped,
                    int32_t* radius, int32_t* rect, float* depth, uint32_t* tiles, uint8_t* tie, double* cov2d) {
  const int gx = (cam->width + TILE - 1) / TILE, gy = (cam->height + TILE - 1) / TILE;
  double campos[3];
  for (int a = 0; a < 3; ++a) campos[a] = -(Rw[0 * 3 + a] * tw[0] + Rw[1 * 3 + a] * tw[1] + Rw[2 * 3 + a] * tw[2]);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    visible[i] = 0; radius[i] = 0; tiles[i] = 0; clamped[i] = 0; tie[i] = 0; depth[i] = 0;
    for (int a = 0; a < 4; ++a) rect[i * 4 + a] = 0;
    for (int a = 0; a < 2; ++a) mu_p[i * 2 + a] = 0;
    for (int a = 0; a < 3; ++a) { conic[i * 3 + a] = 0; rgb[i * 3 + a] = 0; cov2d[i * 3 + a] = 0; }
    geom g;
    dual Sig[9];
    if (!geometry(i, n, means, scales, quats, opac, Rw, tw, cam, &g, Sig)) continue;
    double mid = 0.5 * (g.Sp[0] + g.Sp[3]);
    double det = g.Sp[0] * g.Sp[3] - g.Sp[1] * g.Sp[2];
    double lam = mid + sqrt(fmax(0.1, mid * mid - det));
    double r3 = 3.0 * sqrt(lam);
    double rad = ceil(r3);
    uint8_t t = 0;
    if (tie_dist(r3) < 1e-9 * r3) t = 1;
    double v[4] = {(g.mu_p[0] - rad) / TILE, (g.mu_p[1] - rad) / TILE, (g.mu_p[0] + rad + TILE - 1) / TILE,
                   (g.mu_p[1] + rad + TILE - 1) / TILE};
    int lim[4] = {gx, gy, gx, gy};
    int rc[4];
    for (int a = 0; a < 4; ++a) {
      double f = floor(v[a]);
      if (f < 0) f = 0;
      if (f > lim[a]) f = lim[a];
      rc[a] = (int)f;
      if (v[a] > -1 && v[a] < lim[a] + 1 && tie_dist(v[a]) < 1e-9 * fmax(1.0, fabs(v[a]))) t = 1;
    }
    int area = (rc[2] - rc[0]) * (rc[3] - rc[1]);
    if (area == 0) continue;
    dual col[3];
    double Yv[16];
    double mu[3] = {means[i], means[n + i], means[2 * n + i]};
    sh_color(sh_degree, mu, campos, sh, n, i, col, Yv);
    int ok = 1;
    for (int c = 0; c < 3; ++c) if (!isfinite(col[c].v)) ok = 0;
    if (!ok) continue;
    uint8_t cl = 0;
    for (int c = 0; c < 3; ++c) {
      double val = col[c].v;
      if (val < 0) { cl |= (uint8_t)(1u << c); val = 0; }
      rgb[i * 3 + c] = val;
    }
    visible[i] = 1;
    clamped[i] = cl;
    tie[i] = t;
    mu_p[i * 2 + 0] = g.mu_p[0];
    mu_p[i * 2 + 1] = g.mu_p[1];
    for (int a = 0; a < 3; ++a) conic[i * 3 + a] = g.conic[a];
    cov2d[i * 3 + 0] = g.Sp[0];
    cov2d[i * 3 + 1] = g.Sp[1];
    cov2d[i * 3 + 2] = g.Sp[3];
    radius[i] = (int32_t)rad;
    for (int a = 0; a < 4; ++a) rect[i * 4 + a] = rc[a];
    depth[i] = (float)sqrt((g.pc[0] * g.pc[0] + g.pc[1] * g.pc[1]) + g.pc[2] * g.pc[2]);
    tiles[i] = (uint32_t)area;
  }
}

/* ------------------------------------------------------------------------ */
/* Tight binning: only the tiles of the rect the splat can reach.             */
/* ------------------------------------------------------------------------ */
/*
 * A pixel (x, y) is blended with a splat only if alpha >= 1/255, that is
 * q = -(A u^2 + 2 B u v + C v^2) / 2 >= ln(1 / (255 o)) with (u, v) = (x, y) -
 * mu_p, i.e. inside the ellipse A u^2 + 2 B u v + C v^2 <= r2 = 2 ln(255 o).
 * A tile (tx, ty) of the 3-sigma rect is kept if that ellipse, grown to
 * r2 * 1.0201 (radius + 1%) and padded by 1/8 px, reaches the tile's
 * pixel-centre box [16 tx, 16 tx + 15] x [16 ty, 16 ty + 15]; dropping the
 * other tiles changes no pixel.  The margin is the library's, so that its
 * float evaluation of the per-pixel test never passes outside the kept
 * tiles.  Conventions shared with it (in log2 units P = r2 / (2 ln 2)):
 * P < 0 keeps no tile, 0 <= P <= 1e-6 and |B / A| > 1e3 keep the whole rect.
 *
 * Per row of tiles the reached columns are one interval: the ellipse's
 * u-extent over the row's v-range.  u_max(v) = (-B v + sqrt(A r2 - det v^2)) / A
 * is concave with its peak at v = -B sqrt(r2 / (det C)), u_min(v) =
 * (-B v - sqrt(A r2 - det v^2)) / A convex with its trough at the opposite
 * v, det = A C - B^2; each is clamped to the row's v-range.
 */
static const double kTightGrow = 1.0201, kTightPad = 0.125, kTightP0 = 1e-6, kTightBeta = 1e3;

/* 0: no tile, 1: per-row intervals, 2: the whole rect. */
static int tight_kind(const double* con, double opac) {
  const double P = log2(255.0 * opac);
  if (!(P >= 0.0)) return 0;
  if (P <= kTightP0) return 2;
  if (!(fabs(con[1] / con[0]) <= kTightBeta)) return 2;
  return 1;
}

/* Columns [c0, c1) of tile row ty reached within [x0, x1) (kind 1). */
static void tight_row(const double* mu, const double* con, double opac, int ty, int x0, int x1, double grow,
                      double pad, int* c0, int* c1) {
  const double A = con[0], B = con[1], C = con[2], det = A * C - B * B;
  const double r2 = 2.0 * log(255.0 * opac) * grow;
  *c0 = *c1 = x0;
  const double vmax = sqrt(A * r2 / det);
  const double vlo = fmax(TILE * ty - pad - mu[1], -vmax), vhi = fmin(TILE * ty + TILE - 1 + pad - mu[1], vmax);
  if (!(vlo <= vhi)) return;
  const double vs = B * sqrt(r2 / (det * C));
  const double va = fmin(fmax(-vs, vlo), vhi), vb = fmin(fmax(vs, vlo), vhi);
  const double umax = (-B * va + sqrt(fmax(0.0, A * r2 - det * va * va))) / A;
  const double umin = (-B * vb - sqrt(fmax(0.0, A * r2 - det * vb * vb))) / A;
  const double xlo = mu[0] + umin - pad, xhi = mu[0] + umax + pad;
  const int lo = (int)fmin(fmax(ceil((xlo - (TILE - 1)) / TILE), x0), x1);
  const int hi = (int)fmin(fmax(floor(xhi / TILE) + 1, x0), x1);
  if (hi > lo) { *c0 = lo; *c1 = hi; }
}

/* Counts the kept tiles of every visible Gaussian into tiles[] (a Gaussian
 * with none becomes invisible) and flags (tie bit 4) any whose count or
 * intervals move when the margins move by 1e-4 (relative) / 4e-3 px, well
 * beyond what a binary32 evaluation of the rule can move them: outside those
 * Gaussians any such evaluation keeps the same tiles as this one. */
void orc_tighten(int64_t n, uint8_t* visible, const double* mu_p, const double* conic, const double* opac,
                 const int32_t* rect, uint32_t* tiles, uint8_t* tie) {
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    if (!visible[i]) continue;
    const int32_t* rc = &rect[i * 4];
    const double* con = &conic[i * 3];
    const double P = log2(255.0 * opac[i]);
    if (fabs(P) < 1e-9 || fabs(P - kTightP0) < 1e-9 ||
        fabs(fabs(con[1] / con[0]) - kTightBeta) < 1e-6 * kTightBeta)
      tie[i] |= 4;
    const int kind = tight_kind(con, opac[i]);
    int64_t count = 0;
    if (kind == 2) {
      count = (int64_t)(rc[2] - rc[0]) * (rc[3] - rc[1]);
    } else if (kind == 1) {
      for (int ty = rc[1]; ty < rc[3]; ++ty) {
        int a0, a1, b0, b1, d0, d1;
        tight_row(&mu_p[i * 2], con, opac[i], ty, rc[0], rc[2], kTightGrow, kTightPad, &a0, &a1);
        tight_row(&mu_p[i * 2], con, opac[i], ty, rc[0], rc[2], kTightGrow * (1 + 1e-4), kTightPad + 4e-3, &b0, &b1);
        tight_row(&mu_p[i * 2], con, opac[i], ty, rc[0], rc[2], kTightGrow * (1 - 1e-4), kTightPad - 4e-3, &d0, &d1);
        if (a1 - a0 != b1 - b0 || a1 - a0 != d1 - d0 || (a1 > a0 && (a0 != b0 || a0 != d0))) tie[i] |= 4;
        count += a1 - a0;
      }
    }
    tiles[i] = (uint32_t)count;
    if (count == 0) visible[i] = 0;
  }
}

/* ------------------------------------------------------------------------ */
/* FP32 key recipe of the tight binning.                                      */
/* ------------------------------------------------------------------------ */
/*
 * The rule above decides in exact arithmetic (here fp64).  A renderer that
 * decides in binary32 from a float record of the splat keeps the same tiles
 * except where a margin lands within float rounding of a tile edge.  This
 * mode fixes one such float evaluation completely, so that its decisions are
 * reproducible bit for bit by any IEEE binary32 implementation of the same
 * steps (each step one correctly rounded operation, nothing contracted):
 *
 *   record, the fp64 values rounded once to float:
 *     mx = hi + lo (float add) with hi = f(mu_x), lo = f(mu_x - hi); my alike;
 *     a = f(A log2(e) / 2);  beta = f(B / A);  d = f((C - B^2 / A) log2(e) / 2);
 *     P = f(log2(255 o32)), 255 o32 the float product of the float opacity;
 *   setup:  P < 0 (or NaN): no tile;  P <= 1e-6, |beta| > 1e3, a or d not
 *     positive: the whole rect;  else Pg = P * 1.0201, ia = 1 / a,
 *     Pa = Pg * ia, da = d * ia, ry = sqrt(Pg * (1 / d)),
 *     ds = beta * sqrt((a * Pg) * (1 / (d * fma(beta * beta, a, d))));
 *     the whole rect again if ry, |ds|, Pa or da exceeds 1e30 or is NaN;
 *   per tile row ty of the rect [x0, x1):  with pad = 0.125,
 *     lo_y = max((my - (16 ty + 15)) - pad, -ry), hi_y = min((my - 16 ty) + pad, ry),
 *     none if !(lo_y <= hi_y);  ya = min(max(ds, lo_y), hi_y),
 *     yb = min(max(-ds, lo_y), hi_y), sa = sqrt(max(0, Pa - (da * ya) * ya)),
 *     sb likewise at yb, xhi = ((mx + beta * ya) + sa) + pad,
 *     xlo = ((mx + beta * yb) - sb) - pad; the whole row if !(xhi >= xlo);
 *     columns [clamp(ceil((xlo - 15) * (1/16))), clamp(floor(xhi * (1/16)) + 1))
 *     clamped to [x0, x1] in float, kept if the interval is not empty.
 *
 * The record's dy is mean minus pixel (dy = my - py), as in the blend's
 * exponent; the ellipse is |a| t^2 + |d| dy^2 <= P in log2 units with
 * t = dx + beta dy, the alpha >= 1/255 region of Eq. 3's weights, grown and
 * padded as above.
 *
 * Ties.  The renderer's fp64 geometry is another evaluation of the same
 * formulas, so its record may round the other way where the fp64 value lies
 * within a few fp64 ulps of a float rounding midpoint.  Each record value
 * within kRecTie (relative) of a midpoint gets both neighbours; a Gaussian
 * is a tie if any combination of them keeps other tiles.
 */
static const double kRecTie = 1e-9;

typedef struct { float mx, my, a, beta, d, P; } rec32;

/* The float of the fp64 value v and, if v lies within kRecTie of the
 * midpoint between two floats, the other of the two (else alt = f). */
static void round_both(double v, double rel, float* f, float* alt) {
  *f = (float)v;
  *alt = *f;
  if (!isfinite(*f)) return;
  const float up = nextafterf(*f, INFINITY), dn = nextafterf(*f, -INFINITY);
  const double mup = 0.5 * ((double)*f + (double)up), mdn = 0.5 * ((double)*f + (double)dn);
  const double tol = rel * fabs(v);
  if (fabs(v - mup) <= tol) *alt = up;
  else if (fabs(v - mdn) <= tol) *alt = dn;
}

static float mean32(float hi, double mu) { return hi + (float)(mu - (double)hi); }

typedef struct { float mx, my, Pa, da, beta, ry, ds; int kind; } reach32;

static reach32 reach32_setup(const rec32* r) {
  reach32 z;
  z.mx = r->mx; z.my = r->my; z.beta = r->beta;
  z.Pa = z.da = z.ry = z.ds = 0.0f;
  const float a = r->a, d = r->d, P = r->P;
  if (!(P >= 0.0f)) { z.kind = 0; return z; }
  z.kind = 2;
  if (P <= 1e-6f || !(fabsf(r->beta) <= 1e3f) || !(a > 0.0f) || !(d > 0.0f)) return z;
  const float Pg = P * 1.0201f;
  const float ia = 1.0f / a;
  z.Pa = Pg * ia;
  z.da = d * ia;
  z.ry = sqrtf(Pg * (1.0f / d));
  const float bb = r->beta * r->beta;
  const float den = d * fmaf(bb, a, d);
  const float aP = a * Pg;
  z.ds = r->beta * sqrtf(aP * (1.0f / den));
  if (!(z.ry <= 1e30f) || !(fabsf(z.ds) <= 1e30f) || !(z.Pa <= 1e30f) || !(z.da <= 1e30f)) return z;
  z.kind = 1;
  return z;
}

static void reach32_row(const reach32* z, int ty, int x0, int x1, int* c0, int* c1) {
  *c0 = *c1 = x0;
  if (z->kind != 1) {
    if (z->kind == 2) *c1 = x1;
    return;
  }
  const float pad = 0.125f;
  const float lo_y = fmaxf((z->my - (float)(TILE * ty + TILE - 1)) - pad, -z->ry);
  const float hi_y = fminf((z->my - (float)(TILE * ty)) + pad, z->ry);
  if (!(lo_y <= hi_y)) return;
  const float ya = fminf(fmaxf(z->ds, lo_y), hi_y), yb = fminf(fmaxf(-z->ds, lo_y), hi_y);
  const float sa = sqrtf(fmaxf(0.0f, z->Pa - (z->da * ya) * ya));
  const float sb = sqrtf(fmaxf(0.0f, z->Pa - (z->da * yb) * yb));
  const float xhi = ((z->mx + z->beta * ya) + sa) + pad;
  const float xlo = ((z->mx + z->beta * yb) - sb) - pad;
  if (!(xhi >= xlo)) { *c1 = x1; return; }
  const float fx0 = (float)x0, fx1 = (float)x1;
  const int lo = (int)fminf(fmaxf(ceilf((xlo - 15.0f) * 0.0625f), fx0), fx1);
  const int hi = (int)fminf(fmaxf(floorf(xhi * 0.0625f) + 1.0f, fx0), fx1);
  if (hi > lo) { *c0 = lo; *c1 = hi; }
}

/* The record's six values (mx, my, a, beta, d, P) from the fp64 splat, each
 * with its alternative rounding (equal to it unless near a midpoint).
 * C - B^2 / A equals 1 / Sigma'_yy exactly, which is how it is taken here
 * (the difference cancels for thin splats).  A = Sigma'_yy / det(Sigma')
 * inherits the conditioning of the determinant, (|xx yy| + xy^2) / det, so
 * its tie band widens with it. */
static void record32_both(const double* mu, const double* con, const double* cov, double opac, float v[6],
                          float alt[6]) {
  const double l2e = 1.4426950408889634;
  const double A = con[0], B = con[1];
  const double det = cov[0] * cov[2] - cov[1] * cov[1];
  const double cond = (fabs(cov[0] * cov[2]) + cov[1] * cov[1]) / det;
  float hx, hx2, hy, hy2;
  round_both(mu[0], kRecTie, &hx, &hx2);
  round_both(mu[1], kRecTie, &hy, &hy2);
  v[0] = mean32(hx, mu[0]); alt[0] = mean32(hx2, mu[0]);
  v[1] = mean32(hy, mu[1]); alt[1] = mean32(hy2, mu[1]);
  round_both(0.5 * l2e * A, kRecTie + 1e-14 * cond, &v[2], &alt[2]);
  round_both(B / A, kRecTie, &v[3], &alt[3]);
  round_both(0.5 * l2e / cov[2], kRecTie, &v[4], &alt[4]);
  const float o32 = (float)opac;
  const float p255 = 255.0f * o32;
  round_both(log2((double)p255), kRecTie, &v[5], &alt[5]);
}

static rec32 rec_of(const float v[6]) {
  rec32 r = {v[0], v[1], v[2], v[3], v[4], v[5]};
  return r;
}

/* Kept tiles of one Gaussian under the recipe: total count, and first and
 * last + 1 kept tile row (ya = yb = 0 if none); cols[2 * (ty - y0) + k] the
 * row's interval if cols != NULL. */
static int64_t recipe_tiles(const rec32* r, const int32_t* rc, int* ya, int* yb, int* cols) {
  const reach32 z = reach32_setup(r);
  int64_t count = 0;
  *ya = *yb = 0;
  for (int ty = rc[1]; ty < rc[3]; ++ty) {
    int c0, c1;
    reach32_row(&z, ty, rc[0], rc[2], &c0, &c1);
    if (cols) { cols[2 * (ty - rc[1])] = c0; cols[2 * (ty - rc[1]) + 1] = c1; }
    if (c1 > c0) {
      if (count == 0) *ya = ty;
      *yb = ty + 1;
      count += c1 - c0;
    }
  }
  return count;
}

/* Counts the kept tiles of every visible Gaussian under the fp32 recipe (a
 * Gaussian with none becomes invisible); tie[i] |= 2 if another rounding of
 * its record keeps other tiles. */
void orc_tighten32(int64_t n, uint8_t* visible, const double* mu_p, const double* conic, const double* cov2d,
                   const double* opac, const int32_t* rect, uint32_t* tiles, uint8_t* tie) {
#pragma omp parallel
  {
    int cap = 0;
    int* ref = NULL;
    int* oth = NULL;
#pragma omp for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
      if (!visible[i]) continue;
      const int32_t* rc = &rect[i * 4];
      const int rows = rc[3] - rc[1];
      if (2 * rows > cap) {
        cap = 2 * rows;
        ref = (int*)realloc(ref, sizeof(int) * (size_t)cap);
        oth = (int*)realloc(oth, sizeof(int) * (size_t)cap);
      }
      float v[6], alt[6];
      record32_both(&mu_p[i * 2], &conic[i * 3], &cov2d[i * 3], opac[i], v, alt);
      rec32 r = rec_of(v);
      int ya, yb;
      const int64_t count = recipe_tiles(&r, rc, &ya, &yb, ref);
      int near[6], m = 0;
      for (int k = 0; k < 6; ++k)
        if (alt[k] != v[k]) near[m++] = k;
      for (int combo = 1; combo < (1 << m); ++combo) {
        float w[6];
        for (int k = 0; k < 6; ++k) w[k] = v[k];
        for (int b = 0; b < m; ++b)
          if (combo & (1 << b)) w[near[b]] = alt[near[b]];
        rec32 ra = rec_of(w);
        int ya2, yb2;
        recipe_tiles(&ra, rc, &ya2, &yb2, oth);
        for (int row = 0; row < rows; ++row) {
          const int* p = &ref[2 * row];
          const int* q = &oth[2 * row];
          if (p[0] == p[1] && q[0] == q[1]) continue; /* both empty */
          if (p[0] != q[0] || p[1] != q[1]) tie[i] |= 2;
        }
      }
      tiles[i] = (uint32_t)count;
      if (count == 0) visible[i] = 0;
    }
    free(ref);
    free(oth);
  }
}

/* Kept tiles of Gaussian i under the recipe for every rounding of its record
 * (up to 64 alternatives): out[alt][row][2] intervals over the rect's rows,
 * returns the number of alternatives written (at most max_alt). */
int orc_tight32_alternatives(const double* mu_p, const double* conic, const double* cov2d, double opac,
                             const int32_t* rect, int max_alt, int32_t* out) {
  float v[6], alt[6];
  record32_both(mu_p, conic, cov2d, opac, v, alt);
  int near[6], m = 0;
  for (int k = 0; k < 6; ++k)
    if (alt[k] != v[k]) near[m++] = k;
  const int rows = rect[3] - rect[1];
  int count = 0;
  for (int combo = 0; combo < (1 << m) && count < max_alt; ++combo) {
    float w[6];
    for (int k = 0; k < 6; ++k) w[k] = v[k];
    for (int b = 0; b < m; ++b)
      if (combo & (1 << b)) w[near[b]] = alt[near[b]];
    rec32 r = rec_of(w);
    int ya, yb;
    recipe_tiles(&r, rect, &ya, &yb, &out[(size_t)count * 2 * rows]);
    ++count;
  }
  return count;
}

/* ------------------------------------------------------------------------ */
/* Tile binning and sort (Sec. 3.1 "Rendering").                              */
/* ------------------------------------------------------------------------ */
int64_t orc_count_pairs(int64_t n, const uint8_t* visible, const uint32_t* tiles) {
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i)
    if (visible[i]) k += tiles[i];
  return k;
}

typedef struct { uint64_t key; uint32_t val; } pair_t;

static int cmp_pair(const void* a, const void* b) {
  const pair_t* x = (const pair_t*)a;
  const pair_t* y = (const pair_t*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->val != y->val) return x->val < y->val ? -1 : 1;
  return 0;
}

/* Emit one (key, id) pair per (Gaussian, tile of its rect; with tight = 1 per
 * tile the fp32 recipe keeps, with tight = 2 per tile the fp64 rule keeps), key =
 * tile_id << 32 | float bits of depth, then sort by (key, id) and find
 * each tile's [start, end) in the sorted list.  ranges is [ntiles][2]. */
void orc_bin(int64_t n, const uint8_t* visible, const int32_t* rect, const float* depth, int32_t width,
             int32_t height, int64_t kcount, uint64_t* keys, uint32_t* vals, uint32_t* ranges, int tight,
             const double* mu_p, const double* conic, const double* cov2d, const double* opac) {
  const int gx = (width + TILE - 1) / TILE, gy = (height + TILE - 1) / TILE;
  pair_t* p = (pair_t*)malloc(sizeof(pair_t) * (size_t)(kcount > 0 ? kcount : 1));
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!visible[i]) continue;
    uint32_t bits;
    memcpy(&bits, &depth[i], 4);
    const int kind = tight == 2 ? tight_kind(&conic[i * 3], opac[i]) : 2;
    reach32 z;
    if (tight == 1) {
      float v[6], alt[6];
      record32_both(&mu_p[i * 2], &conic[i * 3], &cov2d[i * 3], opac[i], v, alt);
      const rec32 r = rec_of(v);
      z = reach32_setup(&r);
    }
    for (int ty = rect[i * 4 + 1]; ty < rect[i * 4 + 3]; ++ty) {
      int c0 = rect[i * 4 + 0], c1 = rect[i * 4 + 2];
      if (tight == 1) {
        reach32_row(&z, ty, rect[i * 4 + 0], rect[i * 4 + 2], &c0, &c1);
      } else {
        if (kind == 0) c1 = c0;
        if (kind == 1)
          tight_row(&mu_p[i * 2], &conic[i * 3], opac[i], ty, rect[i * 4 + 0], rect[i * 4 + 2], kTightGrow,
                    kTightPad, &c0, &c1);
      }
      for (int tx = c0; tx < c1; ++tx) {
        p[k].key = ((uint64_t)(uint32_t)(ty * gx + tx) << 32) | bits;
        p[k].val = (uint32_t)i;
        ++k;
      }
    }
  }
  qsort(p, (size_t)k, sizeof(pair_t), cmp_pair);
  for (int64_t t = 0; t < (int64_t)gx * gy * 2; ++t) ranges[t] = 0;
  for (int64_t j = 0; j < k; ++j) {
    keys[j] = p[j].key;
    vals[j] = p[j].val;
    uint32_t tile = (uint32_t)(p[j].key >> 32);
    if (j == 0 || (uint32_t)(p[j - 1].key >> 32) != tile) ranges[tile * 2] = (uint32_t)j;
    if (j == k - 1 || (uint32_t)(p[j + 1].key >> 32) != tile) ranges[tile * 2 + 1] = (uint32_t)(j + 1);
  }
  free(p);
}

/* ------------------------------------------------------------------------ */
/* Alpha blending (Eq. 3), per pixel of each 16x16 tile, front to back.      */
/* ------------------------------------------------------------------------ */
/*
 * Ambiguity flags.  A renderer that evaluates the per-pixel decisions in
 * binary32 takes them differently from this fp64 walk only where a compared
 * value lies within its rounding error of the threshold.  Each decision is
 * flagged when it lies within
 *   fixed margin + err_scale * (a first-order bound of that rounding error)
 * (relative).  The bound, with u = 2^-24:
 *   alpha: the exponent q in binary32 has error <= 8 u (1 + |q|) from its own
 *     operations (record values rounded once, a handful of products and sums
 *     of like-signed terms, exp and the product o e^q included), plus
 *     |dq/d delta| times the error of the pixel offset delta = mu_p - p, which
 *     is formed tile-relative (the mean's float high part minus the tile
 *     origin is exact, then the low part is added and the pixel's offset in
 *     the tile subtracted: two roundings at magnitude <= |delta| + 16):
 *     e_alpha = u (8 (1 + |q|) + sum_k |dq/d delta_k| (2 |delta_k| + 16));
 *   T: each blended step multiplies T by 1 - alpha, whose relative error is
 *     alpha / (1 - alpha) e_alpha plus one rounding, and rounds the product:
 *     e_T accumulates alpha / (1 - alpha) e_alpha + 3 u per step.
 * The transmittance stop of a step is flagged with the e_T of the value it
 * compares, the alpha cut and the clamp with that pixel's e_alpha.
 */
typedef struct {
  double tol_alpha; /* fixed relative margin around 1/255 */
  double tol_T;     /* fixed relative margin around the 1e-4 transmittance stop */
  double tol_clamp; /* fixed relative margin around the 0.99 alpha clamp */
  double err_scale; /* multiple of the binary32 error bound added to each margin (0: none) */
} orc_tol;

#define U32 5.9604644775390625e-08 /* 2^-24 */

#define ALPHA_MIN (1.0 / 255.0)
#define ALPHA_MAX 0.99
#define T_MIN 1e-4

typedef struct {
  uint32_t id;
  double alpha, T, eq, dx, dy;
  int clampd;
} contrib;

/* Walks one pixel's list; if rec != NULL stores every blended Gaussian.
 * Returns number blended; writes colour, final T, last (1 + list index of
 * the last blended Gaussian) and the ambiguity flags (1 alpha cut, 2 T stop,
 * 4 alpha clamp, 8 q ~ 0). */
static int walk_pixel(double px, double py, const uint32_t* ids, int64_t count, const double* mu_p,
                      const double* conic, const double* opac, const double* rgb, const orc_tol* tol,
                      double C[3], double* Tout, int64_t* last, uint8_t* flag, int64_t* evals, contrib* rec,
                      int64_t rec_cap) {
  double T = 1.0;
  int nb = 0;
  C[0] = C[1] = C[2] = 0;
  *last = 0;
  *flag = 0;
  int64_t ev = 0;
  double eT = 0.0; /* relative binary32 error bound of T */
  for (int64_t j = 0; j < count; ++j) {
    uint32_t g = ids[j];
    ++ev;
    double dx = mu_p[g * 2 + 0] - px, dy = mu_p[g * 2 + 1] - py;
    double A = conic[g * 3 + 0], B = conic[g * 3 + 1], Cc = conic[g * 3 + 2];
    double q = -0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy;
    if (fabs(q) < 1e-10) *flag |= 8;
    if (q > 0) continue;
    double ea = 0.0;
    if (tol->err_scale > 0) {
      const double gx = A * dx + B * dy, gy = B * dx + Cc * dy;
      ea = U32 * (8.0 * (1.0 + fabs(q)) + fabs(gx) * (2.0 * fabs(dx) + 16.0) + fabs(gy) * (2.0 * fabs(dy) + 16.0));
    }
    double eq = exp(q);
    double raw = opac[g] * eq;
    double alpha = raw < ALPHA_MAX ? raw : ALPHA_MAX;
    if (fabs(alpha - ALPHA_MIN) <= (tol->tol_alpha + tol->err_scale * ea) * ALPHA_MIN) *flag |= 1;
    if (alpha < ALPHA_MIN) continue;
    if (fabs(raw - ALPHA_MAX) <= (tol->tol_clamp + tol->err_scale * ea) * ALPHA_MAX) *flag |= 4;
    double tn = T * (1.0 - alpha);
    const double etn = eT + alpha / (1.0 - alpha) * ea + 3.0 * U32;
    if (fabs(tn - T_MIN) <= (tol->tol_T + tol->err_scale * etn) * T_MIN) *flag |= 2;
    if (tn < T_MIN) break;
    eT = etn;
    for (int c = 0; c < 3; ++c) C[c] += rgb[g * 3 + c] * alpha * T;
    if (rec && nb < rec_cap) {
      rec[nb].id = g; rec[nb].alpha = alpha; rec[nb].T = T; rec[nb].eq = eq;
      rec[nb].dx = dx; rec[nb].dy = dy; rec[nb].clampd = !(raw < ALPHA_MAX);
    }
    ++nb;
    T = tn;
    *last = j + 1;
  }
  *Tout = T;
  if (evals) *evals = ev;
  return nb;
}

/* image [3][H][W]; T_final [H][W]; last [H][W] (int32); flags [H][W]. */
void orc_blend(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* vals, const double* mu_p,
               const double* conic, const double* opac, const double* rgb, const float bg[3], const orc_tol* tol,
               double* image, double* T_final, int32_t* last, uint8_t* flags, int64_t* eval_total) {
  const int gx = (width + TILE - 1) / TILE, gy = (height + TILE - 1) / TILE;
  int64_t evsum = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : evsum)
  for (int t = 0; t < gx * gy; ++t) {
    int tx = t % gx, ty = t / gx;
    uint32_t s = ranges[t * 2], e = ranges[t * 2 + 1];
    for (int j = 0; j < TILE; ++j)
      for (int i = 0; i < TILE; ++i) {
        int px = tx * TILE + i, py = ty * TILE + j;
        if (px >= width || py >= height) continue;
        double C[3], T;
        int64_t lst, ev;
        uint8_t f;
        walk_pixel(px, py, vals + s, (int64_t)e - s, mu_p, conic, opac, rgb, tol, C, &T, &lst, &f, &ev, NULL, 0);
        int64_t pix = (int64_t)py * width + px;
        for (int c = 0; c < 3; ++c) image[(int64_t)c * width * height + pix] = C[c] + T * bg[c];
        T_final[pix] = T;
        last[pix] = (int32_t)lst;
        flags[pix] = f;
        evsum += ev;
      }
  }
  if (eval_total) *eval_total = evsum;
}

/* Untiled reference: each pixel walks every visible Gaussian in (depth, id)
 * order, keeping those whose rect contains the pixel's tile. */
void orc_blend_bruteforce(int64_t n, int32_t width, int32_t height, const uint8_t* visible, const int32_t* rect,
                          const float* depth, const double* mu_p, const double* conic, const double* opac,
                          const double* rgb, const float bg[3], const orc_tol* tol, double* image) {
  int64_t nv = 0;
  for (int64_t i = 0; i < n; ++i) nv += visible[i];
  pair_t* order = (pair_t*)malloc(sizeof(pair_t) * (size_t)(nv > 0 ? nv : 1));
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i)
    if (visible[i]) {
      uint32_t bits;
      memcpy(&bits, &depth[i], 4);
      order[k].key = bits;
      order[k].val = (uint32_t)i;
      ++k;
    }
  qsort(order, (size_t)nv, sizeof(pair_t), cmp_pair);
  uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(nv > 0 ? nv : 1));
  for (int py = 0; py < height; ++py)
    for (int px = 0; px < width; ++px) {
      int tx = px / TILE, ty = py / TILE;
      int64_t c = 0;
      for (int64_t j = 0; j < nv; ++j) {
        uint32_t g = order[j].val;
        if (tx >= rect[g * 4 + 0] && tx < rect[g * 4 + 2] && ty >= rect[g * 4 + 1] && ty < rect[g * 4 + 3])
          ids[c++] = g;
      }
      double C[3], T;
      int64_t lst;
      uint8_t f;
      walk_pixel(px, py, ids, c, mu_p, conic, opac, rgb, tol, C, &T, &lst, &f, NULL, NULL, 0);
      int64_t pix = (int64_t)py * width + px;
      for (int ch = 0; ch < 3; ++ch) image[(int64_t)ch * width * height + pix] = C[ch] + T * bg[ch];
    }
  free(ids);
  free(order);
}

/* ------------------------------------------------------------------------ */
/* Blend backward: exact derivatives of walk_pixel, per pixel last to first. */
/* Outputs per Gaussian (accumulated, caller zeroes): g_mu_p [n][2],          */
/* g_conic [n][3] (d/dA, d/dB, d/dC), g_opac [n], g_rgb [n][3].  If g_abs     */
/* is not NULL it receives [n][18]: per Gaussian and component in the order   */
/* (mu_x, mu_y, A, B, C, o, r, g, b), first the sum over pixels of the         */
/* magnitudes of each term's operands (|rgb| + |B| in place of rgb - B), the   */
/* scale of the rounding error of any floating-point evaluation; then the sum  */
/* of |d term / d delta_x| + |d term / d delta_y|, the sensitivity of each     */
/* term to the rounding of the pixel offset delta = mu_p - pixel.              */
/* ------------------------------------------------------------------------ */
void orc_blend_backward(int32_t width, int32_t height, const uint32_t* ranges, const uint32_t* vals,
                        const double* mu_p, const double* conic, const double* opac, const double* rgb,
                        const float bg[3], const float* dL_dimg, double* g_mu_p, double* g_conic, double* g_opac,
                        double* g_rgb, double* g_abs) {
  const int gx = (width + TILE - 1) / TILE, gy = (height + TILE - 1) / TILE;
  orc_tol tol = {0, 0, 0, 0};
#pragma omp parallel
  {
    int64_t cap = 1 << 16;
    contrib* rec = (contrib*)malloc(sizeof(contrib) * (size_t)cap);
#pragma omp for schedule(dynamic, 1)
    for (int t = 0; t < gx * gy; ++t) {
      int tx = t % gx, ty = t / gx;
      uint32_t s = ranges[t * 2], e = ranges[t * 2 + 1];
      if ((int64_t)(e - s) > cap) {
        cap = (int64_t)(e - s);
        rec = (contrib*)realloc(rec, sizeof(contrib) * (size_t)cap);
      }
      for (int j = 0; j < TILE; ++j)
        for (int i = 0; i < TILE; ++i) {
          int px = tx * TILE + i, py = ty * TILE + j;
          if (px >= width || py >= height) continue;
          int64_t pix = (int64_t)py * width + px;
          double C[3], T;
          int64_t lst;
          uint8_t f;
          int nb = walk_pixel(px, py, vals + s, (int64_t)e - s, mu_p, conic, opac, rgb, &tol, C, &T, &lst, &f,
                              NULL, rec, cap);
          double G[3];
          for (int c = 0; c < 3; ++c) G[c] = dL_dimg[(int64_t)c * width * height + pix];
          double Bk[3] = {bg[0], bg[1], bg[2]}; /* colour seen behind the current Gaussian */
          for (int k = nb - 1; k >= 0; --k) {
            const contrib* r = &rec[k];
            uint32_t g = r->id;
            double a = r->alpha, Ti = r->T;
            double dLda = 0, dLda_abs = 0;
            for (int c = 0; c < 3; ++c) {
              double col = rgb[g * 3 + c];
#pragma omp atomic
              g_rgb[g * 3 + c] += a * Ti * G[c];
              if (g_abs) {
#pragma omp atomic
                g_abs[g * 18 + 6 + c] += fabs(a * Ti * G[c]);
              }
              dLda += Ti * (col - Bk[c]) * G[c];
              dLda_abs += Ti * (fabs(col) + fabs(Bk[c])) * fabs(G[c]);
              Bk[c] = a * col + (1.0 - a) * Bk[c];
            }
            if (r->clampd) continue; /* alpha = 0.99 does not depend on o or q */
            double dLdq = dLda * a;
            double dLdo = dLda * r->eq;
            double A = conic[g * 3 + 0], B = conic[g * 3 + 1], Cc = conic[g * 3 + 2];
            double dx = r->dx, dy = r->dy;
#pragma omp atomic
            g_opac[g] += dLdo;
#pragma omp atomic
            g_mu_p[g * 2 + 0] += dLdq * -(A * dx + B * dy);
#pragma omp atomic
            g_mu_p[g * 2 + 1] += dLdq * -(B * dx + Cc * dy);
#pragma omp atomic
            g_conic[g * 3 + 0] += dLdq * -0.5 * dx * dx;
#pragma omp atomic
            g_conic[g * 3 + 1] += dLdq * -dx * dy;
#pragma omp atomic
            g_conic[g * 3 + 2] += dLdq * -0.5 * dy * dy;
            if (g_abs) {
              /* magnitudes of the operands, not of the result: dL/dalpha
               * carries the difference rgb - B */
              const double q_abs = dLda_abs * a, o_abs = dLda_abs * r->eq;
              const double t[6] = {q_abs * (fabs(A * dx) + fabs(B * dy)), q_abs * (fabs(B * dx) + fabs(Cc * dy)),
                                   q_abs * 0.5 * dx * dx, q_abs * fabs(dx * dy), q_abs * 0.5 * dy * dy, o_abs};
              const double p[5] = {q_abs * (fabs(A) + fabs(B)), q_abs * (fabs(B) + fabs(Cc)), q_abs * fabs(dx),
                                   q_abs * (fabs(dx) + fabs(dy)), q_abs * fabs(dy)};
              for (int e = 0; e < 6; ++e) {
#pragma omp atomic
                g_abs[g * 18 + e] += t[e];
              }
              for (int e = 0; e < 5; ++e) {
#pragma omp atomic
                g_abs[g * 18 + 9 + e] += p[e];
              }
            }
          }
        }
    }
    free(rec);
  }
}

/* ------------------------------------------------------------------------ */
/* Preprocess backward (Sec. 4.2, 4.3).                                        */
/*   dL/dSigma'  = -Q G Q           (Q = conic matrix, G its gradient)         */
/*   dL/dT       = 2 dL/dSigma_p T Sigma,  dL/dSigma = T^T dL/dSigma_p T       */
/*   dL/dJ       = dL/dT W^T                                                   */
/*   dL/dmu_c    = J_phi^T dL/dmu_p + sum_ij dL/dJ_ij dJ_ij/dmu_c              */
/*   dL/dmu      = W^T dL/dmu_c + (d rgb / d mu)^T dL/drgb                     */
/* Outputs (written, same SoA layout as the parameters): g_means [3][n],       */
/* g_scales [3][n], g_quats [4][n], g_opac [n], g_sh [S][n].                   */
/* ------------------------------------------------------------------------ */
void orc_preprocess_backward(int64_t n, const double* means, const double* scales, const double* quats,
                             const double* opac, const double* sh, int sh_degree, const double* Rw, const double* tw,
                             const orc_camera* cam, const uint8_t* visible, const double* g_mu_p,
                             const double* g_conic, const double* g_opac2d, const double* g_rgb, double* g_means,
                             double* g_scales, double* g_quats, double* g_opac, double* g_sh) {
  const int S = 3 * (sh_degree + 1) * (sh_degree + 1);
  double campos[3];
  for (int a = 0; a < 3; ++a) campos[a] = -(Rw[0 * 3 + a] * tw[0] + Rw[1 * 3 + a] * tw[1] + Rw[2 * 3 + a] * tw[2]);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) { g_means[a * n + i] = 0; g_scales[a * n + i] = 0; }
    for (int a = 0; a < 4; ++a) g_quats[a * n + i] = 0;
    g_opac[i] = 0;
    for (int k = 0; k < S; ++k) g_sh[(int64_t)k * n + i] = 0;
    if (!visible[i]) continue;
    geom g;
    dual Sig[9];
    if (!geometry(i, n, means, scales, quats, opac, Rw, tw, cam, &g, Sig)) continue;
    /* conic gradient as a symmetric matrix: dL = sum_ij G_ij dQ_ij */
    double Q[4] = {g.conic[0], g.conic[1], g.conic[1], g.conic[2]};
    double Gm[4] = {g_conic[i * 3 + 0], 0.5 * g_conic[i * 3 + 1], 0.5 * g_conic[i * 3 + 1], g_conic[i * 3 + 2]};
    double QG[4], H[4];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) QG[r * 2 + c] = Q[r * 2 + 0] * Gm[0 * 2 + c] + Q[r * 2 + 1] * Gm[1 * 2 + c];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) H[r * 2 + c] = -(QG[r * 2 + 0] * Q[0 * 2 + c] + QG[r * 2 + 1] * Q[1 * 2 + c]);
    /* dL/dT = 2 H T Sigma ; dL/dSigma = T^T H T */
    double HT[6], dT[6], dSig[9];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) HT[r * 3 + c] = H[r * 2 + 0] * g.T[0 * 3 + c] + H[r * 2 + 1] * g.T[1 * 3 + c];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += HT[r * 3 + k] * g.Sig[k * 3 + c];
        dT[r * 3 + c] = 2.0 * acc;
      }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) dSig[r * 3 + c] = g.T[0 * 3 + r] * HT[0 * 3 + c] + g.T[1 * 3 + r] * HT[1 * 3 + c];
    /* dL/dJ = dL/dT W^T */
    double dJm[6];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += dT[r * 3 + k] * Rw[c * 3 + k];
        dJm[r * 3 + c] = acc;
      }
    /* dL/dmu_c: mean projection + Jacobian's dependence on mu_c */
    double dJ[18];
    orc_jacobian_grad_model(cam->model, g.pc, cam->fx, cam->fy, dJ);
    double gmc[3];
    for (int c = 0; c < 3; ++c) {
      double acc = g.J[0 * 3 + c] * g_mu_p[i * 2 + 0] + g.J[1 * 3 + c] * g_mu_p[i * 2 + 1];
      for (int e = 0; e < 6; ++e) acc += dJm[e] * dJ[c * 6 + e];
      gmc[c] = acc;
    }
    double gm[3];
    for (int c = 0; c < 3; ++c)
      gm[c] = Rw[0 * 3 + c] * gmc[0] + Rw[1 * 3 + c] * gmc[1] + Rw[2 * 3 + c] * gmc[2];
    /* colour: SH coefficients and the view direction */
    dual col[3];
    double Yv[16];
    double mu[3] = {means[i], means[n + i], means[2 * n + i]};
    sh_color(sh_degree, mu, campos, sh, n, i, col, Yv);
    int nb = (sh_degree + 1) * (sh_degree + 1);
    for (int c = 0; c < 3; ++c) {
      if (col[c].v < 0) continue; /* clamped channel */
      double gc = g_rgb[i * 3 + c];
      for (int k = 0; k < nb; ++k) g_sh[(int64_t)(k * 3 + c) * n + i] = Yv[k] * gc;
      for (int a = 0; a < 3; ++a) gm[a] += col[c].d[a] * gc;
    }
    for (int a = 0; a < 3; ++a) g_means[a * n + i] = gm[a];
    /* scale and rotation through Sigma(s, q) */
    for (int k = 0; k < 7; ++k) {
      double acc = 0;
      for (int e = 0; e < 9; ++e) acc += dSig[e] * Sig[e].d[k];
      if (k < 3) g_scales[k * n + i] = acc;
      else g_quats[(k - 3) * n + i] = acc;
    }
    g_opac[i] = g_opac2d[i];
  }
}

/* Threads of the OpenMP loops above (timing only; results do not depend on it). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
