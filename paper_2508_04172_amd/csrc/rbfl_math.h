// Host/device math of the meshfree likelihood: waveform family, chirp-time
// coordinates, spin-weighted harmonics, detector response.  Used by the
// start-up orchestration on the host and by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace rbfl {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMsunS = 4.925490947641267e-06;                   // G Msun / c^3 [s]
constexpr double kMpcS = 3.0856775814913673e22 / 299792458.0;      // Mpc / c [s]
constexpr double kEulerGamma = 0.5772156649015329;

// Phase and amplitude constants of one (m1, m2, chi1, chi2) point of the
// synthetic family.  The (2,2) SPA phase at template t_c = phi_c = 0 is
//   Psi(f) = -pi/4 + 3/(128 eta v^5) [1 + p2 v^2 + p3 v^3 + p4 v^4
//            + p5 (1 + 3 ln v) v^5 + (p6 + p6l ln(4v)) v^6 + p7 v^7],
// v = (pi M f)^(1/3): 3.5PN non-spinning terms plus aligned-spin
// spin-orbit and spin-spin terms.
struct Binary {
  double m_s;       // total mass [s]
  double eta, delta;
  double pre;       // 3 / (128 eta)
  double p2, p3, p4, p5, p6, p6l, p7;
  double amp;       // sqrt(5/24) pi^(-2/3) Mc^(5/6) in seconds (divide by the distance in seconds)
  double f_isco;    // orbital ISCO frequency 1 / (2 pi 6^(3/2) M)
  // time and phase reference: with f_ref > 0 the template phase is
  // Psi(f) - Psi(f_ref) - Psi'(f_ref) (f - f_ref), so t_c and phi_c are the
  // time and phase at which the (2,2) mode passes f_ref; f_ref = 0 keeps the
  // formal coalescence as the reference
  double f_ref, psi_ref, dpsi_ref;
};

__host__ __device__ inline double phase22_pn(double f, const Binary &b);
__host__ __device__ inline double dphase22_pn(double f, const Binary &b);

__host__ __device__ inline Binary make_binary(double m1, double m2, double c1, double c2, double f_ref) {
  Binary b;
  const double mt = m1 + m2;
  b.m_s = mt * kMsunS;
  const double eta = m1 * m2 / (mt * mt);
  const double dl = (m1 - m2) / mt;
  const double cs = 0.5 * (c1 + c2);
  const double ca = 0.5 * (c1 - c2);
  b.eta = eta;
  b.delta = dl;
  b.pre = 3.0 / (128.0 * eta);
  const double e2 = eta * eta, e3 = e2 * eta;
  b.p2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
  b.p3 = -16.0 * kPi + 113.0 / 3.0 * dl * ca + (113.0 / 3.0 - 76.0 / 3.0 * eta) * cs;
  b.p4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * e2 +
         (-405.0 / 8.0 + 200.0 * eta) * ca * ca - 405.0 / 4.0 * dl * ca * cs +
         (-405.0 / 8.0 + 2.5 * eta) * cs * cs;
  b.p5 = kPi * (38645.0 / 756.0 - 65.0 / 9.0 * eta) +
         dl * ca * (-732985.0 / 2268.0 - 140.0 / 9.0 * eta) +
         cs * (-732985.0 / 2268.0 + 24260.0 / 81.0 * eta + 340.0 / 9.0 * e2);
  b.p6 = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * kPi * kPi - 6848.0 / 21.0 * kEulerGamma +
         eta * (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * kPi * kPi) + 76055.0 / 1728.0 * e2 -
         127825.0 / 1296.0 * e3 +
         kPi * (2270.0 / 3.0 * dl * ca + (2270.0 / 3.0 - 520.0 * eta) * cs) +
         (75515.0 / 144.0 - 8225.0 / 18.0 * eta) * dl * ca * cs +
         (75515.0 / 288.0 - 263245.0 / 252.0 * eta - 480.0 * e2) * ca * ca +
         (75515.0 / 288.0 - 232415.0 / 504.0 * eta + 1255.0 / 9.0 * e2) * cs * cs;
  b.p6l = -6848.0 / 21.0;
  b.p7 = kPi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * e2) +
         dl * ca * (-25150083775.0 / 3048192.0 + 26804935.0 / 6048.0 * eta - 1985.0 / 48.0 * e2) +
         cs * (-25150083775.0 / 3048192.0 + 10566655595.0 / 762048.0 * eta -
               1042165.0 / 3024.0 * e2 + 5345.0 / 36.0 * e3);
  const double mc = pow(m1 * m2, 0.6) / pow(mt, 0.2) * kMsunS;
  b.amp = sqrt(5.0 / 24.0) * pow(kPi, -2.0 / 3.0) * pow(mc, 5.0 / 6.0);
  b.f_isco = 1.0 / (2.0 * kPi * pow(6.0, 1.5) * b.m_s);
  b.f_ref = f_ref > 0.0 ? f_ref : 0.0;
  b.psi_ref = f_ref > 0.0 ? phase22_pn(f_ref, b) : 0.0;
  b.dpsi_ref = f_ref > 0.0 ? dphase22_pn(f_ref, b) : 0.0;
  return b;
}

// The PN phase series at the formal coalescence reference.
__host__ __device__ inline double phase22_pn(double f, const Binary &b) {
  const double v = cbrt(kPi * b.m_s * f);
  const double lv = log(v);
  const double v2 = v * v;
  const double v5 = v2 * v2 * v;
  double s = b.p7;
  s = s * v + (b.p6 + b.p6l * (1.3862943611198906 + lv));   // ln 4 = 1.386...
  s = s * v + b.p5 * (1.0 + 3.0 * lv);
  s = s * v + b.p4;
  s = s * v + b.p3;
  s = s * v + b.p2;
  s = s * v2 + 1.0;
  return -0.25 * kPi + b.pre / v5 * s;
}

// dPsi/df of the PN series: with v = (pi M f)^(1/3), dv/df = v / (3 f) and
// Psi = -pi/4 + pre v^-5 S(v), dPsi/df = pre v^-5 (v S'(v) - 5 S(v)) / (3 f).
__host__ __device__ inline double dphase22_pn(double f, const Binary &b) {
  const double v = cbrt(kPi * b.m_s * f);
  const double lv = log(v);
  const double v2 = v * v;
  const double v5 = v2 * v2 * v;
  const double l6 = b.p6 + b.p6l * (1.3862943611198906 + lv);
  double s = b.p7;                       // S(v)
  s = s * v + l6;
  s = s * v + b.p5 * (1.0 + 3.0 * lv);
  s = s * v + b.p4;
  s = s * v + b.p3;
  s = s * v + b.p2;
  s = s * v2 + 1.0;
  double ds = 7.0 * b.p7;                // v S'(v) / v^2
  ds = ds * v + (6.0 * l6 + b.p6l);
  ds = ds * v + b.p5 * (8.0 + 15.0 * lv);
  ds = ds * v + 4.0 * b.p4;
  ds = ds * v + 3.0 * b.p3;
  ds = ds * v + 2.0 * b.p2;
  ds *= v2;
  return b.pre / v5 * (ds - 5.0 * s) / (3.0 * f);
}

// Template phase with the binary's time and phase reference applied.
__host__ __device__ inline double phase22(double f, const Binary &b) {
  return phase22_pn(f, b) - b.psi_ref - b.dpsi_ref * (f - b.f_ref);
}

// Relative amplitudes A22 = 1, A21 = 0.1 delta, A33 = 0.3 delta,
// A32 = 0.05 (1 - 3 eta), A44 = 0.1 (1 - 3 eta).
__host__ __device__ inline double mode_amp(int l, int m, double eta, double delta) {
  if (l == 2 && m == 2) return 1.0;
  if (l == 2 && m == 1) return 0.1 * delta;
  if (l == 3 && m == 3) return 0.3 * delta;
  if (l == 3 && m == 2) return 0.05 * (1.0 - 3.0 * eta);
  if (l == 4 && m == 4) return 0.1 * (1.0 - 3.0 * eta);
  return 0.0;
}

// Chirp-time coordinates (theta0, theta3, theta3s, theta3s_bar) at f0.
__host__ __device__ inline void phys_to_theta(const double p[4], double f0, double th[4]) {
  const double m1 = p[0], m2 = p[1], c1 = p[2], c2 = p[3];
  const double mt = m1 + m2;
  const double eta = m1 * m2 / (mt * mt);
  const double dl = (m1 - m2) / mt;
  const double cs = 0.5 * (c1 + c2), ca = 0.5 * (c1 - c2);
  const double chi_r = cs + dl * ca - 76.0 * eta * cs / 113.0;
  const double chi_eff = (m1 * c1 + m2 * c2) / mt;
  const double u = kPi * mt * kMsunS * f0;
  const double u23 = pow(u, -2.0 / 3.0);
  th[0] = 5.0 / (128.0 * eta) * pow(u, -5.0 / 3.0);
  th[1] = kPi / (4.0 * eta) * u23;
  th[2] = 113.0 * chi_r / (192.0 * eta) * u23;
  th[3] = 113.0 * chi_eff / (192.0 * eta) * u23;
}

// Inverse map.  Returns false where the point is not a physical binary
// (eta > 1/4, |chi| > chi_max, non-finite); p receives m1, m2, chi1, chi2.
__host__ __device__ inline bool theta_to_phys(const double th[4], double f0, double chi_max, double p[4]) {
  const double u = 5.0 * th[1] / (32.0 * kPi * th[0]);       // pi M f0
  if (!(u > 0.0)) return false;
  const double eta = kPi / (4.0 * th[1]) * pow(u, -2.0 / 3.0);
  if (!(eta > 0.0 && eta <= 0.25)) return false;
  const double mt = u / (kPi * f0) / kMsunS;
  const double dl = sqrt(1.0 - 4.0 * eta);
  const double chi_r = 48.0 * kPi * th[2] / (113.0 * th[1]);
  const double chi_eff = 48.0 * kPi * th[3] / (113.0 * th[1]);
  const double cs = 113.0 * (chi_eff - chi_r) / (76.0 * eta);
  const double ca = (chi_eff - cs) / dl;
  p[0] = 0.5 * mt * (1.0 + dl);
  p[1] = 0.5 * mt * (1.0 - dl);
  p[2] = cs + ca;
  p[3] = cs - ca;
  return isfinite(p[2]) && isfinite(p[3]) && fabs(p[2]) <= chi_max && fabs(p[3]) <= chi_max;
}

// Response of one detector to a source at (alpha, dec) with polarisation psi:
// F+ = D:e+, Fx = D:ex with wave axes X = -cos(psi) e_alpha + sin(psi) e_dec,
// Y = sin(psi) e_alpha + cos(psi) e_dec; delay = -r . s_hat.
__host__ __device__ inline void detector_response(const double D[9], const double r[3], double alpha,
                                                  double dec, double psi, double *fp, double *fc,
                                                  double *delay) {
  double sa, ca, sd, cd, sp, cp;
  sincos(alpha, &sa, &ca);
  sincos(dec, &sd, &cd);
  sincos(psi, &sp, &cp);
  const double ea[3] = {-sa, ca, 0.0};
  const double ed[3] = {-sd * ca, -sd * sa, cd};
  double X[3], Y[3];
  for (int i = 0; i < 3; ++i) {
    X[i] = -cp * ea[i] + sp * ed[i];
    Y[i] = sp * ea[i] + cp * ed[i];
  }
  double p = 0.0, c = 0.0;
  for (int i = 0; i < 3; ++i) {
    double dx = 0.0, dy = 0.0;
    for (int j = 0; j < 3; ++j) {
      dx += D[3 * i + j] * X[j];
      dy += D[3 * i + j] * Y[j];
    }
    p += X[i] * dx - Y[i] * dy;
    c += X[i] * dy + Y[i] * dx;
  }
  *fp = p;
  *fc = c;
  *delay = -(r[0] * cd * ca + r[1] * cd * sa + r[2] * sd);
}

// One spin -2 harmonic as a short sum: -2Y_lm(iota, phi) = norm *
// sum_k coef_k cos(iota/2)^cpow_k sin(iota/2)^spow_k * e^{i m phi}.
struct YlmTerms {
  int m;
  int n;
  double coef[9];
  int cpow[9];
  int spow[9];
};

__host__ __device__ inline void eval_ylm(const YlmTerms &t, double ch, double sh, double phi,
                                         double *re, double *im) {
  double s = 0.0;
  for (int k = 0; k < t.n; ++k) {
    double a = t.coef[k];
    for (int e = 0; e < t.cpow[k]; ++e) a *= ch;
    for (int e = 0; e < t.spow[k]; ++e) a *= sh;
    s += a;
  }
  double sm, cm;
  sincos((double)t.m * phi, &sm, &cm);
  *re = s * cm;
  *im = s * sm;
}

}  // namespace rbfl
