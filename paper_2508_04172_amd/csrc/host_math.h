// Host FP64 pieces of the start-up stage that need neither a device nor a
// handle: the analytic PSD, detector geometry, spin -2 harmonics, the spline
// table, Halton points, the polynomial tail's monomials, the symmetric 4x4
// eigen-decomposition of the metric, the templates' reference frequency and
// the time bands of the antenna patterns.  Built into the library, and
// host-only into the shim through which the CPU tests compare them with the
// oracle.
#pragma once

#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

#include "rbfl_internal.h"
#include "rbfl_math.h"

namespace rbfl {

// aLIGO-like analytic PSD, x = f / 215 Hz (scaled by `scale`).
double psd_analytic(double f, double scale);

// Detector tensor D = (u u^T - v v^T) / 2 and position r [light-seconds] from
// (latitude, longitude, x-arm azimuth from north toward east, opening angle,
// distance from the geocentre).
void detector_geometry(const double g[5], double D[9], double r[3]);

// -2Y_{l m} as a short sum of powers of cos(iota/2), sin(iota/2) times
// e^{i m phi}, and its value.
YlmTerms ylm_terms(int l, int m);
void ylm_value(const YlmTerms &t, double iota, double phi, double *re, double *im);

// Weights of the not-a-knot spline through 10 unit-spaced samples at
// fraction f of the central interval: w_s(f) = sum_p tab[s][p] f^p.
void spline_table(double tab[kSplineTaps][4]);

// Radical inverse of i in `base` (exact integer ratio rounded once), and the
// i-th Halton point in [-1, 1]^4 (bases 2, 3, 5, 7).
double radical_inverse(uint64_t i, uint64_t base);
void halton_point(uint64_t i, double x[4]);

// Monomials of degree <= `degree` in 4 variables, graded lexicographic: the
// variable indices of each (-1 = unused); returns their number.
int monomials(int degree, int idx[kMaxPoly][3]);

// Cyclic Jacobi eigen-decomposition of a symmetric 4x4 matrix (row-major):
// eigenvalues lam (unsorted) and eigenvectors as the columns of V.
void jacobi_eigen(const double a_in[16], double lam[4], double V[16]);

// Mean frequency of the centre's (2,2) band under f^(-7/3) / S_0.
double reference_frequency(double f_low, double seg_len, int64_t n_s, const double *psd0, const double center[4]);

// Time bands of the antenna patterns: edges [n_bands + 1] bin indices and
// the band time of every (band, mode) relative to t_c.
void time_bands(const double centre[4], double f_ref, double f_low, double seg_len, int64_t n_s, int n_modes,
                const int modes[][2], int n_bands, const double *psd0, std::vector<int64_t> &edges,
                double times[RBFL_MAX_BANDS][RBFL_MAX_MODES]);

// ---- metric: generic-real versions of the phase and the inverse map, so the
// derivatives can be taken by the complex step.
template <class R>
R phase22_generic(R f, R m1, R m2, R c1, R c2) {
  using std::log;
  using std::pow;
  const double pi = kPi;
  const R mt = m1 + m2;
  const R eta = m1 * m2 / (mt * mt);
  const R dl = (m1 - m2) / mt;
  const R cs = 0.5 * (c1 + c2), ca = 0.5 * (c1 - c2);
  const R v = pow(pi * mt * kMsunS * f, 1.0 / 3.0);
  const R lv = log(v);
  const R e2 = eta * eta, e3 = e2 * eta;
  const R p2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
  const R p3 = -16.0 * pi + 113.0 / 3.0 * dl * ca + (113.0 / 3.0 - 76.0 / 3.0 * eta) * cs;
  const R p4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * e2 +
               (-405.0 / 8.0 + 200.0 * eta) * ca * ca - 405.0 / 4.0 * dl * ca * cs +
               (-405.0 / 8.0 + 2.5 * eta) * cs * cs;
  const R p5 = pi * (38645.0 / 756.0 - 65.0 / 9.0 * eta) + dl * ca * (-732985.0 / 2268.0 - 140.0 / 9.0 * eta) +
               cs * (-732985.0 / 2268.0 + 24260.0 / 81.0 * eta + 340.0 / 9.0 * e2);
  const R p6 = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * pi * pi - 6848.0 / 21.0 * kEulerGamma +
               eta * (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * pi * pi) + 76055.0 / 1728.0 * e2 -
               127825.0 / 1296.0 * e3 + pi * (2270.0 / 3.0 * dl * ca + (2270.0 / 3.0 - 520.0 * eta) * cs) +
               (75515.0 / 144.0 - 8225.0 / 18.0 * eta) * dl * ca * cs +
               (75515.0 / 288.0 - 263245.0 / 252.0 * eta - 480.0 * e2) * ca * ca +
               (75515.0 / 288.0 - 232415.0 / 504.0 * eta + 1255.0 / 9.0 * e2) * cs * cs;
  const double p6l = -6848.0 / 21.0;
  const R p7 = pi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * e2) +
               dl * ca * (-25150083775.0 / 3048192.0 + 26804935.0 / 6048.0 * eta - 1985.0 / 48.0 * e2) +
               cs * (-25150083775.0 / 3048192.0 + 10566655595.0 / 762048.0 * eta - 1042165.0 / 3024.0 * e2 +
                     5345.0 / 36.0 * e3);
  const R v2 = v * v;
  R s = p7;
  s = s * v + (p6 + p6l * (std::log(4.0) + lv));
  s = s * v + p5 * (1.0 + 3.0 * lv);
  s = s * v + p4;
  s = s * v + p3;
  s = s * v + p2;
  s = s * v2 + 1.0;
  return -0.25 * pi + 3.0 / (128.0 * eta * v2 * v2 * v) * s;
}

template <class R>
void theta_to_phys_generic(const R th[4], double f0, R p[4]) {
  using std::pow;
  using std::sqrt;
  const R u = 5.0 * th[1] / (32.0 * kPi * th[0]);
  const R eta = kPi / (4.0 * th[1]) * pow(u, -2.0 / 3.0);
  const R mt = u / (kPi * f0) / kMsunS;
  const R dl = sqrt(1.0 - 4.0 * eta);
  const R chi_r = 48.0 * kPi * th[2] / (113.0 * th[1]);
  const R chi_eff = 48.0 * kPi * th[3] / (113.0 * th[1]);
  const R cs = 113.0 * (chi_eff - chi_r) / (76.0 * eta);
  const R ca = (chi_eff - cs) / dl;
  p[0] = 0.5 * mt * (1.0 + dl);
  p[1] = 0.5 * mt * (1.0 - dl);
  p[2] = cs + ca;
  p[3] = cs - ca;
}

// Neumaier-compensated sum.
struct Sum {
  double s = 0.0, c = 0.0;
  void add(double v) {
    const double t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};


}  // namespace rbfl
