// Host FP64 start-up pieces declared in host_math.h.
#include "host_math.h"

#include <algorithm>

namespace rbfl {

// aLIGO-like analytic PSD, x = f / 215 Hz.
double psd_analytic(double f, double scale) {
  const double x = f / 215.0;
  return scale * 1e-49 *
         (pow(x, -4.14) - 5.0 / (x * x) + 111.0 * (1.0 - x * x + 0.5 * x * x * x * x) / (1.0 + 0.5 * x * x));
}

// Detector tensor and position from (lat, lon, x-arm azimuth, opening, radius).
void detector_geometry(const double g[5], double D[9], double r[3]) {
  const double lat = g[0], lon = g[1], az = g[2], op = g[3], rad = g[4];
  const double east[3] = {-sin(lon), cos(lon), 0.0};
  const double north[3] = {-sin(lat) * cos(lon), -sin(lat) * sin(lon), cos(lat)};
  const double up[3] = {cos(lat) * cos(lon), cos(lat) * sin(lon), sin(lat)};
  double u[3], v[3];
  for (int i = 0; i < 3; ++i) {
    u[i] = cos(az) * north[i] + sin(az) * east[i];
    v[i] = cos(az + op) * north[i] + sin(az + op) * east[i];
    r[i] = rad * up[i];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) D[3 * i + j] = 0.5 * (u[i] * u[j] - v[i] * v[j]);
}

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// -2Y_{l m}(iota, phi) = sqrt((2l+1)/4pi) d^l_{m,2}(iota) e^{i m phi}, with the
// Wigner small-d element written as its finite sum over k.
YlmTerms ylm_terms(int l, int m) {
  YlmTerms t{};
  t.m = m;
  t.n = 0;
  const int m1 = m, m2 = 2;
  const double norm = sqrt((2.0 * l + 1.0) / (4.0 * kPi));
  const double pre = sqrt(factorial(l + m1) * factorial(l - m1) * factorial(l + m2) * factorial(l - m2));
  for (int k = 0; k <= 2 * l; ++k) {
    const int a1 = l + m2 - k, a2 = k, a3 = m1 - m2 + k, a4 = l - m1 - k;
    if (a1 < 0 || a2 < 0 || a3 < 0 || a4 < 0) continue;
    const double sign = ((k + m1 - m2) & 1) ? -1.0 : 1.0;
    t.coef[t.n] = norm * sign * pre / (factorial(a1) * factorial(a2) * factorial(a3) * factorial(a4));
    t.cpow[t.n] = 2 * l + m2 - m1 - 2 * k;
    t.spow[t.n] = m1 - m2 + 2 * k;
    ++t.n;
  }
  return t;
}

void ylm_value(const YlmTerms &t, double iota, double phi, double *re, double *im) {
  eval_ylm(t, cos(0.5 * iota), sin(0.5 * iota), phi, re, im);
}

// Not-a-knot cubic spline through 10 unit-spaced samples, evaluated in the
// central interval [4, 5]: its value is linear in the samples, sum_s w_s(f) y_s,
// with each w_s a cubic in f.  Second derivatives m_i solve
// m_{i-1} + 4 m_i + m_{i+1} = 6 (y_{i+1} - 2 y_i + y_{i-1}) (i = 1..8) with the
// not-a-knot conditions m_0 - 2 m_1 + m_2 = 0 and m_7 - 2 m_8 + m_9 = 0; on
// [4, 5], S(f) = y4 + (y5 - y4 - m4/3 - m5/6) f + m4/2 f^2 + (m5 - m4)/6 f^3.
void spline_table(double tab[kSplineTaps][4]) {
  constexpr int n = kSplineTaps;
  for (int s = 0; s < n; ++s) {
    double A[n][n + 1] = {};
    double y[n] = {};
    y[s] = 1.0;
    A[0][0] = 1.0;
    A[0][1] = -2.0;
    A[0][2] = 1.0;
    A[n - 1][n - 3] = 1.0;
    A[n - 1][n - 2] = -2.0;
    A[n - 1][n - 1] = 1.0;
    for (int i = 1; i < n - 1; ++i) {
      A[i][i - 1] = 1.0;
      A[i][i] = 4.0;
      A[i][i + 1] = 1.0;
      A[i][n] = 6.0 * (y[i + 1] - 2.0 * y[i] + y[i - 1]);
    }
    // Gaussian elimination with partial pivoting
    for (int c = 0; c < n; ++c) {
      int piv = c;
      for (int r = c + 1; r < n; ++r)
        if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
      if (piv != c)
        for (int k = 0; k <= n; ++k) std::swap(A[c][k], A[piv][k]);
      for (int r = c + 1; r < n; ++r) {
        const double f = A[r][c] / A[c][c];
        for (int k = c; k <= n; ++k) A[r][k] -= f * A[c][k];
      }
    }
    double m[n];
    for (int r = n - 1; r >= 0; --r) {
      double v = A[r][n];
      for (int k = r + 1; k < n; ++k) v -= A[r][k] * m[k];
      m[r] = v / A[r][r];
    }
    tab[s][0] = y[4];
    tab[s][1] = y[5] - y[4] - m[4] / 3.0 - m[5] / 6.0;
    tab[s][2] = 0.5 * m[4];
    tab[s][3] = (m[5] - m[4]) / 6.0;
  }
}

// Van der Corput radical inverse as an exact integer ratio, rounded once.
double radical_inverse(uint64_t i, uint64_t base) {
  uint64_t num = 0, den = 1;
  while (i > 0) {
    num = num * base + i % base;
    den *= base;
    i /= base;
  }
  return (double)num / (double)den;
}

void halton_point(uint64_t i, double x[4]) {
  const uint64_t bases[4] = {2, 3, 5, 7};
  for (int d = 0; d < 4; ++d) x[d] = 2.0 * radical_inverse(i, bases[d]) - 1.0;
}

int monomials(int degree, int idx[kMaxPoly][3]) {
  int n = 0;
  for (int d = 0; d <= degree; ++d) {
    if (d == 0) {
      idx[n][0] = idx[n][1] = idx[n][2] = -1;
      ++n;
    } else if (d == 1) {
      for (int i = 0; i < 4; ++i, ++n) {
        idx[n][0] = i;
        idx[n][1] = idx[n][2] = -1;
      }
    } else if (d == 2) {
      for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j, ++n) {
          idx[n][0] = i;
          idx[n][1] = j;
          idx[n][2] = -1;
        }
    } else {
      for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j)
          for (int k = j; k < 4; ++k, ++n) {
            idx[n][0] = i;
            idx[n][1] = j;
            idx[n][2] = k;
          }
    }
  }
  return n;
}

// Cyclic Jacobi eigen-decomposition of a symmetric 4x4 matrix.
void jacobi_eigen(const double a_in[16], double lam[4], double V[16]) {
  double a[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      a[i][j] = a_in[4 * i + j];
      V[4 * i + j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) (i == j ? diag : off) += a[i][j] * a[i][j];
    if (off <= 1e-34 * diag) break;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        if (a[p][q] == 0.0) continue;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < 4; ++k) {
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = cs * akp - sn * akq;
          a[k][q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < 4; ++k) {
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = cs * apk - sn * aqk;
          a[q][k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < 4; ++k) {
          const double vkp = V[4 * k + p], vkq = V[4 * k + q];
          V[4 * k + p] = cs * vkp - sn * vkq;
          V[4 * k + q] = sn * vkp + cs * vkq;
        }
      }
  }
  for (int i = 0; i < 4; ++i) lam[i] = a[i][i];
}

// Reference frequency of the template time and phase: the mean frequency of
// the centre's (2,2) band under the metric's weights |h22|^2 / S_0, i.e.
// f^(-7/3) / S_0.  There the time and constant-phase shifts that the match
// maximises over are uncorrelated, so with the template phase referenced
// there the overlap series of neighbouring templates stay aligned in time
// and phase across the ellipsoid.
double reference_frequency(double f_low, double seg_len, int64_t n_s, const double *psd0, const double center[4]) {
  const Binary b = make_binary(center[0], center[1], center[2], center[3], 0.0);
  const int64_t j0 = std::max<int64_t>(1, (int64_t)ceil(f_low * seg_len - 1e-9));
  int64_t j1 = (int64_t)ceil(2.0 * b.f_isco * seg_len);
  j1 = std::min<int64_t>(std::max<int64_t>(j1, j0), n_s / 2);
  if (j1 <= j0) throw Error(RBFL_E_INVALID_ARG, "the (2,2) band at the centre is empty");
  Sum w, fw;
  for (int64_t j = j0; j < j1; ++j) {
    const double f = (double)j / seg_len;
    const double v = pow(f, -7.0 / 3.0) / psd0[j];
    w.add(v);
    fw.add(f * v);
  }
  return fw.value() / w.value();
}

// Time bands of the antenna patterns (rbfl_build_spec.n_bands > 1).  The
// centre's (2,2) stationary-phase track t(f) = Psi'(f) / (2 pi) carries the
// gravitational-wave phase Phi(f) = f Psi'(f) - Psi(f); the bands cut
// [lowest bin, (2,2) cut-off) into equal shares of Phi, so the phase error
// of a delay drifting linearly in time has the same bound in every band, and
// the last band runs on to the top of the grid.  Mode (l, m) passes f at the
// (2,2) track time of 2 f / m; its time in band b is the mean of that time
// over its own bins there under f^(-1/3) / S_0 (the delay error's weight
// f^2 |h|^2 / S), or 0 where it has no bins.  edges: [B + 1] bin indices.
void time_bands(const double centre[4], double f_ref, double f_low, double seg_len, int64_t n_s, int n_modes,
                const int modes[][2], int n_bands, const double *psd0, std::vector<int64_t> &edges,
                double times[RBFL_MAX_BANDS][RBFL_MAX_MODES]) {
  const int B = n_bands;
  const double df = 1.0 / seg_len;
  const Binary b = make_binary(centre[0], centre[1], centre[2], centre[3], f_ref);
  const int64_t j_lo = std::max<int64_t>(1, (int64_t)ceil(f_low * seg_len - 1e-9));
  const int64_t j_hi = n_s / 2;
  auto cut_bin = [&](int m) {
    const int64_t jc = (int64_t)ceil((double)m * b.f_isco * seg_len);
    return std::min(std::max(jc, j_lo), j_hi);
  };
  const int64_t j22 = cut_bin(2);
  if (j22 - j_lo < 2) throw Error(RBFL_E_INVALID_ARG, "the (2,2) band at the centre is too short for time bands");
  std::vector<double> phi((size_t)(j22 - j_lo));
  for (int64_t j = j_lo; j < j22; ++j) {
    const double f = (double)j * df;
    phi[(size_t)(j - j_lo)] = f * (dphase22_pn(f, b) - b.dpsi_ref) - phase22(f, b);
  }
  edges.assign((size_t)B + 1, 0);
  edges[0] = j_lo;
  edges[(size_t)B] = j_hi;
  const double p0 = phi.front(), p1 = phi.back();
  for (int i = 1; i < B; ++i) {
    const double cut = p0 + (p1 - p0) * (double)i / (double)B;
    const auto it = std::lower_bound(phi.begin(), phi.end(), cut);
    edges[(size_t)i] = j_lo + (int64_t)(it - phi.begin());
  }
  for (int a = 0; a < n_modes; ++a) {
    const int m = modes[a][1];
    const int64_t jc = cut_bin(m);
    for (int i = 0; i < B; ++i) {
      const int64_t lo = std::max(edges[(size_t)i], j_lo), hi = std::min(edges[(size_t)i + 1], jc);
      Sum w, tw;
      for (int64_t j = lo; j < hi; ++j) {
        const double f = (double)j * df;
        const double v = pow(f, -1.0 / 3.0) / psd0[j];
        const double t = (dphase22_pn(2.0 * f / (double)m, b) - b.dpsi_ref) / (2.0 * kPi);
        w.add(v);
        tw.add(v * t);
      }
      times[i][a] = hi > lo ? tw.value() / w.value() : 0.0;
    }
  }
}

}  // namespace rbfl
