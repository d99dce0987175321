// Host side of the rbfl C ABI: spec validation, the start-up stage
// orchestration (frame, nodes and data on the host in FP64; templates,
// overlaps, time series, SVD and RBF solve on the GPU), the exact ln L and
// method-error split, and the C entry points (the online stage is in
// rbfl_eval.hip, the surrogate's training driver in surrogate_host.hip, the
// artefact export in rbfl_query.hip).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "host_math.h"
#include "host_util.h"
#include "rbfl_internal.h"
#include "sampler.h"

namespace rbfl {

thread_local std::string g_last_error;

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    const char *msg = hipGetErrorString(e);
    (void)hipGetLastError();
    throw Error(e == hipErrorOutOfMemory ? RBFL_E_OUT_OF_MEMORY : RBFL_E_DEVICE,
                std::string(what) + ": " + (msg ? msg : "unknown HIP error"));
  }
}


// ---------------------------------------------------------------------------
// Host FP64 pieces of the start-up stage
// ---------------------------------------------------------------------------

// Projected metric of the normalised (2,2) template (Eq. MisMatch): half the
// weighted inner products of the Theta-derivatives of the phase after their
// components along 1 and 2 pi f are removed (weighted Gram-Schmidt), weights
// |h22|^2/S.  Derivatives by the complex step Im Psi(Theta + i h e_i)/h.
static void compute_metric(const Ctx &c, const std::vector<double> &psd0, const double center[4], double g[16]) {
  const Binary b = make_binary(center[0], center[1], center[2], center[3], 0.0);   // band only
  const int64_t j0 = std::max<int64_t>(1, (int64_t)ceil(c.f_low * c.seg_len - 1e-9));
  int64_t j1 = (int64_t)ceil(2.0 * b.f_isco * c.seg_len);
  j1 = std::min<int64_t>(std::max<int64_t>(j1, j0), c.n_s / 2);
  const int64_t n = j1 - j0;
  if (n < 8) throw Error(RBFL_E_INVALID_ARG, "the (2,2) band at the centre has fewer than 8 bins");
  std::vector<double> w(n), t(n);
  Sum ws;
  for (int64_t k = 0; k < n; ++k) {
    const double f = (double)(j0 + k) * c.df;
    w[k] = pow(f, -7.0 / 3.0) / psd0[j0 + k];
    ws.add(w[k]);
  }
  const double wsum = ws.value();
  for (auto &v : w) v /= wsum;
  Sum tm;
  for (int64_t k = 0; k < n; ++k) tm.add(w[k] * 2.0 * kPi * (double)(j0 + k) * c.df);
  const double tmean = tm.value();
  Sum tt;
  for (int64_t k = 0; k < n; ++k) {
    t[k] = 2.0 * kPi * (double)(j0 + k) * c.df - tmean;
    tt.add(w[k] * t[k] * t[k]);
  }
  double th_c[4];
  phys_to_theta(center, c.f_low, th_c);
  std::vector<std::vector<double>> d(4, std::vector<double>(n));
  typedef std::complex<double> cd;
  const double h = 1e-20 * fabs(th_c[1]);
  for (int i = 0; i < 4; ++i) {
    cd th[4] = {th_c[0], th_c[1], th_c[2], th_c[3]};
    th[i] += cd(0.0, h);
    cd p[4];
    theta_to_phys_generic<cd>(th, c.f_low, p);
    Sum mean;
    for (int64_t k = 0; k < n; ++k) {
      const cd ph = phase22_generic<cd>(cd((double)(j0 + k) * c.df, 0.0), p[0], p[1], p[2], p[3]);
      d[i][k] = ph.imag() / h;
      mean.add(w[k] * d[i][k]);
    }
    const double mu = mean.value();
    Sum dt;
    for (int64_t k = 0; k < n; ++k) {
      d[i][k] -= mu;
      dt.add(w[k] * d[i][k] * t[k]);
    }
    const double beta = dt.value() / tt.value();
    for (int64_t k = 0; k < n; ++k) d[i][k] -= beta * t[k];
  }
  for (int i = 0; i < 4; ++i)
    for (int j = i; j < 4; ++j) {
      Sum s;
      for (int64_t k = 0; k < n; ++k) s.add(w[k] * d[i][k] * d[j][k]);
      g[4 * i + j] = g[4 * j + i] = 0.5 * s.value();
    }
}

// ---- true match (Eq. Match) and the squeeze of the longest axis (Sec. II C.1)

typedef std::complex<double> cplx;

// In-place radix-2 transform y_m = sum_j x_j e^{+2 pi i j m / L}, L a power of
// two; bit-reversal permutation then butterflies with a table of the L/2
// twiddles e^{2 pi i k / L}.
static void fft_plus_pow2(std::vector<cplx> &x) {
  const size_t L = x.size();
  for (size_t i = 1, j = 0; i < L; ++i) {
    size_t bit = L >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(x[i], x[j]);
  }
  std::vector<cplx> tw(L / 2);
  for (size_t k = 0; k < L / 2; ++k) {
    const double a = 2.0 * kPi * (double)k / (double)L;
    tw[k] = cplx(cos(a), sin(a));
  }
  for (size_t len = 2; len <= L; len <<= 1) {
    const size_t half = len >> 1, stride = L / len;
    for (size_t i = 0; i < L; i += len)
      for (size_t k = 0; k < half; ++k) {
        const cplx u = x[i + k], v = x[i + k + half] * tw[k * stride];
        x[i + k] = u + v;
        x[i + k + half] = u - v;
      }
  }
}

// Match of the normalised (2,2) templates of a and b under detector 0's PSD,
// maximised over phase (the modulus) and time: the coarse peak of
// |sum_j X_j e^{2 pi i f_j t}| on a grid of seg_len / L (L >= 2 n_s) from one
// transform, then a golden-section refinement within one grid step.
static double match22(const Ctx &c, const std::vector<double> &psd0, const Binary &a, const Binary &b) {
  const int64_t j_lo = std::max<int64_t>(1, (int64_t)ceil(c.f_low * c.seg_len - 1e-9));
  auto band_end = [&](const Binary &x) {
    return std::min<int64_t>(std::max<int64_t>((int64_t)ceil(2.0 * x.f_isco * c.seg_len), j_lo), c.n_s / 2);
  };
  const int64_t ja = band_end(a), jb = band_end(b), jc = std::min(ja, jb);
  auto tmpl = [&](const Binary &x, int64_t j) {
    const double f = (double)j * c.df;
    return std::polar(pow(f, -7.0 / 6.0), -phase22(f, x));
  };
  Sum na, nb;
  for (int64_t j = j_lo; j < ja; ++j) na.add(std::norm(tmpl(a, j)) / psd0[j]);
  for (int64_t j = j_lo; j < jb; ++j) nb.add(std::norm(tmpl(b, j)) / psd0[j]);
  const double norm = 1.0 / sqrt(na.value() * nb.value());
  if (jc <= j_lo) return 0.0;
  std::vector<cplx> X((size_t)(jc - j_lo));
  for (int64_t j = j_lo; j < jc; ++j) X[j - j_lo] = std::conj(tmpl(a, j)) * tmpl(b, j) / psd0[j] * norm;
  size_t L = 1;
  while (L < (size_t)(2 * c.n_s)) L <<= 1;
  std::vector<cplx> y(L, cplx(0.0, 0.0));
  for (int64_t j = j_lo; j < jc; ++j) y[(size_t)j] = X[j - j_lo];
  fft_plus_pow2(y);
  size_t best = 0;
  for (size_t m = 1; m < L; ++m)
    if (std::abs(y[m]) > std::abs(y[best])) best = m;
  // |sum_j X_j e^{2 pi i j t / seg_len}|, phases re-seeded every 256 bins
  auto g = [&](double t) {
    cplx s(0.0, 0.0);
    const double w = 2.0 * kPi * t / c.seg_len;
    const cplx step = std::polar(1.0, w);
    cplx e(0.0, 0.0);
    for (int64_t j = j_lo; j < jc; ++j) {
      if (((j - j_lo) & 255) == 0) e = std::polar(1.0, w * (double)j);
      s += X[j - j_lo] * e;
      e *= step;
    }
    return std::abs(s);
  };
  const double dt = c.seg_len / (double)L;
  double lo = ((double)best - 1.0) * dt, hi = ((double)best + 1.0) * dt;
  const double r = 0.5 * (sqrt(5.0) - 1.0);
  double x1 = hi - r * (hi - lo), x2 = lo + r * (hi - lo);
  double g1 = g(x1), g2 = g(x2);
  for (int it = 0; it < 80 && hi - lo > 1e-13 * c.seg_len; ++it) {
    if (g1 >= g2) {
      hi = x2;
      x2 = x1;
      g2 = g1;
      x1 = hi - r * (hi - lo);
      g1 = g(x1);
    } else {
      lo = x1;
      x1 = x2;
      g1 = g2;
      x2 = lo + r * (hi - lo);
      g2 = g(x2);
    }
  }
  return std::max({g1, g2, std::abs(y[best])});
}

// Squeeze (Fig. 2): scale of the longest semi-axis (index 3) such that the
// true match with the centre template first falls to M0 there.  Outward
// scan s = i/64 along +e and -e with the family's formulas taken at face
// value in the spins (the spin bound acts through node rejection).  The first
// point below M0 brackets the crossing with the point before it; a step that
// leaves the binaries (eta > 1/4) is cut at that boundary (bisected to
// 1e-12) and brackets a crossing only if the match there is below M0, else
// the direction sets no limit.  The crossing is bisected to 1e-12.  Returns
// the smaller crossing, 1 if none; *tip_match receives the match at the tip.
static double squeeze_factor(const Ctx &c, const std::vector<double> &psd0, const double center[4],
                             double *tip_match) {
  const Binary bc = make_binary(center[0], center[1], center[2], center[3], c.f_ref);
  auto at = [&](double s, bool *ok) {
    double th[4], p[4];
    for (int i = 0; i < 4; ++i) th[i] = c.theta_c[i] + c.V[4 * i + 3] * s * c.semi[3];
    *ok = theta_to_phys(th, c.f_low, std::numeric_limits<double>::infinity(), p);
    if (!*ok) return 0.0;
    return match22(c, psd0, bc, make_binary(p[0], p[1], p[2], p[3], c.f_ref));
  };
  double factor = 1.0, factor_sign = 1.0;
  const int n_scan = 64;
  for (const double sign : {1.0, -1.0}) {
    double lo = 0.0;
    for (int i = 1; i <= n_scan; ++i) {
      const double s = (double)i / n_scan;
      bool ok = false;
      double m = at(sign * s, &ok);
      double hi = s;
      if (!ok) {
        // the step leaves the binaries: cut it at the boundary
        double a = lo, b = s;
        while (b - a > 1e-12) {
          const double mid = 0.5 * (a + b);
          double th[4], p[4];
          for (int r = 0; r < 4; ++r) th[r] = c.theta_c[r] + c.V[4 * r + 3] * sign * mid * c.semi[3];
          if (theta_to_phys(th, c.f_low, std::numeric_limits<double>::infinity(), p))
            a = mid;
          else
            b = mid;
        }
        m = at(sign * a, &ok);
        if (!ok || m >= c.match) break;
        hi = a;
      }
      if (m < c.match) {
        double a = lo, b = hi;
        while (b - a > 1e-12) {
          const double mid = 0.5 * (a + b);
          bool okm = false;
          const double mm = at(sign * mid, &okm);
          if (okm && mm >= c.match)
            a = mid;
          else
            b = mid;
        }
        if (0.5 * (a + b) < factor) {
          factor = 0.5 * (a + b);
          factor_sign = sign;
        }
        break;
      }
      lo = s;
    }
  }
  bool ok = false;
  *tip_match = factor < 1.0 ? at(factor_sign * factor, &ok) : 0.0;
  return factor;
}

// Synthetic data: coloured noise + the projected injection (Eq. projected_h_fd).
// Projected signal of detector k in bin j on a rotating Earth: each mode a
// contributes at its stationary-phase time t_a = t_c + Psi'(2f/m) / (2 pi)
// (the referenced phase's slope), with the antenna pattern and delay of the
// source at Earth-fixed longitude alpha - earth_rate (t_a - t_trig):
// sum_a A_ka(t_a) h_a(f) e^{-2 pi i f (t_c + dt_k(t_a))}; amp scales h_a.
static double2 rotating_signal_bin(const Ctx &c, const Binary &b, const YlmTerms *yneg, const YlmTerms *ypos, int k,
                                   double alpha, double dec, double psi, double iota, double phi, double tc, int64_t j,
                                   double amp) {
  const double f = (double)j * c.df;
  double hr = 0.0, hi = 0.0;
  for (int a = 0; a < c.n_modes; ++a) {
    const int l = c.modes[a][0], m = c.modes[a][1];
    if (!(f < (double)m * b.f_isco)) continue;
    const double x = 2.0 * f / (double)m;
    const double ta = tc + (dphase22_pn(x, b) - b.dpsi_ref) / (2.0 * kPi);
    double fp, fc, dt;
    detector_response(c.D[k], c.r[k], alpha - c.earth_rate * (ta - c.t_trig), dec, psi, &fp, &fc, &dt);
    double nr, ni, pr, pi;
    ylm_value(yneg[a], iota, phi, &nr, &ni);
    ylm_value(ypos[a], iota, phi, &pr, &pi);
    const double sg = (l & 1) ? -1.0 : 1.0;
    const double Ar = 0.5 * ((fp * nr - fc * ni) + sg * (fp * pr - fc * pi));
    const double Ai = 0.5 * ((fp * ni + fc * nr) + sg * (-fp * pi - fc * pr));
    const double ph = 0.5 * (double)m * phase22(x, b);
    const double am = mode_amp(l, m, b.eta, b.delta) * amp * exp(-7.0 / 6.0 * log(f));
    const double xr = am * cos(ph), xi = -am * sin(ph);   // h = am e^{-i ph}
    // e^{-2 pi i f tau}, tau = t_c + dt: whole samples reduced exactly, then the remainder
    const double tau = tc + dt;
    const int64_t nsh = (int64_t)llround(tau * c.fs);
    const double rem = tau - (double)nsh / c.fs;
    int64_t jm = (j % c.n_s) * (((nsh % c.n_s) + c.n_s) % c.n_s) % c.n_s;
    const double frac = (double)jm / (double)c.n_s + f * rem;
    double sn, cs;
    sincos(-2.0 * kPi * frac, &sn, &cs);
    const double vr = Ar * xr - Ai * xi, vi = Ar * xi + Ai * xr;
    hr += vr * cs - vi * sn;
    hi += vr * sn + vi * cs;
  }
  return make_double2(hr, hi);
}

static void synthesise_data(const rbfl_build_spec &s, const Ctx &c, const std::vector<std::vector<double>> &psd,
                            const YlmTerms *yneg, const YlmTerms *ypos, std::vector<std::vector<double2>> &data,
                            double *d_inj) {
  const Binary b = make_binary(s.inj_phys[0], s.inj_phys[1], s.inj_phys[2], s.inj_phys[3], c.f_ref);
  const int64_t j_lo = std::max<int64_t>(1, (int64_t)ceil(c.f_low * c.seg_len - 1e-9));
  const int64_t j_hi = c.n_s / 2;
  const double alpha = s.inj_ext[0], dec = s.inj_ext[1], psi = s.inj_ext[2], iota = s.inj_ext[3],
               phi = s.inj_ext[4];
  std::vector<std::vector<double2>> sig(c.n_det, std::vector<double2>(c.n_f, make_double2(0.0, 0.0)));
  Sum rho2;
  const double amp1 = b.amp / kMpcS;   // at 1 Mpc
  for (int k = 0; k < c.n_det; ++k) {
    if (c.earth_rate != 0.0) {
      // rotating Earth: every (bin, mode) at its own stationary-phase time
      Sum e;
      for (int64_t j = j_lo; j < j_hi; ++j) {
        const double f = (double)j * c.df;
        const double2 v = rotating_signal_bin(c, b, yneg, ypos, k, alpha, dec, psi, iota, phi, s.t_trig, j, amp1);
        sig[k][j] = v;
        e.add((v.x * v.x + v.y * v.y) / psd[k][j]);
        (void)f;
      }
      rho2.add(4.0 * c.df * e.value());
      continue;
    }
    double fp, fc, dt;
    detector_response(c.D[k], c.r[k], alpha, dec, psi, &fp, &fc, &dt);
    double Ar[RBFL_MAX_MODES], Ai[RBFL_MAX_MODES];
    for (int a = 0; a < c.n_modes; ++a) {
      double nr, ni, pr, pi;
      ylm_value(yneg[a], iota, phi, &nr, &ni);
      ylm_value(ypos[a], iota, phi, &pr, &pi);
      const double sg = (c.modes[a][0] & 1) ? -1.0 : 1.0;
      Ar[a] = 0.5 * ((fp * nr - fc * ni) + sg * (fp * pr - fc * pi));
      Ai[a] = 0.5 * ((fp * ni + fc * nr) + sg * (-fp * pi - fc * pr));
    }
    const double tau = s.t_trig + dt;
    const int64_t nsh = (int64_t)llround(tau * c.fs);
    const double rem = tau - (double)nsh / c.fs;
    Sum e;
    for (int64_t j = j_lo; j < j_hi; ++j) {
      const double f = (double)j * c.df;
      double hr = 0.0, hi = 0.0;
      for (int a = 0; a < c.n_modes; ++a) {
        const int l = c.modes[a][0], m = c.modes[a][1];
        if (!(f < (double)m * b.f_isco)) continue;
        const double ph = 0.5 * (double)m * phase22(2.0 * f / (double)m, b);
        const double am = mode_amp(l, m, b.eta, b.delta) * amp1 * exp(-7.0 / 6.0 * log(f));
        const double xr = am * cos(ph), xi = -am * sin(ph);   // h = am e^{-i ph}
        hr += Ar[a] * xr - Ai[a] * xi;
        hi += Ar[a] * xi + Ai[a] * xr;
      }
      // time shift e^{-2 pi i f tau}: whole samples reduced exactly, then the remainder
      int64_t jm = (j % c.n_s) * (nsh % c.n_s) % c.n_s;
      if (jm < 0) jm += c.n_s;
      const double frac = (double)jm / (double)c.n_s + f * rem;
      double sn, cs;
      sincos(-2.0 * kPi * frac, &sn, &cs);
      const double2 v = make_double2(hr * cs - hi * sn, hr * sn + hi * cs);
      sig[k][j] = v;
      e.add((v.x * v.x + v.y * v.y) / psd[k][j]);
    }
    rho2.add(4.0 * c.df * e.value());
  }
  *d_inj = sqrt(rho2.value()) / s.inj_snr;
  data.assign(c.n_det, std::vector<double2>(c.n_f, make_double2(0.0, 0.0)));
  for (int k = 0; k < c.n_det; ++k) {
    for (int64_t j = 0; j < c.n_f; ++j) {
      double2 v = make_double2(sig[k][j].x / *d_inj, sig[k][j].y / *d_inj);
      if (s.noise_white && j >= 1) {
        const double am = sqrt(psd[k][j] / (4.0 * c.df));
        v.x += am * s.noise_white[((int64_t)k * c.n_f + j) * 2];
        v.y += am * s.noise_white[((int64_t)k * c.n_f + j) * 2 + 1];
      }
      data[k][j] = v;
    }
  }
}

static void validate(const rbfl_build_spec *s) {
  require(s != nullptr, "spec is NULL");
  require(s->abi_version == RBFL_ABI_VERSION, "abi_version mismatch");
  require(std::isfinite(s->f_ref) && s->f_ref < 0.5 * s->fs, "f_ref must be finite and below fs / 2");
  require(std::isfinite(s->earth_rate) && fabs(s->earth_rate) < 1.0, "earth_rate must be finite, |rate| < 1 rad/s");
  require((s->flags & ~(uint32_t)(RBFL_FLAG_CENTER_NODE | RBFL_FLAG_SQUEEZE | RBFL_FLAG_OPTIMISE_CENTRE)) == 0,
          "unknown flag bits");
  require(s->n_det >= 1 && s->n_det <= RBFL_MAX_DET, "n_det out of range");
  require(s->n_bands >= 0 && s->n_bands <= RBFL_MAX_BANDS && s->n_det * std::max(1, s->n_bands) <= RBFL_MAX_BLOCKS,
          "n_bands must be in 0 .. RBFL_MAX_BANDS with n_det * n_bands <= RBFL_MAX_BLOCKS");
  require(s->n_modes >= 1 && s->n_modes <= RBFL_MAX_MODES, "n_modes out of range");
  for (int a = 0; a < s->n_modes; ++a) {
    const int l = s->modes[a][0], m = s->modes[a][1];
    require((l == 2 && (m == 2 || m == 1)) || (l == 3 && (m == 3 || m == 2)) || (l == 4 && m == 4),
            "unsupported mode (l, |m|)");
    for (int b = 0; b < a; ++b)
      require(!(s->modes[b][0] == l && s->modes[b][1] == m), "duplicate mode");
  }
  require(std::isfinite(s->fs) && s->fs > 0 && std::isfinite(s->seg_len) && s->seg_len > 0, "fs/seg_len");
  const double ns = s->fs * s->seg_len;
  require(fabs(ns - std::round(ns)) < 1e-6 && ((int64_t)std::llround(ns)) % 2 == 0 && ns >= 16,
          "fs * seg_len must be an even integer >= 16");
  require(std::isfinite(s->f_low) && s->f_low > 0 && s->f_low < 0.5 * s->fs, "f_low out of range");
  require(s->det_geom != nullptr, "det_geom is NULL");
  for (int i = 0; i < 5 * s->n_det; ++i) require(std::isfinite(s->det_geom[i]), "det_geom has non-finite values");
  if (!s->psd) require(std::isfinite(s->psd_scale) && s->psd_scale > 0, "psd_scale must be > 0");
  if (s->data_fd) {
    require(std::isfinite(s->d_ref) && s->d_ref > 0, "d_ref must be > 0 when data_fd is given");
  } else {
    require(std::isfinite(s->inj_snr) && s->inj_snr > 0, "inj_snr must be > 0");
    require(s->inj_phys[0] > 0 && s->inj_phys[1] > 0 && s->inj_phys[0] >= s->inj_phys[1], "injection masses");
    for (int i = 0; i < 5; ++i) require(std::isfinite(s->inj_ext[i]), "injection extrinsics");
  }
  require(s->center_phys[0] > 0 && s->center_phys[1] > 0 && s->center_phys[0] > s->center_phys[1],
          "centre masses must satisfy m1 > m2 > 0");
  require(fabs(s->center_phys[2]) < 1 && fabs(s->center_phys[3]) < 1, "centre spins");
  require(std::isfinite(s->match) && s->match > 0 && s->match < 1, "match must be in (0, 1)");
  require(std::isfinite(s->t_trig) && s->t_trig >= 0 && s->t_trig < s->seg_len, "t_trig out of the segment");
  const double ntr = s->t_trig * s->fs;
  require(fabs(ntr - std::round(ntr)) < 1e-6, "t_trig must be on the sample grid");
  require(std::isfinite(s->half_window) && s->half_window > 0, "half_window must be > 0");
  const int W = (int)floor(s->half_window * s->fs + 1e-9);
  require(W >= 6 && 2 * W + 1 < ns, "half_window must span at least 6 samples and fit in the segment");
  require(s->poly_degree >= 0 && s->poly_degree <= 3, "poly_degree must be 0..3");
  const int M = (int)(s->poly_degree == 0 ? 1 : s->poly_degree == 1 ? 5 : s->poly_degree == 2 ? 15 : 35);
  require(s->n_nodes > M && s->n_nodes <= 20000, "n_nodes must exceed the number of monomials (and <= 20000)");
  require(s->q >= 1 && s->q <= std::min(s->n_nodes, 2 * W + 1), "q must be in 1 .. min(N, 2W+1)");
  require(std::isfinite(s->eps) && s->eps >= 0, "eps must be >= 0 (0: chosen by the condition of the system)");
  require(std::isfinite(s->chi_max) && s->chi_max > 0 && s->chi_max <= 1, "chi_max must be in (0, 1]");
  if (s->psd) {
    const int64_t nf = (int64_t)std::llround(ns) / 2 + 1;
    for (int64_t i = 0; i < nf * s->n_det; ++i)
      require((std::isfinite(s->psd[i]) && s->psd[i] > 0) || (i % nf) == 0, "psd must be finite and > 0");
  }
}


// ---- SNR-optimised centre (Sec. II C.1) -------------------------------------

// Window-sample series z_ka(t) ([k][a][nb][T]) and mode overlaps sigma_k,ab
// ([k][nb][a][b]) of templates at host-given binaries, whole band: the
// start-up kernels with the data rotated to the window's first sample.
static void ensure_win_D(Ctx &c, hipStream_t s) {
  if (c.win_D.p) return;
  const int64_t n_trig = (int64_t)std::llround(c.t_trig * c.fs);
  const int64_t n0 = ((n_trig - c.half_w) % c.n_s + c.n_s) % c.n_s;
  c.win_D.alloc((size_t)c.n_det * c.brute_J);
  launch_rotate_band(c.brute_D.p, c.n_det, c.brute_J, c.brute_j_lo, n0, c.n_s, c.win_D.p, s);
}

// Device buffers of template_series, kept across calls of one search.
struct SeriesWork {
  int nb = 0;
  DevBuf<int> modes;
  DevBuf<Binary> bins;
  DevBuf<double2> A, Z, S, part;
};

static void template_series(Ctx &c, const std::vector<Binary> &bins, std::vector<double2> &Z,
                            std::vector<double2> &S, hipStream_t s, SeriesWork &w) {
  const int nb = (int)bins.size(), nm = c.n_modes, nd = c.n_det, T = c.T;
  const int64_t J = c.brute_J;
  ensure_win_D(c, s);
  int mode_lm[2 * RBFL_MAX_MODES] = {};
  for (int a = 0; a < nm; ++a) {
    mode_lm[2 * a] = c.modes[a][0];
    mode_lm[2 * a + 1] = c.modes[a][1];
  }
  // A is [a][binary][J]: its nm * nb rows go through one windowed DFT per
  // detector, which writes that detector's [a][binary][T] block of Z
  const int rows = nm * nb;
  const int n_split = window_dft_splits(rows, T, J);
  if (w.nb != nb) {
    w.modes.alloc(2 * RBFL_MAX_MODES);
    w.bins.alloc(nb);
    w.A.alloc((size_t)rows * J);
    w.Z.alloc((size_t)nd * rows * T);
    w.S.alloc((size_t)nd * nb * nm * nm);
    w.part.alloc((size_t)n_split * rows * T);
    w.nb = nb;
  }
  auto &d_modes = w.modes;
  auto &d_bins = w.bins;
  auto &A = w.A;
  auto &dZ = w.Z;
  auto &dS = w.S;
  auto &part = w.part;
  RBFL_HIP(hipMemcpyAsync(d_modes.p, mode_lm, sizeof(mode_lm), hipMemcpyHostToDevice, s));
  RBFL_HIP(hipMemcpyAsync(d_bins.p, bins.data(), sizeof(Binary) * nb, hipMemcpyHostToDevice, s));
  launch_waveforms(d_bins.p, nb, d_modes.p, nm, c.brute_j_lo, (int)J, c.df, 1.0, A.p, s);
  launch_sigma(A.p, nb, nm, (int)J, 0, (int)J, c.brute_w.p, nd, nb, 0, dS.p, s);
  for (int k = 0; k < nd; ++k) {
    launch_window_dft(A.p, rows, (int)J, (int)J, c.win_D.p + (size_t)k * J, c.brute_j_lo, c.n_s, T, n_split, part.p,
                      s);
    launch_reduce_splits(part.p, n_split, rows, T, dZ.p + (size_t)k * rows * T, s);
  }
  Z.resize(dZ.n);
  S.resize(dS.n);
  RBFL_HIP(hipMemcpyAsync(Z.data(), dZ.p, sizeof(double2) * dZ.n, hipMemcpyDeviceToHost, s));
  RBFL_HIP(hipMemcpyAsync(S.data(), dS.p, sizeof(double2) * dS.n, hipMemcpyDeviceToHost, s));
  RBFL_HIP(hipStreamSynchronize(s));
}

// Network SNR^2 of point p of a batch at inclination iota and phase phi:
// per detector the SNR maximised over the plane of the two polarisations
// h+ = sum_a c+_a h_a, hx = sum_a cx_a h_a (the mode factors of
// Eq. logl_complete at (F+, Fx) = (1, 0) and (0, 1): c+ = [Y_{l,-m} +
// (-1)^l conj(Y_lm)] / 2, cx = i [Y_{l,-m} - (-1)^l conj(Y_lm)] / 2), i.e.
// q = v^H G^+ v with v = (<h+|d>, <hx|d>) and G their Gram matrix
// (pseudo-inverse: a rank-one G, as for the (2,2) mode alone, keeps its
// leading direction), and over time: the best window sample b, then the
// maximum of q along the not-a-knot spline of v through the window samples
// on [b - 1, b + 1] (golden section, 60 steps; the sample value where the
// stencil would leave the window).  Summed over the detectors.  w holds the
// spline weights and the per-sample work arrays, kept across the calls of
// one search.
struct SnrWork {
  double tab[kSplineTaps][4];
  std::vector<double> r0, i0, r1, i1;
  std::vector<cplx> v0, v1;
  explicit SnrWork(int T) : r0(T), i0(T), r1(T), i1(T), v0(T), v1(T) { spline_table(tab); }
};

static double network_snr2(const Ctx &c, const YlmTerms *yneg, const YlmTerms *ypos, const std::vector<double2> &Z,
                           const std::vector<double2> &S, int nb, int p, double iota, double phi, SnrWork &w) {
  const int nm = c.n_modes, T = c.T;
  cplx cp[RBFL_MAX_MODES], cx[RBFL_MAX_MODES];
  for (int a = 0; a < nm; ++a) {
    double nr, ni, pr, pi;
    ylm_value(yneg[a], iota, phi, &nr, &ni);
    ylm_value(ypos[a], iota, phi, &pr, &pi);
    const double sg = (c.modes[a][0] & 1) ? -1.0 : 1.0;
    cp[a] = 0.5 * (cplx(nr, ni) + sg * cplx(pr, -pi));
    cx[a] = cplx(0.0, 0.5) * (cplx(nr, ni) - sg * cplx(pr, -pi));
  }
  const double(&tab)[kSplineTaps][4] = w.tab;
  std::vector<cplx> &v0 = w.v0, &v1 = w.v1;
  double total = 0.0;
  for (int k = 0; k < c.n_det; ++k) {
    cplx G00(0.0, 0.0), G01(0.0, 0.0), G11(0.0, 0.0);
    for (int a = 0; a < nm; ++a)
      for (int b = 0; b < nm; ++b) {
        const double2 sv = S[(((size_t)k * nb + p) * nm + a) * nm + b];
        const cplx sg(sv.x, sv.y);
        G00 += std::conj(cp[a]) * cp[b] * sg;
        G01 += std::conj(cp[a]) * cx[b] * sg;
        G11 += std::conj(cx[a]) * cx[b] * sg;
      }
    const double ga = G00.real(), gd = G11.real();
    const double disc = sqrt(0.25 * (ga - gd) * (ga - gd) + std::norm(G01));
    const double l1 = 0.5 * (ga + gd) + disc, l2 = 0.5 * (ga + gd) - disc;
    if (!(l1 > 0.0)) continue;
    const bool full = l2 > 1e-10 * l1;
    cplx e0(1.0, 0.0), e1(0.0, 0.0);   // leading eigenvector when G is (nearly) rank one
    if (!full) {
      if (std::abs(G01) > 0.0) {
        e0 = G01;
        e1 = cplx(l1 - ga, 0.0);
      } else if (gd > ga) {
        e0 = 0.0;
        e1 = 1.0;
      }
      const double nrm = sqrt(std::norm(e0) + std::norm(e1));
      e0 /= nrm;
      e1 /= nrm;
    }
    auto q = [&](cplx a0, cplx a1) {
      if (full) return (gd * std::norm(a0) + ga * std::norm(a1) - 2.0 * (std::conj(a0) * G01 * a1).real()) / (l1 * l2);
      return std::norm(std::conj(e0) * a0 + std::conj(e1) * a1) / l1;
    };
    int best = 0;
    double qb = -1.0;
    // v(t) = (sum_a conj(c+_a) z_a(t), sum_a conj(cx_a) z_a(t)), mode by mode
    // over contiguous sample rows
    double *r0 = w.r0.data(), *i0 = w.i0.data(), *r1 = w.r1.data(), *i1 = w.i1.data();
    std::fill(r0, r0 + T, 0.0);
    std::fill(i0, i0 + T, 0.0);
    std::fill(r1, r1 + T, 0.0);
    std::fill(i1, i1 + T, 0.0);
    for (int a = 0; a < nm; ++a) {
      const double2 *za = &Z[(((size_t)k * nm + a) * nb + p) * T];
      const double pr = cp[a].real(), pi = -cp[a].imag(), xr = cx[a].real(), xi = -cx[a].imag();
      for (int t = 0; t < T; ++t) {
        const double zx = za[t].x, zy = za[t].y;
        r0[t] += pr * zx - pi * zy;
        i0[t] += pr * zy + pi * zx;
        r1[t] += xr * zx - xi * zy;
        i1[t] += xr * zy + xi * zx;
      }
    }
    for (int t = 0; t < T; ++t) {
      const cplx a0(r0[t], i0[t]), a1(r1[t], i1[t]);
      v0[t] = a0;
      v1[t] = a1;
      const double qt = q(a0, a1);
      if (qt > qb) {
        qb = qt;
        best = t;
      }
    }
    double peak = qb;
    if (best - 5 >= 0 && best + 5 <= T - 1) {
      // q along the spline at position x in [best - 1, best + 1]
      auto at = [&](double x) {
        int n0 = (int)floor(x);
        if (n0 > best) n0 = best;   // x = best + 1 stays in the last interval
        const double f = x - n0;
        cplx a0(0.0, 0.0), a1(0.0, 0.0);
        for (int t = 0; t < kSplineTaps; ++t) {
          const double w = tab[t][0] + f * (tab[t][1] + f * (tab[t][2] + f * tab[t][3]));
          a0 += w * v0[n0 - 4 + t];
          a1 += w * v1[n0 - 4 + t];
        }
        return q(a0, a1);
      };
      const double r = 0.5 * (sqrt(5.0) - 1.0);
      double lo = best - 1.0, hi = best + 1.0;
      double x1 = hi - r * (hi - lo), x2 = lo + r * (hi - lo);
      double q1 = at(x1), q2 = at(x2);
      for (int it = 0; it < 60; ++it) {
        if (q1 >= q2) {
          hi = x2;
          x2 = x1;
          q2 = q1;
          x1 = hi - r * (hi - lo);
          q1 = at(x1);
        } else {
          lo = x1;
          x1 = x2;
          q1 = q2;
          x2 = lo + r * (hi - lo);
          q2 = at(x2);
        }
      }
      peak = std::max(q1, q2);
    }
    total += peak;
  }
  return total;
}

// Nelder-Mead maximisation of f over n coordinates from x0 with initial steps
// `step` (reflection 1, expansion 2, contraction 1/2, shrink 1/2); stops when
// the simplex's values agree to ftol relative and its extent is below xtol,
// or after max_evals evaluations.  Returns the best value; x0 receives its
// point.
template <class F>
static double nelder_mead_max(F &&f, std::vector<double> &x0, const std::vector<double> &step, double ftol,
                              double xtol, int max_evals) {
  const int n = (int)x0.size();
  std::vector<std::vector<double>> X(n + 1, x0);
  std::vector<double> V(n + 1);
  int evals = 0;
  for (int i = 0; i <= n; ++i) {
    if (i > 0) X[i][i - 1] += step[i - 1];
    V[i] = f(X[i]);
    ++evals;
  }
  std::vector<int> idx(n + 1);
  while (evals < max_evals) {
    for (int i = 0; i <= n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return V[a] > V[b]; });
    std::vector<std::vector<double>> Xs(n + 1);
    std::vector<double> Vs(n + 1);
    for (int i = 0; i <= n; ++i) {
      Xs[i] = X[idx[i]];
      Vs[i] = V[idx[i]];
    }
    X.swap(Xs);
    V.swap(Vs);
    double extent = 0.0;
    for (int i = 1; i <= n; ++i)
      for (int d = 0; d < n; ++d) extent = std::max(extent, fabs(X[i][d] - X[0][d]));
    if (fabs(V[0] - V[n]) <= ftol * fabs(V[0]) && extent < xtol) break;
    std::vector<double> cen(n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int d = 0; d < n; ++d) cen[d] += X[i][d] / n;
    auto along = [&](double t) {
      std::vector<double> y(n);
      for (int d = 0; d < n; ++d) y[d] = cen[d] + t * (X[n][d] - cen[d]);
      return y;
    };
    const std::vector<double> xr = along(-1.0);
    const double fr = f(xr);
    ++evals;
    if (fr > V[0]) {
      const std::vector<double> xe = along(-2.0);
      const double fe = f(xe);
      ++evals;
      X[n] = fe > fr ? xe : xr;
      V[n] = std::max(fe, fr);
    } else if (fr > V[n - 1]) {
      X[n] = xr;
      V[n] = fr;
    } else {
      const bool outside = fr > V[n];
      const std::vector<double> xc = along(outside ? -0.5 : 0.5);
      const double fc = f(xc);
      ++evals;
      if (fc > (outside ? fr : V[n])) {
        X[n] = xc;
        V[n] = fc;
      } else {
        for (int i = 1; i <= n; ++i) {
          for (int d = 0; d < n; ++d) X[i][d] = X[0][d] + 0.5 * (X[i][d] - X[0][d]);
          V[i] = f(X[i]);
          ++evals;
        }
      }
    }
  }
  int b = 0;
  for (int i = 1; i <= n; ++i)
    if (V[i] > V[b]) b = i;
  x0 = X[b];
  return V[b];
}

// The SNR-optimised centre (Sec. II C.1 seeds the search with the best
// template, iota and phi zero).  Outer Nelder-Mead over the intrinsic
// coordinates u = Delta e / a of the seed's eigen-frame at M0 (initial steps
// 0.1, tolerances 1e-12 relative in SNR^2 and 1e-7 in u, at most 800
// templates), restarted once from its result with steps 0.02; for each
// template, the SNR^2 maximised over (iota, phi): the
// best of a 7 x 8 grid (iota = j pi / 6, phi = k pi / 4), then a Nelder-Mead
// from it (steps 0.1 rad, 1e-12, 1e-8, 300 evaluations), all on the host from
// the template's series.  Points outside the physical region count as 0.
// centre[] is updated.
static void optimise_centre(Ctx &c, const std::vector<double> &psd0, const YlmTerms *yneg, const YlmTerms *ypos,
                            double centre[4], hipStream_t s) {
  double g[16], lam[4], vec[16], V0[16], semi0[4], th0[4];
  compute_metric(c, psd0, centre, g);
  jacobi_eigen(g, lam, vec);
  int order[4] = {0, 1, 2, 3};
  std::sort(order, order + 4, [&](int x, int y) { return lam[x] > lam[y]; });
  for (int i = 0; i < 4; ++i) {
    const int o = order[i];
    for (int r = 0; r < 4; ++r) V0[4 * r + i] = vec[4 * r + o];
    semi0[i] = sqrt((1.0 - c.match) / lam[o]);
  }
  phys_to_theta(centre, c.f_low, th0);
  auto to_phys = [&](const double *u, double p[4]) {
    double th[4];
    for (int r = 0; r < 4; ++r) {
      th[r] = th0[r];
      for (int j = 0; j < 4; ++j) th[r] += V0[4 * r + j] * u[j] * semi0[j];
    }
    return theta_to_phys(th, c.f_low, c.chi_max, p);
  };
  SeriesWork work;
  SnrWork snr_work(c.T);
  std::vector<double2> Z, S;
  double cur_angles[2] = {0.0, 0.0};   // the inner search's angles for the last template
  auto inner = [&]() {
    double b = -1.0;
    std::vector<double> a0 = {0.0, 0.0};
    for (int j = 0; j <= 6; ++j)
      for (int k = 0; k < 8; ++k) {
        const double v = network_snr2(c, yneg, ypos, Z, S, 1, 0, j * kPi / 6.0, k * kPi / 4.0, snr_work);
        if (v > b) {
          b = v;
          a0 = {j * kPi / 6.0, k * kPi / 4.0};
        }
      }
    b = nelder_mead_max(
        [&](const std::vector<double> &a) { return network_snr2(c, yneg, ypos, Z, S, 1, 0, a[0], a[1], snr_work); },
        a0, {0.1, 0.1}, 1e-12, 1e-8, 300);
    cur_angles[0] = a0[0];
    cur_angles[1] = a0[1];
    return b;
  };
  auto outer = [&](const std::vector<double> &u) {
    double p[4];
    if (!to_phys(u.data(), p)) return 0.0;
    template_series(c, {make_binary(p[0], p[1], p[2], p[3], c.f_ref)}, Z, S, s, work);
    return inner();
  };
  {
    double p[4];
    to_phys(std::vector<double>(4, 0.0).data(), p);
    template_series(c, {make_binary(p[0], p[1], p[2], p[3], c.f_ref)}, Z, S, s, work);
    c.centre_snr[0] = sqrt(std::max(network_snr2(c, yneg, ypos, Z, S, 1, 0, 0.0, 0.0, snr_work), 0.0));
  }
  std::vector<double> u(4, 0.0);
  double v = nelder_mead_max(outer, u, {0.1, 0.1, 0.1, 0.1}, 1e-12, 1e-7, 800);
  v = nelder_mead_max(outer, u, {0.02, 0.02, 0.02, 0.02}, 1e-12, 1e-7, 800);   // a restart: the simplex may collapse early
  outer(u);   // the angles of the returned vertex
  double p[4];
  to_phys(u.data(), p);
  for (int i = 0; i < 4; ++i) centre[i] = c.centre_opt[i] = p[i];
  c.centre_opt[4] = cur_angles[0];
  c.centre_opt[5] = cur_angles[1];
  c.centre_snr[1] = sqrt(std::max(v, 0.0));
}

// ---- RBFL_DEBUG: host-side bounds checks of everything the kernels index
// with.  With the environment variable RBFL_DEBUG set (to anything but "0"),
// every handle's output layout, sizes, band table and device constants are
// checked after rbfl_build and rbfl_load, and every work item of a
// multi-event plan is replayed through the kernels' own event lookup
// (work_event) against the plan's buffers; the first violation is
// RBFL_E_STATE.  The epilogues' spline stencils need no table: a stencil
// outside the window marks the proposal -inf before any row is read.

bool debug_mode() {
  const char *v = std::getenv("RBFL_DEBUG");
  return v != nullptr && *v != 0 && std::strcmp(v, "0") != 0;
}

void debug_require(bool ok, const std::string &what) {
  if (!ok) throw Error(RBFL_E_STATE, "RBFL_DEBUG: " + what);
}

void debug_check_layout(const Ctx &c) {
  const EvalConsts &e = c.host_consts;
  const int nm = c.n_modes, q = c.q;
  debug_require(c.n_v == c.n_det * c.n_bands && c.n_v >= 1 && c.n_v <= RBFL_MAX_BLOCKS && e.n_v == c.n_v &&
                    e.n_bands == c.n_bands && e.n_det == c.n_det && e.n_modes == nm,
                "block counts");
  debug_require(c.K == c.n_v * (2 * q * nm + nm * nm) && e.K == c.K && c.Kp >= c.K && c.Kp % kColTile == 0,
                "output width");
  // every output column in exactly one (block, mode) coefficient range or one
  // block's overlap range
  std::vector<int> cover((size_t)c.K, 0);
  auto mark = [&](int off, int len, const char *what) {
    debug_require(off >= 0 && off + len <= c.K, std::string(what) + " offset out of range");
    for (int i = off; i < off + len; ++i) ++cover[(size_t)i];
  };
  for (int v = 0; v < c.n_v; ++v) {
    for (int a = 0; a < nm; ++a) mark(e.coef_off[v][a], 2 * q, "coefficient");
    mark(e.sig_off[v], nm * nm, "overlap");
  }
  for (int x : cover) debug_require(x == 1, "output columns not covered exactly once");
  // buffers the epilogues and contractions index
  const size_t pairs = (size_t)c.n_v * nm;
  debug_require(c.T >= 11 && e.T == c.T && e.q == q, "window too short for the 10-tap spline stencil");
  debug_require(c.basis.n == pairs * c.T * q && c.basis4.n == pairs * c.T * q * 4, "basis sizes");
  debug_require(c.W.n == (size_t)c.rows * c.Kp && c.nodes.n == (size_t)c.rows * 4 && c.coldesc.n == (size_t)c.K,
                "weight, node or layout sizes");
  debug_require(c.rows >= c.N + c.M && c.rows % kRowChunk == 0, "padded rows");
  // band table
  debug_require((int)c.band_edges.size() == c.n_bands + 1 && c.band_edges.front() == c.brute_j_lo &&
                    c.band_edges.back() == c.n_s / 2,
                "band edges");
  for (int b = 0; b < c.n_bands; ++b) {
    debug_require(c.band_edges[b + 1] >= c.band_edges[b], "band edges decrease");
    for (int a = 0; a < nm; ++a) debug_require(std::isfinite(e.band_t[b][a]), "band time not finite");
  }
  // the device copy of the constants is the host's
  EvalConsts d;
  RBFL_HIP(hipMemcpy(&d, c.consts.p, sizeof(EvalConsts), hipMemcpyDeviceToHost));
  debug_require(std::memcmp(&d, &e, sizeof(EvalConsts)) == 0, "device constants differ from the host copy");
}

// What the start-up's stages hand on: the mode overlaps and SVD coefficients
// at the nodes, the bands' reference times and the start-up's start.
struct BuildCarry {
  DevBuf<double2> sig, C;
  double band_t[RBFL_MAX_BANDS][RBFL_MAX_MODES] = {};
  Clock::time_point t_all;
};

// Start-up up to the window series at the nodes: data, frame, nodes,
// templates, overlaps and windowed DFT.
static void build_front(const rbfl_build_spec *s, hipStream_t stream, Ctx &c, BuildCarry &carry) {
  carry.t_all = Clock::now();
  validate(s);
  RBFL_HIP(hipGetDevice(&c.device));
  c.n_det = s->n_det;
  c.n_modes = s->n_modes;
  for (int a = 0; a < c.n_modes; ++a) {
    c.modes[a][0] = s->modes[a][0];
    c.modes[a][1] = s->modes[a][1];
  }
  c.fs = s->fs;
  c.seg_len = s->seg_len;
  c.f_low = s->f_low;
  c.n_s = (int64_t)std::llround(s->fs * s->seg_len);
  c.n_f = c.n_s / 2 + 1;
  c.df = 1.0 / s->seg_len;
  c.eps = s->eps;   // 0: chosen with the RBF system (the smallest integer keeping it well conditioned)
  c.chi_max = s->chi_max;
  c.t_trig = s->t_trig;
  c.earth_rate = s->earth_rate;
  c.match = s->match;
  c.q = s->q;
  c.half_w = (int)floor(s->half_window * s->fs + 1e-9);
  c.T = 2 * c.half_w + 1;
  c.degree = s->poly_degree;
  int poly[kMaxPoly][3];
  c.M = monomials(c.degree, poly);
  c.N = s->n_nodes;
  c.n_bands = std::max(1, s->n_bands);
  c.n_v = c.n_det * c.n_bands;
  c.K = c.n_v * (2 * c.q * c.n_modes + c.n_modes * c.n_modes);
  c.Kp = ((c.K + kColTile - 1) / kColTile) * kColTile;
  c.rows = ((c.N + c.M + kRowChunk - 1) / kRowChunk) * kRowChunk;
  for (int k = 0; k < c.n_det; ++k) detector_geometry(s->det_geom + 5 * k, c.D[k], c.r[k]);

  YlmTerms yneg[RBFL_MAX_MODES], ypos[RBFL_MAX_MODES];
  for (int a = 0; a < c.n_modes; ++a) {
    yneg[a] = ylm_terms(c.modes[a][0], -c.modes[a][1]);
    ypos[a] = ylm_terms(c.modes[a][0], c.modes[a][1]);
  }

  // PSD and data
  auto t0 = Clock::now();
  std::vector<std::vector<double>> psd(c.n_det, std::vector<double>(c.n_f));
  for (int k = 0; k < c.n_det; ++k) {
    psd[k][0] = std::numeric_limits<double>::infinity();
    for (int64_t j = 1; j < c.n_f; ++j)
      psd[k][j] = s->psd ? s->psd[(int64_t)k * c.n_f + j] : psd_analytic((double)j * c.df, s->psd_scale);
  }
  if (s->f_ref > 0.0)
    c.f_ref = s->f_ref;
  else if (s->f_ref == 0.0)
    c.f_ref = reference_frequency(c.f_low, c.seg_len, c.n_s, psd[0].data(), s->center_phys);
  else
    c.f_ref = 0.0;
  std::vector<std::vector<double2>> data;
  if (s->data_fd) {
    c.d_ref = s->d_ref;
    data.assign(c.n_det, std::vector<double2>(c.n_f));
    for (int k = 0; k < c.n_det; ++k)
      for (int64_t j = 0; j < c.n_f; ++j)
        data[k][j] = make_double2(s->data_fd[((int64_t)k * c.n_f + j) * 2], s->data_fd[((int64_t)k * c.n_f + j) * 2 + 1]);
  } else {
    synthesise_data(*s, c, psd, yneg, ypos, data, &c.d_ref);
  }
  {
    // whole band, 4 df d_k / S_k and 4 df / S_k: the exact ln L at arbitrary
    // proposals, the exact outputs and the centre's network SNR
    const int64_t j_lo = std::max<int64_t>(1, (int64_t)ceil(c.f_low * c.seg_len - 1e-9));
    const int64_t j_hi = c.n_s / 2;
    c.brute_j_lo = j_lo;
    c.brute_J = j_hi - j_lo;
    std::vector<double2> bd((size_t)c.n_det * c.brute_J);
    std::vector<double> bw((size_t)c.n_det * c.brute_J);
    for (int k = 0; k < c.n_det; ++k)
      for (int64_t j = j_lo; j < j_hi; ++j) {
        const double sc = 4.0 * c.df / psd[k][j];
        bd[(size_t)k * c.brute_J + (j - j_lo)] = make_double2(sc * data[k][j].x, sc * data[k][j].y);
        bw[(size_t)k * c.brute_J + (j - j_lo)] = sc;
      }
    c.brute_D.alloc(bd.size());
    c.brute_w.alloc(bw.size());
    RBFL_HIP(hipMemcpyAsync(c.brute_D.p, bd.data(), sizeof(double2) * bd.size(), hipMemcpyHostToDevice, stream));
    RBFL_HIP(hipMemcpyAsync(c.brute_w.p, bw.data(), sizeof(double) * bw.size(), hipMemcpyHostToDevice, stream));
    RBFL_HIP(hipStreamSynchronize(stream));
  }
  c.timing[0] = seconds_since(t0);

  // frame, at the given centre or at the network-SNR optimum reached from it
  t0 = Clock::now();
  double centre[4] = {s->center_phys[0], s->center_phys[1], s->center_phys[2], s->center_phys[3]};
  for (int i = 0; i < 4; ++i) c.centre_opt[i] = centre[i];
  c.centre_snr[0] = c.centre_snr[1] = 0.0;
  if (s->flags & RBFL_FLAG_OPTIMISE_CENTRE) optimise_centre(c, psd[0], yneg, ypos, centre, stream);
  phys_to_theta(centre, c.f_low, c.theta_c);
  if (s->metric) {
    for (int i = 0; i < 16; ++i) c.metric[i] = s->metric[i];
  } else {
    compute_metric(c, psd[0], centre, c.metric);
  }
  double lam[4], vec[16];
  jacobi_eigen(c.metric, lam, vec);
  int order[4] = {0, 1, 2, 3};
  std::sort(order, order + 4, [&](int x, int y) { return lam[x] > lam[y]; });
  for (int i = 0; i < 4; ++i) {
    const int o = order[i];
    c.lam[i] = lam[o];
    if (!(lam[o] > 0.0)) throw Error(RBFL_E_NUMERICAL, "metric is not positive definite");
    int kmax = 0;
    for (int r = 1; r < 4; ++r)
      if (fabs(vec[4 * r + o]) > fabs(vec[4 * kmax + o])) kmax = r;
    const double sg = vec[4 * kmax + o] < 0 ? -1.0 : 1.0;
    for (int r = 0; r < 4; ++r) c.V[4 * r + i] = sg * vec[4 * r + o];
    c.semi[i] = sqrt((1.0 - c.match) / lam[o]);
  }
  c.squeeze[0] = 1.0;
  c.squeeze[1] = 0.0;
  if (s->flags & RBFL_FLAG_SQUEEZE) {
    c.squeeze[0] = squeeze_factor(c, psd[0], centre, &c.squeeze[1]);
    c.semi[3] *= c.squeeze[0];
  }

  // Halton nodes in the ball, physical only
  c.x_nodes.assign((size_t)c.N * 4, 0.0);
  c.phys_nodes.assign((size_t)c.N * 4, 0.0);
  int have = 0;
  auto try_point = [&](const double x[4]) -> bool {
    double th[4], p[4];
    for (int i = 0; i < 4; ++i) {
      double v = c.theta_c[i];
      for (int j = 0; j < 4; ++j) v += c.V[4 * i + j] * (x[j] * c.semi[j]);
      th[i] = v;
    }
    if (!theta_to_phys(th, c.f_low, c.chi_max, p)) return false;
    for (int d = 0; d < 4; ++d) {
      c.x_nodes[4 * have + d] = x[d];
      c.phys_nodes[4 * have + d] = p[d];
    }
    ++have;
    return true;
  };
  if (s->flags & RBFL_FLAG_CENTER_NODE) {
    const double zero[4] = {0, 0, 0, 0};
    if (!try_point(zero)) throw Error(RBFL_E_INVALID_ARG, "centre is not a physical point");
  }
  for (uint64_t i = 1; have < c.N; ++i) {
    if (i > 50000000ull) throw Error(RBFL_E_NUMERICAL, "too few physical Halton points in the ellipsoid");
    double x[4];
    halton_point(i, x);
    const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3];
    if (r2 <= 1.0) try_point(x);
  }
  c.timing[1] = seconds_since(t0);

  // ---- device: templates, overlaps and windowed DFT at the nodes, per
  // output block (detector, or detector and time band)
  t0 = Clock::now();
  const int64_t j_lo = std::max<int64_t>(1, (int64_t)ceil(c.f_low * c.seg_len - 1e-9));
  const int64_t j_hi = c.n_s / 2;
  double(&band_t)[RBFL_MAX_BANDS][RBFL_MAX_MODES] = carry.band_t;
  if (c.n_bands > 1)
    time_bands(centre, c.f_ref, c.f_low, c.seg_len, c.n_s, c.n_modes, c.modes, c.n_bands, psd[0].data(), c.band_edges,
               band_t);
  else
    c.band_edges = {j_lo, j_hi};
  std::vector<Binary> bins(c.N);
  int J_mode[RBFL_MAX_MODES] = {};
  for (int i = 0; i < c.N; ++i) {
    bins[i] = make_binary(c.phys_nodes[4 * i], c.phys_nodes[4 * i + 1], c.phys_nodes[4 * i + 2], c.phys_nodes[4 * i + 3],
                          c.f_ref);
    for (int a = 0; a < c.n_modes; ++a) {
      int64_t jc = (int64_t)ceil((double)c.modes[a][1] * bins[i].f_isco * c.seg_len);
      jc = std::min(std::max(jc, j_lo), j_hi);
      J_mode[a] = std::max<int>(J_mode[a], (int)(jc - j_lo));
    }
  }
  int J = 1;
  for (int a = 0; a < c.n_modes; ++a) J = std::max(J, J_mode[a]);
  const int64_t n_trig = (int64_t)std::llround(c.t_trig * c.fs);
  int64_t n0 = ((n_trig - c.half_w) % c.n_s + c.n_s) % c.n_s;
  std::vector<double2> Dk((size_t)c.n_det * J);
  std::vector<double> wk((size_t)c.n_det * J);
  for (int k = 0; k < c.n_det; ++k)
    for (int jj = 0; jj < J; ++jj) {
      const int64_t j = j_lo + jj;
      const double sc = 4.0 * c.df / psd[k][j];
      const int64_t ph = (j % c.n_s) * n0 % c.n_s;
      double sn, cs;
      const double ang = 2.0 * kPi * ((double)ph / (double)c.n_s);
      sn = sin(ang);
      cs = cos(ang);
      const double2 d = data[k][j];
      Dk[(size_t)k * J + jj] = make_double2(sc * (d.x * cs - d.y * sn), sc * (d.x * sn + d.y * cs));
      wk[(size_t)k * J + jj] = sc;
    }
  DevBuf<Binary> d_bins;
  d_bins.alloc(c.N);
  RBFL_HIP(hipMemcpyAsync(d_bins.p, bins.data(), sizeof(Binary) * c.N, hipMemcpyHostToDevice, stream));
  int mode_lm[2 * RBFL_MAX_MODES];
  for (int a = 0; a < c.n_modes; ++a) {
    mode_lm[2 * a] = c.modes[a][0];
    mode_lm[2 * a + 1] = c.modes[a][1];
  }
  DevBuf<int> d_modes;
  d_modes.alloc(2 * RBFL_MAX_MODES);
  RBFL_HIP(hipMemcpyAsync(d_modes.p, mode_lm, sizeof(mode_lm), hipMemcpyHostToDevice, stream));
  DevBuf<double2> d_Dk;
  d_Dk.alloc(Dk.size());
  RBFL_HIP(hipMemcpyAsync(d_Dk.p, Dk.data(), sizeof(double2) * Dk.size(), hipMemcpyHostToDevice, stream));
  DevBuf<double> d_wk;
  d_wk.alloc(wk.size());
  RBFL_HIP(hipMemcpyAsync(d_wk.p, wk.data(), sizeof(double) * wk.size(), hipMemcpyHostToDevice, stream));
  const int nm2 = c.n_modes * c.n_modes;
  c.z_nodes.alloc((size_t)c.n_v * c.n_modes * c.N * c.T);
  DevBuf<double2> &d_sig = carry.sig;
  d_sig.alloc((size_t)c.n_v * c.N * nm2);
  RBFL_HIP(hipMemsetAsync(d_sig.p, 0, sizeof(double2) * d_sig.n, stream));
  // node batches sized so the templates of a batch stay within 32 GiB of the
  // 288 GB of HBM: long segments (2048 s at 4096 Hz from 5 Hz: ~150 MB of
  // templates per node) then still fill the windowed DFT's 64-node tiles
  const size_t budget = (size_t)32 << 30;
  int nb_max = (int)std::max<size_t>(1, std::min<size_t>(c.N, budget / ((size_t)c.n_modes * J * sizeof(double2))));
  // whole 64-node tiles of the windowed DFT where the batch is cut by the budget
  if (nb_max < c.N && nb_max >= 64) nb_max &= ~63;
  DevBuf<double2> d_A;
  d_A.alloc((size_t)c.n_modes * nb_max * J);
  // split the bin range of the windowed DFT so each launch fills the GPU
  // (a band's bins: no more splits than its whole mode's)
  auto n_splits = [&](int nb, int len) { return window_dft_splits(nb, c.T, len); };
  size_t part_elems = 1;
  for (int base = 0; base < c.N; base += nb_max) {
    const int nb = std::min(nb_max, c.N - base);
    for (int a = 0; a < c.n_modes; ++a)
      part_elems = std::max(part_elems, (size_t)n_splits(nb, J_mode[a]) * nb * c.T);
  }
  DevBuf<double2> d_part;
  d_part.alloc(part_elems);
  RBFL_HIP(hipMemsetAsync(c.z_nodes.p, 0, sizeof(double2) * c.z_nodes.n, stream));
  for (int base = 0; base < c.N; base += nb_max) {
    const int nb = std::min(nb_max, c.N - base);
    launch_waveforms(d_bins.p + base, nb, d_modes.p, c.n_modes, j_lo, J, c.df, 1.0 / (c.d_ref * kMpcS), d_A.p, stream);
    for (int b = 0; b < c.n_bands; ++b) {
      // band b's bins, relative to j_lo, within the templates' extent
      const int jb0 = (int)std::min<int64_t>(c.band_edges[b] - j_lo, J);
      const int jb1 = (int)std::min<int64_t>(c.band_edges[b + 1] - j_lo, J);
      if (jb1 <= jb0) continue;
      // block v = k B + b: detector k's results at stride B N
      launch_sigma(d_A.p, nb, c.n_modes, J, jb0, jb1, d_wk.p, c.n_det, (int64_t)c.n_bands * c.N, base,
                   d_sig.p + (size_t)b * c.N * nm2, stream);
      for (int a = 0; a < c.n_modes; ++a) {
        const int len = std::min(J_mode[a], jb1) - jb0;
        if (len <= 0) continue;
        const int n_split = n_splits(nb, len);
        for (int k = 0; k < c.n_det; ++k) {
          const size_t v = (size_t)k * c.n_bands + b;
          launch_window_dft(d_A.p + (size_t)a * nb * J + jb0, nb, len, J, d_Dk.p + (size_t)k * J + jb0, j_lo + jb0,
                            c.n_s, c.T, n_split, d_part.p, stream);
          launch_reduce_splits(d_part.p, n_split, nb, c.T, c.z_nodes.p + ((v * c.n_modes + a) * c.N + base) * c.T,
                               stream);
        }
      }
    }
  }
  RBFL_HIP(hipStreamSynchronize(stream));
  d_A.reset();
  d_part.reset();
  c.timing[2] = seconds_since(t0);
}

// SVD per (block, mode) of one or more start-ups (Eq. SVD), and each one's
// basis and coefficients at the nodes.  The pairs of all start-ups with the
// same window length T go through one batched call: each pair's row-major
// N x T block of window series is a column-major T x N matrix, padded with
// zero columns to the largest N among them (zero columns change neither the
// left singular vectors nor the nonzero singular values); its left singular
// vectors are the conjugated right singular vectors of Z.  A single start-up
// is not padded.
static void svd_stage(const std::vector<std::pair<Ctx *, BuildCarry *>> &jobs, hipStream_t stream) {
  const auto t0 = Clock::now();
  BlasHandle bh;
  blas_check(rocblas_set_stream(bh.h, stream), "rocblas_set_stream");
  std::vector<bool> taken(jobs.size(), false);
  for (size_t g = 0; g < jobs.size(); ++g) {
    if (taken[g]) continue;
    const int T = jobs[g].first->T;
    std::vector<size_t> grp;
    int N_max = 0, n_prob = 0;
    for (size_t i = g; i < jobs.size(); ++i)
      if (!taken[i] && jobs[i].first->T == T) {
        const Ctx &c = *jobs[i].first;
        taken[i] = true;
        grp.push_back(i);
        N_max = std::max(N_max, c.N);
        n_prob += c.n_v * c.n_modes;
      }
    const int mn = std::min(N_max, T);
    DevBuf<double2> d_work, d_U;
    d_work.alloc((size_t)n_prob * N_max * T);
    d_U.alloc((size_t)n_prob * T * mn);
    DevBuf<double> d_S, d_E;
    d_S.alloc((size_t)n_prob * mn);
    d_E.alloc((size_t)n_prob * std::max(1, mn - 1));
    DevBuf<int> d_info;
    d_info.alloc(n_prob);
    int first = 0;
    for (size_t i : grp) {
      const Ctx &c = *jobs[i].first;
      const int n_pairs = c.n_v * c.n_modes;
      double2 *dst = d_work.p + (size_t)first * N_max * T;
      if (c.N == N_max) {
        RBFL_HIP(hipMemcpyAsync(dst, c.z_nodes.p, sizeof(double2) * n_pairs * c.N * T, hipMemcpyDeviceToDevice,
                                stream));
      } else {
        for (int ka = 0; ka < n_pairs; ++ka) {
          double2 *d = dst + (size_t)ka * N_max * T;
          RBFL_HIP(hipMemcpyAsync(d, c.z_nodes.p + (size_t)ka * c.N * T, sizeof(double2) * c.N * T,
                                  hipMemcpyDeviceToDevice, stream));
          RBFL_HIP(hipMemsetAsync(d + (size_t)c.N * T, 0, sizeof(double2) * (N_max - c.N) * T, stream));
        }
      }
      first += n_pairs;
    }
    blas_check(rocsolver_zgesvd_strided_batched(
                   bh.h, rocblas_svect_singular, rocblas_svect_none, T, N_max,
                   reinterpret_cast<rocblas_double_complex *>(d_work.p), T, (rocblas_stride)N_max * T, d_S.p,
                   (rocblas_stride)mn, reinterpret_cast<rocblas_double_complex *>(d_U.p), T, (rocblas_stride)T * mn,
                   nullptr, 1, 1, d_E.p, (rocblas_stride)std::max(1, mn - 1), rocblas_outofplace, d_info.p, n_prob),
               "rocsolver_zgesvd_strided_batched");
    std::vector<int> info_h(n_prob);
    std::vector<double> S_h(d_S.n);
    RBFL_HIP(hipMemcpyAsync(info_h.data(), d_info.p, sizeof(int) * n_prob, hipMemcpyDeviceToHost, stream));
    RBFL_HIP(hipMemcpyAsync(S_h.data(), d_S.p, sizeof(double) * d_S.n, hipMemcpyDeviceToHost, stream));
    RBFL_HIP(hipStreamSynchronize(stream));
    d_work.reset();
    first = 0;
    for (size_t i : grp) {
      Ctx &c = *jobs[i].first;
      DevBuf<double2> &d_C = jobs[i].second->C;
      const int n_pairs = c.n_v * c.n_modes, mn_c = std::min(c.N, T);
      for (int ka = 0; ka < n_pairs; ++ka)
        if (info_h[first + ka] != 0)
          throw Error(RBFL_E_NUMERICAL, "SVD of pair " + std::to_string(ka) + " did not converge (info " +
                                            std::to_string(info_h[first + ka]) + ")");
      c.singular.assign((size_t)n_pairs * mn_c, 0.0);
      for (int ka = 0; ka < n_pairs; ++ka)
        for (int j = 0; j < mn_c; ++j) c.singular[(size_t)ka * mn_c + j] = S_h[(size_t)(first + ka) * mn + j];
      c.basis.alloc((size_t)n_pairs * T * c.q);
      d_C.alloc((size_t)n_pairs * c.N * c.q);
      for (int ka = 0; ka < n_pairs; ++ka) {
        const double2 *Z = c.z_nodes.p + (size_t)ka * c.N * T;
        launch_basis_from_u(d_U.p + (size_t)(first + ka) * T * mn, T, T, c.q, c.basis.p + (size_t)ka * T * c.q,
                            stream);
        launch_coeffs(Z, c.basis.p + (size_t)ka * T * c.q, c.N, T, c.q, d_C.p + (size_t)ka * c.N * c.q, stream);
      }
      first += n_pairs;
    }
    RBFL_HIP(hipStreamSynchronize(stream));
  }
  const double dt = seconds_since(t0);
  for (const auto &j : jobs) j.first->timing[3] = dt;
}

// RBF system (Eq. rbfcoeff) and FP64 LU solve, then the online stage's
// constants and spline-folded basis.
static void build_back(const rbfl_build_spec *s, hipStream_t stream, Ctx &c, BuildCarry &carry) {
  const auto t0 = Clock::now();
  int poly[kMaxPoly][3];
  monomials(c.degree, poly);
  const int NM = c.N + c.M;
  YlmTerms yneg[RBFL_MAX_MODES], ypos[RBFL_MAX_MODES];
  for (int a = 0; a < c.n_modes; ++a) {
    yneg[a] = ylm_terms(c.modes[a][0], -c.modes[a][1]);
    ypos[a] = ylm_terms(c.modes[a][0], c.modes[a][1]);
  }
  const double(&band_t)[RBFL_MAX_BANDS][RBFL_MAX_MODES] = carry.band_t;
  const DevBuf<double2> &d_C = carry.C, &d_sig = carry.sig;
  BlasHandle bh;
  blas_check(rocblas_set_stream(bh.h, stream), "rocblas_set_stream");
  DevBuf<int> d_info;
  d_info.alloc(1);
  std::vector<int4> coldesc;
  int coef_off[RBFL_MAX_BLOCKS][RBFL_MAX_MODES], sig_off[RBFL_MAX_BLOCKS];
  for (int k = 0; k < c.n_v; ++k) {
    for (int a = 0; a < c.n_modes; ++a) {
      coef_off[k][a] = (int)coldesc.size();
      for (int i = 0; i < c.q; ++i) {
        coldesc.push_back(make_int4(0, k, a, i));
        coldesc.push_back(make_int4(1, k, a, i));
      }
    }
    sig_off[k] = (int)coldesc.size();
    for (int a = 0; a < c.n_modes; ++a) coldesc.push_back(make_int4(2, k, a, a));
    for (int a = 0; a < c.n_modes; ++a)
      for (int b = a + 1; b < c.n_modes; ++b) {
        coldesc.push_back(make_int4(2, k, a, b));
        coldesc.push_back(make_int4(3, k, a, b));
      }
  }
  if ((int)coldesc.size() != c.K) throw Error(RBFL_E_INVALID_ARG, "internal: output layout size");
  c.coldesc.alloc(coldesc.size());
  RBFL_HIP(hipMemcpyAsync(c.coldesc.p, coldesc.data(), sizeof(int4) * coldesc.size(), hipMemcpyHostToDevice, stream));
  DevBuf<double> d_R;
  d_R.alloc((size_t)c.K * NM);
  launch_assemble_rhs(d_C.p, d_sig.p, c.coldesc.p, c.N, c.K, NM, c.q, c.n_modes, d_R.p, stream);
  std::vector<double> Rh((size_t)c.K * NM);
  RBFL_HIP(hipMemcpyAsync(Rh.data(), d_R.p, sizeof(double) * Rh.size(), hipMemcpyDeviceToHost, stream));
  c.nodes.alloc((size_t)c.rows * 4);
  RBFL_HIP(hipMemsetAsync(c.nodes.p, 0, sizeof(double) * c.rows * 4, stream));
  RBFL_HIP(hipMemcpyAsync(c.nodes.p, c.x_nodes.data(), sizeof(double) * c.N * 4, hipMemcpyHostToDevice, stream));
  DevBuf<int> d_poly;
  d_poly.alloc(kMaxPoly * 3);
  RBFL_HIP(hipMemcpyAsync(d_poly.p, poly, sizeof(poly), hipMemcpyHostToDevice, stream));
  c.node_values.assign((size_t)c.N * c.K, 0.0);
  RBFL_HIP(hipStreamSynchronize(stream));
  for (int n = 0; n < c.N; ++n)
    for (int col = 0; col < c.K; ++col) c.node_values[(size_t)n * c.K + col] = Rh[(size_t)col * NM + n];
  DevBuf<double> d_A2, d_A0, d_F, d_res;
  d_A2.alloc((size_t)NM * NM);
  d_A0.alloc((size_t)NM * NM);
  DevBuf<int> d_ipiv;
  d_ipiv.alloc(NM);
  // Hager-Higham estimate of ||A^{-1}||_1 from solves with the LU factors of
  // A and A^T, times ||A||_1: the 1-norm condition estimate
  auto cond_estimate = [&](double anorm) {
    DevBuf<double> d_v;
    d_v.alloc(NM);
    std::vector<double> x(NM, 1.0 / NM), y(NM), z(NM);
    double est = 0.0;
    for (int it = 0; it < 5; ++it) {
      RBFL_HIP(hipMemcpyAsync(d_v.p, x.data(), sizeof(double) * NM, hipMemcpyHostToDevice, stream));
      blas_check(rocsolver_dgetrs(bh.h, rocblas_operation_none, NM, 1, d_A2.p, NM, d_ipiv.p, d_v.p, NM), "getrs");
      RBFL_HIP(hipMemcpyAsync(y.data(), d_v.p, sizeof(double) * NM, hipMemcpyDeviceToHost, stream));
      RBFL_HIP(hipStreamSynchronize(stream));
      double ny = 0.0;
      for (double v : y) ny += fabs(v);
      est = std::max(est, ny);
      std::vector<double> xi(NM);
      for (int i = 0; i < NM; ++i) xi[i] = y[i] >= 0 ? 1.0 : -1.0;
      RBFL_HIP(hipMemcpyAsync(d_v.p, xi.data(), sizeof(double) * NM, hipMemcpyHostToDevice, stream));
      blas_check(rocsolver_dgetrs(bh.h, rocblas_operation_transpose, NM, 1, d_A2.p, NM, d_ipiv.p, d_v.p, NM),
                 "getrs");
      RBFL_HIP(hipMemcpyAsync(z.data(), d_v.p, sizeof(double) * NM, hipMemcpyDeviceToHost, stream));
      RBFL_HIP(hipStreamSynchronize(stream));
      int jmax = 0;
      double zx = 0.0;
      for (int i = 0; i < NM; ++i) {
        if (fabs(z[i]) > fabs(z[jmax])) jmax = i;
        zx += z[i] * x[i];
      }
      if (fabs(z[jmax]) <= zx) break;
      std::fill(x.begin(), x.end(), 0.0);
      x[jmax] = 1.0;
    }
    return anorm * est;
  };
  // the shape parameter: as given, or (eps = 0 in the spec) the smallest
  // integer from 1 whose system has a 1-norm condition estimate <= kAutoEpsCond
  const bool auto_eps = !(s->eps > 0.0);
  c.eps = auto_eps ? 1.0 : s->eps;
  for (;;) {
    launch_assemble_system(c.nodes.p, c.N, c.M, d_poly.p, c.eps * c.eps, d_A2.p, stream);
    std::vector<double> Ah((size_t)NM * NM);
    RBFL_HIP(hipMemcpyAsync(Ah.data(), d_A2.p, sizeof(double) * Ah.size(), hipMemcpyDeviceToHost, stream));
    // unfactored copy of the system for the refinement's residuals
    RBFL_HIP(hipMemcpyAsync(d_A0.p, d_A2.p, sizeof(double) * NM * NM, hipMemcpyDeviceToDevice, stream));
    RBFL_HIP(hipStreamSynchronize(stream));
    double anorm = 0.0;
    for (int j = 0; j < NM; ++j) {
      double a = 0.0;
      for (int i = 0; i < NM; ++i) a += fabs(Ah[(size_t)j * NM + i]);
      anorm = std::max(anorm, a);
    }
    blas_check(rocsolver_dgetrf(bh.h, NM, NM, d_A2.p, NM, d_ipiv.p, d_info.p), "rocsolver_dgetrf");
    int info = 0;
    RBFL_HIP(hipMemcpyAsync(&info, d_info.p, sizeof(int), hipMemcpyDeviceToHost, stream));
    RBFL_HIP(hipStreamSynchronize(stream));
    const bool last = !auto_eps || c.eps >= kAutoEpsMax;
    if (info != 0) {
      if (last) throw Error(RBFL_E_NUMERICAL, "RBF system is singular (zero pivot " + std::to_string(info) + ")");
      c.eps += 1.0;
      continue;
    }
    c.cond = cond_estimate(anorm);
    if (last || c.cond <= kAutoEpsCond) break;
    c.eps += 1.0;
  }
  d_F.alloc((size_t)c.K * NM);
  d_res.alloc((size_t)c.K * NM);
  RBFL_HIP(hipMemcpyAsync(d_F.p, d_R.p, sizeof(double) * c.K * NM, hipMemcpyDeviceToDevice, stream));
  blas_check(rocsolver_dgetrs(bh.h, rocblas_operation_none, NM, c.K, d_A2.p, NM, d_ipiv.p, d_R.p, NM),
             "rocsolver_dgetrs");
  // two steps of iterative refinement with double-double residuals: LU alone
  // leaves a forward error ~ cond(A) * eps; refinement takes W to FP64 rounding
  for (int it = 0; it < 2; ++it) {
    launch_residual_dd(d_A0.p, d_F.p, d_R.p, NM, c.K, d_res.p, stream);
    blas_check(rocsolver_dgetrs(bh.h, rocblas_operation_none, NM, c.K, d_A2.p, NM, d_ipiv.p, d_res.p, NM),
               "rocsolver_dgetrs");
    launch_add(d_R.p, d_res.p, (int64_t)c.K * NM, stream);
  }
  d_A0.reset();
  d_F.reset();
  d_res.reset();
  c.W.alloc((size_t)c.rows * c.Kp);
  launch_transpose_weights(d_R.p, NM, c.K, c.rows, c.Kp, c.W.p, stream);
  RBFL_HIP(hipStreamSynchronize(stream));
  c.timing[4] = seconds_since(t0);

  // ---- constants for the online stage
  EvalConsts &e = c.host_consts;
  std::memset(&e, 0, sizeof(e));
  e.n_det = c.n_det;
  e.n_modes = c.n_modes;
  e.N = c.N;
  e.M = c.M;
  e.K = c.K;
  e.Kp = c.Kp;
  e.rows = c.rows;
  e.q = c.q;
  e.T = c.T;
  e.half_w = c.half_w;
  e.degree = c.degree;
  for (int p = 0; p < kMaxPoly; ++p)
    for (int t = 0; t < 3; ++t) e.poly_idx[p][t] = p < c.M ? poly[p][t] : -1;
  e.eps2 = c.eps * c.eps;
  e.fs = c.fs;
  e.t_trig = c.t_trig;
  e.d_ref = c.d_ref;
  e.f0 = c.f_low;
  e.chi_max = c.chi_max;
  e.f_ref = c.f_ref;
  e.earth_rate = c.earth_rate;
  for (int i = 0; i < 4; ++i) {
    e.theta_c[i] = c.theta_c[i];
    e.semi[i] = c.semi[i];
  }
  for (int i = 0; i < 16; ++i) e.V[i] = c.V[i];
  for (int k = 0; k < c.n_det; ++k) {
    for (int i = 0; i < 9; ++i) e.D[k][i] = c.D[k][i];
    for (int i = 0; i < 3; ++i) e.r[k][i] = c.r[k][i];
  }
  e.n_bands = c.n_bands;
  e.n_v = c.n_v;
  for (int v = 0; v < c.n_v; ++v) {
    for (int a = 0; a < c.n_modes; ++a) e.coef_off[v][a] = coef_off[v][a];
    e.sig_off[v] = sig_off[v];
  }
  for (int b = 0; b < RBFL_MAX_BANDS; ++b)
    for (int a = 0; a < RBFL_MAX_MODES; ++a) e.band_t[b][a] = band_t[b][a];
  for (int a = 0; a < c.n_modes; ++a) {
    e.mode_l[a] = c.modes[a][0];
    e.mode_m[a] = c.modes[a][1];
    e.ylm_neg[a] = yneg[a];
    e.ylm_pos[a] = ypos[a];
  }
  spline_table(e.spline);
  c.consts.alloc(1);
  RBFL_HIP(hipMemcpyAsync(c.consts.p, &e, sizeof(e), hipMemcpyHostToDevice, stream));
  c.basis4.alloc((size_t)c.n_v * c.n_modes * c.T * c.q * 4);
  launch_fold_spline(c.basis.p, c.n_v * c.n_modes, c.T, c.q, c.consts.p, c.basis4.p, stream);
  c.nan_part.alloc(kNanParts);
  launch_count_nan(nullptr, 0, c.nan_part.p, stream);
  RBFL_HIP(hipStreamSynchronize(stream));
  c.timing[5] = seconds_since(carry.t_all);
  if (debug_mode()) debug_check_layout(c);
}

static void build(const rbfl_build_spec *s, hipStream_t stream, Ctx &c) {
  BuildCarry carry;
  build_front(s, stream, c, carry);
  svd_stage({{&c, &carry}}, stream);
  build_back(s, stream, c, carry);
}

// Runs fn(i, stream) for i = 0 .. n-1 on up to n_threads host threads, each
// with the given device current and a stream of its own; the first failure
// stops the others from taking further items and is rethrown here.
template <class F>
static void run_on_threads(int n, int n_threads, int device, F &&fn) {
  std::atomic<int> next{0};
  std::atomic<bool> stop{false};
  std::mutex mu;
  int32_t err_code = RBFL_OK;
  std::string err_msg;
  auto fail = [&](int32_t code, const std::string &msg) {
    std::lock_guard<std::mutex> lock(mu);
    if (err_code == RBFL_OK) {
      err_code = code;
      err_msg = msg;
    }
    stop = true;
  };
  auto worker = [&]() {
    hipStream_t st = nullptr;
    try {
      RBFL_HIP(hipSetDevice(device));
      RBFL_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      for (int i = next++; i < n && !stop; i = next++) fn(i, st);
    } catch (const Error &e) {
      fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
      fail(RBFL_E_OUT_OF_MEMORY, "host allocation failed");
    } catch (const std::exception &e) {
      fail(RBFL_E_DEVICE, e.what());
    }
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  };
  std::vector<std::thread> pool;
  const int nt = std::max(1, std::min(n_threads, n));
  try {
    for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  } catch (const std::exception &) {
    // fewer threads than asked: the ones running (and this one) take every item
  }
  worker();
  for (auto &t : pool) t.join();
  if (err_code != RBFL_OK) throw Error(err_code, err_msg);
}

// Several start-ups at once: the stages before and after the SVD run on
// n_threads host threads (one stream each), and the SVDs of all start-ups
// go through one batched call per window length on the caller's stream.
static void build_many(const rbfl_build_spec *specs, int n, int n_threads, hipStream_t stream,
                       std::vector<std::unique_ptr<rbfl_ctx>> &hs) {
  for (int i = 0; i < n; ++i) validate(specs + i);   // every spec checked before any device call
  int device = 0;
  RBFL_HIP(hipGetDevice(&device));
  hs.clear();
  for (int i = 0; i < n; ++i) hs.emplace_back(new rbfl_ctx());
  std::vector<BuildCarry> carry(n);
  run_on_threads(n, n_threads, device,
                 [&](int i, hipStream_t st) { build_front(specs + i, st, hs[i]->c, carry[i]); });
  std::vector<std::pair<Ctx *, BuildCarry *>> jobs;
  for (int i = 0; i < n; ++i) jobs.emplace_back(&hs[i]->c, &carry[i]);
  svd_stage(jobs, stream);
  run_on_threads(n, n_threads, device,
                 [&](int i, hipStream_t st) { build_back(specs + i, st, hs[i]->c, carry[i]); });
}

// The quantities the interpolants approximate, computed exactly at each
// proposal with the start-up kernels (templates, overlaps, windowed DFT, time
// basis coefficients), then turned into ln L two ways: out[0..n) through the
// online stage's own epilogue (only the time basis and the spline remain
// approximate), out[n..2n) from the window samples with the spline alone.
static void exact_parts(Ctx &c, const double *params, int64_t n, double *out, hipStream_t s) {
  if (n <= 0) return;
  const int64_t J = c.brute_J, j_lo = c.brute_j_lo;
  const int nm = c.n_modes, nd = c.n_det, T = c.T, q = c.q;
  if (!c.win_D.p) {
    const int64_t n_trig = (int64_t)std::llround(c.t_trig * c.fs);
    const int64_t n0 = ((n_trig - c.half_w) % c.n_s + c.n_s) % c.n_s;
    c.win_D.alloc((size_t)nd * J);
    launch_rotate_band(c.brute_D.p, nd, J, j_lo, n0, c.n_s, c.win_D.p, s);
  }
  // proposals per batch: templates within ~2 GiB
  const size_t budget = (size_t)2 << 30;
  const int nb_max = (int)std::max<int64_t>(
      1, std::min<int64_t>({n, 4096, (int64_t)(budget / ((size_t)nm * J * sizeof(double2)))}));
  auto n_splits = [&](int nb) { return window_dft_splits(nb, T, J); };
  DevBuf<Binary> bins;
  bins.alloc(nb_max);
  DevBuf<double2> A, Z, sig, C, part;
  A.alloc((size_t)nm * nb_max * J);
  Z.alloc((size_t)nd * nm * nb_max * T);
  sig.alloc((size_t)nd * nb_max * nm * nm);
  C.alloc((size_t)nd * nm * nb_max * q);
  const int nb_last = (int)(n - (n - 1) / nb_max * nb_max);   // the last batch may split further
  part.alloc((size_t)std::max<int64_t>((int64_t)n_splits(nb_max) * nb_max, (int64_t)n_splits(nb_last) * nb_last) * T);
  DevBuf<double> Yb;
  Yb.alloc((size_t)nb_max * c.Kp);
  int mode_lm[2 * RBFL_MAX_MODES] = {};
  for (int a = 0; a < nm; ++a) {
    mode_lm[2 * a] = c.modes[a][0];
    mode_lm[2 * a + 1] = c.modes[a][1];
  }
  DevBuf<int> d_modes;
  d_modes.alloc(2 * RBFL_MAX_MODES);
  RBFL_HIP(hipMemcpyAsync(d_modes.p, mode_lm, sizeof(mode_lm), hipMemcpyHostToDevice, s));
  for (int64_t b0 = 0; b0 < n; b0 += nb_max) {
    const int nb = (int)std::min<int64_t>(nb_max, n - b0);
    launch_proposal_bins(c.consts.p, params, n, b0, nb, bins.p, s);
    launch_waveforms(bins.p, nb, d_modes.p, nm, j_lo, (int)J, c.df, 1.0 / (c.d_ref * kMpcS), A.p, s);
    launch_sigma(A.p, nb, nm, (int)J, 0, (int)J, c.brute_w.p, nd, nb, 0, sig.p, s);
    const int n_split = n_splits(nb);
    for (int a = 0; a < nm; ++a)
      for (int k = 0; k < nd; ++k) {
        launch_window_dft(A.p + (size_t)a * nb * J, nb, (int)J, (int)J, c.win_D.p + (size_t)k * J, j_lo, c.n_s, T,
                          n_split, part.p, s);
        launch_reduce_splits(part.p, n_split, nb, T, Z.p + ((size_t)k * nm + a) * nb * T, s);
      }
    for (int k = 0; k < nd; ++k)
      for (int a = 0; a < nm; ++a) {
        const size_t ka = (size_t)k * nm + a;
        launch_coeffs(Z.p + ka * nb * T, c.basis.p + ka * T * q, nb, T, q, C.p + ka * nb * q, s);
      }
    launch_outputs_rows(C.p, sig.p, c.coldesc.p, nb, c.K, c.Kp, q, nm, Yb.p, s);
    launch_epilogue(c.consts.p, c.host_consts, params, n, b0, nb, Yb.p, c.basis4.p, out, s);
    launch_series_lnl(c.consts.p, params, n, b0, nb, Z.p, sig.p, out + n, s);
  }
  RBFL_HIP(hipStreamSynchronize(s));
}

}  // namespace rbfl

struct rbfl_mlp_ctx {
  rbfl::Mlp m;
};


extern "C" {

const char *rbfl_last_error(void) { return rbfl::g_last_error.c_str(); }

int32_t rbfl_build(const rbfl_build_spec *spec, void *stream, rbfl_handle *out) {
  return rbfl::guarded([&] {
    rbfl::require(out != nullptr, "out is NULL");
    *out = nullptr;
    std::unique_ptr<rbfl_ctx> h(new rbfl_ctx());
    rbfl::build(spec, reinterpret_cast<hipStream_t>(stream), h->c);
    *out = h.release();
  });
}

int32_t rbfl_build_many(const rbfl_build_spec *specs, int32_t n, int32_t n_threads, void *stream, rbfl_handle *out) {
  return rbfl::guarded([&] {
    rbfl::require(out != nullptr, "out is NULL");
    rbfl::require(n >= 1 && n <= 4096, "n must be in 1 .. 4096");
    for (int i = 0; i < n; ++i) out[i] = nullptr;
    rbfl::require(specs != nullptr, "specs is NULL");
    rbfl::require(n_threads >= 1 && n_threads <= 16, "n_threads must be in 1 .. 16");
    std::vector<std::unique_ptr<rbfl_ctx>> hs;
    rbfl::build_many(specs, n, n_threads, reinterpret_cast<hipStream_t>(stream), hs);
    for (int i = 0; i < n; ++i) out[i] = hs[i].release();
  });
}

int32_t rbfl_brute(rbfl_handle h, const double *params, int64_t n, double *lnl, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::require(params != nullptr && lnl != nullptr, "params/lnl is NULL");
    rbfl::require(n >= 0 && n <= 2147483647, "n must be in 0 .. 2^31 - 1");
    rbfl::Ctx &c = h->c;
    rbfl::launch_brute(c.consts.p, params, n, n, c.brute_D.p, c.brute_w.p, c.brute_j_lo, c.brute_J, c.n_s, c.df,
                       1.0 / (c.d_ref * rbfl::kMpcS), lnl, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_exact_parts(rbfl_handle h, const double *params, int64_t n, double *out, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::require(params != nullptr && out != nullptr, "params/out is NULL");
    rbfl::require(n >= 0 && n <= 2147483647, "n must be in 0 .. 2^31 - 1");
    rbfl::require(h->c.n_bands == 1, "rbfl_exact_parts covers frozen antenna patterns only (n_bands = 1)");
    rbfl::exact_parts(h->c, params, n, out, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_eval(rbfl_handle h, const double *params, int64_t n, double *lnl, int32_t form, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::eval(h->c, params, n, lnl, form, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_interp(rbfl_handle h, const double *params, int64_t n, double *out, int32_t form, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::interp(h->c, params, n, out, form, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_prepare(rbfl_handle h, int32_t form) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::prepare(h->c, form);
  });
}

int32_t rbfl_reserve(rbfl_handle h, int64_t n) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::require(n >= 1, "n must be >= 1");
    rbfl::reserve(h->c, n);
  });
}

int32_t rbfl_query(rbfl_handle h, int32_t what, void *out, size_t bytes) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::query(h->c, what, out, bytes);
  });
}

int32_t rbfl_autotune(rbfl_handle h, const double *params, int64_t n, int32_t form, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::autotune(h->c, params, n, form, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_variants(int32_t form) {
  if (form < 0 || form > RBFL_FORM_SPLIT) return -RBFL_E_INVALID_ARG;
  return rbfl::contract_variants(form);
}

int32_t rbfl_set_variant(rbfl_handle h, int32_t form, int32_t variant) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    if (form < 0 || form > RBFL_FORM_SPLIT) throw rbfl::Error(RBFL_E_INVALID_ARG, "unknown or untunable form");
    if (!h->c.prepared[form]) throw rbfl::Error(RBFL_E_STATE, "form not prepared (call rbfl_prepare)");
    rbfl::require(variant >= 0 && variant < rbfl::contract_variants(form), "variant out of range");
    h->c.variant[form] = variant;
  });
}

int32_t rbfl_set_split_tol(rbfl_handle h, double tol) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::require(std::isfinite(tol) && tol > 0.0 && tol <= 1e-3, "tol must be in (0, 1e-3]");
    h->c.split_tol = tol;
  });
}

int32_t rbfl_fuse_epilogue(rbfl_handle h, int32_t on) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::require(on >= 0 && on <= 3, "on must be 0..3 (bit 0 the FP64 form, bit 1 the split form)");
    rbfl::require(!(on && h->c.n_bands > 1), "the fused epilogue covers frozen antenna patterns only (n_bands = 1)");
    h->c.lnl_gemm = (on & 1) != 0;
    h->c.split_lnl = (on & 2) != 0;
  });
}

int32_t rbfl_pipeline(rbfl_handle h, int32_t chunks) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::require(chunks >= 1 && chunks <= 64, "chunks must be in 1..64");
    h->c.pipe = chunks;
  });
}

int32_t rbfl_profile(rbfl_handle h, int32_t on) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    h->c.profile = on != 0;
  });
}

int32_t rbfl_surrogate_train(rbfl_handle h, const rbfl_train_spec *spec, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::require(h->c.n_bands == 1, "the surrogate covers frozen antenna patterns only (n_bands = 1)");
    rbfl::surrogate_train(h->c, spec, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_surrogate_force(rbfl_handle h, int32_t on) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    if (!h->c.sur) throw rbfl::Error(RBFL_E_STATE, "no surrogate trained");
    h->c.sur_ok = on ? true : (h->c.sur_stats[0] != 0.0);
  });
}

int32_t rbfl_mlp_create(int32_t n_in, int32_t hidden, int32_t n_out, const double *normals, rbfl_mlp *out) {
  return rbfl::guarded([&] {
    rbfl::require(out != nullptr && normals != nullptr, "NULL argument");
    rbfl::require(n_in >= 1 && hidden >= 1 && n_out >= 1 && hidden <= 4096 && n_out <= 65536, "sizes");
    std::unique_ptr<rbfl_mlp_ctx> m(new rbfl_mlp_ctx());
    m->m.init(n_in, hidden, n_out, normals);
    *out = m.release();
  });
}

int32_t rbfl_mlp_forward(rbfl_mlp m, const float *x, int64_t B, float *y, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(m != nullptr && x != nullptr && y != nullptr && B >= 1 && B <= 65536, "arguments");
    m->m.forward(x, B, y, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_mlp_loss_grad(rbfl_mlp m, const float *x, const float *t, int64_t B, double *loss, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(m != nullptr && x != nullptr && t != nullptr && B >= 1 && B <= 65536, "arguments");
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    m->m.loss_grad(x, t, B, s);
    double l = 0.0;
    RBFL_HIP(hipMemcpyAsync(&l, m->m.loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
    RBFL_HIP(hipStreamSynchronize(s));
    if (loss) *loss = l;
  });
}

int32_t rbfl_mlp_adam(rbfl_mlp m, double lr, double beta1, double beta2, double eps, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(m != nullptr, "NULL mlp");
    m->m.adam(lr, beta1, beta2, eps, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_mlp_get(rbfl_mlp m, int32_t what, float *out, size_t bytes) {
  return rbfl::guarded([&] {
    rbfl::require(m != nullptr && out != nullptr && (what == 0 || what == 1), "arguments");
    const size_t need = sizeof(float) * (size_t)m->m.np;
    rbfl::require(bytes >= need, "output buffer too small");
    RBFL_HIP(hipDeviceSynchronize());
    RBFL_HIP(hipMemcpy(out, what == 0 ? m->m.p.p : m->m.g.p, need, hipMemcpyDeviceToHost));
  });
}

int32_t rbfl_mlp_destroy(rbfl_mlp m) {
  return rbfl::guarded([&] { delete m; });
}

int32_t rbfl_destroy(rbfl_handle h) {
  return rbfl::guarded([&] { delete h; });
}

}  // extern "C"
