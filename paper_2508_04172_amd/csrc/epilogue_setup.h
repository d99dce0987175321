// Per-proposal setup of the online stage's epilogue (Sec. II D): domain
// flags, each detector's arrival-time position in the window and each
// (detector, mode) amplitude of Eq. logl_complete (corrected reading).
// Shared by the epilogue kernels and the contraction kernel that finishes
// ln L in its own epilogue.
#pragma once

#include "rbfl_internal.h"
#include "rbfl_math.h"

namespace rbfl {

struct EpiSetup {
  int status;                       // 0 evaluate, 1 outside the domain (-inf), 2 NaN input
  int event;                        // multi-event batches: the proposal's event
  int n0[RBFL_MAX_DET];             // spline stencil base sample per detector
  double f[RBFL_MAX_DET];           // fractional sample position per detector
  double rr;                        // d_ref / d_L
  double Ar[RBFL_MAX_DET][RBFL_MAX_MODES], Ai[RBFL_MAX_DET][RBFL_MAX_MODES];
};

// a1 for proposal g: loads its 11 parameters into p; 2 for a NaN input, else
// 1 outside the ellipsoid or the physical region, else 0.
__device__ __forceinline__ int epi_prelude(const EvalConsts &c, const double *__restrict__ params, int64_t ld,
                                           int64_t g, double p[11]) {
  bool any_nan = false;
#pragma unroll
  for (int i = 0; i < 11; ++i) {
    p[i] = params[i * ld + g];
    any_nan |= isnan(p[i]);
  }
  if (any_nan) return 2;
  double r2 = 0.0;
  for (int d = 0; d < 4; ++d) {
    const double x = p[d] / c.semi[d];
    r2 += x * x;
  }
  bool valid = r2 <= 1.0;
  {
    double th[4], phys[4];
    for (int i = 0; i < 4; ++i) {
      double t = c.theta_c[i];
      for (int j = 0; j < 4; ++j) t += c.V[4 * i + j] * p[j];
      th[i] = t;
    }
    valid = valid && theta_to_phys(th, c.f0, c.chi_max, phys);
  }
  return valid ? 0 : 1;
}

__device__ __forceinline__ void epi_setup(const EvalConsts &c, const double *__restrict__ params, int64_t ld,
                                          int64_t g, EpiSetup &o) {
  double p[11];
  const int pre = epi_prelude(c, params, ld, g, p);
  if (pre == 2) {
    o.status = 2;
    return;
  }
  bool valid = pre == 0;
  const double alpha = p[4], dec = p[5], psi = p[6], iota = p[7], phi = p[8], tc = p[9], dl = p[10];
  o.rr = c.d_ref / dl;
  double ch, sh;
  sincos(0.5 * iota, &sh, &ch);
  double ynr[RBFL_MAX_MODES], yni[RBFL_MAX_MODES], ypr[RBFL_MAX_MODES], ypi[RBFL_MAX_MODES];
  for (int a = 0; a < c.n_modes; ++a) {
    eval_ylm(c.ylm_neg[a], ch, sh, phi, &ynr[a], &yni[a]);
    eval_ylm(c.ylm_pos[a], ch, sh, phi, &ypr[a], &ypi[a]);
  }
  const int T = c.T;
  for (int k = 0; k < c.n_det; ++k) {
    // a4: detector response, arrival time and spline stencil
    double fp, fc, dt;
    detector_response(c.D[k], c.r[k], alpha, dec, psi, &fp, &fc, &dt);
    const double s = (tc + dt - c.t_trig) * c.fs + (double)c.half_w;
    const double fl = floor(s);
    valid = valid && fl >= 4.0 && fl <= (double)(T - 6);
    o.n0[k] = valid ? (int)fl : 4;
    o.f[k] = s - fl;
    // a6: amplitudes of every mode at this detector
    for (int a = 0; a < c.n_modes; ++a) {
      const double sg = (c.mode_l[a] & 1) ? -1.0 : 1.0;
      o.Ar[k][a] = 0.5 * ((fp * ynr[a] - fc * yni[a]) + sg * (fp * ypr[a] - fc * ypi[a]));
      o.Ai[k][a] = 0.5 * ((fp * yni[a] + fc * ynr[a]) + sg * (-fp * ypi[a] - fc * ypr[a]));
    }
  }
  o.status = valid ? 0 : 1;
}

}  // namespace rbfl
