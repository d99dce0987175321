// Per-proposal setup of the online stage's epilogue (Sec. II D): domain
// flags, each detector's arrival-time position in the window and each
// (detector, mode) amplitude of Eq. logl_complete (corrected reading).
// Shared by the epilogue kernels and the contraction kernels that finish
// ln L in their own epilogues.
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

// Weight of one interpolated output in ln L = sum_c w_c Y[c] (Eq.
// logl_complete, corrected reading, frozen antenna patterns) for a proposal
// with setup o, r = d_ref / d_L, amplitudes A_{k,a} and spline position
// n0 + f at detector k.  d is the output's column descriptor: d.x = 0 / 1 for
// Re / Im of SVD coefficient d.w of mode d.z at detector d.y,
//   w = r Re(conj(A) b) / r (Ai br - Ar bi),  b = sum_p f^p B4[n0][d.w][p];
// d.x = 2 / 3 for Re / Im of the overlap of modes d.z, d.w,
//   w = -r^2 |A_a|^2 / 2 on the diagonal, else -r^2 Re(conj(A_a) A_b) /
//   r^2 Im(conj(A_a) A_b).
__device__ __forceinline__ double lnl_weight(const int4 d, const EpiSetup &o, int n_modes, int T, int q,
                                             const double2 *__restrict__ basis4) {
  const int k = d.y, a = d.z;
  const double rr = o.rr;
  const double ara = o.Ar[k][a], aia = o.Ai[k][a];
  if (d.x <= 1) {
    const double f = o.f[k];
    const double2 *v = basis4 + (((int64_t)(k * n_modes + a) * T + o.n0[k]) * q + d.w) * 4;
    const double2 v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3];
    const double br = fma(fma(fma(v3.x, f, v2.x), f, v1.x), f, v0.x);
    const double bi = fma(fma(fma(v3.y, f, v2.y), f, v1.y), f, v0.y);
    return d.x == 0 ? rr * (ara * br + aia * bi) : rr * (aia * br - ara * bi);
  }
  const double arb = o.Ar[k][d.w], aib = o.Ai[k][d.w];
  if (d.x == 2 && a == d.w) return -0.5 * rr * rr * (ara * ara + aia * aia);
  if (d.x == 2) return -rr * rr * (ara * arb + aia * aib);
  return rr * rr * (ara * aib - aia * arb);
}

}  // namespace rbfl
