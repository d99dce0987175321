// Exact ln L at each proposal without the interpolant (the reference the
// meshfree method approximates): the templates of every mode are formed on the
// frequency grid at the proposal's own intrinsic parameters, and
//   z_ka(tau_k) = 4 df sum_f conj(h_a) d_k e^{+2 pi i f tau_k} / S_k,
//   sigma_k,ab  = 4 df sum_f conj(h_a) h_b / S_k
// are direct sums over the band, combined as in Eq. logl_complete (corrected
// reading; equal to Eq. logl_basic for the projected signal of
// Eq. projected_h_fd).  tau_k = t_c + dt_k is absolute time in the segment;
// the phase f tau is split into a whole number of samples, reduced exactly in
// integers, plus a remainder, so long segments keep full precision.
//
// One workgroup per proposal; the threads stride over the bins, one pass per
// detector (20 complex accumulators per thread), fixed-order reductions.
// With the Earth's rotation switched on the antenna factors and delays vary
// along the band (each mode's frequency at its own stationary-phase time), so
// <h_k|d_k> and <h_k|h_k> are summed directly instead.
#include "rbfl_internal.h"

namespace rbfl {

namespace {

constexpr int kBruteThreads = 256;

// Sums v over the workgroup (fixed order); result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kBruteThreads / 64; ++w) t += red[w];
  return t;
}

__global__ void __launch_bounds__(kBruteThreads) k_brute(const EvalConsts *__restrict__ cp,
                                                         const double *__restrict__ params, int64_t ld,
                                                         const double2 *__restrict__ Dd,
                                                         const double *__restrict__ wk, int64_t j_lo, int64_t J,
                                                         int64_t n_s, double df, double inv_dref_s,
                                                         double *__restrict__ lnl) {
  __shared__ double red[kBruteThreads / 64];
  const EvalConsts &c = *cp;
  const int64_t g = blockIdx.x;
  double p[11];
  bool any_nan = false;
#pragma unroll
  for (int i = 0; i < 11; ++i) {
    p[i] = params[i * ld + g];
    any_nan |= isnan(p[i]);
  }
  if (any_nan) {
    if (threadIdx.x == 0) lnl[g] = __builtin_nan("");
    return;
  }
  double th[4], phys[4];
  for (int i = 0; i < 4; ++i) {
    double t = c.theta_c[i];
    for (int j = 0; j < 4; ++j) t += c.V[4 * i + j] * p[j];
    th[i] = t;
  }
  if (!theta_to_phys(th, c.f0, c.chi_max, phys)) {
    if (threadIdx.x == 0) lnl[g] = -__builtin_huge_val();
    return;
  }
  const Binary b = make_binary(phys[0], phys[1], phys[2], phys[3], c.f_ref);
  const double alpha = p[4], dec = p[5], psi = p[6], iota = p[7], phi = p[8], tc = p[9], dl = p[10];
  const double rr = c.d_ref / dl;
  const int n_modes = c.n_modes;
  // band end of each mode: f < m F_isco
  int64_t jend[RBFL_MAX_MODES];
  int64_t jmax = j_lo;
#pragma unroll
  for (int a = 0; a < RBFL_MAX_MODES; ++a) {
    if (a >= n_modes) break;
    jend[a] = std::min<int64_t>(j_lo + J, (int64_t)ceil((double)c.mode_m[a] * b.f_isco / df));
    jmax = std::max(jmax, jend[a]);
  }
  double ch, sh;
  sincos(0.5 * iota, &sh, &ch);
  const double fs = (double)n_s * df;
  double total = 0.0, comp = 0.0;
  if (c.earth_rate != 0.0) {
    // rotating Earth: A and the delay of every (bin, mode) at the mode's
    // stationary-phase time t_a = t_c + Psi'(2f/m) / (2 pi); <h_k|d_k> and
    // <h_k|h_k> summed directly over the band
    double ynr[RBFL_MAX_MODES], yni[RBFL_MAX_MODES], ypr[RBFL_MAX_MODES], ypi[RBFL_MAX_MODES];
    for (int a = 0; a < n_modes; ++a) {
      eval_ylm(c.ylm_neg[a], ch, sh, phi, &ynr[a], &yni[a]);
      eval_ylm(c.ylm_pos[a], ch, sh, phi, &ypr[a], &ypi[a]);
    }
    for (int k = 0; k < c.n_det; ++k) {
      const double2 *Dk = Dd + (int64_t)k * J;
      const double *wkk = wk + (int64_t)k * J;
      double zr = 0.0, sw = 0.0;
      for (int64_t j = j_lo + threadIdx.x; j < jmax; j += kBruteThreads) {
        const double f = (double)j * df;
        double hr = 0.0, hi = 0.0;
        for (int a = 0; a < n_modes; ++a) {
          if (!(j < jend[a])) continue;
          const int l = c.mode_l[a], m = c.mode_m[a];
          const double x = 2.0 * f / (double)m;
          const double ta = tc + (dphase22_pn(x, b) - b.dpsi_ref) / (2.0 * kPi);
          double fp, fc, dt;
          detector_response(c.D[k], c.r[k], alpha - c.earth_rate * (ta - c.t_trig), dec, psi, &fp, &fc, &dt);
          const double sg = (l & 1) ? -1.0 : 1.0;
          const double Ar = 0.5 * ((fp * ynr[a] - fc * yni[a]) + sg * (fp * ypr[a] - fc * ypi[a]));
          const double Ai = 0.5 * ((fp * yni[a] + fc * ynr[a]) + sg * (-fp * ypi[a] - fc * ypr[a]));
          const double ph = 0.5 * (double)m * phase22(x, b);
          const double amp = mode_amp(l, m, b.eta, b.delta) * b.amp * inv_dref_s * exp(-7.0 / 6.0 * log(f));
          double sn, cs;
          sincos(ph, &sn, &cs);
          const double xr = amp * cs, xi = -amp * sn;   // h_a = amp e^{-i ph}
          const double tau = tc + dt;
          const int64_t nsh = (int64_t)llrint(tau * fs);
          const double rem = tau - (double)nsh / fs;
          const int64_t nm_ = ((nsh % n_s) + n_s) % n_s;
          const int64_t ph_int = ((j % n_s) * nm_) % n_s;
          double se, ce;
          sincospi(-2.0 * ((double)ph_int / (double)n_s + f * rem), &se, &ce);
          const double vr = Ar * xr - Ai * xi, vi = Ar * xi + Ai * xr;
          hr += vr * ce - vi * se;
          hi += vr * se + vi * ce;
        }
        const double2 d = Dk[j - j_lo];
        zr += hr * d.x + hi * d.y;                       // Re(conj(h) d)
        sw += (hr * hr + hi * hi) * wkk[j - j_lo];
      }
      const double v = rr * block_sum(zr, red) - 0.5 * rr * rr * block_sum(sw, red);
      const double t = total + v;
      comp += fabs(total) >= fabs(v) ? (total - t) + v : (v - t) + total;
      total = t;
    }
    if (threadIdx.x == 0) lnl[g] = total + comp;
    return;
  }
  for (int k = 0; k < c.n_det; ++k) {
    double fp, fc, dt;
    detector_response(c.D[k], c.r[k], alpha, dec, psi, &fp, &fc, &dt);
    const double tau = tc + dt;
    const int64_t nsh = (int64_t)llrint(tau * fs);
    const double rem = tau - (double)nsh / fs;
    const int64_t nmod = ((nsh % n_s) + n_s) % n_s;
    double zr[RBFL_MAX_MODES] = {}, zi[RBFL_MAX_MODES] = {};
    double sr[RBFL_MAX_MODES * (RBFL_MAX_MODES + 1) / 2] = {}, si[RBFL_MAX_MODES * (RBFL_MAX_MODES + 1) / 2] = {};
    const double2 *Dk = Dd + (int64_t)k * J;
    const double *wkk = wk + (int64_t)k * J;
    for (int64_t j = j_lo + threadIdx.x; j < jmax; j += kBruteThreads) {
      const double f = (double)j * df;
      // conj(h_a) = amp e^{+i ph} (zero beyond the mode's band)
      double hr[RBFL_MAX_MODES], hi[RBFL_MAX_MODES];
#pragma unroll
      for (int a = 0; a < RBFL_MAX_MODES; ++a) {
        hr[a] = 0.0;
        hi[a] = 0.0;
        if (a < n_modes && j < jend[a]) {
          const int l = c.mode_l[a], m = c.mode_m[a];
          const double ph = 0.5 * (double)m * phase22(2.0 * f / (double)m, b);
          const double amp = mode_amp(l, m, b.eta, b.delta) * b.amp * inv_dref_s * exp(-7.0 / 6.0 * log(f));
          double sn, cs;
          sincos(ph, &sn, &cs);
          hr[a] = amp * cs;
          hi[a] = amp * sn;
        }
      }
      // e^{+2 pi i f tau} with the whole samples reduced exactly
      const int64_t ph_int = ((j % n_s) * nmod) % n_s;     // product < n_s^2 / 2: fits in 64 bits
      double se, ce;
      sincospi(2.0 * ((double)ph_int / (double)n_s + f * rem), &se, &ce);
      const double2 d = Dk[j - j_lo];
      const double dr = d.x * ce - d.y * se, di = d.x * se + d.y * ce;
      const double w = wkk[j - j_lo];
      int pi = 0;
#pragma unroll
      for (int a = 0; a < RBFL_MAX_MODES; ++a) {
        if (a >= n_modes) break;
        zr[a] += hr[a] * dr - hi[a] * di;
        zi[a] += hr[a] * di + hi[a] * dr;
#pragma unroll
        for (int bb = a; bb < RBFL_MAX_MODES; ++bb) {
          if (bb >= n_modes) break;
          // conj(h_a) h_b = (hr_a + i hi_a)(hr_b - i hi_b)
          sr[pi] += (hr[a] * hr[bb] + hi[a] * hi[bb]) * w;
          si[pi] += (hi[a] * hr[bb] - hr[a] * hi[bb]) * w;
          ++pi;
        }
      }
    }
    // amplitudes of this detector's modes
    double Ar[RBFL_MAX_MODES], Ai[RBFL_MAX_MODES];
#pragma unroll
    for (int a = 0; a < RBFL_MAX_MODES; ++a) {
      if (a >= n_modes) break;
      double ynr, yni, ypr, ypi;
      eval_ylm(c.ylm_neg[a], ch, sh, phi, &ynr, &yni);
      eval_ylm(c.ylm_pos[a], ch, sh, phi, &ypr, &ypi);
      const double sg = (c.mode_l[a] & 1) ? -1.0 : 1.0;
      Ar[a] = 0.5 * ((fp * ynr - fc * yni) + sg * (fp * ypr - fc * ypi));
      Ai[a] = 0.5 * ((fp * yni + fc * ynr) + sg * (-fp * ypi - fc * ypr));
    }
    double zt = 0.0, st = 0.0;
    int pi = 0;
#pragma unroll
    for (int a = 0; a < RBFL_MAX_MODES; ++a) {
      if (a >= n_modes) break;
      const double zra = block_sum(zr[a], red), zia = block_sum(zi[a], red);
      zt += Ar[a] * zra + Ai[a] * zia;                           // Re(conj(A_a) z_a)
#pragma unroll
      for (int bb = a; bb < RBFL_MAX_MODES; ++bb, ++pi) {
        if (bb >= n_modes) break;
        const double sre = block_sum(sr[pi], red), sim = block_sum(si[pi], red);
        // conj(A_a) A_b sigma_ab + (b != a) its conjugate partner
        const double pr = Ar[a] * Ar[bb] + Ai[a] * Ai[bb];
        const double pim = Ar[a] * Ai[bb] - Ai[a] * Ar[bb];
        const double term = pr * sre - pim * sim;
        st += bb == a ? term : 2.0 * term;
      }
    }
    const double v = rr * zt - 0.5 * rr * rr * st;
    const double t = total + v;
    comp += fabs(total) >= fabs(v) ? (total - t) + v : (v - t) + total;
    total = t;
  }
  if (threadIdx.x == 0) lnl[g] = total + comp;
}

}  // namespace

void launch_brute(const EvalConsts *c, const double *params, int64_t ld, int64_t n, const double2 *Dd,
                  const double *wk, int64_t j_lo, int64_t J, int64_t n_s, double df, double inv_dref_s, double *lnl,
                  hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_brute, dim3((unsigned)n), dim3(kBruteThreads), 0, s, c, params, ld, Dd, wk, j_lo, J, n_s, df,
                     inv_dref_s, lnl);
  RBFL_HIP(hipGetLastError());
}

}  // namespace rbfl
