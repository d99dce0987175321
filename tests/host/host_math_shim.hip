// C entry points over the library's host start-up math (host_math.h), built
// host-only for the CPU tests that compare it with the oracle.  Test
// infrastructure: not part of the library.
#include <cstring>
#include <vector>

#include "host_math.h"

using namespace rbfl;

extern "C" {

double hm_psd(double f, double scale) { return psd_analytic(f, scale); }

void hm_geometry(const double *g, double *D, double *r) { detector_geometry(g, D, r); }

void hm_ylm(int l, int m, double iota, double phi, double *out) {
  const YlmTerms t = ylm_terms(l, m);
  ylm_value(t, iota, phi, &out[0], &out[1]);
}

void hm_spline_table(double *out) {
  double tab[kSplineTaps][4];
  spline_table(tab);
  std::memcpy(out, tab, sizeof(tab));
}

void hm_halton(unsigned long long i, double *x) { halton_point(i, x); }

int hm_monomials(int degree, int *idx) {
  int t[kMaxPoly][3];
  const int n = monomials(degree, t);
  std::memcpy(idx, t, sizeof(int) * 3 * n);
  return n;
}

void hm_jacobi(const double *a, double *lam, double *V) { jacobi_eigen(a, lam, V); }

double hm_reference_frequency(double f_low, double seg_len, long long n_s, const double *psd0, const double *c) {
  return reference_frequency(f_low, seg_len, n_s, psd0, c);
}

// edges: [n_bands + 1]; times: [n_bands][n_modes]
void hm_time_bands(const double *centre, double f_ref, double f_low, double seg_len, long long n_s, int n_modes,
                   const int *modes, int n_bands, const double *psd0, long long *edges, double *times) {
  int md[RBFL_MAX_MODES][2] = {};
  for (int a = 0; a < n_modes; ++a) {
    md[a][0] = modes[2 * a];
    md[a][1] = modes[2 * a + 1];
  }
  std::vector<int64_t> e;
  double t[RBFL_MAX_BANDS][RBFL_MAX_MODES] = {};
  time_bands(centre, f_ref, f_low, seg_len, n_s, n_modes, md, n_bands, psd0, e, t);
  for (int b = 0; b <= n_bands; ++b) edges[b] = e[b];
  for (int b = 0; b < n_bands; ++b)
    for (int a = 0; a < n_modes; ++a) times[b * n_modes + a] = t[b][a];
}

void hm_phys_to_theta(const double *p, double f0, double *th) { phys_to_theta(p, f0, th); }

int hm_theta_to_phys(const double *th, double f0, double chi_max, double *p) {
  return theta_to_phys(th, f0, chi_max, p) ? 1 : 0;
}

}  // extern "C"
