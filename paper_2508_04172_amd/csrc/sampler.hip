// GPU-resident ensemble sampler in the eigen-axis coordinates (Sec. II D:
// proposals are drawn in the Delta e coordinates of the ellipsoid), driving
// the online stage.  Differential-evolution Metropolis moves (ter Braak 2006):
// the walkers are split into two halves; each walker i of one half proposes
//   Y = X_i + g (X_j - X_k),  j != k drawn from the other half,
// with g = gamma (1 + 0.01 n), n standard normal, and g = 1 with probability
// p_jump.  (j, k) and (k, j) are equally likely, so the proposal is symmetric
// (also with the periodic angles wrapped) and the Metropolis ratio is the
// posterior ratio.  Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and
// Shaw, SC 2011), keyed by the seed, counter (walker, step low word, step
// high word | half << 31, call).
#include "sampler.h"

namespace rbfl {

namespace {

constexpr int kSBlock = 256;

// Two uniforms of call t of a walker's counter for (step, half).
struct Draw {
  uint64_t seed, step;
  uint32_t walker;
  int half;
  __device__ void pair(uint32_t t, double *u0, double *u1) const { philox_pair(seed, walker, step, half, t, u0, u1); }
};

__device__ __forceinline__ Draw make_draw(uint64_t seed, uint32_t walker, uint64_t step, int half) {
  Draw d;
  d.seed = seed;
  d.step = step;
  d.walker = walker;
  d.half = half;
  return d;
}

// Periods of the angles: alpha 2 pi, psi pi (the response has period pi in
// psi), phi 2 pi; 0 for the other parameters.
__device__ __forceinline__ double period(int m) {
  return m == 4 ? 2.0 * kPi : m == 6 ? kPi : m == 8 ? 2.0 * kPi : 0.0;
}

__device__ __forceinline__ double wrap(double v, double P) {
  v = fmod(v, P);
  return v < 0.0 ? v + P : v;
}

// Log prior density (up to a constant) of the sampled parameters: uniform in
// Delta e inside the unit ball of x = Delta e / a and the physical region,
// alpha, psi, phi uniform (periodic), dec with density cos(dec), iota with
// sin(iota) (isotropic sky and orientation), t_c uniform in [t_lo, t_hi],
// d_L with density d_L^d_exp in [d_lo, d_hi].
__device__ double sampler_log_prior(const EvalConsts &c, const SamplerPrior &pr, const double p[11]) {
  double r2 = 0.0;
  for (int d = 0; d < 4; ++d) {
    const double x = p[d] / c.semi[d];
    r2 += x * x;
  }
  if (!(r2 <= 1.0)) return -__builtin_huge_val();
  double th[4], phys[4];
  for (int i = 0; i < 4; ++i) {
    double t = c.theta_c[i];
    for (int j = 0; j < 4; ++j) t += c.V[4 * i + j] * p[j];
    th[i] = t;
  }
  if (!theta_to_phys(th, c.f0, c.chi_max, phys)) return -__builtin_huge_val();
  const double dec = p[5], iota = p[7], tc = p[9], dl = p[10];
  if (!(dec > -0.5 * kPi && dec < 0.5 * kPi && iota > 0.0 && iota < kPi)) return -__builtin_huge_val();
  if (!(tc >= pr.t_lo && tc <= pr.t_hi && dl >= pr.d_lo && dl <= pr.d_hi)) return -__builtin_huge_val();
  return log(cos(dec)) + log(sin(iota)) + pr.d_exp * log(dl);
}

// Walkers drawn from the prior: x uniform in the unit ball by rejection from
// the cube, kept if physical (up to 4096 tries), the extrinsic parameters by
// inverse transforms.  Counter step = 2^63 - 1 (never reached by a run).
__global__ void __launch_bounds__(kSBlock) k_sampler_init(const EvalConsts *__restrict__ cp, SamplerPrior pr,
                                                          uint64_t seed, int W, double *__restrict__ X,
                                                          double *__restrict__ lp) {
  const int w = blockIdx.x * kSBlock + threadIdx.x;
  if (w >= W) return;
  const EvalConsts &c = *cp;
  const Draw dr = make_draw(seed, (uint32_t)w, 0x7FFFFFFFFFFFFFFFull, 1);
  double p[11];
  uint32_t t = 0;
  bool found = false;
  for (int tries = 0; tries < 4096 && !found; ++tries) {
    double u[4];
    dr.pair(t++, &u[0], &u[1]);
    dr.pair(t++, &u[2], &u[3]);
    double r2 = 0.0;
    double th[4], phys[4];
    for (int d = 0; d < 4; ++d) r2 += (2.0 * u[d] - 1.0) * (2.0 * u[d] - 1.0);
    if (r2 > 1.0) continue;
    for (int d = 0; d < 4; ++d) p[d] = (2.0 * u[d] - 1.0) * c.semi[d];
    for (int i = 0; i < 4; ++i) {
      double v = c.theta_c[i];
      for (int j = 0; j < 4; ++j) v += c.V[4 * i + j] * p[j];
      th[i] = v;
    }
    found = theta_to_phys(th, c.f0, c.chi_max, phys);
  }
  if (!found)
    for (int d = 0; d < 4; ++d) p[d] = 0.0;   // the centre, physical by construction
  double u[8];
  dr.pair(t++, &u[0], &u[1]);
  dr.pair(t++, &u[2], &u[3]);
  dr.pair(t++, &u[4], &u[5]);
  dr.pair(t++, &u[6], &u[7]);
  p[4] = 2.0 * kPi * u[0];
  p[5] = asin(2.0 * u[1] - 1.0);
  p[6] = kPi * u[2];
  p[7] = acos(2.0 * u[3] - 1.0);
  p[8] = 2.0 * kPi * u[4];
  p[9] = pr.t_lo + (pr.t_hi - pr.t_lo) * u[5];
  const double e = pr.d_exp + 1.0;
  const double a = pow(pr.d_lo, e), b = pow(pr.d_hi, e);
  p[10] = pow(a + (b - a) * u[6], 1.0 / e);
  for (int m = 0; m < 11; ++m) X[(int64_t)m * W + w] = p[m];
  lp[w] = sampler_log_prior(c, pr, p);
}

// Proposals of one half: walker i of half h (global index h M + i) with
// partners from the other half.  Calls 0, 1 and 3 of its counter.
__global__ void __launch_bounds__(kSBlock) k_de_propose(const SamplerState *__restrict__ st, uint64_t seed, int M,
                                                        int half, double gamma, double p_jump,
                                                        const double *__restrict__ X, double *__restrict__ Y) {
  const int i = blockIdx.x * kSBlock + threadIdx.x;
  if (i >= M) return;
  const int W = 2 * M;
  const int gi = half * M + i, other = (1 - half) * M;
  const Draw dr = make_draw(seed, (uint32_t)gi, st->step, half);
  double u0, u1, u2, u3, u4, u5;
  dr.pair(0, &u0, &u1);
  dr.pair(1, &u2, &u3);
  dr.pair(3, &u4, &u5);
  const int j = min((int)(u0 * M), M - 1);
  int k = min((int)(u1 * (M - 1)), M - 2);
  if (k >= j) ++k;
  // g = gamma (1 + 0.01 n) with n from the Box-Muller transform of (u2, u3),
  // or 1 (a jump between modes) when u4 < p_jump
  double g = gamma * (1.0 + 0.01 * sqrt(-2.0 * log(u2)) * cospi(2.0 * u3));
  if (u4 < p_jump) g = 1.0;
  (void)u5;
  for (int m = 0; m < 11; ++m) {
    const double xi = X[(int64_t)m * W + gi];
    double dxm = X[(int64_t)m * W + other + j] - X[(int64_t)m * W + other + k];
    const double P = period(m);
    if (P > 0.0) dxm -= P * rint(dxm / P);   // the shorter way round
    double y = xi + g * dxm;
    if (P > 0.0) y = wrap(y, P);
    Y[(int64_t)m * M + i] = y;
  }
}

// Metropolis decision for one half (call 2 of the walker's counter), with ln L
// weighted by the annealing factor beta of the step; on the second half also
// the chain sample of the completed step.
__global__ void __launch_bounds__(kSBlock) k_de_accept(const EvalConsts *__restrict__ cp, SamplerPrior pr,
                                                       const SamplerState *__restrict__ st, uint64_t seed, int M,
                                                       int half, int prior_only, const double *__restrict__ Y,
                                                       const double *__restrict__ lnl_y, double *__restrict__ X,
                                                       double *__restrict__ lnl_x, double *__restrict__ lp_x,
                                                       unsigned long long *__restrict__ acc) {
  const int i = blockIdx.x * kSBlock + threadIdx.x;
  if (i >= M) return;
  const EvalConsts &c = *cp;
  const int W = 2 * M;
  const int gi = half * M + i;
  double p[11];
  for (int m = 0; m < 11; ++m) p[m] = Y[(int64_t)m * M + i];
  const double lpy = sampler_log_prior(c, pr, p);
  double ly = prior_only ? 0.0 : lnl_y[i];
  if (isnan(ly)) ly = -__builtin_huge_val();
  const Draw dr = make_draw(seed, (uint32_t)gi, st->step, half);
  double u, unused;
  dr.pair(2, &u, &unused);
  const double lx = lnl_x[gi], lpx = lp_x[gi];
  const double ninf = -__builtin_huge_val();
  bool take = false;
  if (ly + lpy > ninf) {
    if (!(lx + lpx > ninf)) {
      take = true;   // a walker at zero posterior takes any proposal of non-zero posterior
    } else {
      const double beta = st->beta_fixed >= 0.0 ? st->beta_fixed
                          : st->step < st->anneal_steps
                              ? pow(st->beta0, 1.0 - (double)st->step / (double)st->anneal_steps)
                              : 1.0;
      take = log(u) < beta * (ly - lx) + (lpy - lpx);
    }
  }
  if (take) {
    for (int m = 0; m < 11; ++m) X[(int64_t)m * W + gi] = p[m];
    lnl_x[gi] = ly;
    lp_x[gi] = lpy;
    acc[gi] += 1ull;
  }
  if (half == 1 && st->chain != nullptr) {
    // chain layout [12][slots][W]: row m of every sample contiguous
    const uint64_t done = st->step + 1 - st->run_start;
    if (done % (uint64_t)st->thin == 0) {
      const int64_t slot = (int64_t)(done / (uint64_t)st->thin) - 1;
      if (slot < st->slots) {
        const int64_t row = st->slots * (int64_t)W;
        double *dst = st->chain + slot * (int64_t)W;
        for (int h = 0; h < 2; ++h) {
          const int w = h * M + i;
          for (int m = 0; m < 11; ++m) dst[m * row + w] = X[(int64_t)m * W + w];
          dst[11 * row + w] = lnl_x[w];
        }
      }
    }
  }
}

// Walker w of the resampled ensemble is walker idx[w] of the current one.
__global__ void __launch_bounds__(kSBlock) k_gather_walkers(const double *__restrict__ X,
                                                            const double *__restrict__ lnl,
                                                            const double *__restrict__ lp,
                                                            const int32_t *__restrict__ idx, int W,
                                                            double *__restrict__ Xo, double *__restrict__ lnlo,
                                                            double *__restrict__ lpo) {
  const int w = blockIdx.x * kSBlock + threadIdx.x;
  if (w >= W) return;
  const int src = idx[w];
  for (int m = 0; m < 11; ++m) Xo[(int64_t)m * W + w] = X[(int64_t)m * W + src];
  lnlo[w] = lnl[src];
  lpo[w] = lp[src];
}

__global__ void k_step_advance(SamplerState *st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->step += 1;
}

__global__ void __launch_bounds__(kSBlock) k_fill(double *__restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * kSBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(kSBlock) k_log_prior(const EvalConsts *__restrict__ cp, SamplerPrior pr,
                                                       const double *__restrict__ X, int W,
                                                       double *__restrict__ lp) {
  const int w = blockIdx.x * kSBlock + threadIdx.x;
  if (w >= W) return;
  double p[11];
  for (int m = 0; m < 11; ++m) p[m] = X[(int64_t)m * W + w];
  lp[w] = sampler_log_prior(*cp, pr, p);
}

// Prior reweighting (Sec. III A: w = p_target / p_sampled): the sampled
// intrinsic prior is uniform in Delta e, the target uniform in (m1, m2,
// chi1, chi2) inside box, so log w = log |det d(m1, m2, chi1, chi2) /
// d Delta e| (= log |det d phys / d Theta|, V being orthonormal), from
// central differences with steps 1e-7 |Theta_m|; plus d_exp log d_L for a
// distance prior d^d_exp relative to the sampled one.  -inf outside box.
__global__ void __launch_bounds__(kSBlock) k_prior_weights(const EvalConsts *__restrict__ cp,
                                                           const double *__restrict__ params, int64_t ld, int64_t n,
                                                           PriorBox box, double *__restrict__ logw) {
  const int64_t g = (int64_t)blockIdx.x * kSBlock + threadIdx.x;
  if (g >= n) return;
  const EvalConsts &c = *cp;
  double th[4], phys[4];
  for (int i = 0; i < 4; ++i) {
    double t = c.theta_c[i];
    for (int j = 0; j < 4; ++j) t += c.V[4 * i + j] * params[j * ld + g];
    th[i] = t;
  }
  const double inf = __builtin_huge_val();
  if (!theta_to_phys(th, c.f0, inf, phys)) {
    logw[g] = -inf;
    return;
  }
  for (int d = 0; d < 4; ++d)
    if (!(phys[d] >= box.lo[d] && phys[d] <= box.hi[d])) {
      logw[g] = -inf;
      return;
    }
  double J[4][4];
  for (int m = 0; m < 4; ++m) {
    const double h = 1e-7 * fabs(th[m]);
    double tp[4], tm[4], pp[4], pm[4];
    for (int i = 0; i < 4; ++i) tp[i] = tm[i] = th[i];
    tp[m] += h;
    tm[m] -= h;
    theta_to_phys(tp, c.f0, inf, pp);
    theta_to_phys(tm, c.f0, inf, pm);
    for (int i = 0; i < 4; ++i) J[i][m] = (pp[i] - pm[i]) / (2.0 * h);
  }
  // determinant by Gaussian elimination with partial pivoting
  double det = 1.0;
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (fabs(J[r][col]) > fabs(J[piv][col])) piv = r;
    if (piv != col) {
      for (int k = 0; k < 4; ++k) {
        const double t = J[col][k];
        J[col][k] = J[piv][k];
        J[piv][k] = t;
      }
      det = -det;
    }
    det *= J[col][col];
    if (J[col][col] == 0.0) break;
    for (int r = col + 1; r < 4; ++r) {
      const double f = J[r][col] / J[col][col];
      for (int k = col; k < 4; ++k) J[r][k] -= f * J[col][k];
    }
  }
  logw[g] = log(fabs(det)) + box.d_exp * log(params[10 * ld + g]);
}

}  // namespace

void launch_sampler_init(const EvalConsts *c, const SamplerPrior &pr, uint64_t seed, int W, double *X, double *lp,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_sampler_init, dim3((W + kSBlock - 1) / kSBlock), dim3(kSBlock), 0, s, c, pr, seed, W, X, lp);
  RBFL_HIP(hipGetLastError());
}

void launch_log_prior(const EvalConsts *c, const SamplerPrior &pr, const double *X, int W, double *lp,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_log_prior, dim3((W + kSBlock - 1) / kSBlock), dim3(kSBlock), 0, s, c, pr, X, W, lp);
  RBFL_HIP(hipGetLastError());
}

void launch_de_propose(const SamplerState *st, uint64_t seed, int M, int half, double gamma, double p_jump,
                       const double *X, double *Y, hipStream_t s) {
  hipLaunchKernelGGL(k_de_propose, dim3((M + kSBlock - 1) / kSBlock), dim3(kSBlock), 0, s, st, seed, M, half, gamma,
                     p_jump, X, Y);
  RBFL_HIP(hipGetLastError());
}

void launch_de_accept(const EvalConsts *c, const SamplerPrior &pr, const SamplerState *st, uint64_t seed, int M,
                      int half, int prior_only, const double *Y, const double *lnl_y, double *X, double *lnl_x,
                      double *lp_x, unsigned long long *acc, hipStream_t s) {
  hipLaunchKernelGGL(k_de_accept, dim3((M + kSBlock - 1) / kSBlock), dim3(kSBlock), 0, s, c, pr, st, seed, M, half,
                     prior_only, Y, lnl_y, X, lnl_x, lp_x, acc);
  RBFL_HIP(hipGetLastError());
}

void launch_step_advance(SamplerState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, st);
  RBFL_HIP(hipGetLastError());
}

void launch_gather_walkers(const double *X, const double *lnl, const double *lp, const int32_t *idx, int W,
                           double *Xo, double *lnlo, double *lpo, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_walkers, dim3((W + kSBlock - 1) / kSBlock), dim3(kSBlock), 0, s, X, lnl, lp, idx, W, Xo,
                     lnlo, lpo);
  RBFL_HIP(hipGetLastError());
}

void launch_fill(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + kSBlock - 1) / kSBlock)), dim3(kSBlock), 0, s, p, n, v);
  RBFL_HIP(hipGetLastError());
}

void launch_prior_weights(const EvalConsts *c, const double *params, int64_t ld, int64_t n, const PriorBox &box,
                          double *logw, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_prior_weights, dim3((unsigned)((n + kSBlock - 1) / kSBlock)), dim3(kSBlock), 0, s, c, params,
                     ld, n, box, logw);
  RBFL_HIP(hipGetLastError());
}

}  // namespace rbfl
