// Ensemble sampler and prior reweighting: device-side state and launchers
// (sampler.hip).
#pragma once

#include "rbfl_internal.h"

namespace rbfl {

// One Philox4x32-10 block (Salmon, Moraes, Dror and Shaw, SC 2011): 10 rounds
// of two 32x32 -> 64-bit products with the multipliers 0xD2511F53 and
// 0xCD9E8D57, key bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85
// between rounds.  Host and device.
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Uniform in (0, 1) from two 32-bit words: 53 bits, offset by half an ulp.
__host__ __device__ inline double philox_u01(uint32_t a, uint32_t b) {
  const uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
  return ((double)m + 0.5) * 0x1p-53;
}

// The two uniforms of call t for (walker, step, half) under key = seed.
__host__ __device__ inline void philox_pair(uint64_t seed, uint32_t walker, uint64_t step, int half, uint32_t t,
                                            double *u0, double *u1) {
  uint32_t c[4] = {walker, (uint32_t)step, ((uint32_t)(step >> 32) & 0x7FFFFFFFu) | ((uint32_t)half << 31), t};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  *u0 = philox_u01(c[0], c[1]);
  *u1 = philox_u01(c[2], c[3]);
}

// Sampled prior: t_c uniform in [t_lo, t_hi], d_L with density d_L^d_exp in
// [d_lo, d_hi] (the other parameters as in sampler_log_prior).
struct SamplerPrior {
  double t_lo, t_hi, d_lo, d_hi, d_exp;
};

// Run state read by the step kernels (device memory, so that one captured
// step graph serves every run): completed steps, the step count when the
// current run began, and where the run's chain samples go.
struct SamplerState {
  uint64_t step, run_start;
  double *chain;       // [12][slots][W] or null
  int64_t slots;
  int32_t thin;
  // annealing: ln L enters the acceptance with the weight
  // beta = beta0^(1 - step / anneal_steps) for step < anneal_steps, else 1
  uint64_t anneal_steps;
  double beta0;
  double beta_fixed;   // >= 0: this ln L weight instead of the schedule (tempered SMC stages)
};

// Target prior of the reweighting: uniform in (m1, m2, chi1, chi2) within
// [lo, hi], distance density d_L^d_exp relative to the sampled one.
struct PriorBox {
  double lo[4], hi[4];
  double d_exp;
};

void launch_sampler_init(const EvalConsts *c, const SamplerPrior &pr, uint64_t seed, int W, double *X, double *lp,
                         hipStream_t s);
void launch_log_prior(const EvalConsts *c, const SamplerPrior &pr, const double *X, int W, double *lp,
                      hipStream_t s);
void launch_de_propose(const SamplerState *st, uint64_t seed, int M, int half, double gamma, double p_jump,
                       const double *X, double *Y, hipStream_t s);
void launch_de_accept(const EvalConsts *c, const SamplerPrior &pr, const SamplerState *st, uint64_t seed, int M,
                      int half, int prior_only, const double *Y, const double *lnl_y, double *X, double *lnl_x,
                      double *lp_x, unsigned long long *acc, hipStream_t s);
void launch_step_advance(SamplerState *st, hipStream_t s);
void launch_gather_walkers(const double *X, const double *lnl, const double *lp, const int32_t *idx, int W,
                           double *Xo, double *lnlo, double *lpo, hipStream_t s);
void launch_fill(double *p, int64_t n, double v, hipStream_t s);
void launch_prior_weights(const EvalConsts *c, const double *params, int64_t ld, int64_t n, const PriorBox &box,
                          double *logw, hipStream_t s);

}  // namespace rbfl
