// Ensemble sampler and prior reweighting: device-side state and launchers
// (sampler.hip).
#pragma once

#include "rbfl_internal.h"

namespace rbfl {

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
void launch_fill(double *p, int64_t n, double v, hipStream_t s);
void launch_prior_weights(const EvalConsts *c, const double *params, int64_t ld, int64_t n, const PriorBox &box,
                          double *logw, hipStream_t s);

}  // namespace rbfl
