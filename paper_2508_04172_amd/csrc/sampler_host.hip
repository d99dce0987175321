// GPU-resident ensemble sampler, host side: sampler state, the captured
// step graph, tempered SMC start, queries, prior reweighting, and the
// rbfl_sampler_* and rbfl_prior_weights entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "host_math.h"
#include "rbfl_internal.h"
#include "sampler.h"

struct rbfl_sampler_ctx {
  rbfl::Ctx *c = nullptr;
  rbfl_sampler_spec spec{};
  rbfl::SamplerPrior prior{};
  int W = 0, M = 0;
  double gamma = 0.0;
  rbfl::DevBuf<double> X, Y, lnl_x, lnl_y, lp_x;
  rbfl::DevBuf<unsigned long long> acc;
  rbfl::DevBuf<rbfl::SamplerState> st;
  rbfl::SamplerState stage{};   // host copy staged for the next run
  uint64_t steps = 0;
  double beta_fixed = -1.0;     // ln L weight after a tempered SMC start (1), -1 = the spec's schedule
  uint32_t smc_stages = 0;      // stages run so far (the resampling draws' counter)
  hipStream_t cap = nullptr, last = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~rbfl_sampler_ctx() {
    if (c && exec) c->graph_users -= 1;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace rbfl {
// One sampler step: for each half, proposals, their ln L through the online
// stage (the handle's work space, reserved beforehand), the Metropolis
// decisions; then the step counter.
static void sampler_step(rbfl_sampler_ctx &S, hipStream_t s) {
  const bool prior_only = S.spec.flags & RBFL_SAMPLER_PRIOR_ONLY;
  for (int half = 0; half < 2; ++half) {
    launch_de_propose(S.st.p, S.spec.seed, S.M, half, S.gamma, S.spec.p_jump, S.X.p, S.Y.p, s);
    if (!prior_only) eval(*S.c, S.Y.p, S.M, S.lnl_y.p, S.spec.form, s);
    launch_de_accept(S.c->consts.p, S.prior, S.st.p, S.spec.seed, S.M, half, prior_only ? 1 : 0, S.Y.p, S.lnl_y.p,
                     S.X.p, S.lnl_x.p, S.lp_x.p, S.acc.p, s);
  }
  launch_step_advance(S.st.p, s);
}

static rbfl_sampler_ctx *sampler_create(Ctx &c, const rbfl_sampler_spec *sp, const double *init, hipStream_t s) {
  require(sp != nullptr, "spec is NULL");
  const rbfl_sampler_spec &p = *sp;
  require(p.walkers >= 8 && p.walkers % 2 == 0 && p.walkers <= (1 << 30), "walkers must be even, 8 .. 2^30");
  require(p.form >= 0 && p.form <= RBFL_FORM_SURROGATE, "unknown form");
  require(c.prepared[p.form], "form not prepared (call rbfl_prepare)");
  require(p.t_lo < p.t_hi && std::isfinite(p.t_lo) && std::isfinite(p.t_hi), "need t_lo < t_hi");
  require(p.d_lo > 0.0 && p.d_lo < p.d_hi && std::isfinite(p.d_hi), "need 0 < d_lo < d_hi");
  require(std::isfinite(p.d_exp) && p.d_exp > -1.0, "d_exp must be finite and > -1");
  require(p.gamma >= 0.0 && std::isfinite(p.gamma), "gamma must be >= 0");
  require(p.p_jump >= 0.0 && p.p_jump <= 1.0, "p_jump must be in 0 .. 1");
  require((p.flags & ~RBFL_SAMPLER_PRIOR_ONLY) == 0, "unknown sampler flag bits");
  require(p.anneal_steps >= 0, "anneal_steps must be >= 0");
  require(p.anneal_steps == 0 || (p.beta0 > 0.0 && p.beta0 <= 1.0), "beta0 must be in (0, 1]");
  std::unique_ptr<rbfl_sampler_ctx> S(new rbfl_sampler_ctx());
  S->c = &c;
  S->spec = p;
  S->prior = SamplerPrior{p.t_lo, p.t_hi, p.d_lo, p.d_hi, p.d_exp};
  S->W = p.walkers;
  S->M = p.walkers / 2;
  S->gamma = p.gamma > 0.0 ? p.gamma : 2.38 / sqrt(22.0);
  const int64_t W = S->W, M = S->M;
  S->X.alloc(11 * W);
  S->Y.alloc(11 * M);
  S->lnl_x.alloc(W);
  S->lnl_y.alloc(M);
  S->lp_x.alloc(W);
  S->acc.alloc(W);
  S->st.alloc(1);
  RBFL_HIP(hipMemsetAsync(S->acc.p, 0, sizeof(unsigned long long) * W, s));
  if (init) {
    RBFL_HIP(hipMemcpyAsync(S->X.p, init, sizeof(double) * 11 * W, hipMemcpyDeviceToDevice, s));
    launch_log_prior(c.consts.p, S->prior, S->X.p, S->W, S->lp_x.p, s);
  } else {
    launch_sampler_init(c.consts.p, S->prior, p.seed, S->W, S->X.p, S->lp_x.p, s);
  }
  const bool prior_only = p.flags & RBFL_SAMPLER_PRIOR_ONLY;
  if (prior_only) {
    launch_fill(S->lnl_x.p, W, 0.0, s);
  } else {
    reserve(c, std::min<int64_t>(std::max<int64_t>(M, 1), 1 << 20));
    eval(c, S->X.p, W, S->lnl_x.p, p.form, s);
  }
  S->stage = SamplerState{0, 0, nullptr, 0, 1, (uint64_t)p.anneal_steps, p.beta0, -1.0};
  RBFL_HIP(hipMemcpyAsync(S->st.p, &S->stage, sizeof(SamplerState), hipMemcpyHostToDevice, s));
  RBFL_HIP(hipStreamSynchronize(s));
  // capture one step (profiling off: no events inside the graph)
  const bool prof = c.profile;
  c.profile = false;
  RBFL_HIP(hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking));
  RBFL_HIP(hipStreamBeginCapture(S->cap, hipStreamCaptureModeThreadLocal));
  try {
    sampler_step(*S, S->cap);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(S->cap, &g);
    if (g) (void)hipGraphDestroy(g);
    c.profile = prof;
    throw;
  }
  c.profile = prof;
  RBFL_HIP(hipStreamEndCapture(S->cap, &S->graph));
  RBFL_HIP(hipGraphInstantiate(&S->exec, S->graph, nullptr, nullptr, 0));
  S->last = s;
  c.graph_users += 1;
  return S.release();
}

static void sampler_run(rbfl_sampler_ctx &S, int64_t steps, int thin, double *chain, int64_t slots, hipStream_t s) {
  require(steps >= 0, "steps must be >= 0");
  require(thin >= 1, "thin must be >= 1");
  require(chain == nullptr || slots >= 1, "chain needs slots >= 1");
  if (S.last && S.last != s) RBFL_HIP(hipStreamSynchronize(S.last));
  // the staged state is read by an asynchronous copy: let the previous one finish
  RBFL_HIP(hipStreamSynchronize(s));
  S.stage = SamplerState{S.steps, S.steps, chain, chain ? slots : 0, thin, (uint64_t)S.spec.anneal_steps,
                         S.spec.beta0, S.beta_fixed};
  RBFL_HIP(hipMemcpyAsync(S.st.p, &S.stage, sizeof(SamplerState), hipMemcpyHostToDevice, s));
  for (int64_t i = 0; i < steps; ++i) RBFL_HIP(hipGraphLaunch(S.exec, s));
  S.steps += (uint64_t)steps;
  S.last = s;
}

// Tempered sequential Monte Carlo from the current walkers (Del Moral, Doucet
// and Jasra 2006), taking them as prior draws (weight beta = 0): per stage
// the increment db in (0, 1 - beta] whose weights w = L^db keep an effective
// sample size of ess_frac W (the whole remainder when that stays above),
// found by 60 bisection halvings; ln Z += log mean w; systematic resampling
// at positions (u + i) / W, u = Philox(walker 2^32 - 1, step = stage index,
// half 1, call 4); then `moves` sampler steps at the new beta.
static void sampler_smc(rbfl_sampler_ctx &S, double ess_frac, int moves, int max_stages, hipStream_t s,
                        double *log_z, int32_t *stages_out, double *beta_out) {
  require(!(S.spec.flags & RBFL_SAMPLER_PRIOR_ONLY), "a prior-only sampler has no likelihood to temper");
  require(ess_frac > 0.0 && ess_frac < 1.0, "ess_frac must be in (0, 1)");
  require(moves >= 1 && max_stages >= 1, "moves and max_stages must be >= 1");
  if (S.last && S.last != s) RBFL_HIP(hipStreamSynchronize(S.last));
  const int W = S.W;
  std::vector<double> l(W), w(W), cum(W);
  std::vector<int32_t> idx(W);
  DevBuf<int32_t> d_idx;
  d_idx.alloc(W);
  DevBuf<double> Xt, lt, pt;
  Xt.alloc((size_t)11 * W);
  lt.alloc(W);
  pt.alloc(W);
  double beta = 0.0, lz = 0.0;
  int st = 0;
  for (; st < max_stages && beta < 1.0; ++st) {
    RBFL_HIP(hipMemcpyAsync(l.data(), S.lnl_x.p, sizeof(double) * W, hipMemcpyDeviceToHost, s));
    RBFL_HIP(hipStreamSynchronize(s));
    double m = -std::numeric_limits<double>::infinity();
    for (double v : l)
      if (std::isfinite(v)) m = std::max(m, v);
    require(std::isfinite(m), "no walker has a finite ln L");
    auto ess = [&](double db) {
      Sum s1, s2;
      for (int i = 0; i < W; ++i) {
        const double e = std::isfinite(l[i]) ? exp(db * (l[i] - m)) : 0.0;
        s1.add(e);
        s2.add(e * e);
      }
      return s1.value() * s1.value() / s2.value();
    };
    const double rem = 1.0 - beta;
    double db = rem;
    if (ess(rem) < ess_frac * W) {
      double lo = 0.0, hi = rem;
      for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (ess(mid) >= ess_frac * W)
          lo = mid;
        else
          hi = mid;
      }
      db = lo;
    }
    double c = 0.0;
    Sum tot;
    for (int i = 0; i < W; ++i) {
      w[i] = std::isfinite(l[i]) ? exp(db * (l[i] - m)) : 0.0;
      c += w[i];
      cum[i] = c;
      tot.add(w[i]);
    }
    lz += db * m + log(tot.value() / W);
    for (int i = 0; i < W; ++i) cum[i] /= c;
    double u = 0.0, unused = 0.0;
    philox_pair(S.spec.seed, 0xFFFFFFFFu, S.smc_stages, 1, 4, &u, &unused);
    int j = 0;
    for (int i = 0; i < W; ++i) {
      const double pos = (u + (double)i) / (double)W;
      while (j < W - 1 && cum[j] <= pos) ++j;
      idx[i] = j;
    }
    RBFL_HIP(hipMemcpyAsync(d_idx.p, idx.data(), sizeof(int32_t) * W, hipMemcpyHostToDevice, s));
    launch_gather_walkers(S.X.p, S.lnl_x.p, S.lp_x.p, d_idx.p, W, Xt.p, lt.p, pt.p, s);
    RBFL_HIP(hipMemcpyAsync(S.X.p, Xt.p, sizeof(double) * 11 * W, hipMemcpyDeviceToDevice, s));
    RBFL_HIP(hipMemcpyAsync(S.lnl_x.p, lt.p, sizeof(double) * W, hipMemcpyDeviceToDevice, s));
    RBFL_HIP(hipMemcpyAsync(S.lp_x.p, pt.p, sizeof(double) * W, hipMemcpyDeviceToDevice, s));
    beta = std::min(1.0, beta + db);
    if (rem - db <= 0.0) beta = 1.0;
    S.smc_stages += 1;
    S.beta_fixed = beta;
    sampler_run(S, moves, 1, nullptr, 0, s);
  }
  RBFL_HIP(hipStreamSynchronize(s));
  if (log_z) *log_z = lz;
  if (stages_out) *stages_out = st;
  if (beta_out) *beta_out = beta;
}

static void sampler_query(rbfl_sampler_ctx &S, int what, double *out, size_t bytes) {
  require(out != nullptr, "out is NULL");
  if (S.last) RBFL_HIP(hipStreamSynchronize(S.last));
  const size_t W = (size_t)S.W;
  switch (what) {
    case 0: {
      require(bytes >= sizeof(double) * 12 * W, "buffer too small");
      RBFL_HIP(hipMemcpy(out, S.X.p, sizeof(double) * 11 * W, hipMemcpyDeviceToHost));
      RBFL_HIP(hipMemcpy(out + 11 * W, S.lnl_x.p, sizeof(double) * W, hipMemcpyDeviceToHost));
      return;
    }
    case 1:
    case 2: {
      std::vector<unsigned long long> a(W);
      RBFL_HIP(hipMemcpy(a.data(), S.acc.p, sizeof(unsigned long long) * W, hipMemcpyDeviceToHost));
      if (what == 1) {
        require(bytes >= sizeof(double) * W, "buffer too small");
        for (size_t i = 0; i < W; ++i) out[i] = (double)a[i];
      } else {
        require(bytes >= sizeof(double) * 2, "buffer too small");
        double tot = 0.0;
        for (auto v : a) tot += (double)v;
        out[0] = (double)S.steps;
        out[1] = S.steps ? tot / ((double)S.steps * (double)W) : 0.0;
      }
      return;
    }
    default:
      throw Error(RBFL_E_INVALID_ARG, "unknown sampler query");
  }
}

static void prior_weights(Ctx &c, const double *params, int64_t ld, int64_t n, const double box[8], double d_exp,
                          double *logw, double *n_eff, hipStream_t s) {
  require(params != nullptr && logw != nullptr && box != nullptr, "NULL argument");
  require(n >= 0 && ld >= n, "need 0 <= n <= ld");
  require(std::isfinite(d_exp), "d_exp must be finite");
  PriorBox b;
  for (int d = 0; d < 4; ++d) {
    b.lo[d] = box[2 * d];
    b.hi[d] = box[2 * d + 1];
    require(b.lo[d] <= b.hi[d], "box bounds must satisfy lo <= hi");
  }
  b.d_exp = d_exp;
  launch_prior_weights(c.consts.p, params, ld, n, b, logw, s);
  if (n_eff) {
    std::vector<double> w((size_t)n);
    RBFL_HIP(hipMemcpyAsync(w.data(), logw, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    RBFL_HIP(hipStreamSynchronize(s));
    double mx = -std::numeric_limits<double>::infinity();
    for (double v : w) mx = std::max(mx, v);
    Sum s1, s2;
    if (std::isfinite(mx))
      for (double v : w) {
        const double e = exp(v - mx);
        s1.add(e);
        s2.add(e * e);
      }
    *n_eff = s2.value() > 0.0 ? s1.value() * s1.value() / s2.value() : 0.0;
  }
}
}  // namespace rbfl

extern "C" {

int32_t rbfl_sampler_create(rbfl_handle h, const rbfl_sampler_spec *spec, const double *init, void *stream,
                            rbfl_sampler *out) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr && out != nullptr, "NULL argument");
    *out = nullptr;
    *out = rbfl::sampler_create(h->c, spec, init, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_sampler_run(rbfl_sampler s, int64_t steps, int32_t thin, double *chain, int64_t slots, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(s != nullptr, "sampler is NULL");
    rbfl::sampler_run(*s, steps, thin, chain, slots, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_sampler_smc(rbfl_sampler s, double ess_frac, int32_t moves, int32_t max_stages, void *stream,
                         double *log_evidence, int32_t *stages, double *beta) {
  return rbfl::guarded([&] {
    rbfl::require(s != nullptr, "sampler is NULL");
    rbfl::sampler_smc(*s, ess_frac, moves, max_stages, reinterpret_cast<hipStream_t>(stream), log_evidence, stages,
                      beta);
  });
}

int32_t rbfl_sampler_query(rbfl_sampler s, int32_t what, double *out, size_t bytes) {
  return rbfl::guarded([&] {
    rbfl::require(s != nullptr, "sampler is NULL");
    rbfl::sampler_query(*s, what, out, bytes);
  });
}

int32_t rbfl_sampler_destroy(rbfl_sampler s) {
  return rbfl::guarded([&] {
    if (s && s->last) (void)hipStreamSynchronize(s->last);
    delete s;
  });
}

int32_t rbfl_prior_weights(rbfl_handle h, const double *params, int64_t ld, int64_t n, const double box[8],
                           double d_exp, double *logw, double *n_eff, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::prior_weights(h->c, params, ld, n, box, d_exp, logw, n_eff, reinterpret_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
