// Online stage of the rbfl C ABI (Sec. II D): work space, the contraction of
// every arithmetic form, the evaluation orders (serial chunks, pipelined
// chunks, ln L finished inside the FP64 or split contraction), interpolated
// outputs, the reduced forms' weight preparation and the autotuner that picks
// tiles, digit counts and orders.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "rbfl_internal.h"

namespace rbfl {

// Work space of the orders that finish ln L inside the contraction (FP64 or
// split), for n proposals; allocated on first use of either (and grown with
// the rest): one partial sum per proposal and column tile of the narrower of
// the two tiles.
static void reserve_lnl_gemm(Ctx &c, int64_t n) {
  c.epi_su.alloc(epi_setup_bytes() * (size_t)n);
  c.epi_part.alloc((size_t)(c.Kp / std::min(gemm_lnl_col_tile(), split_col_tile())) * n);
}

void reserve(Ctx &c, int64_t n) {
  if (n <= c.cap) return;
  if (c.graph_users > 0) throw Error(RBFL_E_STATE, "the work space is captured by a sampler: it cannot grow");
  c.Y.alloc((size_t)n * c.Kp);
  c.Bt.alloc((size_t)c.rows * rows_ld(n));
  if (c.epi_su.p) reserve_lnl_gemm(c, n);
  c.cap = n;
  if (c.prepared[RBFL_FORM_BF16]) c.A16.alloc((size_t)c.rows * n);
  if (c.prepared[RBFL_FORM_SPLIT]) {
    c.AS.alloc((size_t)split_max_slices() * n * c.rows);
    c.ASscale.alloc(n);
  }
  if (c.sur) {
    c.sur_x.alloc((size_t)n * 4);
    if (c.sur_nbase) c.sur_U.alloc((size_t)n * c.sur_nbase);
    c.sur->reserve(n);
  }
}

static void contract(Ctx &c, const double *params, int64_t ld, int64_t b0, int64_t nb, int form, hipStream_t s,
                     hipEvent_t *marks = nullptr);

// True when `s` is being captured into a graph (or its capture state cannot
// be read): the pipelined order forks onto a second stream, so such calls
// keep the serial order.
static bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return st != hipStreamCaptureStatusNone;
}

// Pipelined FP64 evaluation of proposals [0, n) (leading dimension ld): the
// basis rows and MFMA product of each chunk run on the caller's stream, its
// epilogue on the handle's side stream, so that the epilogue of chunk i
// (bound by memory latency) runs under the product of chunk i + 1 (bound by
// the matrix cores).  Chunks alternate between the two halves of the work
// space; the product of chunk i + 2 waits for the epilogue of chunk i, and the
// caller's stream waits for the last epilogues before the call returns.  Every
// proposal goes through the same arithmetic as in the serial order, so ln L
// is bit-identical.
static void eval_pipelined(Ctx &c, const double *params, int64_t ld, int64_t n, double *lnl, hipStream_t s) {
  const int64_t half = (c.cap / 2) & ~int64_t(7);
  int64_t ch = (n + c.pipe - 1) / c.pipe;
  ch = std::min(half, (ch + 7) & ~int64_t(7));
  if (!c.side) {
    RBFL_HIP(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking));
    for (int h = 0; h < 2; ++h) {
      RBFL_HIP(hipEventCreateWithFlags(&c.pev_prod[h], hipEventDisableTiming));
      RBFL_HIP(hipEventCreateWithFlags(&c.pev_epi[h], hipEventDisableTiming));
    }
  }
  const int v = c.variant[RBFL_FORM_FP64];
  const bool two_stage = v < gemm_fp64_variants();
  int i = 0;
  for (int64_t b0 = 0; b0 < n; b0 += ch, ++i) {
    const int64_t nb = std::min(ch, n - b0);
    const int h = i & 1;
    double *Y = c.Y.p + (size_t)h * half * c.Kp;
    double *Bt = c.Bt.p + (size_t)h * c.rows * half;
    hipEvent_t ev[6];
    auto mark = [&](int k, hipStream_t st) {
      if (c.profile) RBFL_HIP(hipEventRecord(ev[k], st));
    };
    if (c.profile)
      for (auto &e : ev) {
        RBFL_HIP(hipEventCreate(&e));
        c.timed_events.push_back(e);
      }
    mark(0, s);
    if (two_stage) launch_rows_fp64(c.consts.p, c.host_consts, params, ld, b0, nb, c.nodes.p, Bt, s);
    mark(1, s);
    if (i >= 2) RBFL_HIP(hipStreamWaitEvent(s, c.pev_epi[h], 0));
    mark(2, s);
    if (two_stage) launch_gemm_fp64(Bt, nb, c.host_consts, c.W.p, Y, s, v);
    else launch_contract_fp64(c.consts.p, c.host_consts, params, ld, b0, nb, c.nodes.p, c.W.p, Y, s, 2);
    mark(3, s);
    RBFL_HIP(hipEventRecord(c.pev_prod[h], s));
    RBFL_HIP(hipStreamWaitEvent(c.side, c.pev_prod[h], 0));
    mark(4, c.side);
    launch_epilogue(c.consts.p, c.host_consts, params, ld, b0, nb, Y, c.basis4.p, lnl, c.side);
    mark(5, c.side);
    RBFL_HIP(hipEventRecord(c.pev_epi[h], c.side));
    if (c.profile) {
      if (two_stage) c.timed.push_back(Ctx::Timed{ev[0], ev[1], 2, nb});
      c.timed.push_back(Ctx::Timed{ev[2], ev[3], 0, nb});
      c.timed.push_back(Ctx::Timed{ev[4], ev[5], 1, nb});
    }
  }
  for (int h = 0; h < std::min(i, 2); ++h) RBFL_HIP(hipStreamWaitEvent(s, c.pev_epi[h], 0));
}

// FP64 evaluation with ln L finished inside the contraction: per chunk the
// proposals' setups and basis rows, the contraction that weights its output
// tile by the setups' coefficients and writes one partial sum per proposal
// and column tile, and their compensated sum (see k_gemm_lnl_fp64).
static void eval_lnl_gemm(Ctx &c, const double *params, int64_t ld, int64_t n, double *lnl, hipStream_t s) {
  const int n_ct = c.Kp / gemm_lnl_col_tile();
  if (!c.epi_su.p) {
    if (capturing(s)) throw Error(RBFL_E_STATE, "work space of the fused epilogue not allocated (evaluate once before capture)");
    reserve_lnl_gemm(c, c.cap);
  }
  for (int64_t b0 = 0; b0 < n; b0 += c.cap) {
    const int64_t nb = std::min(c.cap, n - b0);
    hipEvent_t ev[4];
    auto mark = [&](int k) {
      if (c.profile) RBFL_HIP(hipEventRecord(ev[k], s));
    };
    if (c.profile)
      for (auto &e : ev) {
        RBFL_HIP(hipEventCreate(&e));
        c.timed_events.push_back(e);
      }
    mark(0);
    launch_epi_setup(c.consts.p, params, ld, b0, nb, c.epi_su.p, s);
    launch_rows_fp64(c.consts.p, c.host_consts, params, ld, b0, nb, c.nodes.p, c.Bt.p, s);
    mark(1);
    launch_gemm_lnl_fp64(c.Bt.p, nb, c.host_consts, c.W.p, c.consts.p, c.epi_su.p, c.basis4.p, c.coldesc.p,
                         c.epi_part.p, c.cap, s);
    mark(2);
    launch_lnl_tiles(c.epi_su.p, b0, nb, c.epi_part.p, c.cap, n_ct, lnl, s);
    mark(3);
    if (c.profile) {
      // stages: setups + basis rows (kind 2), contraction with the weighting
      // (kind 0), sum of the tile partials (kind 1)
      c.timed.push_back(Ctx::Timed{ev[0], ev[1], 2, nb});
      c.timed.push_back(Ctx::Timed{ev[1], ev[2], 0, nb});
      c.timed.push_back(Ctx::Timed{ev[2], ev[3], 1, nb});
    }
  }
}

// The split form with ln L finished inside its contraction, chunk by chunk.
static void eval_split_lnl(Ctx &c, const double *params, int64_t ld, int64_t n, double *lnl, hipStream_t s) {
  const int n_ct = c.Kp / split_col_tile();
  if (!c.epi_su.p) {
    if (capturing(s)) throw Error(RBFL_E_STATE, "work space of the fused epilogue not allocated (evaluate once before capture)");
    reserve_lnl_gemm(c, c.cap);
  }
  for (int64_t b0 = 0; b0 < n; b0 += c.cap) {
    const int64_t nb = std::min(c.cap, n - b0);
    hipEvent_t ev[4];
    if (c.profile)
      for (auto &e : ev) {
        RBFL_HIP(hipEventCreate(&e));
        c.timed_events.push_back(e);
      }
    if (c.profile) RBFL_HIP(hipEventRecord(ev[0], s));
    launch_epi_setup(c.consts.p, params, ld, b0, nb, c.epi_su.p, s);
    launch_split_lnl(c.consts.p, c.host_consts, params, ld, b0, nb, c.nodes.p, c.AS.p, c.ASscale.p, c.WS.p,
                     c.WSscale.p, c.epi_su.p, c.basis4.p, c.coldesc.p, c.epi_part.p, c.cap, s,
                     c.variant[RBFL_FORM_SPLIT], c.profile ? ev[1] : nullptr);
    if (c.profile) RBFL_HIP(hipEventRecord(ev[2], s));
    launch_lnl_tiles(c.epi_su.p, b0, nb, c.epi_part.p, c.cap, n_ct, lnl, s);
    if (c.profile) {
      RBFL_HIP(hipEventRecord(ev[3], s));
      // stages: setups + digit rows (kind 2), contraction with the weighting
      // (kind 0), sum of the tile partials (kind 1)
      c.timed.push_back(Ctx::Timed{ev[0], ev[1], 2, nb});
      c.timed.push_back(Ctx::Timed{ev[1], ev[2], 0, nb});
      c.timed.push_back(Ctx::Timed{ev[2], ev[3], 1, nb});
    }
  }
}

// ln L of proposals [0, n) of a parameter array with leading dimension ld.
static void eval_range(Ctx &c, const double *params, int64_t ld, int64_t n, double *lnl, int form, hipStream_t s) {
  if (n == 0) return;
  if (c.cap == 0) reserve(c, std::min<int64_t>(n, 65536));
  const bool fp64 = form == RBFL_FORM_FP64 || (form == RBFL_FORM_SURROGATE && !(c.sur && c.sur_ok));
  if (fp64 && c.lnl_gemm) {
    eval_lnl_gemm(c, params, ld, n, lnl, s);
    return;
  }
  if (form == RBFL_FORM_SPLIT && c.split_lnl) {
    eval_split_lnl(c, params, ld, n, lnl, s);
    return;
  }
  if (fp64 && c.pipe > 1 && c.cap / 2 >= 4096 && n > 4096 && !capturing(s)) {
    eval_pipelined(c, params, ld, n, lnl, s);
    return;
  }
  for (int64_t b0 = 0; b0 < n; b0 += c.cap) {
    const int64_t nb = std::min(c.cap, n - b0);
    if (c.profile) {
      // stages: basis rows (kind 2), MFMA contraction (kind 0), epilogue (kind 1)
      hipEvent_t ev[4];
      for (auto &e : ev) {
        RBFL_HIP(hipEventCreate(&e));
        c.timed_events.push_back(e);
      }
      contract(c, params, ld, b0, nb, form, s, ev);
      launch_epilogue(c.consts.p, c.host_consts, params, ld, b0, nb, c.Y.p, c.basis4.p, lnl, s);
      RBFL_HIP(hipEventRecord(ev[3], s));
      c.timed.push_back(Ctx::Timed{ev[0], ev[1], 2, nb});
      c.timed.push_back(Ctx::Timed{ev[1], ev[2], 0, nb});
      c.timed.push_back(Ctx::Timed{ev[2], ev[3], 1, nb});
      continue;
    }
    contract(c, params, ld, b0, nb, form, s);
    launch_epilogue(c.consts.p, c.host_consts, params, ld, b0, nb, c.Y.p, c.basis4.p, lnl, s);
  }
}

void eval(Ctx &c, const double *params, int64_t n, double *lnl, int form, hipStream_t s) {
  require(params != nullptr && lnl != nullptr, "params/lnl is NULL");
  require(n >= 0, "n must be >= 0");
  if (form < 0 || form > RBFL_FORM_SURROGATE) throw Error(RBFL_E_INVALID_ARG, "unknown form");
  if (!c.prepared[form]) throw Error(RBFL_E_STATE, "form not prepared (call rbfl_prepare)");
  eval_range(c, params, n, n, lnl, form, s);
  launch_count_nan(lnl, n, c.nan_part.p, s);
}

// The contraction of proposals [b0, b0 + nb) into the work space Y, in two
// stages where the form has them (basis rows, then the MFMA product); marks,
// when given, are recorded before, between and after the stages.
static void contract(Ctx &c, const double *params, int64_t ld, int64_t b0, int64_t nb, int form, hipStream_t s,
                     hipEvent_t *marks) {
  auto mark = [&](int i) {
    if (marks) RBFL_HIP(hipEventRecord(marks[i], s));
  };
  auto fp64 = [&]() {
    const int v = c.variant[RBFL_FORM_FP64];
    if (v < gemm_fp64_variants()) {
      launch_rows_fp64(c.consts.p, c.host_consts, params, ld, b0, nb, c.nodes.p, c.Bt.p, s);
      mark(1);
      launch_gemm_fp64(c.Bt.p, nb, c.host_consts, c.W.p, c.Y.p, s, v);
    } else {
      mark(1);
      launch_contract_fp64(c.consts.p, c.host_consts, params, ld, b0, nb, c.nodes.p, c.W.p, c.Y.p, s, 2);
    }
  };
  mark(0);
  switch (form) {
    case RBFL_FORM_FP64:
      fp64();
      break;
    case RBFL_FORM_FP32:
      mark(1);
      launch_contract_fp32(c.consts.p, c.host_consts, params, ld, b0, nb, c.nodes.p, c.W32.p, c.Y.p, s,
                           c.variant[form]);
      break;
    case RBFL_FORM_SPLIT:
      launch_contract_split(c.consts.p, c.host_consts, params, ld, b0, nb, c.nodes.p, c.AS.p, c.ASscale.p, c.WS.p,
                            c.WSscale.p, c.Y.p, s, c.variant[form], marks ? marks[1] : nullptr);
      break;
    case RBFL_FORM_SURROGATE:
      if (c.sur && c.sur_ok) {
        launch_sur_inputs(params, ld, b0, nb, c.consts.p, c.sur_x.p, s);
        if (c.sur_nbase)
          launch_sur_base_inputs(params, ld, b0, nb, c.consts.p, c.sur_ms_d.p, c.sur_poly.p, c.sur_nbase, c.sur_U.p,
                                 s);
        mark(1);
        c.sur->infer(c.sur_x.p, nb, c.sur_mu.p, c.sur_sd.p, c.Y.p, c.Kp, s, c.sur_nbase ? c.sur_U.p : nullptr,
                     c.sur_nbase ? c.sur_B.p : nullptr, c.sur_nbase);
      } else {
        fp64();
      }
      break;
    default:
      launch_contract_bf16(c.consts.p, c.host_consts, params, ld, b0, nb, c.nodes.p, c.A16.p, c.W16.p, c.Y.p, s,
                           marks ? marks[1] : nullptr);
  }
  mark(2);
}

void interp(Ctx &c, const double *params, int64_t n, double *out, int form, hipStream_t s) {
  require(params != nullptr && out != nullptr, "params/out is NULL");
  require(n >= 0, "n must be >= 0");
  if (form < 0 || form > RBFL_FORM_SURROGATE) throw Error(RBFL_E_INVALID_ARG, "unknown form");
  if (!c.prepared[form]) throw Error(RBFL_E_STATE, "form not prepared (call rbfl_prepare)");
  if (n == 0) return;
  if (c.cap == 0) reserve(c, std::min<int64_t>(n, 65536));
  for (int64_t b0 = 0; b0 < n; b0 += c.cap) {
    const int64_t nb = std::min(c.cap, n - b0);
    contract(c, params, n, b0, nb, form, s);
    RBFL_HIP(hipMemcpy2DAsync(out + b0 * c.K, sizeof(double) * c.K, c.Y.p, sizeof(double) * c.Kp,
                              sizeof(double) * c.K, nb, hipMemcpyDeviceToDevice, s));
  }
}

// Times every contraction tile variant of `form` on the first min(n, work
// capacity) proposals of `params` (HIP events, median of 3 after a warm-up)
// and keeps the fastest for later rbfl_eval/rbfl_interp calls.
// ln L of the first nb proposals with the current variant of `form`, to host.
static std::vector<double> lnl_probe(Ctx &c, const double *params, int64_t n, int64_t nb, int form, double *dev,
                                     hipStream_t s) {
  contract(c, params, n, 0, nb, form, s);
  launch_epilogue(c.consts.p, c.host_consts, params, n, 0, nb, c.Y.p, c.basis4.p, dev, s);
  std::vector<double> h(nb);
  RBFL_HIP(hipMemcpyAsync(h.data(), dev, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  RBFL_HIP(hipStreamSynchronize(s));
  return h;
}

void autotune(Ctx &c, const double *params, int64_t n, int form, hipStream_t s) {
  require(params != nullptr && n >= 1, "autotune needs proposals");
  if (form < 0 || form > RBFL_FORM_SPLIT) throw Error(RBFL_E_INVALID_ARG, "unknown or untunable form");
  if (!c.prepared[form]) throw Error(RBFL_E_STATE, "form not prepared (call rbfl_prepare)");
  if (c.cap == 0) reserve(c, std::min<int64_t>(n, 65536));
  const int64_t nb = std::min(c.cap, n);
  const int nv = contract_variants(form);
  // The split form's slice count sets its accuracy: a variant is eligible
  // only if its ln L stays within split_tol of the FP64 form's on these
  // proposals (same domain flags, finite entries compared).
  std::vector<double> ref;
  DevBuf<double> probe;
  if (form == RBFL_FORM_SPLIT) {
    probe.alloc(nb);
    ref = lnl_probe(c, params, n, nb, RBFL_FORM_FP64, probe.p, s);
  }
  hipEvent_t e0, e1;
  RBFL_HIP(hipEventCreate(&e0));
  RBFL_HIP(hipEventCreate(&e1));
  int best = -1;
  double best_ms = 1e300;
  // accuracy of each split variant, and one warm-up launch of every variant
  bool eligible[8];
  for (int v = 0; v < nv && v < 8; ++v) {
    c.variant[form] = v;
    eligible[v] = true;
    if (form == RBFL_FORM_SPLIT) {
      const std::vector<double> got = lnl_probe(c, params, n, nb, form, probe.p, s);
      double err = 0.0;
      for (int64_t i = 0; i < nb; ++i) {
        if (std::isfinite(ref[i]) != std::isfinite(got[i]) || std::isnan(ref[i]) != std::isnan(got[i])) {
          err = INFINITY;
          break;
        }
        if (std::isfinite(ref[i])) err = std::max(err, std::fabs(got[i] - ref[i]));
      }
      c.split_err[v] = err;
      eligible[v] = err <= c.split_tol;
    }
    contract(c, params, n, 0, nb, form, s);
  }
  // two interleaved rounds of three timed launches per variant (so that no
  // variant is timed alone while the clocks settle); keep each variant's
  // smaller round median
  double med[8];
  for (int v = 0; v < 8; ++v) med[v] = 1e300;
  for (int round = 0; round < 2; ++round)
    for (int v = 0; v < nv && v < 8; ++v) {
      c.variant[form] = v;
      double t[3];
      for (int r = 0; r < 3; ++r) {
        RBFL_HIP(hipEventRecord(e0, s));
        contract(c, params, n, 0, nb, form, s);
        RBFL_HIP(hipEventRecord(e1, s));
        RBFL_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        RBFL_HIP(hipEventElapsedTime(&ms, e0, e1));
        t[r] = ms;
      }
      std::sort(t, t + 3);
      med[v] = std::min(med[v], t[1]);
    }
  for (int v = 0; v < nv && v < 8; ++v) {
    c.tune_ms[form][v] = med[v];
    if (eligible[v] && med[v] < best_ms) {
      best_ms = med[v];
      best = v;
    }
  }
  // FP64 GEMM tiles within 3% of the fastest time: keep the one whose larger
  // workgroup tile re-reads the least (the difference is within run-to-run
  // noise, about 2-3% between launches of the same tile; the bandwidth saved,
  // up to 3x, is not)
  if (form == RBFL_FORM_FP64 && best >= 0 && best < gemm_fp64_variants()) {
    for (int v = 0; v < gemm_fp64_variants() && v < nv && v < 8; ++v)
      if (med[v] <= 1.03 * best_ms && gemm_fp64_reuse(v) > gemm_fp64_reuse(best)) best = v;
  }
  if (best < 0) {
    // no split variant within split_tol: keep the most accurate one
    // (ties to more digits) and leave split_ok false for RBFL_Q_SPLIT_STATE
    best = 0;
    for (int v = 1; v < nv && v < 8; ++v)
      if (c.split_err[v] <= c.split_err[best]) best = v;
  }
  if (form == RBFL_FORM_SPLIT) {
    c.split_tuned = true;
    c.split_ok = eligible[best];
  }
  c.variant[form] = best;
  // FP64: with the chosen tile, time whole evaluations of the nb proposals in
  // 1 (serial), 2, 4 and 8 pipelined chunks and keep the fastest
  if (form == RBFL_FORM_FP64 && c.cap / 2 >= 4096 && nb > 4096 && !capturing(s)) {
    static const int depths[4] = {1, 2, 4, 8};
    DevBuf<double> out;
    out.alloc(nb);
    const bool prof = c.profile;
    c.profile = false;
    double pm[4] = {1e300, 1e300, 1e300, 1e300};
    for (int round = 0; round < 2; ++round)
      for (int d = 0; d < 4; ++d) {
        c.pipe = depths[d];
        if (round == 0) eval_range(c, params, n, nb, out.p, form, s);
        double t[3];
        for (int r = 0; r < 3; ++r) {
          RBFL_HIP(hipEventRecord(e0, s));
          eval_range(c, params, n, nb, out.p, form, s);
          RBFL_HIP(hipEventRecord(e1, s));
          RBFL_HIP(hipEventSynchronize(e1));
          float ms = 0.0f;
          RBFL_HIP(hipEventElapsedTime(&ms, e0, e1));
          t[r] = ms;
        }
        std::sort(t, t + 3);
        pm[d] = std::min(pm[d], t[1]);
      }
    // a pipelined order must beat the serial one by 3% (the spread of these
    // timings between runs is 2-3%, and the overlap slows each kernel it
    // runs beside): otherwise the serial order is kept
    int bd = 0;
    for (int d = 1; d < 4; ++d)
      if (pm[d] < 0.97 * pm[0] && pm[d] < pm[bd]) bd = d;
    c.pipe = depths[bd];
    for (int d = 0; d < 4; ++d) c.pipe_ms[d] = pm[d];
    // then ln L finished inside the contraction, kept if 1% faster still
    // (frozen patterns only: its per-proposal setup has one arrival time per
    // detector)
    c.lnl_gemm = c.n_bands == 1;
    double fm = 1e300;
    for (int round = 0; round < 2 && c.lnl_gemm; ++round) {
      if (round == 0) eval_range(c, params, n, nb, out.p, form, s);
      double t[3];
      for (int r = 0; r < 3; ++r) {
        RBFL_HIP(hipEventRecord(e0, s));
        eval_range(c, params, n, nb, out.p, form, s);
        RBFL_HIP(hipEventRecord(e1, s));
        RBFL_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        RBFL_HIP(hipEventElapsedTime(&ms, e0, e1));
        t[r] = ms;
      }
      std::sort(t, t + 3);
      fm = std::min(fm, t[1]);
    }
    c.lnl_gemm_ms = fm < 1e300 ? fm : 0.0;
    c.lnl_gemm = fm < 0.99 * pm[bd];
    if (c.lnl_gemm) {
      c.pipe = 1;
    } else if (c.graph_users == 0 && !c.split_lnl) {
      // its work space is not kept for an order not chosen (unless a captured
      // sampler step may be using it)
      RBFL_HIP(hipStreamSynchronize(s));
      c.epi_su.reset();
      c.epi_part.reset();
    }
    c.profile = prof;
    RBFL_HIP(hipStreamSynchronize(s));
  }
  // split form: with the chosen digit count, time whole evaluations with the
  // separate epilogue and with ln L finished inside the contraction (frozen
  // patterns only) and keep the latter if 1% faster
  if (form == RBFL_FORM_SPLIT && c.n_bands == 1 && nb > 4096 && !capturing(s)) {
    DevBuf<double> out;
    out.alloc(nb);
    const bool prof = c.profile;
    c.profile = false;
    double om[2] = {1e300, 1e300};
    for (int round = 0; round < 2; ++round)
      for (int o = 0; o < 2; ++o) {
        c.split_lnl = o == 1;
        if (round == 0) eval_range(c, params, n, nb, out.p, form, s);
        double t[3];
        for (int r = 0; r < 3; ++r) {
          RBFL_HIP(hipEventRecord(e0, s));
          eval_range(c, params, n, nb, out.p, form, s);
          RBFL_HIP(hipEventRecord(e1, s));
          RBFL_HIP(hipEventSynchronize(e1));
          float ms = 0.0f;
          RBFL_HIP(hipEventElapsedTime(&ms, e0, e1));
          t[r] = ms;
        }
        std::sort(t, t + 3);
        om[o] = std::min(om[o], t[1]);
      }
    c.split_order_ms[0] = om[0];
    c.split_order_ms[1] = om[1];
    c.split_lnl = om[1] < 0.99 * om[0];
    RBFL_HIP(hipStreamSynchronize(s));
    if (!c.split_lnl && !c.lnl_gemm && c.graph_users == 0) {
      c.epi_su.reset();
      c.epi_part.reset();
    }
    c.profile = prof;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

void prepare(Ctx &c, int form) {
  if (form < 0 || form > RBFL_FORM_SPLIT) throw Error(RBFL_E_INVALID_ARG, "unknown form");
  if (c.prepared[form]) return;
  const size_t n = (size_t)c.rows * c.Kp;
  if (form == RBFL_FORM_BF16) {
    c.W16.alloc(n);
    launch_bf16_prepare(c.W.p, c.rows, c.Kp, c.W16.p, 0);
    // the chunk buffer follows the work space (reserve allocates it for a prepared form)
    if (c.cap > 0) c.A16.alloc((size_t)c.rows * c.cap);
    RBFL_HIP(hipDeviceSynchronize());
    c.prepared[RBFL_FORM_BF16] = true;
    return;
  }
  if (form == RBFL_FORM_SPLIT) {
    if (c.rows > split_max_rows())
      throw Error(RBFL_E_UNSUPPORTED, "the split form needs N + M <= " + std::to_string(split_max_rows()));
    c.WS.alloc((size_t)split_max_slices() * c.Kp * c.rows);
    c.WSscale.alloc(c.Kp);
    launch_split_prepare(c.W.p, c.rows, c.Kp, c.WSscale.p, c.WS.p, 0);
    if (c.cap > 0) {
      c.AS.alloc((size_t)split_max_slices() * c.cap * c.rows);
      c.ASscale.alloc(c.cap);
    }
    RBFL_HIP(hipDeviceSynchronize());
    c.variant[RBFL_FORM_SPLIT] = kSplitDefaultVariant;
    c.prepared[RBFL_FORM_SPLIT] = true;
    return;
  }
  if (!c.W32.p) c.W32.alloc(n);
  launch_convert_weights(c.W.p, n, c.W32.p, nullptr, 0);
  RBFL_HIP(hipDeviceSynchronize());
  c.prepared[RBFL_FORM_FP32] = true;
}

}  // namespace rbfl
