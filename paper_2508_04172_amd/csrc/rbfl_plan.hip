// Multi-event batches, host side: plans over several handles, their event
// descriptors and work lists (FP64 and split forms), HIP-graph capture,
// per-event digit tuning, the RBFL_DEBUG work-list checks, and the
// rbfl_plan_* and rbfl_eval_ragged entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "host_math.h"
#include "rbfl_internal.h"

namespace rbfl {

// ---- multi-event batches -----------------------------------------------------

struct Plan {
  std::vector<Ctx *> ctx;
  std::vector<int64_t> counts;
  int64_t total = 0;
  const double *params = nullptr;
  double *lnl = nullptr;
  DevBuf<EventDesc> ev_work, ev_param;
  DevBuf<double> Y, Bt;
  int64_t total_groups = 0, max_ldb = 0;
  DevBuf<unsigned long long> counter;
  int64_t total_items = 0;
  int grid = 0;
  int variant = 0;              // FP64 tile variant; -1 for the split form
  double tune_ms[8] = {};
  // split form (RBFL_PLAN_SPLIT): digits per event (caller order), the digit
  // rows and row scales of every event, and the work lists of the events
  // grouped by digit count (one persistent launch per group)
  bool split = false;
  std::vector<int> S;
  DevBuf<int8_t> AS;
  DevBuf<double> rscale;
  int64_t split_threads = 0;
  int n_groups = 0;
  int group_S[4] = {}, group_n[4] = {}, group_off[4] = {}, group_grid[4] = {};
  int64_t group_items[4] = {};
  DevBuf<EventDesc> ev_group;
  int split_tol_state = -1;     // 1: every event within RBFL_SPLIT_TOL of the FP64 plan, 0: not, -1: not tuned
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

// A plan's caller-order descriptors d and its work lists (work order, one
// per group of items): proposal ranges partition [0, total), each event's
// rows of the shared buffers lie inside them without overlap, and every
// work item maps through work_event to a tile inside its event.
static void debug_check_plan(const Plan &p, const std::vector<EventDesc> &d,
                             const std::vector<std::pair<std::vector<EventDesc>, int64_t>> &lists) {
  const int n_ev = (int)d.size();
  int64_t q0 = 0;
  const double *y_end = p.Y.p;
  const double *b_end = p.Bt.p;
  for (int e = 0; e < n_ev; ++e) {
    const EventDesc &x = d[e];
    const Ctx &c = *p.ctx[e];
    debug_require(x.q0 == q0 && x.n == p.counts[e] && x.n >= 1, "proposal ranges");
    debug_require(x.Kp == c.Kp && x.rows == c.rows && x.consts == c.consts.p && x.W == c.W.p, "event constants");
    debug_require(x.Y == y_end && x.Y + x.n * x.Kp <= p.Y.p + p.Y.n, "output rows outside the plan's buffer");
    y_end = x.Y + x.n * x.Kp;
    if (!p.split) {
      debug_require(x.Bt == b_end && x.ldb >= x.n && x.Bt + (int64_t)x.rows * x.ldb <= p.Bt.p + p.Bt.n,
                    "basis rows outside the plan's buffer");
      b_end = x.Bt + (int64_t)x.rows * x.ldb;
    } else {
      const int8_t *as = static_cast<const int8_t *>(x.AS);
      debug_require(x.S >= 5 && x.S <= split_max_slices() && as >= p.AS.p &&
                        as + (int64_t)split_max_slices() * x.rows * x.n <= p.AS.p + p.AS.n &&
                        x.rscale == p.rscale.p + x.q0 && x.q0 + x.n <= (int64_t)p.rscale.n,
                    "digit rows outside the plan's buffers");
    }
    q0 += x.n;
  }
  debug_require(q0 == p.total, "proposal ranges do not cover the batch");
  for (const auto &lw : lists) {
    const std::vector<EventDesc> &w = lw.first;
    const int nw = (int)w.size();
    int64_t next = 0;
    for (int i = 0; i < nw; ++i) {
      debug_require(w[i].item0 == next && w[i].tiles_q >= 1 && w[i].tiles_c >= 1, "work list ranges");
      next += (int64_t)w[i].tiles_q * w[i].tiles_c;
    }
    debug_require(next == lw.second, "work list length");
    for (int64_t item = 0; item < lw.second; ++item) {
      const int e = work_event(w.data(), nw, item);
      const int64_t local = item - w[e].item0;
      debug_require(e >= 0 && e < nw && local >= 0 && local < (int64_t)w[e].tiles_q * w[e].tiles_c,
                    "work item " + std::to_string(item) + " outside its event's tiles");
    }
  }
}

// Event descriptors for tile variant v: caller order (for the epilogue) and
// decreasing-cost order with consecutive work-item ranges (for the persistent
// contraction).  Cost of an event = proposals x (N+M) x K.
static void plan_layout(Plan &p, int v, hipStream_t s) {
  int qt, cw;
  ragged_tile(v, &qt, &cw);
  const int n_ev = (int)p.ctx.size();
  std::vector<EventDesc> d(n_ev);
  int64_t q0 = 0, yoff = 0, boff = 0, rg = 0;
  p.max_ldb = 0;
  for (int e = 0; e < n_ev; ++e) {
    Ctx &c = *p.ctx[e];
    std::memset(&d[e], 0, sizeof(EventDesc));
    d[e].consts = c.consts.p;
    d[e].nodes = c.nodes.p;
    d[e].W = c.W.p;
    d[e].basis = c.basis4.p;
    d[e].Y = p.Y.p + yoff;
    d[e].Bt = p.Bt.p + boff;
    d[e].q0 = q0;
    d[e].n = p.counts[e];
    d[e].ldb = rows_ld(p.counts[e]);
    d[e].rg0 = rg;
    d[e].tiles_q = (int)((p.counts[e] + qt - 1) / qt);
    d[e].tiles_c = c.Kp / cw;
    d[e].Kp = c.Kp;
    d[e].rows = c.rows;
    q0 += p.counts[e];
    yoff += p.counts[e] * c.Kp;
    boff += (int64_t)c.rows * d[e].ldb;
    rg += c.rows / 16;
    p.max_ldb = std::max(p.max_ldb, d[e].ldb);
  }
  p.total_groups = rg;
  std::vector<int> order(n_ev);
  for (int e = 0; e < n_ev; ++e) order[e] = e;
  auto cost = [&](int e) { return (double)p.counts[e] * (p.ctx[e]->N + p.ctx[e]->M) * p.ctx[e]->K; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  std::vector<EventDesc> w(n_ev);
  int64_t item = 0;
  for (int i = 0; i < n_ev; ++i) {
    w[i] = d[order[i]];
    w[i].item0 = item;
    item += (int64_t)w[i].tiles_q * w[i].tiles_c;
  }
  p.total_items = item;
  int dev = 0, cus = 0;
  RBFL_HIP(hipGetDevice(&dev));
  RBFL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  p.grid = (int)std::max<int64_t>(1, std::min<int64_t>(p.total_items, (int64_t)cus * ragged_blocks_per_cu(v)));
  if (debug_mode()) debug_check_plan(p, d, {{w, p.total_items}});
  RBFL_HIP(hipMemcpyAsync(p.ev_work.p, w.data(), sizeof(EventDesc) * n_ev, hipMemcpyHostToDevice, s));
  RBFL_HIP(hipMemcpyAsync(p.ev_param.p, d.data(), sizeof(EventDesc) * n_ev, hipMemcpyHostToDevice, s));
  RBFL_HIP(hipStreamSynchronize(s));
  p.variant = v;
}

// Split-form layout with the digit counts p.S: caller-order descriptors for
// the digit rows and the epilogue, and per digit count a work list of its
// events in decreasing cost with consecutive item ranges.
static void plan_layout_split(Plan &p, hipStream_t s) {
  const int qt = split_ragged_tile_q(), cw = split_ragged_tile_c();
  const int n_ev = (int)p.ctx.size();
  std::vector<EventDesc> d(n_ev);
  int64_t q0 = 0, yoff = 0, aoff = 0, t0 = 0;
  for (int e = 0; e < n_ev; ++e) {
    Ctx &c = *p.ctx[e];
    EventDesc &x = d[e];
    std::memset(&x, 0, sizeof(x));
    x.consts = c.consts.p;
    x.nodes = c.nodes.p;
    x.W = c.W.p;
    x.basis = c.basis4.p;
    x.Y = p.Y.p + yoff;
    x.q0 = q0;
    x.n = p.counts[e];
    x.tiles_q = (int)((p.counts[e] + qt - 1) / qt);
    x.tiles_c = c.Kp / cw;
    x.Kp = c.Kp;
    x.rows = c.rows;
    x.BS = c.WS.p;
    x.cscale = c.WSscale.p;
    x.AS = p.AS.p + aoff;
    x.rscale = p.rscale.p + q0;
    x.S = p.S[e];
    x.t0 = t0;
    q0 += p.counts[e];
    yoff += p.counts[e] * c.Kp;
    aoff += (int64_t)split_max_slices() * c.rows * p.counts[e];
    t0 += (int64_t)(c.rows / 16) * p.counts[e];
  }
  p.split_threads = t0;
  int dev = 0, cus = 0;
  RBFL_HIP(hipGetDevice(&dev));
  RBFL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  auto cost = [&](int e) { return (double)p.counts[e] * (p.ctx[e]->N + p.ctx[e]->M) * p.ctx[e]->K; };
  std::vector<EventDesc> w;
  p.n_groups = 0;
  for (int S = 8; S >= 5; --S) {
    std::vector<int> order;
    for (int e = 0; e < n_ev; ++e)
      if (p.S[e] == S) order.push_back(e);
    if (order.empty()) continue;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    const int g = p.n_groups++;
    p.group_S[g] = S;
    p.group_n[g] = (int)order.size();
    p.group_off[g] = (int)w.size();
    int64_t item = 0;
    for (int e : order) {
      EventDesc x = d[e];
      x.item0 = item;
      item += (int64_t)x.tiles_q * x.tiles_c;
      w.push_back(x);
    }
    p.group_items[g] = item;
    p.group_grid[g] = (int)std::max<int64_t>(1, std::min<int64_t>(item, (int64_t)cus * split_ragged_blocks_per_cu()));
  }
  p.total_items = 0;
  p.grid = 0;
  for (int g = 0; g < p.n_groups; ++g) {
    p.total_items += p.group_items[g];
    p.grid = std::max(p.grid, p.group_grid[g]);
  }
  if (debug_mode()) {
    std::vector<std::pair<std::vector<EventDesc>, int64_t>> lists;
    for (int g = 0; g < p.n_groups; ++g)
      lists.push_back({std::vector<EventDesc>(w.begin() + p.group_off[g], w.begin() + p.group_off[g] + p.group_n[g]),
                       p.group_items[g]});
    debug_check_plan(p, d, lists);
  }
  RBFL_HIP(hipMemcpyAsync(p.ev_param.p, d.data(), sizeof(EventDesc) * n_ev, hipMemcpyHostToDevice, s));
  RBFL_HIP(hipMemcpyAsync(p.ev_group.p, w.data(), sizeof(EventDesc) * n_ev, hipMemcpyHostToDevice, s));
  RBFL_HIP(hipStreamSynchronize(s));
  p.variant = -1;
}

static void plan_run(Plan &p, hipStream_t s) {
  const int n_ev = (int)p.ctx.size();
  if (p.split) {
    launch_ragged_split_rows(p.ev_param.p, n_ev, p.split_threads, p.params, p.total, s);
    launch_zero_counters(p.counter.p, p.n_groups, s);
    for (int g = 0; g < p.n_groups; ++g)
      launch_ragged_split_contract(p.group_S[g], p.ev_group.p + p.group_off[g], p.group_n[g], p.group_items[g],
                                   p.counter.p + g, p.group_grid[g], s);
    launch_ragged_epilogue(p.ev_param.p, n_ev, p.params, p.total, p.lnl, s);
    return;
  }
  if (p.variant < ragged_fused_variants()) {
    launch_ragged_contract(p.variant, p.ev_work.p, n_ev, p.total_items, p.counter.p, p.params, p.total, p.grid, s);
  } else {
    launch_ragged_rows_fp64(p.ev_param.p, n_ev, p.total_groups, p.max_ldb, p.params, p.total, s);
    launch_ragged_gemm_fp64(p.variant - ragged_fused_variants(), p.ev_work.p, n_ev, p.total_items, p.counter.p,
                            p.grid, s);
  }
  launch_ragged_epilogue(p.ev_param.p, n_ev, p.params, p.total, p.lnl, s);
}

}  // namespace rbfl

struct rbfl_plan_ctx {
  rbfl::Plan p;
};

namespace rbfl {
// Captures one launch of the plan into a HIP graph on the plan's own stream.
static void plan_capture(Plan &p) {
  if (!p.cap_stream) RBFL_HIP(hipStreamCreateWithFlags(&p.cap_stream, hipStreamNonBlocking));
  RBFL_HIP(hipStreamBeginCapture(p.cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    plan_run(p, p.cap_stream);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(p.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  RBFL_HIP(hipStreamEndCapture(p.cap_stream, &p.graph));
  RBFL_HIP(hipGraphInstantiate(&p.exec, p.graph, nullptr, nullptr, 0));
}

// Split-form digit counts per event: ln L of the whole batch with every event
// at S = 5 .. 8 digits (each timed, median of 3) against the FP64 plan's.  An
// event with at least kTuneMinValid in-domain proposals takes the fewest
// digits whose ln L stays within RBFL_SPLIT_TOL / 10 of the FP64 form's on
// them (same domain flags; the margin of a decade covers proposals the tuner
// did not see), down to no fewer than 5; with fewer in-domain proposals it
// keeps the default 7 digits unless 7 misses RBFL_SPLIT_TOL.  When no count
// meets RBFL_SPLIT_TOL the most accurate one is kept (split_tol_state then
// says so).
static void plan_tune_split(Plan &p, hipStream_t s) {
  constexpr int64_t kTuneMinValid = 256;
  const int n_ev = (int)p.ctx.size();
  p.split = false;
  plan_layout(p, ragged_fused_variants(), s);
  plan_run(p, s);
  std::vector<double> ref(p.total), got(p.total);
  RBFL_HIP(hipMemcpyAsync(ref.data(), p.lnl, sizeof(double) * p.total, hipMemcpyDeviceToHost, s));
  RBFL_HIP(hipStreamSynchronize(s));
  p.split = true;
  std::vector<std::array<double, 4>> err(n_ev);
  std::vector<int64_t> valid(n_ev, 0);
  {
    int64_t q0 = 0;
    for (int e = 0; e < n_ev; ++e) {
      for (int64_t i = q0; i < q0 + p.counts[e]; ++i) valid[e] += std::isfinite(ref[i]) ? 1 : 0;
      q0 += p.counts[e];
    }
  }
  hipEvent_t e0, e1;
  RBFL_HIP(hipEventCreate(&e0));
  RBFL_HIP(hipEventCreate(&e1));
  for (int v = 0; v < 4; ++v) {
    std::fill(p.S.begin(), p.S.end(), split_variant_slices(v));
    plan_layout_split(p, s);
    plan_run(p, s);
    RBFL_HIP(hipMemcpyAsync(got.data(), p.lnl, sizeof(double) * p.total, hipMemcpyDeviceToHost, s));
    RBFL_HIP(hipStreamSynchronize(s));
    int64_t q0 = 0;
    for (int e = 0; e < n_ev; ++e) {
      double m = 0.0;
      for (int64_t i = q0; i < q0 + p.counts[e]; ++i) {
        if (std::isfinite(ref[i]) != std::isfinite(got[i]) || std::isnan(ref[i]) != std::isnan(got[i])) {
          m = INFINITY;
          break;
        }
        if (std::isfinite(ref[i])) m = std::max(m, std::fabs(got[i] - ref[i]));
      }
      err[e][v] = m;
      q0 += p.counts[e];
    }
    double t[3];
    for (int r = 0; r < 3; ++r) {
      RBFL_HIP(hipEventRecord(e0, s));
      plan_run(p, s);
      RBFL_HIP(hipEventRecord(e1, s));
      RBFL_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      RBFL_HIP(hipEventElapsedTime(&ms, e0, e1));
      t[r] = ms;
    }
    std::sort(t, t + 3);
    p.tune_ms[v] = t[1];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  bool all_ok = true;
  for (int e = 0; e < n_ev; ++e) {
    int pick = -1;
    if (valid[e] >= kTuneMinValid) {
      for (int v = 0; v < 4 && pick < 0; ++v)
        if (err[e][v] <= 0.1 * RBFL_SPLIT_TOL) pick = v;
    }
    if (pick < 0) {
      for (int v = kSplitDefaultVariant; v < 4 && pick < 0; ++v)
        if (err[e][v] <= RBFL_SPLIT_TOL) pick = v;
    }
    if (pick < 0) {
      all_ok = false;
      pick = 3;
      for (int v = 2; v >= 0; --v)
        if (err[e][v] < err[e][pick]) pick = v;
    }
    p.S[e] = split_variant_slices(pick);
  }
  p.split_tol_state = all_ok ? 1 : 0;
}

static rbfl_plan_ctx *plan_create(const rbfl_handle *hs, int n_ev, const int64_t *counts, const double *params,
                                  double *lnl, uint32_t flags, hipStream_t s) {
  require(hs != nullptr && counts != nullptr && params != nullptr && lnl != nullptr, "NULL argument");
  require(n_ev >= 1 && n_ev <= 4096, "n_events must be in 1 .. 4096");
  require((flags & ~(uint32_t)(RBFL_PLAN_GRAPH | RBFL_PLAN_AUTOTUNE | RBFL_PLAN_SPLIT)) == 0, "unknown plan flags");
  std::unique_ptr<rbfl_plan_ctx> pc(new rbfl_plan_ctx());
  Plan &p = pc->p;
  int64_t yelems = 0, belems = 0;
  for (int e = 0; e < n_ev; ++e) {
    require(hs[e] != nullptr, "NULL handle in the event list");
    require(hs[e]->c.n_bands == 1, "multi-event plans cover frozen antenna patterns only (n_bands = 1)");
    require(counts[e] >= 1, "every event needs at least one proposal");
    p.ctx.push_back(&hs[e]->c);
    p.counts.push_back(counts[e]);
    p.total += counts[e];
    yelems += counts[e] * hs[e]->c.Kp;
    belems += (int64_t)hs[e]->c.rows * rows_ld(counts[e]);
  }
  p.params = params;
  p.lnl = lnl;
  p.ev_work.alloc(n_ev);
  p.ev_param.alloc(n_ev);
  p.Y.alloc((size_t)yelems);
  p.Bt.alloc((size_t)belems);
  p.counter.alloc(4);
  if (flags & RBFL_PLAN_SPLIT) {
    int64_t aelems = 0;
    for (int e = 0; e < n_ev; ++e) {
      prepare(*p.ctx[e], RBFL_FORM_SPLIT);
      aelems += (int64_t)split_max_slices() * p.ctx[e]->rows * counts[e];
    }
    p.AS.alloc((size_t)aelems);
    p.rscale.alloc((size_t)p.total);
    p.ev_group.alloc(n_ev);
    p.S.assign(n_ev, split_variant_slices(kSplitDefaultVariant));
    if (flags & RBFL_PLAN_AUTOTUNE) {
      plan_tune_split(p, s);
    } else {
      for (int e = 0; e < n_ev; ++e) p.S[e] = split_variant_slices(p.ctx[e]->variant[RBFL_FORM_SPLIT]);
    }
    p.split = true;
    plan_layout_split(p, s);
    p.Bt.reset();        // the FP64 basis rows served only the tuner's reference
  } else if (flags & RBFL_PLAN_AUTOTUNE) {
    hipEvent_t e0, e1;
    RBFL_HIP(hipEventCreate(&e0));
    RBFL_HIP(hipEventCreate(&e1));
    int best = 0;
    double best_ms = 1e300;
    for (int v = 0; v < ragged_variants() && v < 8; ++v) {
      plan_layout(p, v, s);
      plan_run(p, s);
      double t[3];
      for (int r = 0; r < 3; ++r) {
        RBFL_HIP(hipEventRecord(e0, s));
        plan_run(p, s);
        RBFL_HIP(hipEventRecord(e1, s));
        RBFL_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        RBFL_HIP(hipEventElapsedTime(&ms, e0, e1));
        t[r] = ms;
      }
      std::sort(t, t + 3);
      p.tune_ms[v] = t[1];
      if (t[1] < best_ms) {
        best_ms = t[1];
        best = v;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan_layout(p, best, s);
  } else {
    plan_layout(p, ragged_fused_variants(), s);
  }
  if (flags & RBFL_PLAN_GRAPH) plan_capture(p);
  return pc.release();
}

// Pins the FP64 tile variant of a plan: new layout, and a new graph if the
// plan has one.
static void plan_set_variant(Plan &p, int v, hipStream_t s) {
  if (p.split) throw Error(RBFL_E_STATE, "a split-form plan has no FP64 tile variants");
  require(v >= 0 && v < ragged_variants(), "variant out of range");
  RBFL_HIP(hipStreamSynchronize(s));
  plan_layout(p, v, s);
  if (p.exec) {
    (void)hipGraphExecDestroy(p.exec);
    (void)hipGraphDestroy(p.graph);
    p.exec = nullptr;
    p.graph = nullptr;
    plan_capture(p);
  }
}
}  // namespace rbfl

extern "C" {

int32_t rbfl_plan_create(const rbfl_handle *hs, int32_t n_events, const int64_t *counts, const double *params,
                         double *lnl, uint32_t flags, void *stream, rbfl_plan *out) {
  return rbfl::guarded([&] {
    rbfl::require(out != nullptr, "out is NULL");
    *out = nullptr;
    *out = rbfl::plan_create(hs, n_events, counts, params, lnl, flags, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_plan_launch(rbfl_plan plan, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(plan != nullptr, "plan is NULL");
    rbfl::Plan &p = plan->p;
    if (p.exec)
      RBFL_HIP(hipGraphLaunch(p.exec, reinterpret_cast<hipStream_t>(stream)));
    else
      rbfl::plan_run(p, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_plan_query(rbfl_plan plan, double *out, size_t bytes) {
  return rbfl::guarded([&] {
    rbfl::require(plan != nullptr, "plan is NULL");
    const rbfl::Plan &p = plan->p;
    double v[16] = {(double)p.variant, (double)p.total_items, (double)p.grid, (double)p.total};
    for (int i = 0; i < 8; ++i) v[4 + i] = p.tune_ms[i];
    v[12] = p.split ? 1.0 : 0.0;
    v[13] = p.split ? (double)*std::min_element(p.S.begin(), p.S.end()) : 0.0;
    v[14] = p.split ? (double)*std::max_element(p.S.begin(), p.S.end()) : 0.0;
    v[15] = (double)p.split_tol_state;
    rbfl::require(out != nullptr && bytes >= 12 * sizeof(double), "output buffer too small (need at least 96 bytes)");
    std::memcpy(out, v, std::min(bytes, sizeof(v)));
  });
}

int32_t rbfl_plan_set_variant(rbfl_plan plan, int32_t variant, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(plan != nullptr, "plan is NULL");
    rbfl::plan_set_variant(plan->p, variant, reinterpret_cast<hipStream_t>(stream));
  });
}

int32_t rbfl_plan_destroy(rbfl_plan plan) {
  return rbfl::guarded([&] { delete plan; });
}

int32_t rbfl_eval_ragged(const rbfl_handle *hs, int32_t n_events, const int64_t *counts, const double *params,
                         double *lnl, void *stream) {
  return rbfl::guarded([&] {
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::unique_ptr<rbfl_plan_ctx> hold(rbfl::plan_create(hs, n_events, counts, params, lnl, 0u, s));
    rbfl::plan_run(hold->p, s);
    RBFL_HIP(hipStreamSynchronize(s));
  });
}


}  // extern "C"
