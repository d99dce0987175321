// Internal declarations of the rbfl library: handle layout, the constant
// block the online kernels read, and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rbfl.h"
#include "rbfl_math.h"

namespace rbfl {

constexpr int kMaxPoly = 35;     // monomials of degree <= 3 in 4 variables
constexpr int kSplineTaps = 10;  // samples in the sub-sample spline stencil
constexpr int kRowChunk = 32;    // W rows padded to a multiple of this (every row step divides it)
constexpr int kColTile = 128;    // widest contraction column tile; K is padded to a multiple of it
constexpr double kAutoEpsCond = 1e12;   // automatic shape parameter: largest accepted 1-norm condition
constexpr double kAutoEpsMax = 8.0;     // ... and the largest integer shape parameter tried

// Error carrying an rbfl_status through the host code; converted at the ABI.
struct Error : std::runtime_error {
  int32_t code;
  Error(int32_t c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char *what);
#define RBFL_HIP(x) ::rbfl::hip_check((x), #x)

inline void require(bool ok, const std::string &msg) {
  if (!ok) throw Error(RBFL_E_INVALID_ARG, msg);
}

// Thread-local text behind rbfl_last_error().
extern thread_local std::string g_last_error;

// Runs f and converts what it throws into an rbfl_status (no exception
// crosses the C ABI).
template <class F>
int32_t guarded(F &&f) {
  try {
    f();
    g_last_error.clear();
    return RBFL_OK;
  } catch (const Error &e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return RBFL_E_OUT_OF_MEMORY;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return RBFL_E_DEVICE;
  } catch (...) {
    g_last_error = "unknown failure";
    return RBFL_E_DEVICE;
  }
}

// Everything the online-stage kernels read, resident in device memory (one
// copy per handle, read through a pointer so handles never share state).
struct EvalConsts {
  int n_det, n_modes, N, M, K, Kp, rows;   // rows = N + M padded to kRowChunk
  int q, T, half_w, degree;
  int poly_idx[kMaxPoly][3];                // variable indices of each monomial, -1 = unused
  double eps2, fs, t_trig, d_ref, f0, chi_max;
  double f_ref;                             // template time/phase reference frequency (0: coalescence)
  double earth_rate;                        // Earth rotation [rad/s] in the exact likelihood (0: frozen)
  double theta_c[4], V[16], semi[4];        // V row-major: Theta_i = theta_c_i + sum_j V[i][j] de_j
  double D[RBFL_MAX_DET][9], r[RBFL_MAX_DET][3];
  // blocks of interpolated outputs: detector k (frozen patterns, n_bands = 1)
  // or (detector k, band b) as block v = k n_bands + b (time bands)
  int n_bands, n_v;
  int coef_off[RBFL_MAX_BLOCKS][RBFL_MAX_MODES], sig_off[RBFL_MAX_BLOCKS];
  double band_t[RBFL_MAX_BANDS][RBFL_MAX_MODES];   // time of each (band, mode) relative to t_c
  int mode_l[RBFL_MAX_MODES], mode_m[RBFL_MAX_MODES];
  YlmTerms ylm_neg[RBFL_MAX_MODES];         // -2Y_{l,-m}
  YlmTerms ylm_pos[RBFL_MAX_MODES];         // -2Y_{l,m}
  double spline[kSplineTaps][4];            // w_s(f) = sum_p spline[s][p] f^p
};

// One event of a multi-event batch, as the persistent kernels read it.
struct EventDesc {
  const EvalConsts *consts;
  const double *nodes;
  const double *W;
  const double2 *basis;         // spline-folded basis [pair][T][q][4]
  double *Y;           // this event's rows of the shared work space, [n][Kp]
  double *Bt;          // this event's basis rows (rows + GEMM variants), [rows][ldb]
  int64_t q0, n;       // first proposal (column of the concatenated params) and count
  int64_t item0;       // first work item of this event (work order)
  int64_t ldb;         // leading dimension of Bt
  int64_t rg0;         // first 16-row group of this event in the row kernel's grid
  int tiles_q, tiles_c, Kp, rows;
  // split form (plans with RBFL_PLAN_SPLIT)
  const void *BS;        // the handle's weight digits [8][rows/16][Kp], 16 int8 per entry
  const double *cscale;  // the handle's power-of-two column scales [Kp]
  void *AS;              // this event's row digits [S][rows/16][n], 16 int8 per entry
  double *rscale;        // this event's power-of-two row scales [n]
  int S;                 // digits per value (5 .. 8)
  int64_t t0;            // first thread of this event in the digit-row kernel's flat grid
};

// The event of work item `item` in a work list (events in work order, each
// with the first item of its consecutive range): the last event whose first
// item is <= item.  The persistent kernels and the host's bounds check
// (RBFL_DEBUG) share it.
__host__ __device__ inline int work_event(const EventDesc *ev, int n_ev, int64_t item) {
  int e = 0;
  while (e + 1 < n_ev && ev[e + 1].item0 <= item) ++e;
  return e;
}

template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    reset();
    if (count == 0) return;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw Error(RBFL_E_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    n = count;
  }
};

// Surrogate network in -> H -> H -> out (SiLU), FP32 parameters and Adam
// state on the device (mlp.hip).
struct Mlp {
  int in = 0, hid = 0, out = 0;
  int64_t np = 0, o_w1 = 0, o_b1 = 0, o_w2 = 0, o_b2 = 0, o_w3 = 0, o_b3 = 0;
  DevBuf<float> p, g, m, v;
  DevBuf<float> Z1, H1, Z2, H2, Yb, dY, dA, dB;
  DevBuf<double> part, loss;
  int64_t cap = 0;
  int t = 0;
  void init(int n_in, int hidden, int n_out, const double *normals);
  void reserve(int64_t B);
  void forward(const float *X, int64_t B, float *Y, hipStream_t s);
  // inference into the interpolant's output layout: Y[b][c] = mu[c] + sd[c] y[b][c]
  // in FP64 (row stride ldy) for c < out, y as forward() computes it; no
  // pre-activations stored
  // (residual form: plus the FP64 base sum_j Ub[b][j] Bb[j][c], Bb [nbase][out])
  void infer(const float *X, int64_t B, const float *mu, const float *sd, double *Y, int64_t ldy, hipStream_t s,
             const double *Ub = nullptr, const double *Bb = nullptr, int nbase = 0);
  void loss_grad(const float *X, const float *T, int64_t B, hipStream_t s);   // loss -> this->loss
  void adam(double lr, double b1, double b2, double eps, hipStream_t s);
};

// Partial counts of NaN ln L values of the last evaluation call (one per
// block of the counting kernel, summed by rbfl_query).
constexpr int kNanParts = 256;

struct Ctx {
  int device = 0;              // the device current at rbfl_build / rbfl_load; every artefact lives there
  // sizes and scalars
  int n_det = 0, n_modes = 0;
  int n_bands = 1, n_v = 0;    // time bands of the antenna patterns; output blocks n_det * n_bands
  std::vector<int64_t> band_edges;   // [n_bands + 1] bin index of each band's first bin, then the end
  int modes[RBFL_MAX_MODES][2] = {};
  int N = 0, M = 0, K = 0, Kp = 0, rows = 0, q = 0, T = 0, half_w = 0, degree = 0;
  int64_t n_s = 0, n_f = 0;
  double fs = 0, seg_len = 0, f_low = 0, df = 0;
  double eps = 0, chi_max = 1, t_trig = 0, d_ref = 0, match = 0;
  double f_ref = 0;            // template time/phase reference frequency (0: coalescence)
  double earth_rate = 0;       // Earth rotation [rad/s] in the exact likelihood and the injection
  double squeeze[2] = {1, 0};  // factor applied to the longest semi-axis, true match at its new tip
  double centre_opt[6] = {};   // centre used (m1, m2, chi1, chi2) and the optimiser's iota, phi
  double centre_snr[2] = {};   // network SNR at the given centre (iota = phi = 0) and at the optimum
  // frame
  double theta_c[4] = {}, V[16] = {}, lam[4] = {}, semi[4] = {}, metric[16] = {};
  double D[RBFL_MAX_DET][9] = {}, r[RBFL_MAX_DET][3] = {};
  // host-side artefacts kept for export
  std::vector<double> x_nodes, phys_nodes, node_values, singular;
  double cond = 0;
  double timing[8] = {};
  // device artefacts
  DevBuf<EvalConsts> consts;
  DevBuf<double> nodes;        // [rows][4] unit-ball coordinates, zero-padded
  DevBuf<double> W;            // [rows][Kp] RBF weights, zero-padded
  DevBuf<double2> basis;       // [n_v][n_modes][T][q]
  DevBuf<double2> basis4;      // spline-folded basis [n_v][n_modes][T][q][4]
  DevBuf<double2> z_nodes;     // [n_v][n_modes][N][T] (kept for export)
  DevBuf<double2> brute_D;     // exact ln L: 4 df d_k / S_k over bins j_lo .. n_s/2 - 1, [n_det][brute_J]
  DevBuf<double> brute_w;      // exact ln L: 4 df / S_k, [n_det][brute_J]
  int64_t brute_j_lo = 0, brute_J = 0;
  DevBuf<double2> win_D;       // exact outputs: brute_D with the window start's phase, made on first use
  DevBuf<int4> coldesc;        // output column layout (kind, detector, mode, index), [K]
  DevBuf<unsigned long long> nan_part;   // [kNanParts] NaN counts of the last evaluation call
  // reduced-precision weight copies
  DevBuf<float> W32;           // [rows][Kp]
  DevBuf<uint16_t> W16;        // BF16 form: weights in 8-row groups [rows/8][Kp][8]
  DevBuf<uint16_t> A16;        // BF16 form: kernel rows of one chunk [rows/8][cap][8]
  DevBuf<int8_t> WS;           // split form: weight slices [S][Kp][rows]
  DevBuf<double> WSscale;      // split form: power-of-two column scales [Kp]
  DevBuf<int8_t> AS;           // split form: kernel-row slices of one chunk [S][cap][rows]
  DevBuf<double> ASscale;      // split form: power-of-two row scales of one chunk [cap]
  bool prepared[5] = {true, false, false, false, true};
  int variant[5] = {0, 0, 0, 0, 0};   // contraction tile variant per form (rbfl_autotune)
  double tune_ms[5][8] = {};          // last autotune timings per variant
  double split_err[8] = {};           // last split autotune: max |d ln L| vs the FP64 form per variant
  bool split_tuned = false;           // the split form's digit count was chosen by rbfl_autotune
  bool split_ok = false;              // last split autotune found a variant within split_tol
  double split_tol = RBFL_SPLIT_TOL;  // the split autotune's bar against the FP64 form (rbfl_set_split_tol)
  // work space
  DevBuf<double> Y;            // [cap][Kp]
  DevBuf<double> Bt;           // FP64 basis rows of one chunk [rows][rows_ld(cap)]
  // ln L finished inside the FP64 contraction (rbfl_fuse_epilogue bit 0) and
  // inside the split contraction (bit 1)
  bool lnl_gemm = false;
  double lnl_gemm_ms = 0.0;           // the autotuner's time per evaluation of that order
  bool split_lnl = false;
  double split_order_ms[2] = {};      // the split autotune's ms per evaluation: separate epilogue, fused
  DevBuf<unsigned char> epi_su;       // per-proposal setups [cap]
  DevBuf<double> epi_part;            // partial sums per column tile [Kp / tile][cap]
  int64_t cap = 0;
  int graph_users = 0;         // live samplers whose captured step uses Y / Bt / the weight copies
  // pipelined FP64 evaluation (rbfl_pipeline): chunks per call (1 = serial),
  // the side stream that runs the epilogues, per work-space half the events
  // "product done" and "epilogue done", and the autotuner's timings
  int pipe = 1;
  double pipe_ms[4] = {};
  hipStream_t side = nullptr;
  hipEvent_t pev_prod[2] = {nullptr, nullptr}, pev_epi[2] = {nullptr, nullptr};
  EvalConsts host_consts;
  // surrogate (rbfl_surrogate_train)
  Mlp *sur = nullptr;
  DevBuf<float> sur_mu, sur_sd;       // per-column standardisation of the outputs
  DevBuf<float> sur_x;                // work space [cap][4]
  bool sur_ok = false;                // held-out check passed
  // residual form: FP64 least-squares polynomial base of degree sur_degree in
  // the training set's standardised coordinates u = (x - m) / s
  int sur_degree = 0, sur_nbase = 0;
  double sur_ms[8] = {};              // m[4], s[4]
  DevBuf<double> sur_ms_d;            // the same on the device
  DevBuf<int> sur_poly;               // [kMaxPoly][3] variable indices of the base monomials
  DevBuf<double> sur_B;               // [nbase][K] base coefficients
  DevBuf<double> sur_U;               // work space [cap][nbase] monomials of a chunk
  double sur_stats[8] = {};
  // optional per-launch timing (rbfl_profile)
  bool profile = false;
  struct Timed {
    hipEvent_t a, b;
    int kind;          // 0 MFMA contraction, 1 epilogue, 2 basis rows
    int64_t n;         // proposals in the launch
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> timed_events;   // owned by the handle until the stats are read
  void drop_timed() {
    for (auto e : timed_events) (void)hipEventDestroy(e);
    timed_events.clear();
    timed.clear();
  }
  ~Ctx() {
    delete sur;
    drop_timed();
    for (auto e : pev_prod)
      if (e) (void)hipEventDestroy(e);
    for (auto e : pev_epi)
      if (e) (void)hipEventDestroy(e);
    if (side) (void)hipStreamDestroy(side);
  }
};

// RBFL_DEBUG host-side bounds checks (rbfl_host.hip)
bool debug_mode();
void debug_check_layout(const Ctx &c);
void debug_require(bool ok, const std::string &what);   // RBFL_E_STATE "RBFL_DEBUG: what" unless ok

// Online-stage operations of a handle (rbfl_eval.hip), shared by the host
// files: reduced-precision weights of a form, work space for n proposals, a
// batched evaluation in a form, the interpolated outputs, and the autotuner
// (rbfl_prepare, rbfl_reserve, rbfl_eval, rbfl_interp, rbfl_autotune).
void prepare(Ctx &c, int form);
void reserve(Ctx &c, int64_t n);
void eval(Ctx &c, const double *params, int64_t n, double *lnl, int form, hipStream_t s);
void interp(Ctx &c, const double *params, int64_t n, double *out, int form, hipStream_t s);
void autotune(Ctx &c, const double *params, int64_t n, int form, hipStream_t s);
// The surrogate's training driver (surrogate_host.hip, rbfl_surrogate_train)
// and the artefact export (rbfl_query.hip, rbfl_query).
void surrogate_train(Ctx &c, const rbfl_train_spec *sp, hipStream_t s);
void query(Ctx &c, int what, void *out, size_t bytes);

// ---- start-up kernels (build_kernels.hip) ----
void launch_waveforms(const Binary *bins, int nb, const int *mode_lm, int n_modes, int64_t j_lo, int J,
                      double df, double inv_dref_s, double2 *out, hipStream_t s);
void launch_sigma(const double2 *A, int nb, int n_modes, int J, int j0, int j1, const double *wk, int n_det,
                  int64_t det_stride, int node_base, double2 *sig, hipStream_t s);
// Bin-range splits of the windowed DFT for nb nodes, T taps and len bins:
// enough to fill the GPU, none shorter than 256 bins.
int window_dft_splits(int nb, int T, int64_t len);
void launch_window_dft(const double2 *A_mode, int nb, int J_mode, int J_stride, const double2 *Dk, int64_t j_lo,
                       int64_t n_s, int T, int n_split, double2 *partial, hipStream_t s);
void launch_reduce_splits(const double2 *partial, int n_split, int nb, int T, double2 *Z_rows, hipStream_t s);
void launch_brute(const EvalConsts *c, const double *params, int64_t ld, int64_t n, const double2 *Dd,
                  const double *wk, int64_t j_lo, int64_t J, int64_t n_s, double df, double inv_dref_s, double *lnl,
                  hipStream_t s);
void launch_proposal_bins(const EvalConsts *c, const double *params, int64_t ld, int64_t b0, int nb, Binary *bins,
                          hipStream_t s);
void launch_rotate_band(const double2 *D, int n_det, int64_t J, int64_t j_lo, int64_t n0, int64_t n_s,
                        double2 *out, hipStream_t s);
void launch_outputs_rows(const double2 *C, const double2 *sig, const int4 *coldesc, int nb, int K, int Kp, int q,
                         int n_modes, double *Y, hipStream_t s);
void launch_series_lnl(const EvalConsts *c, const double *params, int64_t ld, int64_t b0, int64_t nb,
                       const double2 *Z, const double2 *sig, double *lnl, hipStream_t s);
void launch_fold_spline(const double2 *B, int n_pairs, int T, int q, const EvalConsts *c, double2 *B4,
                        hipStream_t s);
void launch_basis_from_u(const double2 *U, int T, int ldu, int q, double2 *B, hipStream_t s);
void launch_coeffs(const double2 *Z, const double2 *B, int N, int T, int q, double2 *C, hipStream_t s);
void launch_assemble_rhs(const double2 *C, const double2 *sig, const int4 *coldesc, int N, int K, int NM,
                         int q, int n_modes, double *R, hipStream_t s);
void launch_assemble_system(const double *x, int N, int M, const int *poly_idx, double eps2, double *A,
                            hipStream_t s);
void launch_residual_dd(const double *A, const double *rhs, const double *W, int NM, int K, double *res,
                        hipStream_t s);
void launch_add(double *y, const double *x, int64_t n, hipStream_t s);
void launch_transpose_weights(const double *R, int NM, int K, int rows, int Kp, double *W, hipStream_t s);

// ---- online kernels (eval_kernels.hip) ----
int contract_variants(int form);
const char *contract_variant_name(int form, int variant);
// ---- FP64 rows + GEMM (contract_fp64.hip) ----
int64_t rows_ld(int64_t n);
int gemm_fp64_variants();
const char *gemm_fp64_variant_name(int variant);
double gemm_fp64_reuse(int variant);
void launch_rows_fp64(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                      int64_t nb, const double *nodes, double *Bt, hipStream_t s);
void launch_gemm_fp64(const double *Bt, int64_t nb, const EvalConsts &hc, const double *W, double *Y, hipStream_t s,
                      int variant);
void launch_contract_fp64(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld,
                          int64_t b0, int64_t nb, const double *nodes, const double *W, double *Y,
                          hipStream_t s, int variant);
void launch_contract_fp32(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld,
                          int64_t b0, int64_t nb, const double *nodes, const float *W, double *Y, hipStream_t s,
                          int variant);
void launch_bf16_prepare(const double *W, int rows, int Kp, uint16_t *WB, hipStream_t s);
void launch_contract_bf16(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                          int64_t nb, const double *nodes, uint16_t *AB, const uint16_t *WB, double *Y,
                          hipStream_t s, hipEvent_t mid);
int ragged_variants();
int ragged_fused_variants();          // variants below this use the fused persistent kernel
int ragged_blocks_per_cu(int variant);
void launch_ragged_rows_fp64(const EventDesc *ev, int n_ev, int64_t total_groups, int64_t max_ldb,
                             const double *params, int64_t ld, hipStream_t s);
void launch_ragged_gemm_fp64(int variant, const EventDesc *ev, int n_ev, int64_t total_items,
                             unsigned long long *counter, int grid, hipStream_t s);
void ragged_tile(int variant, int *proposals_per_tile, int *columns_per_tile);
void launch_ragged_contract(int variant, const EventDesc *ev, int n_ev, int64_t total_items,
                            unsigned long long *counter, const double *params, int64_t ld, int grid, hipStream_t s);
void launch_ragged_epilogue(const EventDesc *ev, int n_ev, const double *params, int64_t total, double *lnl,
                            hipStream_t s);
void launch_epilogue(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                     int64_t nb, const double *Y, const double2 *basis, double *lnl, hipStream_t s);
// Epilogue inside the FP64 contraction: per-proposal setups (epi_setup_bytes()
// each), the contraction's partial sums part[column tile][ldp], their sum.
size_t epi_setup_bytes();
int gemm_lnl_col_tile();
void launch_epi_setup(const EvalConsts *c, const double *params, int64_t ld, int64_t b0, int64_t nb, void *setups,
                      hipStream_t s);
void launch_gemm_lnl_fp64(const double *Bt, int64_t nb, const EvalConsts &hc, const double *W, const EvalConsts *c,
                          const void *setups, const double2 *basis4, const int4 *coldesc, double *part, int64_t ldp,
                          hipStream_t s);
void launch_lnl_tiles(const void *setups, int64_t b0, int64_t nb, const double *part, int64_t ldp, int n_ct,
                      double *lnl, hipStream_t s);
// multi-event split form: tile shape of the persistent contraction, its
// resident workgroups per CU, the digit rows of every event in one launch,
// the persistent contraction over the work list of events with S digits, and
// a kernel that zeroes n <= 64 work counters
int split_ragged_tile_q();
int split_ragged_tile_c();
int split_ragged_blocks_per_cu();
void launch_ragged_split_rows(const EventDesc *ev, int n_ev, int64_t total_threads, const double *params, int64_t ld,
                              hipStream_t s);
void launch_ragged_split_contract(int S, const EventDesc *ev, int n_ev, int64_t total_items,
                                  unsigned long long *counter, int grid, hipStream_t s);
void launch_zero_counters(unsigned long long *counter, int n, hipStream_t s);
int split_max_slices();
int split_max_rows();
int split_variant_count();
int split_variant_slices(int variant);
const char *split_variant_name(int variant);
constexpr int kSplitDefaultVariant = 2;    // 7 base-254 digits: within a few units of FP64 rounding
void launch_split_prepare(const double *W, int rows, int Kp, double *scale, int8_t *BS, hipStream_t s);
void launch_contract_split(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                           int64_t nb, const double *nodes, int8_t *AS, double *rscale, const int8_t *BS,
                           const double *scale, double *Y, hipStream_t s, int variant, hipEvent_t mid);
// The split form with ln L finished inside its contraction (frozen patterns):
// digit rows, then one partial sum per proposal and split_col_tile()-column
// tile into part[tile][ldp] from the setups of launch_epi_setup; mid, when
// given, is recorded between the two.
int split_col_tile();
void launch_split_lnl(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                      int64_t nb, const double *nodes, int8_t *AS, double *rscale, const int8_t *BS,
                      const double *cscale, const void *setups, const double2 *basis4, const int4 *coldesc,
                      double *part, int64_t ldp, hipStream_t s, int variant, hipEvent_t mid);
// part[b] = number of NaN entries of lnl[0, n) in block b's grid-stride share
// (kNanParts blocks; every slot is written, so no clearing is needed).
void launch_count_nan(const double *lnl, int64_t n, unsigned long long *part, hipStream_t s);
// The nbase monomials (graded-lexicographic, variable indices poly[p][0..2],
// -1 unused) of u = (x - ms[0..3]) / ms[4..7], x = delta_e / a, in FP64:
// U[b][p] for proposals b0 .. b0 + nb - 1.
void launch_sur_base_inputs(const double *params, int64_t ld, int64_t b0, int64_t nb, const EvalConsts *c,
                            const double *ms, const int *poly, int nbase, double *U, hipStream_t s);
void launch_sur_inputs(const double *params, int64_t ld, int64_t b0, int64_t nb, const EvalConsts *c, float *x,
                       hipStream_t s);
void launch_col_stats(const double *Y, int64_t n, int K, float *mu, float *sd, hipStream_t s);
void launch_standardise(const double *Y, int64_t n, int K, const float *mu, const float *sd, float *T, hipStream_t s);
void launch_convert_weights(const double *W, size_t n, float *hi, uint16_t *b16, hipStream_t s);

}  // namespace rbfl

// The opaque handle of the C ABI.
struct rbfl_ctx {
  rbfl::Ctx c;
};
