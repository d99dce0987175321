/*
 * rbfl -- meshfree RBF likelihood for gravitational-wave parameter estimation
 * (Sharma, Pathak, Roy & Sengupta, arXiv:2508.04172), MI355X (gfx950) build.
 *
 * C ABI.  Every call returns an int32 status (RBFL_OK = 0); no C++ exception
 * crosses this boundary.  On error the outputs are unspecified and
 * rbfl_last_error() describes the failure.  Per-query domain conditions are
 * not errors: a proposal outside the interpolation ellipsoid, outside the
 * physical region or outside the stored time window gets ln L = -inf.
 *
 * Ownership: the caller owns every buffer it passes in or out; the library
 * owns the handle and every device artefact behind it (nodes, RBF weights,
 * SVD basis, frame), released by rbfl_destroy.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  rbfl_build synchronises its stream before returning; rbfl_eval
 * only enqueues work and returns.  Asynchronous device faults surface as
 * RBFL_E_DEVICE from a later call or from the caller's own synchronisation.
 *
 * Threading: a handle owns one work space (the interpolated outputs and
 * basis rows of a chunk), so rbfl_eval and rbfl_interp calls on one handle
 * must not overlap on the device: issue them on one stream, or order calls
 * on different streams with events.  Different handles are independent.
 * rbfl_build, rbfl_prepare, rbfl_autotune, rbfl_pipeline and rbfl_destroy
 * need exclusive use of a handle.
 */
#ifndef RBFL_H
#define RBFL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBFL_ABI_VERSION 7
#define RBFL_MAX_MODES 5
#define RBFL_MAX_DET 4
#define RBFL_MAX_BANDS 16     /* time bands of the antenna patterns (rbfl_build_spec.n_bands) */
#define RBFL_MAX_BLOCKS 64    /* n_det * n_bands: blocks of interpolated outputs */

enum rbfl_status {
  RBFL_OK = 0,
  RBFL_E_INVALID_ARG = 1,   /* malformed spec, NULL pointer, size out of range */
  RBFL_E_OUT_OF_MEMORY = 2, /* a device or host allocation failed */
  RBFL_E_DEVICE = 3,        /* a HIP or rocSOLVER call failed */
  RBFL_E_NUMERICAL = 4,     /* singular RBF system, SVD not converged, metric not positive definite */
  RBFL_E_UNSUPPORTED = 5,   /* a form or option this library does not provide */
  RBFL_E_STATE = 6          /* call out of order (e.g. a form not prepared) */
};

/* Arithmetic form of the online stage. */
enum rbfl_form {
  RBFL_FORM_FP64 = 0,       /* plain: FP64 kernel rows, FP64 MFMA contraction, FP64 epilogue */
  RBFL_FORM_FP32 = 1,       /* FP32 kernel rows and FP32 MFMA contraction, FP64 epilogue */
  RBFL_FORM_BF16 = 2,       /* kernel rows and weights rounded to BF16, FP32-accumulating MFMA
                               16x16x32, FP64 epilogue (for its error report: an 8-bit
                               significand does not carry the interpolant's cancellation) */
  RBFL_FORM_SPLIT = 3,      /* error-free split products: FP64 kernel rows and weight columns, each
                               scaled by a power of two into [-1, 1], written in S signed base-254
                               int8 digits; every digit pair i + j < S on int8 MFMA with exact int32
                               sums per level, levels combined in FP64 (per kernel row at most
                               (S + 3) 254^-S of the two scales); FP64 epilogue.  S is chosen by
                               rbfl_autotune (default 7).  Needs N + M <= 16384 */
  RBFL_FORM_SURROGATE = 4   /* trained surrogate network in place of the interpolant contraction, FP64
                               epilogue; the FP64 interpolant when no surrogate passed its held-out check */
};

/* Spec flags. */
#define RBFL_FLAG_CENTER_NODE 0x1u  /* place the ellipsoid centre as node 0 before the Halton nodes */
#define RBFL_FLAG_OPTIMISE_CENTRE 0x4u  /* move the centre to the network-SNR optimum (Sec. II C.1):
                                           Nelder-Mead from center_phys over the intrinsic parameters
                                           (coordinates Delta e / a of the ellipsoid at the seed), each template's
                                           SNR maximised over (iota, phi) (grid, then Nelder-Mead; the seed's SNR
                                           is reported at iota = phi = 0); per detector the SNR maximised over
                                           the plane of the two
                                           polarisations h+, hx (mode factors at (F+, Fx) = (1, 0), (0, 1)),
                                           over phase, and over time along the spline of the window samples
                                           near the best one; summed over detectors.  RBFL_Q_CENTRE reports
                                           the result.  The reference frequency and the injection stay those
                                           of center_phys. */
#define RBFL_FLAG_SQUEEZE 0x2u      /* squeeze the longest ellipsoid axis (Sec. II C.1, Fig. 2): scale it to
                                       the first point, scanning outward in steps of 1/64 along both
                                       directions, where the true match (Eq. Match) of the (2,2) template
                                       with the centre's falls below M0 (spins taken at face value, a
                                       direction that leaves eta <= 1/4 first sets no limit; the crossing
                                       bisected to 1e-12); RBFL_Q_SQUEEZE reports the factor */

typedef struct rbfl_ctx *rbfl_handle;

/*
 * Start-up specification (Sec. II C of the paper).  All pointers are host
 * pointers, read only during rbfl_build.
 *
 * Frequency grid: f_j = j / seg_len, j = 0 .. n_f - 1, n_f = fs*seg_len/2 + 1.
 * The noise-weighted inner product (Eq. innerProduct) runs over
 * f_low <= f_j < fs/2 (DC and Nyquist excluded).
 *
 * Data: if data_fd is NULL the library synthesises d_k = coloured noise +
 * injection: bin j of detector k gets sqrt(S_k(f_j) / (4 df)) (x + i y) with
 * (x, y) = noise_white[k][j][0..1] (NULL: zero noise), plus the projected
 * injection (Eq. projected_h_fd) at inj_phys, inj_ext, t_c = t_trig, with the
 * distance set so that the network optimal SNR equals inj_snr; that distance
 * is also the template reference distance d_ref.  If data_fd is given,
 * d_ref must be set and the injection fields are ignored.
 *
 * Templates: the library's synthetic multimode inspiral family, h_{l,-m}(f) =
 * A_lm Amp(Mc, d_ref) f^(-7/6) exp(-i (m/2) Psi(2f/m)) for f_low <= f <
 * |m| F_isco, with a 3.5PN aligned-spin TaylorF2-like phase Psi whose time
 * and phase are referenced at f_ref: Psi(f) = Psi_PN(f) - Psi_PN(f_ref) -
 * Psi_PN'(f_ref) (f - f_ref), so t_c and phi_c are the time and phase at
 * which the (2,2) mode passes f_ref (the injection uses the same convention).
 *
 * Ellipsoid: metric g of the (2,2) mode at center_phys in the chirp-time
 * coordinates Theta (Eq. metric_coords), computed unless `metric` is given;
 * the constant-match ellipsoid 1 - match = g dTheta dTheta (Eq. MisMatch).
 * Nodes: unscrambled Halton points (bases 2, 3, 5, 7, index from 1) mapped
 * to the unit ball in the eigen-frame, kept if physical (eta <= 1/4,
 * |chi_i| <= chi_max).  Interpolants: Gaussian RBF exp(-eps^2 r^2) in
 * unit-ball coordinates plus all monomials of degree <= poly_degree
 * (Eq. rbfcoeff), fitted to the first q SVD coefficients of each detector's
 * and mode's time series over t_trig +- half_window (Eq. SVD) and to the
 * mode overlaps (Eq. conjugation_symmetry).
 */
typedef struct {
  int32_t abi_version;                 /* RBFL_ABI_VERSION */
  int32_t n_det;                       /* 1 .. RBFL_MAX_DET */
  int32_t n_modes;                     /* 1 .. RBFL_MAX_MODES */
  int32_t modes[RBFL_MAX_MODES][2];    /* (l, |m|) from {(2,2),(2,1),(3,3),(3,2),(4,4)} */
  double fs;                           /* sample rate [Hz]; fs*seg_len an even integer */
  double seg_len;                      /* segment length [s] */
  double f_low;                        /* lower cut-off [Hz] */
  double psd_scale;                    /* scale of the analytic PSD (used when psd == NULL) */
  const double *psd;                   /* [n_det][n_f] one-sided PSD, or NULL for the analytic model */
  const double *data_fd;               /* [n_det][n_f][2] data (re, im), or NULL to synthesise */
  const double *noise_white;           /* [n_det][n_f][2] standard normal deviates, or NULL (zero noise) */
  double inj_phys[4];                  /* m1, m2 [Msun], chi1z, chi2z */
  double inj_ext[5];                   /* alpha, dec, psi, iota, phi [rad] */
  double inj_snr;                      /* network optimal SNR of the injection (> 0) */
  double d_ref;                        /* template reference distance [Mpc] when data_fd is given */
  const double *det_geom;              /* [n_det][5]: latitude, longitude, x-arm azimuth (from north
                                          toward east), arm opening angle [rad], distance from the
                                          geocentre [light-seconds] */
  double center_phys[4];               /* ellipsoid centre: m1, m2, chi1z, chi2z */
  double match;                        /* M0 in (0, 1) */
  const double *metric;                /* optional [4][4] metric in Theta, or NULL to compute it */
  double t_trig;                       /* trigger time in the segment [s], on the sample grid */
  double half_window;                  /* window half-width [s]; W = floor(half_window * fs) */
  int32_t n_nodes;                     /* N >= 1 + number of monomials */
  int32_t q;                           /* basis size, 1 .. min(N, 2W+1) */
  double eps;                          /* Gaussian shape parameter (> 0), or 0: the smallest integer from 1
                                          whose RBF system has a 1-norm condition estimate <= 1e12 (tried up
                                          to 8, RBFL_Q_EPS reports the value used) */
  int32_t poly_degree;                 /* 0 .. 3 */
  double chi_max;                      /* spin bound of the physical region (0 < chi_max <= 1) */
  uint32_t flags;                      /* RBFL_FLAG_* */
  double f_ref;                        /* template time/phase reference frequency [Hz]: > 0 as given,
                                          0 = the mean frequency of the centre's (2,2) band under the
                                          weights f^(-7/3) / S_0 (the metric's), < 0 = the formal
                                          coalescence (no reference shift) */
  double earth_rate;                   /* Earth's rotation rate [rad/s] for the exact likelihood and the
                                          synthesised injection (0 = antenna patterns frozen at t_c, the
                                          meshfree method's model, 7.2921150e-5 = sidereal): a source at
                                          right ascension alpha has Earth-fixed longitude
                                          alpha - earth_rate (t - t_trig), and each mode's frequency f is
                                          emitted at its stationary-phase time t_c + Psi'(2f/m) / (2 pi) */
  int32_t n_bands;                     /* time bands B of the antenna patterns: 0 or 1 = patterns frozen at
                                          t_c over the whole signal (Sec. II B); 2 .. RBFL_MAX_BANDS with
                                          n_det * B <= RBFL_MAX_BLOCKS = the time-banded form below */
} rbfl_build_spec;

/* Time-banded antenna patterns (n_bands = B > 1).  Sec. II B freezes the
 * patterns over the signal, which Sec. IV names as the limit for long
 * third-generation signals on a rotating Earth.  The banded form cuts the
 * frequency axis into B bands holding equal shares of the centre template's
 * (2,2) gravitational-wave phase f Psi'(f) - Psi(f) (between the lowest bin
 * and the centre's (2,2) cut-off; the last band runs to the top of the
 * grid).  In band b, mode (l, m) takes its antenna factor and delay at one
 * time t_bm relative to t_c: the mean of its stationary-phase time
 * Psi'(2f/m) / (2 pi) over its bins in the band under the weights
 * f^(-1/3) / S_0 (0 where the mode has no bins there); the source's
 * Earth-fixed longitude is then alpha - earth_rate (t_c + t_bm - t_trig).
 * Each (detector k, band b) is one block v = k B + b of Eq. logl_complete's
 * terms, with z and the mode overlaps summed over the band's bins only and
 * interpolated like the frozen form's (K = n_det B (2 q n_modes +
 * n_modes^2) outputs); the overlaps carry no delay, so cross terms between
 * modes drop the small phase their different delays would give them.
 * RBFL_Q_BANDS reports the bands.  A banded handle evaluates through
 * rbfl_eval, rbfl_interp, rbfl_eval_static and the samplers in every form
 * but the surrogate; rbfl_fuse_epilogue(on), rbfl_exact_parts,
 * rbfl_surrogate_train, rbfl_plan_create and rbfl_eval_ragged return
 * RBFL_E_INVALID_ARG for it. */

/* Thread-local description of the last failure on this thread; valid until
 * the next rbfl_* call on the same thread. */
const char *rbfl_last_error(void);

/* Start-up stage (Sec. II C): data, metric frame, Halton nodes, overlap time
 * series at the nodes (windowed DFT on the GPU), mode overlaps, FP64 SVD per
 * detector and mode and FP64 LU solve of the RBF system, all on the GPU.
 * Synchronous on `stream`.  *out receives a new handle. */
int32_t rbfl_build(const rbfl_build_spec *spec, void *stream, rbfl_handle *out);

/* The start-up stage (Sec. II C) of n events at once, for multi-event
 * batches: the stages before and after the SVD run for specs[0 .. n) on
 * n_threads host threads (1 .. 16, each with a stream of its own that the
 * library creates and destroys), and the FP64 SVDs of every event's
 * (detector, mode) pairs (Eq. SVD) go through one batched call per window
 * length on `stream`, each pair's node-by-sample matrix padded with zero node
 * rows to the largest node count of the call (this leaves the time basis and
 * the nonzero singular values as they are; the results agree with rbfl_build's
 * to rounding).  Synchronous; n in 1 .. 4096.  out[0 .. n) receives n new
 * handles, each owned by the caller as if made by rbfl_build; RBFL_Q_TIMING's
 * SVD entry of each is the batched stage's time.  On any failure (the first
 * event's error is returned) every out[i] is NULL and nothing is kept. */
int32_t rbfl_build_many(const rbfl_build_spec *specs, int32_t n, int32_t n_threads, void *stream,
                        rbfl_handle *out);

/* Exact ln L for n proposals, without the interpolant: the reference the
 * meshfree method approximates (Eq. logl_basic for the projected signal of
 * Eq. projected_h_fd, evaluated as Eq. logl_complete with z and the mode
 * overlaps as direct sums over the band at each proposal's own templates).
 * params, lnl: as rbfl_eval (device, SoA [11][n], FP64 [n]).  Defined on the
 * whole physical region (no ellipsoid or window restriction): -inf for an
 * unphysical intrinsic point, NaN for a NaN input.  Enqueued on `stream`,
 * allocates nothing; cost ~ n x bins x modes x detectors (one workgroup per
 * proposal). */
int32_t rbfl_brute(rbfl_handle h, const double *params, int64_t n, double *lnl, void *stream);

/* Where the meshfree ln L loses accuracy (Sec. II D, the three approximations
 * of the online stage): the quantities the interpolants approximate are
 * computed exactly at each proposal with the start-up kernels (its own
 * templates, the mode overlaps, the windowed DFT giving z at the T window
 * samples, and that series' coefficients on the handle's time basis), then
 *   out[0 .. n)   ln L through the online stage's own epilogue from those
 *                 exact coefficients and overlaps: equal to rbfl_eval but for
 *                 the RBF interpolation;
 *   out[n .. 2n)  ln L from the exact window samples with the same spline
 *                 stencil, no time basis: equal to out[0..n) but for the
 *                 truncation to q basis vectors, and to rbfl_brute but for
 *                 the sub-sample spline.
 * params: as rbfl_eval (device, SoA [11][n]); out: device FP64 [2][n].  Same
 * domain, window and NaN rules as rbfl_eval.  Synchronous on `stream`;
 * allocates work space for up to 4096 proposals at a time (templates of a
 * batch kept within ~2 GiB) and frees it before returning.  Cost
 * ~ n x bins x modes x detectors x T: a diagnostic, not a hot path. */
int32_t rbfl_exact_parts(rbfl_handle h, const double *params, int64_t n, double *out, void *stream);

/* Online stage (Sec. II D) for n proposals.
 * params: device, FP64, structure of arrays [11][n] (row stride n):
 *   delta_e0..3 (displacement from the centre along the metric eigenvectors,
 *   ordered by ascending semi-axis, in Theta units), alpha, dec, psi, iota,
 *   phi [rad], t_c (geocentric coalescence time in the segment [s]), d_L [Mpc].
 * lnl: device, FP64 [n]; ln L per proposal (Eq. logl_complete, corrected
 *   reading), -inf outside the ellipsoid, the physical region or the window.
 * form: RBFL_FORM_*; forms other than FP64 need rbfl_prepare first.
 * Enqueued on `stream`; no allocation when n <= the handle's work capacity
 * (rbfl_reserve), so a call can be captured in a HIP graph after a reserve.
 * Each call also counts its NaN results (RBFL_Q_NAN_COUNT). */
int32_t rbfl_eval(rbfl_handle h, const double *params, int64_t n, double *lnl, int32_t form,
                  void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rbfl_eval of
 * the FP64 form with its work space -- each chunk's basis rows and
 * interpolated outputs -- in a fixed device array of RBFL_STATIC_SCRATCH_BYTES
 * compiled into the library (one per GPU, held until the process ends)
 * instead of the handle's work space; it calls nothing that allocates.
 * Proposals run in chunks of floor(RBFL_STATIC_SCRATCH_BYTES / (8 (rows + Kp)))
 * rounded down to a multiple of 8 (rows = N + M padded to 32, Kp = K padded
 * to 128), always in the serial order (basis rows, contraction with the
 * handle's FP64 tile variant, epilogue), then the NaN count
 * (RBFL_Q_NAN_COUNT).  params, n, lnl: as rbfl_eval; ln L equals rbfl_eval's
 * in its default serial order bit for bit (to rounding when rbfl_eval
 * finishes ln L inside the contraction).  Enqueued on `stream`.  The
 * handle's device must be current (else RBFL_E_INVALID_ARG).  Every call on
 * one GPU shares that GPU's array, which keeps the last call's contents:
 * calls that overlap on one GPU (other streams, threads or handles) race and
 * give wrong results, so order them.  RBFL_E_INVALID_ARG when 64 proposals
 * of the handle do not fit the array (8 (rows + Kp) bytes each). */
#define RBFL_STATIC_SCRATCH_BYTES (128u << 20)
int32_t rbfl_eval_static(rbfl_handle h, const double *params, int64_t n, double *lnl, void *stream);

/* Interpolated quantities at n proposals (Eq. rbfcoeff): out[b][c], c < K,
 * device FP64, row stride K.  Per detector k the K reals are, in order, for
 * each mode the interleaved (Re, Im) of the q SVD coefficients (Eq. SVD),
 * then the n_modes^2 overlap reals: the diagonal sigma_aa, then (Re, Im)
 * sigma_ab for a < b in lexicographic order (Eq. conjugation_symmetry).
 * Only rows 0..3 of params (delta_e) are read; no domain check is applied.
 * Enqueued on `stream`. */
int32_t rbfl_interp(rbfl_handle h, const double *params, int64_t n, double *out, int32_t form, void *stream);

/* Converts the weights for a reduced-precision form (RBFL_FORM_FP32/BF16/SPLIT).
 * Synchronous; needs exclusive use of the handle.  RBFL_E_UNSUPPORTED for a
 * form this library or this handle's size does not support. */
int32_t rbfl_prepare(rbfl_handle h, int32_t form);

/* Pre-allocates work space for batches of up to n proposals (optional). */
int32_t rbfl_reserve(rbfl_handle h, int64_t n);

/* Artefact export (host copies), for checks and diagnostics. */
enum rbfl_query_what {
  RBFL_Q_SIZES = 0,        /* int64[8]: N, M, K, q, T, n_det, n_modes, half_window_samples */
  RBFL_Q_FRAME = 1,        /* double[4 + 16 + 4 + 4 + 16]: theta_c, eigenvectors (row-major,
                              column i = axis i), eigenvalues, semi-axes, metric (row-major) */
  RBFL_Q_D_REF = 2,        /* double[1]: template reference distance [Mpc] */
  RBFL_Q_NODES = 3,        /* double[N][4] unit-ball node coordinates */
  RBFL_Q_NODE_PHYS = 4,    /* double[N][4] m1, m2, chi1, chi2 of the nodes */
  RBFL_Q_WEIGHTS = 5,      /* double[N+M][K] RBF weights */
  RBFL_Q_BASIS = 6,        /* double[n_blocks][n_modes][T][q][2] SVD basis (n_blocks = n_det, or
                              n_det * n_bands with time bands, block v = k n_bands + b) */
  RBFL_Q_NODE_VALUES = 7,  /* double[N][K] interpolated quantities at the nodes */
  RBFL_Q_SINGULAR = 8,     /* double[n_blocks][n_modes][min(N,T)] singular values */
  RBFL_Q_COND = 9,         /* double[1]: 1-norm condition estimate of the RBF system */
  RBFL_Q_TIMING = 10,      /* double[8]: start-up stage wall times [s] */
  RBFL_Q_Z_NODES = 11,     /* double[n_blocks][n_modes][N][T][2] time series at the nodes */
  RBFL_Q_KERNEL_STATS = 12, /* double[9]: MFMA contraction ms, launches, proposals; epilogue ms,
                               launches, proposals; basis-row stage ms, launches, proposals (zero time
                               for forms without one) -- summed HIP-event durations since
                               rbfl_profile was switched on (synchronises the recorded events; resets
                               the sums) */
  RBFL_Q_TUNE = 13,         /* double[4][9]: per form, the chosen contraction tile variant and the
                               autotuner's median time [ms] of each variant (0 = not timed) */
  RBFL_Q_SURROGATE = 14,    /* double[8]: accepted (1/0), held-out max |d ln L|, held-out median
                               |d ln L|, first-epoch loss, last-epoch loss, epochs, training seconds,
                               training proposals */
  RBFL_Q_SPLIT_ERR = 15,    /* double[8]: per split-form variant, max |d ln L| against the FP64 form
                               on the last rbfl_autotune's proposals (0 = not measured) */
  RBFL_Q_F_REF = 16,        /* double[1]: template time/phase reference frequency [Hz] (0: coalescence) */
  RBFL_Q_SQUEEZE = 17,      /* double[2]: factor applied to the longest semi-axis (1 = none) and the true
                               match at the squeezed tip (0 when not squeezed) */
  RBFL_Q_CENTRE = 18,       /* double[8]: the ellipsoid centre used (m1, m2, chi1, chi2), the optimiser's
                               iota and phi, the network SNR at center_phys (iota = phi = 0) and at the
                               optimum (0, 0 without RBFL_FLAG_OPTIMISE_CENTRE) */
  RBFL_Q_PIPELINE = 19,     /* double[7]: chunks per FP64 evaluation in use (rbfl_pipeline), the
                               autotuner's median ms per evaluation at 1, 2, 4 and 8 chunks (0 = not
                               timed), 1/0 for ln L finished inside the contraction (rbfl_fuse_epilogue)
                               and the autotuner's ms per evaluation in that order (0 = not timed) */
  RBFL_Q_SURROGATE_NET = 20, /* float[n_params + 2 K]: the surrogate's trained parameters (the layout
                               of rbfl_mlp_get for n_in = 4, the width given to rbfl_surrogate_train,
                               n_out = K), then the per-column mean and standard deviation that map
                               its outputs to the interpolated quantities (out = mean + sd * y);
                               RBFL_E_STATE before rbfl_surrogate_train.  Synchronises the device. */
  RBFL_Q_EPS = 24,          /* double[1]: the Gaussian shape parameter of the interpolants */
  RBFL_Q_SURROGATE_BASE = 23, /* double[10 + nbase K]: the surrogate's base degree, nbase (0 without
                               a base), m[4], s[4], then the base coefficients [nbase][K] row-major;
                               RBFL_E_STATE before rbfl_surrogate_train.  Synchronises the device. */
  RBFL_Q_SPLIT_STATE = 21,  /* double[3]: 1/0 the split form's digit count was chosen by rbfl_autotune,
                               1/0 that choice is within the handle's split tolerance of the FP64 form (when no digit
                               count is, the tuner keeps the most accurate one and reports 0 here:
                               such a split form does not meet the tuner's bar), digits S in use */
  RBFL_Q_NAN_COUNT = 22,    /* int64[1]: NaN ln L values written by the last rbfl_eval call on this
                               handle (a proposal with a NaN parameter gives NaN; any other NaN result
                               is counted too).  Synchronises the device. */
  RBFL_Q_BANDS = 25,        /* double[2 + (B + 1) + B n_modes]: B = n_bands (1 when frozen), n_blocks,
                               the band edges as bin indices [B + 1] (band b holds bins edges[b] ..
                               edges[b+1] - 1), then the band times t_bm relative to t_c [B][n_modes]
                               (rbfl_build_spec.n_bands) */
  RBFL_Q_SPLIT_ORDER = 26   /* double[3]: 1/0 the split form finishes ln L inside its contraction
                               (rbfl_fuse_epilogue bit 1), then the split autotune's ms per evaluation
                               with the separate epilogue and in that order (0 = not timed) */
};
int32_t rbfl_query(rbfl_handle h, int32_t what, void *out, size_t bytes);

/* Tile autotuner: times each contraction tile variant of `form` on the
 * first min(n, work capacity) proposals of `params` (device [11][n]) with HIP
 * events on `stream` and keeps the fastest for this handle (RBFL_Q_TUNE
 * reports the timings).  Split-form variants differ in digit count S (5..8,
 * variant v has S = 5 + v): only those whose ln L on these proposals stays
 * within the handle's split tolerance (rbfl_set_split_tol, default
 * RBFL_SPLIT_TOL) of the FP64 form's (and keeps its domain flags) are
 * eligible (RBFL_Q_SPLIT_ERR reports the differences); with none eligible the
 * most accurate variant is kept and RBFL_Q_SPLIT_STATE says that the bar was
 * missed; without autotuning the split form uses S = 7.  With the chosen S it
 * then times whole split evaluations with the separate epilogue and with ln L
 * inside the contraction (frozen patterns, more than 4096 proposals) and
 * keeps the latter if at least 1% faster (RBFL_Q_SPLIT_ORDER).  For RBFL_FORM_FP64 it then
 * times whole evaluations of those proposals in each evaluation order (serial,
 * rbfl_pipeline with 2, 4 and 8 chunks, rbfl_fuse_epilogue) and keeps a
 * pipelined order only if it is at least 3% faster than the serial one, ln L
 * inside the contraction if it is at least 1% faster than the best of those
 * (RBFL_Q_PIPELINE reports the timings).  Synchronous; needs exclusive use of the handle. */
#define RBFL_SPLIT_TOL 1e-4
int32_t rbfl_autotune(rbfl_handle h, const double *params, int64_t n, int32_t form, void *stream);

/* The bar rbfl_autotune holds split-form digit counts to against the FP64
 * form on its tuning proposals, for this handle: RBFL_SPLIT_TOL (a tenth of
 * the online stage's 1e-3 accuracy target) until set.  A looser bar lets the
 * tuner keep fewer digits (faster, each proposal's ln L further from the FP64
 * form's, but never by more than tol on the tuning proposals).  Takes effect
 * at the next rbfl_autotune of RBFL_FORM_SPLIT; multi-event plans keep
 * RBFL_SPLIT_TOL.  RBFL_E_INVALID_ARG for a NULL handle or tol outside
 * (0, 1e-3]; needs exclusive use of the handle. */
int32_t rbfl_set_split_tol(rbfl_handle h, double tol);

/* Number of contraction tile variants (at least 1) of `form` (RBFL_FORM_FP64
 * .. SPLIT), or -RBFL_E_INVALID_ARG (negative) for another form. */
int32_t rbfl_variants(int32_t form);

/* Pins the contraction tile variant of `form` (0 <= variant <
 * rbfl_variants(form)) instead of the autotuner's choice.  FP64 variants are
 * tile shapes of one arithmetic (ln L identical); split-form variants are
 * digit counts (S = 5 + variant).  RBFL_E_STATE if the form is not prepared;
 * needs exclusive use of the handle. */
int32_t rbfl_set_variant(rbfl_handle h, int32_t form, int32_t variant);

/* Pipelined FP64 evaluation (Sec. II D's online stage, reordered, not changed):
 * rbfl_eval of the FP64 form splits a call into `chunks` chunks (1 = the
 * serial order, at most 64) whose epilogues (arrival times, reconstruction
 * and Eq. logl_complete) run on a second, handle-owned stream of default
 * priority under the next chunk's basis rows and MFMA product; the work space
 * is split in two halves that the chunks alternate between, and the caller's
 * stream waits for every epilogue before the call returns, so the call stays
 * ordered on `stream` as before.  ln L is bit-identical to the serial order.
 * Used only when the work capacity holds two halves of at least 4096
 * proposals, for calls of more than 4096 proposals, and never while `stream`
 * is being captured.  rbfl_autotune of RBFL_FORM_FP64 times 1, 2, 4 and 8
 * chunks (RBFL_Q_PIPELINE).  Needs exclusive use of the handle;
 * RBFL_E_INVALID_ARG for chunks outside 1..64. */
int32_t rbfl_pipeline(rbfl_handle h, int32_t chunks);

/* ln L finished inside the FP64 or split contraction (Sec. II D's online stage, same
 * terms regrouped): ln L of Eq. logl_complete (corrected reading) is linear in
 * the interpolated outputs, ln L = sum_c coef_c Y[c], with coef_c formed from
 * the proposal's distance ratio, amplitudes and spline-folded basis value.
 * `on` is a bit mask: bit 0 for the FP64 form, bit 1 for the split form
 * (0..3; each call sets both).  In that order rbfl_eval writes each
 * proposal's setup, contracts with a kernel that weights its output tile by
 * coef_c and writes one partial sum per proposal and column tile (128 columns
 * for FP64, 64 for the split form) instead of the outputs, and adds the
 * tiles' partials (compensated, in tile order).  Its work space, 384 bytes +
 * 8 Kp / 64 bytes per proposal of capacity (rbfl_reserve), is allocated by
 * the first evaluation in either order.  ln L agrees with the default order
 * to rounding (the summation order differs); domain flags are the same.
 * Takes precedence over rbfl_pipeline; allowed under graph capture once that
 * work space exists (else RBFL_E_STATE).  rbfl_autotune times each form's
 * order and keeps it if 1% faster than the best other order
 * (RBFL_Q_PIPELINE, RBFL_Q_SPLIT_ORDER).  RBFL_E_INVALID_ARG for `on` outside
 * 0..3, or nonzero on a banded handle.  Needs exclusive use of the handle. */
int32_t rbfl_fuse_epilogue(rbfl_handle h, int32_t on);

/* Switches per-launch timing of the online kernels on (1) or off (0): with it
 * on, rbfl_eval records HIP events around the basis-row, contraction and
 * epilogue launches of every chunk, each on the stream the launch runs on
 * (the caller's; the handle's second stream for pipelined epilogues; with
 * ln L inside the contraction the stages are setups + basis rows, the
 * contraction, and the sum of its partials); RBFL_Q_KERNEL_STATS reports the
 * sums.  Not for use under graph capture. */
int32_t rbfl_profile(rbfl_handle h, int32_t on);

/*
 * Multi-event batches: one launch evaluates the proposals of several events
 * (handles of different N, K, q, mode sets), each event's proposals a
 * contiguous range of one concatenated parameter array.
 *
 * A plan fixes the events, their proposal counts and the device buffers
 * params (FP64 [11][total], row stride total = sum of counts, event e's
 * proposals in columns [sum_{e'<e} counts[e'], ...)) and lnl (FP64 [total]).
 * Execution: one launch writes the FP64 basis rows of every event; a
 * persistent FP64 GEMM kernel then takes (event, proposal tile, column tile)
 * items, events ordered by decreasing cost proposals x (N+M) x K, from an
 * atomic counter (reset by a kernel); then the epilogue finishes ln L of each
 * proposal with its own event's frame and basis.  Variants 0-2 instead form
 * the rows inside the persistent contraction (fused), variants 3-4 are the
 * rows + GEMM tiles (the default).  RBFL_PLAN_AUTOTUNE times each variant on
 * the whole batch (HIP events) and keeps the fastest; RBFL_PLAN_GRAPH captures
 * the launch in a HIP graph, replayed by rbfl_plan_launch -- a sampler step
 * writes new proposals into `params` and launches again, without
 * re-capturing.  The handles must outlive the plan; plan creation allocates
 * (work space for every event's rows and outputs), launches do not.  Launches
 * of one plan must not overlap.
 */
#define RBFL_PLAN_GRAPH 0x1u
#define RBFL_PLAN_AUTOTUNE 0x2u
#define RBFL_PLAN_SPLIT 0x4u      /* contraction in the split form (RBFL_FORM_SPLIT's arithmetic): each
                                     event's weight digits are prepared if needed (rbfl_prepare); one
                                     launch writes the S digits of every event's kernel rows, then one
                                     persistent int8 contraction per digit count S in use takes the
                                     (event, 128 proposals, 64 columns) items of its events.  With
                                     RBFL_PLAN_AUTOTUNE the batch runs at S = 5, 6, 7, 8 against the FP64
                                     plan; an event with at least 256 in-domain proposals takes the fewest
                                     digits whose ln L stays within RBFL_SPLIT_TOL / 10 of it, any other
                                     event 7 digits (8 if 7 misses RBFL_SPLIT_TOL; the most accurate count
                                     when none meets it); without it each event uses its handle's split
                                     variant (default 7) */
typedef struct rbfl_plan_ctx *rbfl_plan;
int32_t rbfl_plan_create(const rbfl_handle *hs, int32_t n_events, const int64_t *counts, const double *params,
                         double *lnl, uint32_t flags, void *stream, rbfl_plan *out);
int32_t rbfl_plan_launch(rbfl_plan plan, void *stream);
/* out double[16] (at least 12): tile variant (-1 for the split form), work items, persistent grid
 * size, proposals, then the autotuner's median time [ms] of each tile variant (split form: of the
 * whole batch at S = 5 .. 8; 0 = not timed), then 1/0 split form, the smallest and largest digit
 * count of its events, and 1/0 every event within RBFL_SPLIT_TOL of the FP64 plan (-1 when the
 * digit counts were not tuned). */
int32_t rbfl_plan_query(rbfl_plan plan, double *out, size_t bytes);
/* Pins the FP64 tile variant of a plan (0 .. 5: variants 0-2 fused rows, 3-4 rows + 64 x 128 GEMM
 * tiles of 4 waves, 5 rows + 128 x 128 tiles of 8 waves) instead of the autotuner's choice,
 * re-capturing its graph if it has one; synchronises `stream` first.  RBFL_E_STATE for a split-form
 * plan, RBFL_E_INVALID_ARG for a variant out of range. */
int32_t rbfl_plan_set_variant(rbfl_plan plan, int32_t variant, void *stream);
int32_t rbfl_plan_destroy(rbfl_plan plan);
/* One-shot multi-event evaluation (creates a plan without graph or autotune,
 * runs it and synchronises `stream`). */
int32_t rbfl_eval_ragged(const rbfl_handle *hs, int32_t n_events, const int64_t *counts, const double *params,
                         double *lnl, void *stream);

/*
 * Learned surrogate (not in the paper: a network that replaces the
 * interpolant contraction, keeping the interpolant as fallback and reference).
 * A multilayer perceptron x -> H -> H -> K with SiLU activations maps the
 * unit-ball coordinates x = delta_e / a to the K interpolated reals
 * (standardised per column by the training set's mean and deviation).  It is
 * trained on proposals whose targets the handle's FP64 interpolant computes,
 * with mean-squared error and Adam, by the library's own FP32 kernels.  After
 * training, ln L of the held-out proposals through the network is compared
 * with ln L through the interpolant; the surrogate is used by
 * RBFL_FORM_SURROGATE only if the largest |difference| (and every domain
 * decision) stays within `threshold`, otherwise that form evaluates the FP64
 * interpolant.  The surrogate form's work space is per handle: calls with it
 * on one handle must not overlap.
 *
 * Parameters (shared layout): W1 [H][4], b1 [H], W2 [H][H], b2 [H],
 * W3 [K][H], b3 [K], weights row-major; initialised from standard normal
 * deviates z in the same layout as W = z / sqrt(fan_in), b = 0.
 */
typedef struct {
  int32_t hidden;                /* H, 8 .. 1024 */
  int32_t batch;                 /* mini-batch size */
  int32_t epochs;                /* passes over the training proposals */
  double lr, beta1, beta2, adam_eps;
  const double *init_normals;    /* host [n_params] standard normal deviates */
  const double *train_params;    /* device FP64 [11][n_train]; rows 0..3 (delta_e) are read */
  int64_t n_train;               /* >= batch */
  const double *holdout_params;  /* device FP64 [11][n_holdout] proposals, or NULL (then never accepted) */
  int64_t n_holdout;
  double threshold;              /* acceptance bar on max |d ln L| over the held-out proposals */
  int32_t base_degree;           /* 0: the network's outputs are the standardised interpolated reals;
                                    1 .. 3 (residual form): an FP64 least-squares polynomial of this degree
                                    (all monomials, graded-lexicographic) in the training proposals'
                                    standardised coordinates u = (x - m) / s (m, s their per-axis mean and
                                    deviation) is fitted to each real, and the network learns the
                                    standardised residual; inference adds the base back in FP64 */
} rbfl_train_spec;
int32_t rbfl_surrogate_train(rbfl_handle h, const rbfl_train_spec *spec, void *stream);
/* Overrides the held-out check (on = 1: the surrogate form uses the network
 * even if it failed the check; 0: back to the check's decision).  For
 * measuring the network path; RBFL_E_STATE if no surrogate was trained. */
int32_t rbfl_surrogate_force(rbfl_handle h, int32_t on);

/* The surrogate network on its own (for checks of its forward and backward
 * passes): x device FP32 [B][n_in], y/t device FP32 [B][n_out]; loss is a
 * host double (the call synchronises); rbfl_mlp_get copies the parameters
 * (what = 0) or the last gradients (what = 1) to host FP32 [n_params]. */
typedef struct rbfl_mlp_ctx *rbfl_mlp;
int32_t rbfl_mlp_create(int32_t n_in, int32_t hidden, int32_t n_out, const double *normals, rbfl_mlp *out);
int32_t rbfl_mlp_forward(rbfl_mlp m, const float *x, int64_t B, float *y, void *stream);
int32_t rbfl_mlp_loss_grad(rbfl_mlp m, const float *x, const float *t, int64_t B, double *loss, void *stream);
int32_t rbfl_mlp_adam(rbfl_mlp m, double lr, double beta1, double beta2, double eps, void *stream);
int32_t rbfl_mlp_get(rbfl_mlp m, int32_t what, float *out, size_t bytes);
int32_t rbfl_mlp_destroy(rbfl_mlp m);

/*
 * Ensemble sampler on the GPU (Sec. II D: sampling in the Delta e
 * coordinates of the ellipsoid; the paper drives a nested sampler on the CPU,
 * this drives the online stage from device-resident walkers).  Parameters as
 * rbfl_eval's 11 rows.  Sampled prior: uniform in Delta e within the unit
 * ball and the physical region, alpha, psi, phi uniform (periods 2 pi, pi,
 * 2 pi), dec with density cos(dec), iota with sin(iota), t_c uniform in
 * [t_lo, t_hi], d_L with density d_L^d_exp in [d_lo, d_hi] (Table I; the
 * paper's runs use d_exp = 0).  Moves: differential-evolution Metropolis
 * (ter Braak 2006) over two halves of the ensemble: walker i of one half
 * proposes X_i + g (X_j - X_k) with j != k from the other half, g = gamma
 * (1 + 0.01 n), n standard normal, or g = 1 with probability p_jump; the
 * angles wrap.  The proposal is symmetric, so a proposal is accepted with
 * probability min(1, posterior ratio) (with ln L weighted by beta during an
 * annealed start); a walker at zero posterior takes any proposal of non-zero
 * posterior.  Random numbers: Philox4x32-10 (Salmon et
 * al. 2011), key = seed, counter = (walker, step mod 2^32, step / 2^32 mod
 * 2^31 | half << 31, call): call 0 gives the partner indices
 * j = floor(u0 M), k = floor(u1 (M - 1)) (+1 if k >= j), call 1 the
 * Box-Muller pair (u2, u3) of n, call 3 the jump draw u4, call 2 the
 * acceptance uniform; u = ((a >> 5) 2^26 + (b >> 6) + 1/2) 2^-53 from each
 * pair of 32-bit words.  Walkers 0 .. M-1 move first, M .. 2M-1 second.
 */
#define RBFL_SAMPLER_PRIOR_ONLY 0x1u   /* ln L taken as 0: samples the prior (for checks) */
typedef struct {
  int32_t walkers;      /* W, even, 8 .. 2^30 */
  int32_t form;         /* RBFL_FORM_* used for ln L (prepared) */
  uint64_t seed;
  double t_lo, t_hi;    /* t_c prior range [s] */
  double d_lo, d_hi;    /* d_L prior range [Mpc], 0 < d_lo < d_hi */
  double d_exp;         /* d_L prior density exponent (0: uniform, 2: uniform in volume) */
  double gamma;         /* differential-evolution scale; 0 = 2.38 / sqrt(2 * 11) */
  double p_jump;        /* probability of a g = 1 move, 0 .. 1 */
  uint32_t flags;       /* RBFL_SAMPLER_* */
  int64_t anneal_steps; /* steps 0 .. anneal_steps-1 accept with ln L weighted by
                           beta = beta0^(1 - step / anneal_steps) (a tempered start from the prior) */
  double beta0;         /* first annealing weight, (0, 1] (unused without annealing) */
} rbfl_sampler_spec;
typedef struct rbfl_sampler_ctx *rbfl_sampler;

/* Creates the walkers: from init (device FP64 [11][W], copied) or, if init is
 * NULL, drawn from the prior (Delta e by rejection from the cube to the unit
 * ball and the physical region, the rest by inverse transforms; Philox
 * counter step 2^63 - 1, half 1), evaluates their ln L, and captures one
 * sampler step (both halves) as a HIP graph over the handle's work space
 * (reserved here for W/2 proposals, at most 2^20 per launch).  The handle
 * must outlive the sampler and is not to be used on another stream while the
 * sampler runs; while a sampler exists the handle refuses calls that would
 * reallocate what the graph uses (rbfl_reserve beyond the reserved size,
 * rbfl_surrogate_train: RBFL_E_STATE; preparing another form only adds
 * buffers).  Synchronous on `stream`. */
int32_t rbfl_sampler_create(rbfl_handle h, const rbfl_sampler_spec *spec, const double *init, void *stream,
                            rbfl_sampler *out);

/* Runs `steps` steps (graph replays) on `stream`, asynchronously.  Every
 * `thin` steps the walkers' positions and ln L go to chain (device FP64
 * [12][slots][W]: row m of sample (s, w) at m * slots * W + s * W + w, row 11
 * = ln L; at most `slots` samples kept; chain may be NULL). */
int32_t rbfl_sampler_run(rbfl_sampler s, int64_t steps, int32_t thin, double *chain, int64_t slots, void *stream);

/* Tempered sequential Monte Carlo start (Del Moral, Doucet and Jasra 2006)
 * from the current walkers, taken as prior draws (ln L weight beta = 0):
 * per stage, the increment db in (0, 1 - beta] for which the weights
 * w = L^db keep an effective sample size ess_frac W (all of the remainder if
 * it stays above that), found by 60 bisection halvings; log Z += log mean w
 * (the evidence of the likelihood ratio relative to the prior); systematic
 * resampling at positions (u + i) / W with u the first uniform of Philox call
 * 4 of (walker 2^32 - 1, step = index of the stage over the sampler's life,
 * half 1); then `moves` sampler steps with ln L weighted by the new beta.
 * Stops at beta = 1 or after max_stages; later rbfl_sampler_run steps keep
 * the final beta.  Synchronous on `stream`; log_evidence, stages and beta
 * (host, optional) receive the results. */
int32_t rbfl_sampler_smc(rbfl_sampler s, double ess_frac, int32_t moves, int32_t max_stages, void *stream,
                         double *log_evidence, int32_t *stages, double *beta);

/* what = 0: walkers, host FP64 [12][W] (positions, ln L); 1: accepted moves
 * per walker, host FP64 [W]; 2: host FP64 [2] = steps run, mean acceptance
 * fraction.  Synchronises the sampler's last stream. */
int32_t rbfl_sampler_query(rbfl_sampler s, int32_t what, double *out, size_t bytes);
int32_t rbfl_sampler_destroy(rbfl_sampler s);

/* Prior reweighting (Sec. III A: w = p_target / p_sampled) of n samples
 * (device FP64, rows of stride ld: the 11 parameters): the sampled intrinsic
 * prior is uniform in Delta e, the target uniform in (m1, m2, chi1, chi2)
 * inside box = {m1_lo, m1_hi, m2_lo, m2_hi, chi1_lo, chi1_hi, chi2_lo,
 * chi2_hi}, and the target distance density is d_L^d_exp times the sampled
 * one: logw = log |det d(m1, m2, chi1, chi2) / d Delta e| + d_exp log d_L
 * (central differences, steps 1e-7 |Theta|), -inf outside the box.  logw:
 * device FP64 [n].  If n_eff is not NULL the call synchronises and stores
 * (sum w)^2 / sum w^2 there. */
int32_t rbfl_prior_weights(rbfl_handle h, const double *params, int64_t ld, int64_t n, const double box[8],
                           double d_exp, double *logw, double *n_eff, void *stream);

/* Start-up reuse (Sec. II D: the interpolants are built once in the start-up
 * stage and then only evaluated while sampling).  rbfl_save writes every
 * artefact of a built handle -- sizes, frame, the online stage's constants,
 * nodes (unit-ball and physical), RBF weights, SVD basis and its
 * spline-folded copy, singular values, node values and node series, output
 * layout, and the exact likelihood's band data -- to `path` (a versioned file
 * with a checksum; written to path + ".tmp" and renamed, so a failed save
 * leaves no partial file at `path`).  Synchronises the device.  Reduced-
 * precision weight copies, tile choices and a trained surrogate are not
 * stored: a loaded handle starts with the FP64 form only (rbfl_prepare and
 * rbfl_autotune again as needed).  RBFL_E_INVALID_ARG if the file cannot be
 * written.
 *
 * rbfl_load creates a handle on the current device from such a file.  Its
 * rbfl_eval, rbfl_interp, rbfl_brute, rbfl_exact_parts and rbfl_query results
 * equal the saved handle's bit for bit.  RBFL_E_INVALID_ARG, with nothing
 * allocated on the device, for a missing, truncated or damaged file (checksum),
 * another format or ABI version, or sizes this library cannot have built;
 * synchronous on `stream`. */
int32_t rbfl_save(rbfl_handle h, const char *path);
int32_t rbfl_load(const char *path, void *stream, rbfl_handle *out);

/* Releases the handle and its device memory (NULL is allowed). */
int32_t rbfl_destroy(rbfl_handle h);

#ifdef __cplusplus
}
#endif

#endif /* RBFL_H */
