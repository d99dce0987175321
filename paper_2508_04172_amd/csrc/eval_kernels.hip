// Online-stage kernels (Sec. II D).
//
// contract_*: Y[b][c] = sum_r B_r(x_b) W[r][c] with the interpolation basis
//   B_r(x) = exp(-eps^2 |x - x_r|^2) for node rows r < N and the monomials
//   p_{r-N}(x) for N <= r < N + M (Eq. rbfcoeff).  The basis rows are formed
//   in registers directly in the MFMA A-operand layout (never stored), W is
//   staged through LDS in chunks of 64 rows.
// epilogue: per proposal, arrival times and spline weights, reconstruction
//   of each detector's and mode's z(tau) from the interpolated SVD
//   coefficients (Eq. SVD) and the extrinsic combination of Eq. logl_complete
//   (corrected reading) with compensated summation.
#include "basis_rows.h"
#include "epilogue_setup.h"
#include "rbfl_internal.h"

namespace rbfl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kLdsPad = 16;   // doubles of padding per LDS row (bank spread across the 4 k-groups)

// Block tile: kWaves waves along the proposals, each wave RT x 16 proposals
// by CT x 16 outputs; the block covers kWaves*RT*16 proposals and CT*16
// outputs.  MFMA f64 16x16x4 operand layout (measured on gfx950): lane l
// holds A[l%16][l/16] and B[l/16][l%16]; accumulator element i of lane l is
// D[l/16 + 4i][l%16].  Weight rows stream through two LDS buffers of CH rows:
// while the MFMAs consume one, each thread's share of the next chunk is
// already in flight from global memory into registers.
// One (proposal tile, column tile) of the FP64 contraction; called by the
// per-handle kernel and by the persistent multi-event kernel.  Must be entered
// by the whole block; ends with a block barrier, so the block may run another
// tile right after.
template <int RT, int CT, int CH>
__device__ __forceinline__ void contract_tile_fp64(const EvalConsts &c, const double *__restrict__ params,
                                                   int64_t ld, int64_t b0, int64_t nb,
                                                   const double *__restrict__ nodes, const double *__restrict__ W,
                                                   double *__restrict__ Y, int tile_q, int tile_c) {
  constexpr int CW = CT * 16;
  constexpr int QT = kWaves * RT * 16;
  constexpr int PER = CH * CW / kThreads;
  static_assert(kRowChunk % CH == 0 && (CH * CW) % kThreads == 0 && CH * 4 <= kThreads, "tile");
  __shared__ double Ws[2][CH][CW + kLdsPad];
  __shared__ double Xs[2][CH][4];
  __shared__ int poly[kMaxPoly][3];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col0 = tile_c * CW;
  const int64_t qbase = (int64_t)tile_q * QT + wave * RT * 16;
  const int N = c.N, NM = c.N + c.M, rows = c.rows, Kp = c.Kp;
  const double eps2 = c.eps2;
  for (int e = threadIdx.x; e < kMaxPoly * 3; e += kThreads) poly[e / 3][e % 3] = c.poly_idx[e / 3][e % 3];

  double xq[RT][4];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t b = qbase + rt * 16 + (lane & 15);
#pragma unroll
    for (int d = 0; d < 4; ++d) xq[rt][d] = b < nb ? params[d * ld + b0 + b] / c.semi[d] : 0.0;
  }
  d4 acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = d4{0.0, 0.0, 0.0, 0.0};

  double wreg[PER];
  double xreg = 0.0;
  auto fetch = [&](int r0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * kThreads;
      wreg[u] = W[(int64_t)(r0 + e / CW) * Kp + col0 + e % CW];
    }
    if (threadIdx.x < CH * 4) xreg = nodes[(int64_t)r0 * 4 + threadIdx.x];
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * kThreads;
      Ws[buf][e / CW][e % CW] = wreg[u];
    }
    if (threadIdx.x < CH * 4) Xs[buf][threadIdx.x >> 2][threadIdx.x & 3] = xreg;
  };
  fetch(0);
  stash(0);
  __syncthreads();
  const int kk = lane >> 4;
  const int n_chunks = rows / CH;
  for (int ch = 0; ch < n_chunks; ++ch) {
    const int cur = ch & 1;
    const int r0 = ch * CH;
    if (ch + 1 < n_chunks) fetch(r0 + CH);
#pragma unroll 2
    for (int s = 0; s < CH / 4; ++s) {
      const int rr = 4 * s + kk;
      double a[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) a[rt] = basis_row_fp64(r0 + rr, N, NM, xq[rt], Xs[cur][rr], eps2, poly);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const double bv = Ws[cur][rr][ct * 16 + (lane & 15)];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt], bv, acc[rt][ct], 0, 0, 0);
      }
    }
    if (ch + 1 < n_chunks) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t b = qbase + rt * 16 + (lane >> 4) + 4 * i;
      if (b >= nb) continue;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) Y[b * Kp + col0 + ct * 16 + (lane & 15)] = acc[rt][ct][i];
    }
  }
}

template <int RT, int CT, int CH>
__global__ void __launch_bounds__(kThreads) k_contract_fp64(const EvalConsts *__restrict__ cp,
                                                            const double *__restrict__ params, int64_t ld,
                                                            int64_t b0, int64_t nb,
                                                            const double *__restrict__ nodes,
                                                            const double *__restrict__ W, double *__restrict__ Y) {
  contract_tile_fp64<RT, CT, CH>(*cp, params, ld, b0, nb, nodes, W, Y, blockIdx.x, blockIdx.y);
}

// FP32 form: basis rows in FP32 (hardware exp), FP32 weights, FP32-accumulating
// MFMA 16x16x4 (operands as the f64 instruction; accumulator element i of
// lane l is D[4(l/16) + i][l%16]).
template <int RT, int CT, int CH>
__global__ void __launch_bounds__(kThreads) k_contract_fp32(const EvalConsts *__restrict__ cp,
                                                            const double *__restrict__ params, int64_t ld,
                                                            int64_t b0, int64_t nb,
                                                            const double *__restrict__ nodes,
                                                            const float *__restrict__ W,
                                                            double *__restrict__ Y) {
  constexpr int CW = CT * 16;
  constexpr int QT = kWaves * RT * 16;
  __shared__ float Ws[CH][CW + kLdsPad];
  __shared__ float Xs[CH][4];
  __shared__ int poly[kMaxPoly][3];
  const EvalConsts &c = *cp;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col0 = blockIdx.y * CW;
  const int64_t qbase = (int64_t)blockIdx.x * QT + wave * RT * 16;
  const int N = c.N, NM = c.N + c.M, rows = c.rows, Kp = c.Kp;
  const float eps2 = (float)c.eps2;
  for (int e = threadIdx.x; e < kMaxPoly * 3; e += kThreads) poly[e / 3][e % 3] = c.poly_idx[e / 3][e % 3];
  float xq[RT][4];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t b = qbase + rt * 16 + (lane & 15);
#pragma unroll
    for (int d = 0; d < 4; ++d) xq[rt][d] = b < nb ? (float)(params[d * ld + b0 + b] / c.semi[d]) : 0.0f;
  }
  f4 acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  const int kk = lane >> 4;
  for (int r0 = 0; r0 < rows; r0 += CH) {
    __syncthreads();
    for (int e = threadIdx.x; e < CH * CW; e += kThreads) {
      const int r = e / CW, cc = e % CW;
      Ws[r][cc] = W[(int64_t)(r0 + r) * Kp + col0 + cc];
    }
    for (int e = threadIdx.x; e < CH * 4; e += kThreads)
      Xs[e >> 2][e & 3] = (float)nodes[(int64_t)r0 * 4 + e];
    __syncthreads();
#pragma unroll 2
    for (int s = 0; s < CH / 4; ++s) {
      const int rr = 4 * s + kk;
      float a[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) a[rt] = basis_row_fp32(r0 + rr, N, NM, xq[rt], Xs[rr], eps2, poly);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const float bv = Ws[rr][ct * 16 + (lane & 15)];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt], bv, acc[rt][ct], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t b = qbase + rt * 16 + 4 * (lane >> 4) + i;
      if (b >= nb) continue;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) Y[b * Kp + col0 + ct * 16 + (lane & 15)] = (double)acc[rt][ct][i];
    }
  }
}

// The epilogue runs in two phases per block of kEpiBatch proposals.
//
// Setup (one lane per proposal): the proposal's domain flags (inside the
// ellipsoid, physical, every detector's spline stencil inside the window, no
// NaN input), each detector's arrival-time position (stencil base and
// fraction), each (detector, mode) amplitude A_{k,lm} =
// [(F+ + iFx) Y_{l,-m} + (-1)^l (F+ - iFx) conj(Y_lm)] / 2 (Eq. logl_complete,
// corrected reading) and d_ref / d_L, into LDS.  These need transcendental
// functions but not the interpolated coefficients, so a lane per proposal
// does them once instead of a wave per proposal.
//
// Reduction (one wave per proposal): the lanes are split over the (detector,
// mode) pairs -- G = 64 / (n_det * n_modes) lanes per pair -- and each pair's
// lanes stride over its q basis coefficients: lane g of pair (k, a)
// accumulates sum_i C_i sum_p f^p B4[n0][i][p] over i = g, g+G, ... with the
// spline-folded basis B4 (the entries of one row are contiguous in i, so the
// G lanes of a pair read adjacent 64-byte groups).  Partial sums meet in the pair's first lane by shuffles; that lane
// forms Re(conj(A) z), the detector's first lane the overlap term, lane 0 the
// sum, all with compensated (Neumaier) additions.
constexpr int kEpiBatch = 64;
static_assert(kEpiBatch + RBFL_MAX_DET * RBFL_MAX_MODES <= kThreads, "offset copy threads");

// ln L of one proposal from its setup o and interpolated row y; one whole
// wave per call, result written to *out by lane 0.  The loads of each stage
// are issued together before their values are used (kEpiUnroll coefficients
// per lane at a time, the detector's overlap reals one per lane), so a
// proposal waits for a few memory round trips instead of one per coefficient.
constexpr int kEpiUnroll = 2;

// coef_off / sig_off: the output offsets of the consts (an LDS copy where the
// block has one).
__device__ __forceinline__ void epi_reduce(const EvalConsts &c, const EpiSetup &o, const double *__restrict__ y,
                                           const double2 *__restrict__ basis4, double *__restrict__ out,
                                           const int (*coef_off)[RBFL_MAX_MODES], const int *sig_off) {
  const int lane = threadIdx.x & 63;
  if (o.status != 0) {
    if (lane == 0) *out = o.status == 2 ? __builtin_nan("") : -__builtin_huge_val();
    return;
  }
  const int n_modes = c.n_modes, q = c.q, T = c.T;
  const int P = c.n_det * n_modes;
  const int G = 64 / P;
  const int pair = lane / G;
  const int gl = lane - pair * G;
  const bool active = pair < P;
  const int k = active ? pair / n_modes : 0;
  const int a = active ? pair - k * n_modes : 0;
  const double f = o.f[k];
  const int n0 = o.n0[k];
  const double ar = o.Ar[k][a], ai = o.Ai[k][a];
  const int det_lead = k * n_modes * G;
  // detector k's overlap reals: lane det_lead + t holds term t (t < n_modes:
  // sigma_tt; then (Re, Im) sigma_ab for a < b in lexicographic order).  A
  // detector owns n_modes * G >= n_modes (n_modes + 1) / 2 lanes for up to 4
  // detectors and 5 modes.
  const int n_terms = n_modes * (n_modes + 1) / 2;
  const int t_own = lane - det_lead;
  double sg_a = 0.0, sg_b = 0.0;
  if (active && t_own < n_terms) {
    const int so = sig_off[k];
    if (t_own < n_modes) {
      sg_a = y[so + t_own];
    } else {
      const int pidx = so + n_modes + 2 * (t_own - n_modes);
      sg_a = y[pidx];
      sg_b = y[pidx + 1];
    }
  }
  // a5: partial reconstruction of z_{k,a} over this lane's coefficients; the
  // spline-folded basis gives the interpolated basis value as a cubic in f
  double zr = 0.0, zi = 0.0;
  if (active) {
    const int off = coef_off[k][a];
    const double2 *base = basis4 + ((int64_t)(k * n_modes + a) * T + n0) * q * 4;
    for (int i0 = gl; i0 < q; i0 += kEpiUnroll * G) {
      double2 cc[kEpiUnroll], v[kEpiUnroll][4];
#pragma unroll
      for (int u = 0; u < kEpiUnroll; ++u) {
        // past the end: a valid entry is loaded and its coefficient zeroed,
        // so that every load is issued before the first use
        const bool ok = i0 + u * G < q;
        const int i = ok ? i0 + u * G : i0;
        const double2 cv = *reinterpret_cast<const double2 *>(y + off + 2 * i);
        cc[u].x = ok ? cv.x : 0.0;
        cc[u].y = ok ? cv.y : 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[u][j] = base[4 * i + j];
      }
#pragma unroll
      for (int u = 0; u < kEpiUnroll; ++u) {
        const double br = fma(fma(fma(v[u][3].x, f, v[u][2].x), f, v[u][1].x), f, v[u][0].x);
        const double bi = fma(fma(fma(v[u][3].y, f, v[u][2].y), f, v[u][1].y), f, v[u][0].y);
        zr += cc[u].x * br - cc[u].y * bi;
        zi += cc[u].x * bi + cc[u].y * br;
      }
    }
  }
  // combine the G partials of each pair in its first lane (fixed order)
  const int lead = pair * G;
  double tr = 0.0, ti = 0.0;
  for (int j = 0; j < G; ++j) {
    tr += __shfl(zr, lead + j, 64);
    ti += __shfl(zi, lead + j, 64);
  }
  const double zterm = ar * tr + ai * ti;   // Re(conj(A) z), valid in pair leaders
  // overlap term of detector k: every A_{k,b} is in the setup
  double st_s = 0.0, st_c = 0.0, zt_s = 0.0, zt_c = 0.0;
  {
    auto add = [](double &sum, double &comp, double v) {
      const double t = sum + v;
      comp += fabs(sum) >= fabs(v) ? (sum - t) + v : (v - t) + sum;
      sum = t;
    };
    for (int m = 0; m < n_modes; ++m) {
      add(zt_s, zt_c, __shfl(zterm, det_lead + m * G, 64));
      add(st_s, st_c, (o.Ar[k][m] * o.Ar[k][m] + o.Ai[k][m] * o.Ai[k][m]) * __shfl(sg_a, det_lead + m, 64));
    }
    int t = n_modes;
    for (int m = 0; m < n_modes; ++m)
      for (int mm = m + 1; mm < n_modes; ++mm) {
        const double sr = __shfl(sg_a, det_lead + t, 64), si = __shfl(sg_b, det_lead + t, 64);
        ++t;
        const double pr = o.Ar[k][m] * o.Ar[k][mm] + o.Ai[k][m] * o.Ai[k][mm];
        const double pi = o.Ar[k][m] * o.Ai[k][mm] - o.Ai[k][m] * o.Ar[k][mm];
        add(st_s, st_c, 2.0 * (pr * sr - pi * si));
      }
  }
  const double rr = o.rr;
  const double term = rr * (zt_s + zt_c) - 0.5 * rr * rr * (st_s + st_c);   // valid in detector leaders
  double tot = 0.0, comp = 0.0;
  for (int kk = 0; kk < c.n_det; ++kk) {
    const double v = __shfl(term, kk * n_modes * G, 64);
    const double t = tot + v;
    comp += fabs(tot) >= fabs(v) ? (tot - t) + v : (v - t) + tot;
    tot = t;
  }
  if (lane == 0) *out = tot + comp;
}

__global__ void __launch_bounds__(kThreads) k_epilogue(const EvalConsts *__restrict__ cp,
                                                       const double *__restrict__ params, int64_t ld, int64_t b0,
                                                       int64_t nb, const double *__restrict__ Y,
                                                       const double2 *__restrict__ basis4, double *__restrict__ lnl) {
  __shared__ EpiSetup su[kEpiBatch];
  __shared__ int coef_off[RBFL_MAX_DET][RBFL_MAX_MODES], sig_off[RBFL_MAX_DET];
  const EvalConsts &c = *cp;
  const int64_t first = (int64_t)blockIdx.x * kEpiBatch;
  if (threadIdx.x < kEpiBatch && first + threadIdx.x < nb) epi_setup(c, params, ld, b0 + first + threadIdx.x, su[threadIdx.x]);
  if (threadIdx.x >= kEpiBatch && threadIdx.x < kEpiBatch + RBFL_MAX_DET * RBFL_MAX_MODES) {
    const int e = threadIdx.x - kEpiBatch;
    coef_off[e / RBFL_MAX_MODES][e % RBFL_MAX_MODES] = c.coef_off[e / RBFL_MAX_MODES][e % RBFL_MAX_MODES];
    if (e < RBFL_MAX_DET) sig_off[e] = c.sig_off[e];
  }
  __syncthreads();
  for (int j = threadIdx.x >> 6; j < kEpiBatch; j += kWaves) {
    const int64_t b = first + j;
    if (b >= nb) break;   // whole wave leaves together
    epi_reduce(c, su[j], Y + b * c.Kp, basis4, lnl + b0 + b, coef_off, sig_off);
  }
}

// Epilogue of the time-banded form (n_bands = B > 1): one wave per proposal,
// one lane per (block v, mode a) pair at a time.  Block v = k B + b is
// detector k over band b, where mode a sees the source at right ascension
// alpha - rate (t_c + t_ba - t_trig); that gives the lane its own antenna
// factor A_va and arrival-time stencil.  The lane reconstructs z_va from all
// q coefficients (spline-folded basis, as the frozen epilogue) and forms
// r Re(conj(A_va) z_va) - r^2/2 [|A_va|^2 sigma_aa + 2 sum_{c > a}
// Re(conj(A_va) A_vc sigma_ac)], taking A_vc from the lanes of the same block
// (a chunk of lanes holds whole blocks, floor(64 / n_modes) of them).  A
// stencil outside the window makes the proposal -inf, as in the frozen form;
// the lanes' terms meet in lane order with compensated additions.
__global__ void __launch_bounds__(kThreads) k_epilogue_banded(const EvalConsts *__restrict__ cp,
                                                              const double *__restrict__ params, int64_t ld,
                                                              int64_t b0, int64_t nb, const double *__restrict__ Y,
                                                              const double2 *__restrict__ basis4,
                                                              double *__restrict__ lnl) {
  const EvalConsts &c = *cp;
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (g >= nb) return;   // whole wave leaves together
  double p[11];
  const int pre = epi_prelude(c, params, ld, b0 + g, p);
  if (pre != 0) {   // NaN input, or outside the ellipsoid or the physical region
    if (lane == 0) lnl[b0 + g] = pre == 2 ? __builtin_nan("") : -__builtin_huge_val();
    return;
  }
  const double alpha = p[4], dec = p[5], psi = p[6], iota = p[7], phi = p[8], tc = p[9], dl = p[10];
  const double rr = c.d_ref / dl;
  double ch, sh;
  sincos(0.5 * iota, &sh, &ch);
  const int nm = c.n_modes, q = c.q, T = c.T, B = c.n_bands;
  const int per = (64 / nm) * nm;
  const int n_pairs = c.n_v * nm;
  const double *y = Y + g * c.Kp;
  bool ok = true;
  double sum = 0.0, comp = 0.0;
  for (int p0 = 0; p0 < n_pairs; p0 += per) {
    const int pr = p0 + lane;
    const bool active = lane < per && pr < n_pairs;
    const int v = active ? pr / nm : 0;
    const int a = active ? pr - v * nm : 0;
    const int k = v / B, bd = v - k * B;
    double ar = 0.0, ai = 0.0, term = 0.0;
    if (active) {
      const double al = alpha - c.earth_rate * (tc + c.band_t[bd][a] - c.t_trig);
      double fp, fc, dt;
      detector_response(c.D[k], c.r[k], al, dec, psi, &fp, &fc, &dt);
      double ynr, yni, ypr, ypi;
      eval_ylm(c.ylm_neg[a], ch, sh, phi, &ynr, &yni);
      eval_ylm(c.ylm_pos[a], ch, sh, phi, &ypr, &ypi);
      const double sg = (c.mode_l[a] & 1) ? -1.0 : 1.0;
      ar = 0.5 * ((fp * ynr - fc * yni) + sg * (fp * ypr - fc * ypi));
      ai = 0.5 * ((fp * yni + fc * ynr) + sg * (-fp * ypi - fc * ypr));
      const double s = (tc + dt - c.t_trig) * c.fs + (double)c.half_w;
      const double fl = floor(s);
      const bool in = fl >= 4.0 && fl <= (double)(T - 6);
      ok = ok && in;
      if (in) {
        const double f = s - fl;
        const double2 *base = basis4 + ((int64_t)pr * T + (int)fl) * q * 4;   // pair pr = v n_modes + a
        const double *cf = y + c.coef_off[v][a];
        double zr = 0.0, zi = 0.0;
        for (int i = 0; i < q; ++i) {
          const double cr = cf[2 * i], ci = cf[2 * i + 1];
          const double2 w0 = base[4 * i], w1 = base[4 * i + 1], w2 = base[4 * i + 2], w3 = base[4 * i + 3];
          const double br = fma(fma(fma(w3.x, f, w2.x), f, w1.x), f, w0.x);
          const double bi = fma(fma(fma(w3.y, f, w2.y), f, w1.y), f, w0.y);
          zr += cr * br - ci * bi;
          zi += cr * bi + ci * br;
        }
        term = rr * (ar * zr + ai * zi);
      }
    }
    // the pair's row of the overlap term; the block's lanes are lead .. lead + nm - 1
    const int lead = lane - a;
    const int so = c.sig_off[v];
    double st = active ? (ar * ar + ai * ai) * y[so + a] : 0.0;
    for (int cc = 1; cc < nm; ++cc) {
      const double br = __shfl(ar, (lead + cc) & 63, 64), bi = __shfl(ai, (lead + cc) & 63, 64);
      if (active && cc > a) {
        const int idx = a * nm - a * (a + 1) / 2 + (cc - a - 1);   // (a, cc) in lexicographic order
        const double sr = y[so + nm + 2 * idx], si = y[so + nm + 2 * idx + 1];
        const double pr_ = ar * br + ai * bi, pi_ = ar * bi - ai * br;
        st += 2.0 * (pr_ * sr - pi_ * si);
      }
    }
    term -= 0.5 * rr * rr * st;
    const double t = sum + term;
    comp += fabs(sum) >= fabs(term) ? (sum - t) + term : (term - t) + sum;
    sum = t;
  }
  const bool all_ok = __all(ok ? 1 : 0) != 0;
  const double mine = sum + comp;
  double tot = 0.0, tc_ = 0.0;
  for (int j = 0; j < 64; ++j) {
    const double vj = __shfl(mine, j, 64);
    const double t = tot + vj;
    tc_ += fabs(tot) >= fabs(vj) ? (tot - t) + vj : (vj - t) + tot;
    tot = t;
  }
  if (lane == 0) lnl[b0 + g] = all_ok ? tot + tc_ : -__builtin_huge_val();
}

// Epilogue finished inside the contraction (FP64 form, optional): ln L is
// linear in the interpolated outputs, ln L = sum_c coef_c(proposal) Y[c], so
// the contraction kernel forms coef_c from each proposal's setup and sums
// coef_c Y[c] over its column tile instead of writing Y; these two kernels
// write the setups before it and add the column tiles' partial sums after it
// (compensated, in tile order).
__global__ void __launch_bounds__(kThreads) k_epi_setup(const EvalConsts *__restrict__ cp,
                                                        const double *__restrict__ params, int64_t ld, int64_t b0,
                                                        int64_t nb, EpiSetup *__restrict__ setups) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b < nb) epi_setup(*cp, params, ld, b0 + b, setups[b]);
}

__global__ void __launch_bounds__(kThreads) k_lnl_tiles(const EpiSetup *__restrict__ setups, int64_t b0, int64_t nb,
                                                        const double *__restrict__ part, int64_t ldp, int n_ct,
                                                        double *__restrict__ lnl) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= nb) return;
  const int st = setups[b].status;
  if (st != 0) {
    lnl[b0 + b] = st == 2 ? __builtin_nan("") : -__builtin_huge_val();
    return;
  }
  double tot = 0.0, comp = 0.0;
  for (int t = 0; t < n_ct; ++t) {
    const double v = part[(int64_t)t * ldp + b];
    const double u = tot + v;
    comp += fabs(tot) >= fabs(v) ? (tot - u) + v : (v - u) + tot;
    tot = u;
  }
  lnl[b0 + b] = tot + comp;
}

// ln L of a batch straight from window samples (no time basis): per detector
// and mode, z at the arrival time is the spline through the 10 samples of
// Z[n_det][n_modes][nb][T] around it; overlaps sig[n_det][nb][n_modes][n_modes].
// Domain, window and NaN handling as in the epilogue.  One thread per
// proposal (a reference path, not a tuned one).
__global__ void __launch_bounds__(kThreads) k_series_lnl(const EvalConsts *__restrict__ cp,
                                                         const double *__restrict__ params, int64_t ld, int64_t b0,
                                                         int64_t nb, const double2 *__restrict__ Z,
                                                         const double2 *__restrict__ sig, double *__restrict__ lnl) {
  const int64_t b = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (b >= nb) return;
  const EvalConsts &c = *cp;
  EpiSetup o;
  epi_setup(c, params, ld, b0 + b, o);
  if (o.status != 0) {
    lnl[b0 + b] = o.status == 2 ? __builtin_nan("") : -__builtin_huge_val();
    return;
  }
  const int n_modes = c.n_modes, T = c.T;
  double tot = 0.0, comp = 0.0;
  for (int k = 0; k < c.n_det; ++k) {
    const double f = o.f[k];
    double w[kSplineTaps];
    for (int t = 0; t < kSplineTaps; ++t)
      w[t] = fma(fma(fma(c.spline[t][3], f, c.spline[t][2]), f, c.spline[t][1]), f, c.spline[t][0]);
    double zt = 0.0, st = 0.0;
    for (int a = 0; a < n_modes; ++a) {
      const double2 *za = Z + ((int64_t)(k * n_modes + a) * nb + b) * T + o.n0[k] - 4;
      double zr = 0.0, zi = 0.0;
      for (int t = 0; t < kSplineTaps; ++t) {
        zr = fma(w[t], za[t].x, zr);
        zi = fma(w[t], za[t].y, zi);
      }
      zt += o.Ar[k][a] * zr + o.Ai[k][a] * zi;                       // Re(conj(A_a) z_a)
      for (int m = 0; m < n_modes; ++m) {
        const double2 sv = sig[(((int64_t)k * nb + b) * n_modes + a) * n_modes + m];
        const double pr = o.Ar[k][a] * o.Ar[k][m] + o.Ai[k][a] * o.Ai[k][m];
        const double pim = o.Ar[k][a] * o.Ai[k][m] - o.Ai[k][a] * o.Ar[k][m];
        st += pr * sv.x - pim * sv.y;                                 // Re(conj(A_a) A_m sigma_am)
      }
    }
    const double v = o.rr * zt - 0.5 * o.rr * o.rr * st;
    const double t = tot + v;
    comp += fabs(tot) >= fabs(v) ? (tot - t) + v : (v - t) + tot;
    tot = t;
  }
  lnl[b0 + b] = tot + comp;
}

// ---- multi-event (ragged) batch --------------------------------------------

// Persistent contraction over the work list of every event: items are
// (event, proposal tile, column tile), numbered event by event in the
// caller's cost order; each block takes the next item from an atomic counter
// until the list is exhausted (every block reaches that exit).
template <int RT, int CT, int CH>
__global__ void __launch_bounds__(kThreads) k_ragged_contract_fp64(const EventDesc *__restrict__ ev, int n_ev,
                                                                   int64_t total_items,
                                                                   unsigned long long *__restrict__ counter,
                                                                   const double *__restrict__ params, int64_t ld) {
  __shared__ long long item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t item = item_s;
    __syncthreads();
    if (item >= total_items) break;
    const EventDesc &d = ev[work_event(ev, n_ev, item)];
    const int64_t local = item - d.item0;
    const int tq = (int)(local % d.tiles_q);
    const int tc = (int)(local / d.tiles_q);
    contract_tile_fp64<RT, CT, CH>(*d.consts, params, ld, d.q0, d.n, d.nodes, d.W, d.Y, tq, tc);
  }
}

__global__ void k_zero_counter(unsigned long long *counter) {
  if (threadIdx.x == 0) *counter = 0ull;
}

// The epilogue's two phases over the concatenated batch; each proposal's
// event is found in the setup phase by binary search over the events' first
// proposals (caller order).
__global__ void __launch_bounds__(kThreads) k_ragged_epilogue(const EventDesc *__restrict__ ev, int n_ev,
                                                              const double *__restrict__ params, int64_t total,
                                                              double *__restrict__ lnl) {
  __shared__ EpiSetup su[kEpiBatch];
  const int64_t first = (int64_t)blockIdx.x * kEpiBatch;
  if (threadIdx.x < kEpiBatch && first + threadIdx.x < total) {
    const int64_t g = first + threadIdx.x;
    int lo = 0, hi = n_ev - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ev[mid].q0 <= g) lo = mid;
      else hi = mid - 1;
    }
    epi_setup(*ev[lo].consts, params, total, g, su[threadIdx.x]);
    su[threadIdx.x].event = lo;
  }
  __syncthreads();
  for (int j = threadIdx.x >> 6; j < kEpiBatch; j += kWaves) {
    const int64_t g = first + j;
    if (g >= total) break;   // whole wave leaves together
    const EventDesc &d = ev[su[j].event];
    epi_reduce(*d.consts, su[j], d.Y + (g - d.q0) * d.Kp, d.basis, lnl + g, d.consts->coef_off, d.consts->sig_off);
  }
}

// NaN entries of lnl[0, n): block b writes its grid-stride share's count to
// part[b] (every block writes, so the slots need no clearing).
__global__ void __launch_bounds__(256) k_count_nan(const double *__restrict__ lnl, int64_t n,
                                                   unsigned long long *__restrict__ part) {
  __shared__ unsigned long long cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  unsigned long long mine = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    mine += isnan(lnl[i]) ? 1ull : 0ull;
  if (mine) atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = cnt;
}

// Surrogate inputs: x = delta_e / a in FP32, [nb][4].
__global__ void k_sur_inputs(const double *__restrict__ params, int64_t ld, int64_t b0, int64_t nb,
                             const EvalConsts *__restrict__ c, float *__restrict__ x) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= nb) return;
  for (int d = 0; d < 4; ++d) x[b * 4 + d] = (float)(params[d * ld + b0 + b] / c->semi[d]);
}

// Residual-form surrogate: the base monomials of u = (x - m) / s in FP64.
__global__ void k_sur_base_inputs(const double *__restrict__ params, int64_t ld, int64_t b0, int64_t nb,
                                  const EvalConsts *__restrict__ c, const double *__restrict__ ms,
                                  const int *__restrict__ poly, int nbase, double *__restrict__ U) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= nb) return;
  double u[4];
  for (int d = 0; d < 4; ++d) u[d] = (params[d * ld + b0 + b] / c->semi[d] - ms[d]) / ms[4 + d];
  for (int p = 0; p < nbase; ++p) {
    double v = 1.0;
    for (int t = 0; t < 3; ++t) {
      const int i = poly[3 * p + t];
      if (i >= 0) v *= u[i];
    }
    U[b * nbase + p] = v;
  }
}

// Per-column mean and standard deviation of Y [n][K] (two passes, FP64).
__global__ void k_col_stats(const double *__restrict__ Y, int64_t n, int K, float *__restrict__ mu,
                            float *__restrict__ sd) {
  const int k = blockIdx.x;
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < n; b += 256) s += Y[b * K + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double mean = red[0] / (double)n;
  __syncthreads();
  double v = 0.0;
  for (int64_t b = threadIdx.x; b < n; b += 256) {
    const double d = Y[b * K + k] - mean;
    v += d * d;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mu[k] = (float)mean;
    const double sdev = sqrt(red[0] / (double)n);
    sd[k] = (float)(sdev > 0.0 ? sdev : 1.0);
  }
}

__global__ void k_standardise(const double *__restrict__ Y, int64_t n, int K, const float *__restrict__ mu,
                              const float *__restrict__ sd, float *__restrict__ T) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * K) return;
  const int k = (int)(e % K);
  T[e] = (float)((Y[e] - (double)mu[k]) / (double)sd[k]);
}

__global__ void k_convert_weights(const double *__restrict__ W, size_t n, float *__restrict__ hi,
                                  uint16_t *__restrict__ b16) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double v = W[e];
  const float h = (float)v;
  if (hi) hi[e] = h;
  if (b16) {
    // round to nearest even on the upper 16 bits of the FP32 value
    uint32_t u = __float_as_uint((float)v);
    const uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
    b16[e] = (uint16_t)((u + r) >> 16);
  }
}

}  // namespace

template <int RT, int CT, int CH>
static void launch_fp64_variant(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld,
                                int64_t b0, int64_t nb, const double *nodes, const double *W, double *Y,
                                hipStream_t s) {
  static_assert(kColTile % (CT * 16) == 0, "K is padded to a multiple of every column tile");
  const int64_t qt = kWaves * RT * 16;
  const int cw = CT * 16;
  dim3 grid((unsigned)((nb + qt - 1) / qt), (unsigned)((hc.Kp + cw - 1) / cw));
  hipLaunchKernelGGL((k_contract_fp64<RT, CT, CH>), grid, dim3(kThreads), 0, s, c, params, ld, b0, nb, nodes, W, Y);
  RBFL_HIP(hipGetLastError());
}

int contract_variants(int form) {
  return form == RBFL_FORM_FP64 ? gemm_fp64_variants() + 1 : form == RBFL_FORM_SPLIT ? split_variant_count() : form == RBFL_FORM_BF16 ? 1 : 2;
}

const char *contract_variant_name(int form, int v) {
  static const char *f64[] = {"fp64 rt2 ct4 ch32", "fp64 rt2 ct4 ch16", "fp64 rt2 ct8 ch16", "fp64 rt4 ct4 ch16",
                              "fp64 rt4 ct2 ch32"};
  static const char *f32[] = {"fp32 rt2 ct4 ch32", "fp32 rt2 ct8 ch32"};
  if (form == RBFL_FORM_FP64) return v < gemm_fp64_variants() ? gemm_fp64_variant_name(v) : "fused rt2 ct8 ch16";
  if (form == RBFL_FORM_BF16) return "bf16 64x64 16x16x32";
  return form == RBFL_FORM_SPLIT ? split_variant_name(v) : f32[v];
}

void launch_contract_fp64(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                          int64_t nb, const double *nodes, const double *W, double *Y, hipStream_t s, int variant) {
  switch (variant) {
    case 1: launch_fp64_variant<2, 4, 16>(c, hc, params, ld, b0, nb, nodes, W, Y, s); break;
    case 2: launch_fp64_variant<2, 8, 16>(c, hc, params, ld, b0, nb, nodes, W, Y, s); break;
    case 3: launch_fp64_variant<4, 4, 16>(c, hc, params, ld, b0, nb, nodes, W, Y, s); break;
    case 4: launch_fp64_variant<4, 2, 32>(c, hc, params, ld, b0, nb, nodes, W, Y, s); break;
    default: launch_fp64_variant<2, 4, 32>(c, hc, params, ld, b0, nb, nodes, W, Y, s);
  }
}

template <int RT, int CT, int CH>
static void launch_fp32_variant(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld,
                                int64_t b0, int64_t nb, const double *nodes, const float *W, double *Y,
                                hipStream_t s) {
  static_assert(kColTile % (CT * 16) == 0 && kRowChunk % CH == 0, "K and the rows are padded to whole tiles");
  const int64_t qt = kWaves * RT * 16;
  const int cw = CT * 16;
  dim3 grid((unsigned)((nb + qt - 1) / qt), (unsigned)((hc.Kp + cw - 1) / cw));
  hipLaunchKernelGGL((k_contract_fp32<RT, CT, CH>), grid, dim3(kThreads), 0, s, c, params, ld, b0, nb, nodes, W, Y);
  RBFL_HIP(hipGetLastError());
}

void launch_contract_fp32(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                          int64_t nb, const double *nodes, const float *W, double *Y, hipStream_t s, int variant) {
  if (variant == 1)
    launch_fp32_variant<2, 8, 32>(c, hc, params, ld, b0, nb, nodes, W, Y, s);
  else
    launch_fp32_variant<2, 4, 32>(c, hc, params, ld, b0, nb, nodes, W, Y, s);
}


// Multi-event variants: 0-2 the fused persistent kernel, 3-4 basis rows +
// persistent GEMM (64 x 128 tiles, 8- and 16-row chunks).
int ragged_variants() { return 6; }
int ragged_fused_variants() { return 3; }
int ragged_blocks_per_cu(int variant) { return variant < 3 ? 2 : variant == 3 ? 4 : variant == 4 ? 3 : 2; }

void ragged_tile(int variant, int *qt, int *cw) {
  static const int q[] = {128, 128, 128, 64, 64, 128}, w[] = {128, 64, 64, 128, 128, 128};
  *qt = q[variant];
  *cw = w[variant];
}

template <int RT, int CT, int CH>
static void launch_ragged_variant(const EventDesc *ev, int n_ev, int64_t total_items, unsigned long long *counter,
                                  const double *params, int64_t ld, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, counter);
  RBFL_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_ragged_contract_fp64<RT, CT, CH>), dim3(grid), dim3(kThreads), 0, s, ev, n_ev, total_items,
                     counter, params, ld);
  RBFL_HIP(hipGetLastError());
}

void launch_ragged_contract(int variant, const EventDesc *ev, int n_ev, int64_t total_items,
                            unsigned long long *counter, const double *params, int64_t ld, int grid, hipStream_t s) {
  switch (variant) {
    case 1: launch_ragged_variant<2, 4, 32>(ev, n_ev, total_items, counter, params, ld, grid, s); break;
    case 2: launch_ragged_variant<2, 4, 16>(ev, n_ev, total_items, counter, params, ld, grid, s); break;
    default: launch_ragged_variant<2, 8, 16>(ev, n_ev, total_items, counter, params, ld, grid, s);
  }
}

void launch_ragged_epilogue(const EventDesc *ev, int n_ev, const double *params, int64_t total, double *lnl,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_ragged_epilogue, dim3((unsigned)((total + kEpiBatch - 1) / kEpiBatch)), dim3(kThreads), 0, s,
                     ev, n_ev, params, total, lnl);
  RBFL_HIP(hipGetLastError());
}

void launch_epilogue(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                     int64_t nb, const double *Y, const double2 *basis, double *lnl, hipStream_t s) {
  if (nb <= 0) return;
  if (hc.n_bands > 1) {
    hipLaunchKernelGGL(k_epilogue_banded, dim3((unsigned)((nb + kWaves - 1) / kWaves)), dim3(kThreads), 0, s, c,
                       params, ld, b0, nb, Y, basis, lnl);
  } else {
    dim3 grid((unsigned)((nb + kEpiBatch - 1) / kEpiBatch));
    hipLaunchKernelGGL(k_epilogue, grid, dim3(kThreads), 0, s, c, params, ld, b0, nb, Y, basis, lnl);
  }
  RBFL_HIP(hipGetLastError());
}

size_t epi_setup_bytes() { return sizeof(EpiSetup); }

void launch_epi_setup(const EvalConsts *c, const double *params, int64_t ld, int64_t b0, int64_t nb, void *setups,
                      hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_epi_setup, dim3((unsigned)((nb + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, c, params,
                     ld, b0, nb, static_cast<EpiSetup *>(setups));
  RBFL_HIP(hipGetLastError());
}

void launch_lnl_tiles(const void *setups, int64_t b0, int64_t nb, const double *part, int64_t ldp, int n_ct,
                      double *lnl, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_lnl_tiles, dim3((unsigned)((nb + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     static_cast<const EpiSetup *>(setups), b0, nb, part, ldp, n_ct, lnl);
  RBFL_HIP(hipGetLastError());
}

void launch_series_lnl(const EvalConsts *c, const double *params, int64_t ld, int64_t b0, int64_t nb,
                       const double2 *Z, const double2 *sig, double *lnl, hipStream_t s) {
  hipLaunchKernelGGL(k_series_lnl, dim3((unsigned)((nb + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, c, params,
                     ld, b0, nb, Z, sig, lnl);
  RBFL_HIP(hipGetLastError());
}

void launch_count_nan(const double *lnl, int64_t n, unsigned long long *part, hipStream_t s) {
  hipLaunchKernelGGL(k_count_nan, dim3(kNanParts), dim3(256), 0, s, lnl, n, part);
  RBFL_HIP(hipGetLastError());
}

void launch_sur_base_inputs(const double *params, int64_t ld, int64_t b0, int64_t nb, const EvalConsts *c,
                            const double *ms, const int *poly, int nbase, double *U, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_sur_base_inputs, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, params, ld, b0, nb, c,
                     ms, poly, nbase, U);
  RBFL_HIP(hipGetLastError());
}

void launch_sur_inputs(const double *params, int64_t ld, int64_t b0, int64_t nb, const EvalConsts *c, float *x,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_sur_inputs, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, params, ld, b0, nb, c, x);
  RBFL_HIP(hipGetLastError());
}

void launch_col_stats(const double *Y, int64_t n, int K, float *mu, float *sd, hipStream_t s) {
  hipLaunchKernelGGL(k_col_stats, dim3(K), dim3(256), 0, s, Y, n, K, mu, sd);
  RBFL_HIP(hipGetLastError());
}

void launch_standardise(const double *Y, int64_t n, int K, const float *mu, const float *sd, float *T,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_standardise, dim3((unsigned)((n * K + 255) / 256)), dim3(256), 0, s, Y, n, K, mu, sd, T);
  RBFL_HIP(hipGetLastError());
}

void launch_convert_weights(const double *W, size_t n, float *hi, uint16_t *b16, hipStream_t s) {
  hipLaunchKernelGGL(k_convert_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, n, hi, b16);
  RBFL_HIP(hipGetLastError());
}

}  // namespace rbfl
