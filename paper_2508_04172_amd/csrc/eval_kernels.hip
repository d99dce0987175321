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
#include "rbfl_internal.h"

namespace rbfl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kLdsPad = 16;   // doubles of padding per LDS row (bank spread across the 4 k-groups)

// Value of basis row `row` at x.  xn: the node's coordinates (row < N).
__device__ __forceinline__ double basis_row_fp64(int row, int N, int NM, const double x[4], const double *xn,
                                                 double eps2, const int (*poly)[3]) {
  if (row < N) {
    double d2 = 0.0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const double t = x[d] - xn[d];
      d2 = fma(t, t, d2);
    }
    return exp(-eps2 * d2);
  }
  if (row < NM) {
    const int p = row - N;
    double v = 1.0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int id = poly[p][s];
      if (id >= 0) v *= x[id];
    }
    return v;
  }
  return 0.0;
}

__device__ __forceinline__ float basis_row_fp32(int row, int N, int NM, const float x[4], const float *xn,
                                                float eps2, const int (*poly)[3]) {
  if (row < N) {
    float d2 = 0.0f;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const float t = x[d] - xn[d];
      d2 = fmaf(t, t, d2);
    }
    return __expf(-eps2 * d2);
  }
  if (row < NM) {
    const int p = row - N;
    float v = 1.0f;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int id = poly[p][s];
      if (id >= 0) v *= x[id];
    }
    return v;
  }
  return 0.0f;
}

// Block tile: kWaves waves along the proposals, each wave RT x 16 proposals
// by CT x 16 outputs; the block covers kWaves*RT*16 proposals and CT*16
// outputs.  MFMA f64 16x16x4 operand layout (measured on gfx950): lane l
// holds A[l%16][l/16] and B[l/16][l%16]; accumulator element i of lane l is
// D[l/16 + 4i][l%16].
template <int RT, int CT>
__global__ void __launch_bounds__(kThreads) k_contract_fp64(const EvalConsts *__restrict__ cp,
                                                            const double *__restrict__ params, int64_t ld,
                                                            int64_t b0, int64_t nb,
                                                            const double *__restrict__ nodes,
                                                            const double *__restrict__ W, double *__restrict__ Y) {
  constexpr int CW = CT * 16;
  constexpr int QT = kWaves * RT * 16;
  __shared__ double Ws[kRowChunk][CW + kLdsPad];
  __shared__ double Xs[kRowChunk][4];
  __shared__ int poly[kMaxPoly][3];
  const EvalConsts &c = *cp;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col0 = blockIdx.y * CW;
  const int64_t qbase = (int64_t)blockIdx.x * QT + wave * RT * 16;
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

  const int kk = lane >> 4;
  for (int r0 = 0; r0 < rows; r0 += kRowChunk) {
    __syncthreads();
    for (int e = threadIdx.x; e < kRowChunk * CW; e += kThreads) {
      const int r = e / CW, cc = e % CW;
      Ws[r][cc] = W[(int64_t)(r0 + r) * Kp + col0 + cc];
    }
    for (int e = threadIdx.x; e < kRowChunk * 4; e += kThreads) Xs[e >> 2][e & 3] = nodes[(int64_t)r0 * 4 + e];
    __syncthreads();
#pragma unroll 2
    for (int s = 0; s < kRowChunk / 4; ++s) {
      const int rr = 4 * s + kk;
      double a[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) a[rt] = basis_row_fp64(r0 + rr, N, NM, xq[rt], Xs[rr], eps2, poly);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const double bv = Ws[rr][ct * 16 + (lane & 15)];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt], bv, acc[rt][ct], 0, 0, 0);
      }
    }
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

// FP32 form: basis rows in FP32 (hardware exp), FP32 weights, FP32-accumulating
// MFMA 16x16x4 (operands as the f64 instruction; accumulator element i of
// lane l is D[4(l/16) + i][l%16]).  With split != 0
// the weights are W32 + W32lo (two FP32 products per step), which removes the
// weight rounding but not the FP32 rounding of the basis rows or of the sums.
template <int RT, int CT>
__global__ void __launch_bounds__(kThreads) k_contract_fp32(const EvalConsts *__restrict__ cp,
                                                            const double *__restrict__ params, int64_t ld,
                                                            int64_t b0, int64_t nb,
                                                            const double *__restrict__ nodes,
                                                            const float *__restrict__ W,
                                                            const float *__restrict__ Wlo, int split,
                                                            double *__restrict__ Y) {
  constexpr int CW = CT * 16;
  constexpr int QT = kWaves * RT * 16;
  __shared__ float Ws[kRowChunk][CW + kLdsPad];
  __shared__ float Wl[kRowChunk][CW + kLdsPad];
  __shared__ float Xs[kRowChunk][4];
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
  for (int r0 = 0; r0 < rows; r0 += kRowChunk) {
    __syncthreads();
    for (int e = threadIdx.x; e < kRowChunk * CW; e += kThreads) {
      const int r = e / CW, cc = e % CW;
      Ws[r][cc] = W[(int64_t)(r0 + r) * Kp + col0 + cc];
      if (split) Wl[r][cc] = Wlo[(int64_t)(r0 + r) * Kp + col0 + cc];
    }
    for (int e = threadIdx.x; e < kRowChunk * 4; e += kThreads)
      Xs[e >> 2][e & 3] = (float)nodes[(int64_t)r0 * 4 + e];
    __syncthreads();
#pragma unroll 2
    for (int s = 0; s < kRowChunk / 4; ++s) {
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
        if (split) {
          const float bl = Wl[rr][ct * 16 + (lane & 15)];
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt], bl, acc[rt][ct], 0, 0, 0);
        }
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Neumaier-compensated accumulation.
struct Comp {
  double s = 0.0, c = 0.0;
  __device__ void add(double v) {
    const double t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
  }
  __device__ double value() const { return s + c; }
};

// One wave per proposal.  Lanes split the q basis coefficients of each
// (detector, mode); the gathered basis rows are contiguous in the
// coefficient index, so the 10-sample stencil loads are coalesced.
__global__ void __launch_bounds__(kThreads) k_epilogue(const EvalConsts *__restrict__ cp,
                                                       const double *__restrict__ params, int64_t ld, int64_t b0,
                                                       int64_t nb, const double *__restrict__ Y,
                                                       const double2 *__restrict__ basis, double *__restrict__ lnl) {
  const EvalConsts &c = *cp;
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (b >= nb) return;
  const int64_t g = b0 + b;
  double p[11];
#pragma unroll
  for (int i = 0; i < 11; ++i) p[i] = params[i * ld + g];
  bool any_nan = false;
#pragma unroll
  for (int i = 0; i < 11; ++i) any_nan |= isnan(p[i]);
  if (any_nan) {
    if (lane == 0) lnl[g] = __builtin_nan("");
    return;
  }
  // a1: inside the ellipsoid and physical
  double r2 = 0.0;
  for (int d = 0; d < 4; ++d) {
    const double x = p[d] / c.semi[d];
    r2 += x * x;
  }
  bool valid = r2 <= 1.0;
  double th[4], phys[4];
  for (int i = 0; i < 4; ++i) {
    double t = c.theta_c[i];
    for (int j = 0; j < 4; ++j) t += c.V[4 * i + j] * p[j];
    th[i] = t;
  }
  valid = valid && theta_to_phys(th, c.f0, c.chi_max, phys);
  const double alpha = p[4], dec = p[5], psi = p[6], iota = p[7], phi = p[8], tc = p[9], dl = p[10];
  const double rr = c.d_ref / dl;
  const int n_modes = c.n_modes, q = c.q, T = c.T;
  // harmonics at (iota, phi)
  double ch, sh;
  sincos(0.5 * iota, &sh, &ch);
  double yn_r[RBFL_MAX_MODES], yn_i[RBFL_MAX_MODES], yp_r[RBFL_MAX_MODES], yp_i[RBFL_MAX_MODES];
  for (int a = 0; a < n_modes; ++a) {
    eval_ylm(c.ylm_neg[a], ch, sh, phi, &yn_r[a], &yn_i[a]);
    eval_ylm(c.ylm_pos[a], ch, sh, phi, &yp_r[a], &yp_i[a]);
  }
  const double *y = Y + b * c.Kp;
  Comp total;
  for (int k = 0; k < c.n_det && valid; ++k) {
    double fp, fc, dt;
    detector_response(c.D[k], c.r[k], alpha, dec, psi, &fp, &fc, &dt);
    const double s = (tc + dt - c.t_trig) * c.fs + (double)c.half_w;
    const double fl = floor(s);
    const double f = s - fl;
    if (!(fl >= 4.0 && fl <= (double)(T - 6))) {
      valid = false;
      break;
    }
    const int n0 = (int)fl;
    double w[kSplineTaps];
#pragma unroll
    for (int t = 0; t < kSplineTaps; ++t)
      w[t] = c.spline[t][0] + f * (c.spline[t][1] + f * (c.spline[t][2] + f * c.spline[t][3]));
    // A_{k,lm} = [(F+ + iFx) Y_{l,-m} + (-1)^l (F+ - iFx) conj(Y_{lm})] / 2
    double ar[RBFL_MAX_MODES], ai[RBFL_MAX_MODES];
    for (int a = 0; a < n_modes; ++a) {
      const double sg = (c.mode_l[a] & 1) ? -1.0 : 1.0;
      ar[a] = 0.5 * ((fp * yn_r[a] - fc * yn_i[a]) + sg * (fp * yp_r[a] - fc * yp_i[a]));
      ai[a] = 0.5 * ((fp * yn_i[a] + fc * yn_r[a]) + sg * (-fp * yp_i[a] - fc * yp_r[a]));
    }
    Comp zt;
    for (int a = 0; a < n_modes; ++a) {
      const int o = c.coef_off[k][a];
      const double2 *base = basis + ((int64_t)(k * n_modes + a) * T + (n0 - 4)) * q;
      double zr = 0.0, zi = 0.0;
      for (int i = lane; i < q; i += 64) {
        const double cr = y[o + 2 * i], ci = y[o + 2 * i + 1];
        double br = 0.0, bi = 0.0;
#pragma unroll
        for (int t = 0; t < kSplineTaps; ++t) {
          const double2 v = base[t * q + i];
          br = fma(w[t], v.x, br);
          bi = fma(w[t], v.y, bi);
        }
        zr += cr * br - ci * bi;
        zi += cr * bi + ci * br;
      }
      zr = wave_sum(zr);
      zi = wave_sum(zi);
      zt.add(ar[a] * zr + ai[a] * zi);   // Re(conj(A) z)
    }
    // sigma term: sum_a |A_a|^2 s_aa + 2 sum_{a<b} Re(conj(A_a) A_b s_ab)
    const int so = c.sig_off[k];
    Comp st;
    for (int a = 0; a < n_modes; ++a) st.add((ar[a] * ar[a] + ai[a] * ai[a]) * y[so + a]);
    int pidx = so + n_modes;
    for (int a = 0; a < n_modes; ++a) {
      for (int bb = a + 1; bb < n_modes; ++bb) {
        const double sr = y[pidx], si = y[pidx + 1];
        pidx += 2;
        // conj(A_a) A_b = (ar_a ar_b + ai_a ai_b) + i (ar_a ai_b - ai_a ar_b)
        const double pr = ar[a] * ar[bb] + ai[a] * ai[bb];
        const double pi = ar[a] * ai[bb] - ai[a] * ar[bb];
        st.add(2.0 * (pr * sr - pi * si));
      }
    }
    total.add(rr * zt.value());
    total.add(-0.5 * rr * rr * st.value());
  }
  if (lane == 0) lnl[g] = valid ? total.value() : -__builtin_huge_val();
}

__global__ void k_convert_weights(const double *__restrict__ W, size_t n, float *__restrict__ hi,
                                  float *__restrict__ lo, uint16_t *__restrict__ b16) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double v = W[e];
  const float h = (float)v;
  if (hi) hi[e] = h;
  if (lo) lo[e] = (float)(v - (double)h);
  if (b16) {
    // round to nearest even on the upper 16 bits of the FP32 value
    uint32_t u = __float_as_uint((float)v);
    const uint32_t r = ((u >> 16) & 1u) + 0x7fffu;
    b16[e] = (uint16_t)((u + r) >> 16);
  }
}

}  // namespace

void launch_contract_fp64(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                          int64_t nb, const double *nodes, const double *W, double *Y, hipStream_t s) {
  constexpr int RT = 2, CT = 4;
  static_assert(CT * 16 == kColTile, "column tile");
  const int64_t qt = kWaves * RT * 16;
  dim3 grid((unsigned)((nb + qt - 1) / qt), (unsigned)(hc.Kp / (CT * 16)));
  hipLaunchKernelGGL((k_contract_fp64<RT, CT>), grid, dim3(kThreads), 0, s, c, params, ld, b0, nb, nodes, W, Y);
  RBFL_HIP(hipGetLastError());
}

void launch_contract_fp32(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                          int64_t nb, const double *nodes, const float *W, const float *Wlo, int split, double *Y,
                          hipStream_t s) {
  constexpr int RT = 2, CT = 4;
  const int64_t qt = kWaves * RT * 16;
  dim3 grid((unsigned)((nb + qt - 1) / qt), (unsigned)(hc.Kp / (CT * 16)));
  hipLaunchKernelGGL((k_contract_fp32<RT, CT>), grid, dim3(kThreads), 0, s, c, params, ld, b0, nb, nodes, W, Wlo,
                     split, Y);
  RBFL_HIP(hipGetLastError());
}

void launch_contract_bf16(const EvalConsts *, const EvalConsts &, const double *, int64_t, int64_t, int64_t,
                          const double *, const uint16_t *, double *, hipStream_t) {
  throw Error(RBFL_E_UNSUPPORTED, "the BF16 form is not available in this build");
}

void launch_epilogue(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                     int64_t nb, const double *Y, const double2 *basis, double *lnl, hipStream_t s) {
  (void)hc;
  dim3 grid((unsigned)((nb + kWaves - 1) / kWaves));
  hipLaunchKernelGGL(k_epilogue, grid, dim3(kThreads), 0, s, c, params, ld, b0, nb, Y, basis, lnl);
  RBFL_HIP(hipGetLastError());
}

void launch_convert_weights(const double *W, size_t n, float *hi, float *lo, uint16_t *b16, hipStream_t s) {
  hipLaunchKernelGGL(k_convert_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, n, hi, lo, b16);
  RBFL_HIP(hipGetLastError());
}

}  // namespace rbfl
