// Start-up stage kernels (Sec. II C): templates at the nodes, mode overlaps,
// windowed DFT for the overlap time series, SVD post-processing and the RBF
// system assembly.  All FP64.
#include "rbfl_internal.h"

namespace rbfl {

namespace {

constexpr int kBlock = 256;

inline unsigned grid1(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// conj(h_{l,-m}(f_j)) for every node of a batch, every mode and bins
// j_lo .. j_lo + J - 1; zero outside the mode's band f < |m| F_isco.
__global__ void __launch_bounds__(kBlock) k_waveforms(const Binary *__restrict__ bins, int nb,
                                                      const int *__restrict__ mode_lm, int64_t j_lo, int J,
                                                      double df, double inv_dref_s, double2 *__restrict__ out) {
  const int jj = blockIdx.x * kBlock + threadIdx.x;
  const int i = blockIdx.y;
  const int a = blockIdx.z;
  if (jj >= J) return;
  const Binary b = bins[i];
  const int l = mode_lm[2 * a], m = mode_lm[2 * a + 1];
  const double f = (double)(j_lo + jj) * df;
  double2 v = make_double2(0.0, 0.0);
  if (f < (double)m * b.f_isco) {
    const double ph = 0.5 * (double)m * phase22(2.0 * f / (double)m, b);
    const double amp = mode_amp(l, m, b.eta, b.delta) * b.amp * inv_dref_s * exp(-7.0 / 6.0 * log(f));
    double sn, cs;
    sincos(ph, &sn, &cs);
    v = make_double2(amp * cs, amp * sn);   // conj(amp e^{-i ph})
  }
  out[((int64_t)a * nb + i) * J + jj] = v;
}

// sigma_k,ab = sum_j conj(h_a) h_b w_k(j) over bins j0 .. j1 - 1 of the
// band (all of it, or one time band), w_k = 4 df / S_k.  A holds conj(h), so
// conj(h_a) h_b = A_a conj(A_b).  One block per (node, detector); the
// detector's results go to sig[k * det_stride + node_base + node]; fixed-order
// tree reduction (deterministic).
__global__ void __launch_bounds__(kBlock) k_sigma(const double2 *__restrict__ A, int nb, int n_modes, int J,
                                                  int j0, int j1, const double *__restrict__ wk,
                                                  int64_t det_stride, int node_base, double2 *__restrict__ sig) {
  const int i = blockIdx.x;
  const int k = blockIdx.y;
  const int npair = n_modes * (n_modes + 1) / 2;
  double2 acc[15];
  for (int p = 0; p < 15; ++p) acc[p] = make_double2(0.0, 0.0);
  const double *w = wk + (int64_t)k * J;
  for (int jj = j0 + threadIdx.x; jj < j1; jj += kBlock) {
    double2 h[RBFL_MAX_MODES];
    for (int a = 0; a < n_modes; ++a) h[a] = A[((int64_t)a * nb + i) * J + jj];
    const double ww = w[jj];
    int p = 0;
    for (int a = 0; a < n_modes; ++a) {
      for (int b = a; b < n_modes; ++b, ++p) {
        // A_a * conj(A_b)
        acc[p].x += (h[a].x * h[b].x + h[a].y * h[b].y) * ww;
        acc[p].y += (h[a].y * h[b].x - h[a].x * h[b].y) * ww;
      }
    }
  }
  __shared__ double2 red[kBlock];
  double2 *out = sig + ((int64_t)k * det_stride + node_base + i) * n_modes * n_modes;
  int p = 0;
  for (int a = 0; a < n_modes; ++a) {
    for (int b = a; b < n_modes; ++b, ++p) {
      red[threadIdx.x] = acc[p];
      __syncthreads();
      for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
          red[threadIdx.x].x += red[threadIdx.x + s].x;
          red[threadIdx.x].y += red[threadIdx.x + s].y;
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        const double2 v = red[0];
        out[a * n_modes + b] = v;
        out[b * n_modes + a] = make_double2(v.x, -v.y);
      }
      __syncthreads();
    }
  }
  (void)npair;
}

// Windowed DFT: partial[s][i][t] = sum_{jj in split s} A[i][jj] Dk[jj] e^{2 pi i (j_lo+jj) t / n_s},
// where Dk already carries 4 df d_k / S_k and the phase of the window start.
// Tile: 64 nodes x 64 taps per block, 16 bins per step; thread (ty, tx)
// owns nodes ty + 16u and taps tx + 16v (u, v < 4).
constexpr int kDftTile = 64;
constexpr int kDftStep = 16;

__global__ void __launch_bounds__(kBlock) k_window_dft(const double2 *__restrict__ A, int nb, int J_mode,
                                                       int J_stride, const double2 *__restrict__ Dk,
                                                       int64_t j_lo, int64_t n_s, int T, int split_len,
                                                       double2 *__restrict__ partial) {
  __shared__ double2 As[kDftTile][kDftStep + 1];
  __shared__ double2 Bs[kDftStep][kDftTile];
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const int node0 = blockIdx.x * kDftTile;
  const int tap0 = blockIdx.y * kDftTile;
  const int split = blockIdx.z;
  const int jb = split * split_len;
  const int je = min(J_mode, jb + split_len);
  double2 acc[4][4];
  for (int u = 0; u < 4; ++u)
    for (int v = 0; v < 4; ++v) acc[u][v] = make_double2(0.0, 0.0);
  const double inv_ns2 = 2.0 / (double)n_s;
  for (int j0 = jb; j0 < je; j0 += kDftStep) {
    for (int e = tid; e < kDftTile * kDftStep; e += kBlock) {
      const int n = e / kDftStep, bb = e % kDftStep;
      const int node = node0 + n, jj = j0 + bb;
      As[n][bb] = (node < nb && jj < je) ? A[(int64_t)node * J_stride + jj] : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < kDftTile * kDftStep; e += kBlock) {
      const int bb = e / kDftTile, t = e % kDftTile;
      const int jj = j0 + bb, tap = tap0 + t;
      double2 v = make_double2(0.0, 0.0);
      if (jj < je && tap < T) {
        const int64_t j = j_lo + jj;
        const int64_t ph = (j * (int64_t)tap) % n_s;
        double sn, cs;
        sincospi((double)ph * inv_ns2, &sn, &cs);
        const double2 d = Dk[jj];
        v = make_double2(d.x * cs - d.y * sn, d.x * sn + d.y * cs);
      }
      Bs[bb][t] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int bb = 0; bb < kDftStep; ++bb) {
      double2 a[4], b[4];
      for (int u = 0; u < 4; ++u) a[u] = As[ty + 16 * u][bb];
      for (int v = 0; v < 4; ++v) b[v] = Bs[bb][tx + 16 * v];
      for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
          acc[u][v].x = fma(a[u].x, b[v].x, fma(-a[u].y, b[v].y, acc[u][v].x));
          acc[u][v].y = fma(a[u].x, b[v].y, fma(a[u].y, b[v].x, acc[u][v].y));
        }
    }
    __syncthreads();
  }
  for (int u = 0; u < 4; ++u) {
    const int node = node0 + ty + 16 * u;
    if (node >= nb) continue;
    for (int v = 0; v < 4; ++v) {
      const int tap = tap0 + tx + 16 * v;
      if (tap < T) partial[((int64_t)split * nb + node) * T + tap] = acc[u][v];
    }
  }
}

__global__ void k_reduce_splits(const double2 *__restrict__ partial, int n_split, int64_t count,
                                double2 *__restrict__ Z) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= count) return;
  double2 s = make_double2(0.0, 0.0);
  for (int p = 0; p < n_split; ++p) {
    const double2 v = partial[(int64_t)p * count + e];
    s.x += v.x;
    s.y += v.y;
  }
  Z[e] = s;
}

// B[t][i] = U[t][i] conj(U[t*][i]) / |U[t*][i]|, t* the first index of the
// largest |U[t][i]|: the basis column rotated so that entry t* is real
// positive.  One block per column.
__global__ void __launch_bounds__(kBlock) k_basis_from_u(const double2 *__restrict__ U, int T, int ldu, int q,
                                                         double2 *__restrict__ B) {
  const int i = blockIdx.x;
  const double2 *col = U + (int64_t)i * ldu;
  double best = -1.0;
  int arg = 0;
  for (int t = threadIdx.x; t < T; t += kBlock) {
    const double m = col[t].x * col[t].x + col[t].y * col[t].y;
    if (m > best) {
      best = m;
      arg = t;
    }
  }
  __shared__ double sb[kBlock];
  __shared__ int sa[kBlock];
  sb[threadIdx.x] = best;
  sa[threadIdx.x] = arg;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double ob = sb[threadIdx.x + s];
      const int oa = sa[threadIdx.x + s];
      if (ob > sb[threadIdx.x] || (ob == sb[threadIdx.x] && oa < sa[threadIdx.x])) {
        sb[threadIdx.x] = ob;
        sa[threadIdx.x] = oa;
      }
    }
    __syncthreads();
  }
  const double2 u = col[sa[0]];
  const double mag = sqrt(u.x * u.x + u.y * u.y);
  const double2 ph = make_double2(u.x / mag, -u.y / mag);
  for (int t = threadIdx.x; t < T; t += kBlock) {
    const double2 v = col[t];
    B[(int64_t)t * q + i] = make_double2(v.x * ph.x - v.y * ph.y, v.x * ph.y + v.y * ph.x);
  }
}

// C[n][i] = sum_t Z[n][t] conj(B[t][i]).
__global__ void k_coeffs(const double2 *__restrict__ Z, const double2 *__restrict__ B, int N, int T, int q,
                         double2 *__restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)N * q) return;
  const int n = (int)(e / q), i = (int)(e % q);
  double sx = 0.0, sy = 0.0;
  for (int t = 0; t < T; ++t) {
    const double2 z = Z[(int64_t)n * T + t];
    const double2 b = B[(int64_t)t * q + i];
    sx += z.x * b.x + z.y * b.y;
    sy += z.y * b.x - z.x * b.y;
  }
  C[e] = make_double2(sx, sy);
}

// Right-hand side, column-major [K][NM]: column c described by coldesc[c] =
// (kind, k, a, i): kind 0 = Re C_{k,a,i}, 1 = Im C_{k,a,i}, 2 = Re sigma_k,ai,
// 3 = Im sigma_k,ai.  Rows >= N (polynomial side conditions) stay zero.
__global__ void k_assemble_rhs(const double2 *__restrict__ C, const double2 *__restrict__ sig,
                               const int4 *__restrict__ coldesc, int N, int K, int NM, int q, int n_modes,
                               int n_det, double *__restrict__ R) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)K * NM) return;
  const int c = (int)(e / NM), n = (int)(e % NM);
  double v = 0.0;
  if (n < N) {
    const int4 d = coldesc[c];
    if (d.x <= 1) {
      const double2 cv = C[(((int64_t)d.y * n_modes + d.z) * N + n) * q + d.w];
      v = d.x == 0 ? cv.x : cv.y;
    } else {
      const double2 sv = sig[((int64_t)d.y * N + n) * n_modes * n_modes + d.z * n_modes + d.w];
      v = d.x == 2 ? sv.x : sv.y;
    }
  }
  R[e] = v;
  (void)n_det;
}

// Saddle-point system [[Phi, P], [P^T, 0]] (symmetric, so row- and
// column-major agree): Phi_ij = exp(-eps^2 |x_i - x_j|^2), P_ij = p_j(x_i).
__global__ void k_assemble_system(const double *__restrict__ x, int N, int M, const int *__restrict__ poly_idx,
                                  double eps2, double *__restrict__ A) {
  const int NM = N + M;
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)NM * NM) return;
  const int i = (int)(e / NM), j = (int)(e % NM);
  double v = 0.0;
  if (i < N && j < N) {
    double d2 = 0.0;
    for (int d = 0; d < 4; ++d) {
      const double t = x[4 * i + d] - x[4 * j + d];
      d2 += t * t;
    }
    v = exp(-eps2 * d2);
  } else if (i < N || j < N) {
    const int node = i < N ? i : j;
    const int p = (i < N ? j : i) - N;
    v = 1.0;
    for (int s = 0; s < 3; ++s) {
      const int id = poly_idx[3 * p + s];
      if (id >= 0) v *= x[4 * node + id];
    }
  }
  A[e] = v;
}

// W[r][c] = R[c][r] for r < NM, c < K; zero padding elsewhere.
__global__ void k_transpose_weights(const double *__restrict__ R, int NM, int K, int rows, int Kp,
                                    double *__restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)rows * Kp) return;
  const int r = (int)(e / Kp), c = (int)(e % Kp);
  W[e] = (r < NM && c < K) ? R[(int64_t)c * NM + r] : 0.0;
}

// res[c][i] = rhs[c][i] - sum_j A[i][j] W[c][j] (column-major, A symmetric)
// accumulated in double-double: each product split exactly with an FMA
// (p + e = a w), each sum with the branch-free two-sum, rounded once at the
// end.  Used for iterative refinement of the RBF solve.
__global__ void k_residual_dd(const double *__restrict__ A, const double *__restrict__ rhs,
                              const double *__restrict__ W, int NM, double *__restrict__ res) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= NM) return;
  const double *w = W + (int64_t)c * NM;
  double hi = rhs[(int64_t)c * NM + i], lo = 0.0;
  for (int j = 0; j < NM; ++j) {
    const double a = A[(int64_t)j * NM + i];
    const double p = -a * w[j];
    const double e = fma(-a, w[j], -p);
    const double t = hi + p;
    const double bp = t - hi;
    lo += ((hi - (t - bp)) + (p - bp)) + e;
    hi = t;
  }
  res[(int64_t)c * NM + i] = hi + lo;
}

__global__ void k_add(double *__restrict__ y, const double *__restrict__ x, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n) y[e] += x[e];
}

}  // namespace

void launch_residual_dd(const double *A, const double *rhs, const double *W, int NM, int K, double *res,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_residual_dd, dim3(grid1(NM, kBlock), K), dim3(kBlock), 0, s, A, rhs, W, NM, res);
  RBFL_HIP(hipGetLastError());
}

void launch_add(double *y, const double *x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_add, dim3(grid1(n, kBlock)), dim3(kBlock), 0, s, y, x, n);
  RBFL_HIP(hipGetLastError());
}

void launch_waveforms(const Binary *bins, int nb, const int *mode_lm, int n_modes, int64_t j_lo, int J,
                      double df, double inv_dref_s, double2 *out, hipStream_t s) {
  dim3 grid(grid1(J, kBlock), nb, n_modes);
  hipLaunchKernelGGL(k_waveforms, grid, dim3(kBlock), 0, s, bins, nb, mode_lm, j_lo, J, df, inv_dref_s, out);
  RBFL_HIP(hipGetLastError());
}

void launch_sigma(const double2 *A, int nb, int n_modes, int J, int j0, int j1, const double *wk, int n_det,
                  int64_t det_stride, int node_base, double2 *sig, hipStream_t s) {
  hipLaunchKernelGGL(k_sigma, dim3(nb, n_det), dim3(kBlock), 0, s, A, nb, n_modes, J, j0, j1, wk, det_stride,
                     node_base, sig);
  RBFL_HIP(hipGetLastError());
}

void launch_window_dft(const double2 *A_mode, int nb, int J_mode, int J_stride, const double2 *Dk, int64_t j_lo,
                       int64_t n_s, int T, int n_split, double2 *partial, hipStream_t s) {
  int split_len = (J_mode + n_split - 1) / n_split;
  split_len = ((split_len + kDftStep - 1) / kDftStep) * kDftStep;
  dim3 grid(grid1(nb, kDftTile), grid1(T, kDftTile), n_split);
  hipLaunchKernelGGL(k_window_dft, grid, dim3(kBlock), 0, s, A_mode, nb, J_mode, J_stride, Dk, j_lo, n_s, T,
                     split_len, partial);
  RBFL_HIP(hipGetLastError());
}

void launch_reduce_splits(const double2 *partial, int n_split, int nb, int T, double2 *Z_rows, hipStream_t s) {
  const int64_t count = (int64_t)nb * T;
  hipLaunchKernelGGL(k_reduce_splits, dim3(grid1(count, kBlock)), dim3(kBlock), 0, s, partial, n_split, count,
                     Z_rows);
  RBFL_HIP(hipGetLastError());
}

// Spline-folded basis for the online reconstruction: with the not-a-knot
// weights w_t(f) = sum_p spline[t][p] f^p of the 10-sample stencil,
//   B4[pair][n][i][p] = sum_t spline[t][p] B[pair][n - 4 + t][i]
// for stencil bases 4 <= n <= T - 6 (zero elsewhere), so that the
// interpolated basis at n + f is sum_p f^p B4[pair][n][i][p].
__global__ void __launch_bounds__(kBlock) k_fold_spline(const double2 *__restrict__ B, int n_pairs, int T, int q,
                                                        const EvalConsts *__restrict__ c, double2 *__restrict__ B4) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)n_pairs * T * q) return;
  const int i = (int)(e % q);
  const int n = (int)((e / q) % T);
  const int64_t pair = e / ((int64_t)q * T);
  double2 out[4] = {};
  if (n >= 4 && n <= T - 6) {
    for (int t = 0; t < kSplineTaps; ++t) {
      const double2 v = B[(pair * T + n - 4 + t) * q + i];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        out[p].x = fma(c->spline[t][p], v.x, out[p].x);
        out[p].y = fma(c->spline[t][p], v.y, out[p].y);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) B4[e * 4 + p] = out[p];
}

void launch_fold_spline(const double2 *B, int n_pairs, int T, int q, const EvalConsts *c, double2 *B4,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_fold_spline, dim3(grid1((int64_t)n_pairs * T * q, kBlock)), dim3(kBlock), 0, s, B, n_pairs,
                     T, q, c, B4);
  RBFL_HIP(hipGetLastError());
}

void launch_basis_from_u(const double2 *U, int T, int ldu, int q, double2 *B, hipStream_t s) {
  hipLaunchKernelGGL(k_basis_from_u, dim3(q), dim3(kBlock), 0, s, U, T, ldu, q, B);
  RBFL_HIP(hipGetLastError());
}

void launch_coeffs(const double2 *Z, const double2 *B, int N, int T, int q, double2 *C, hipStream_t s) {
  hipLaunchKernelGGL(k_coeffs, dim3(grid1((int64_t)N * q, kBlock)), dim3(kBlock), 0, s, Z, B, N, T, q, C);
  RBFL_HIP(hipGetLastError());
}

void launch_assemble_rhs(const double2 *C, const double2 *sig, const int4 *coldesc, int N, int K, int NM, int q,
                         int n_modes, double *R, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble_rhs, dim3(grid1((int64_t)K * NM, kBlock)), dim3(kBlock), 0, s, C, sig, coldesc, N,
                     K, NM, q, n_modes, 0, R);
  RBFL_HIP(hipGetLastError());
}

void launch_assemble_system(const double *x, int N, int M, const int *poly_idx, double eps2, double *A,
                            hipStream_t s) {
  const int64_t NM = N + M;
  hipLaunchKernelGGL(k_assemble_system, dim3(grid1(NM * NM, kBlock)), dim3(kBlock), 0, s, x, N, M, poly_idx, eps2,
                     A);
  RBFL_HIP(hipGetLastError());
}

void launch_transpose_weights(const double *R, int NM, int K, int rows, int Kp, double *W, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose_weights, dim3(grid1((int64_t)rows * Kp, kBlock)), dim3(kBlock), 0, s, R, NM, K,
                     rows, Kp, W);
  RBFL_HIP(hipGetLastError());
}

// ---- exact outputs at arbitrary proposals -----------------------------------
// The start-up kernels above applied to proposals instead of nodes give the
// quantities the interpolants approximate, at the proposal itself: the window
// samples of z, their coefficients on the time basis and the overlaps.

namespace {

// Physical point of each proposal of a batch; an unphysical or NaN proposal
// gets f_isco = 0, so its templates vanish (its ln L is decided by the
// online stage's own domain test).
__global__ void __launch_bounds__(kBlock) k_proposal_bins(const EvalConsts *__restrict__ cp,
                                                          const double *__restrict__ params, int64_t ld, int64_t b0,
                                                          int nb, Binary *__restrict__ bins) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nb) return;
  const EvalConsts &c = *cp;
  double th[4], phys[4];
  bool ok = true;
  for (int r = 0; r < 4; ++r) {
    double t = c.theta_c[r];
    for (int j = 0; j < 4; ++j) t += c.V[4 * r + j] * params[j * ld + b0 + i];
    th[r] = t;
    ok = ok && !isnan(t);
  }
  ok = ok && theta_to_phys(th, c.f0, c.chi_max, phys);
  Binary b = make_binary(ok ? phys[0] : 2.0, ok ? phys[1] : 1.0, ok ? phys[2] : 0.0, ok ? phys[3] : 0.0, c.f_ref);
  if (!ok) b.f_isco = 0.0;
  bins[i] = b;
}

// Band data with the phase of the window's first sample n0 folded in:
// out[k][jj] = D[k][jj] e^{2 pi i j n0 / n_s}, j = j_lo + jj (the product
// j n0 is reduced exactly in integers).
__global__ void k_rotate_band(const double2 *__restrict__ D, int64_t total, int64_t J, int64_t j_lo, int64_t n0,
                              int64_t n_s, double2 *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= total) return;
  const int64_t j = j_lo + e % J;
  const int64_t ph = ((j % n_s) * n0) % n_s;
  double sn, cs;
  sincospi(2.0 * ((double)ph / (double)n_s), &sn, &cs);
  const double2 d = D[e];
  out[e] = make_double2(d.x * cs - d.y * sn, d.x * sn + d.y * cs);
}

// Output rows Y[n][Kp] of a batch in the interpolants' column layout
// (coldesc as for the right-hand side) from coefficients
// C[n_det][n_modes][nb][q] and overlaps sig[n_det][nb][n_modes][n_modes];
// padding columns are zero.
__global__ void k_outputs_rows(const double2 *__restrict__ C, const double2 *__restrict__ sig,
                               const int4 *__restrict__ coldesc, int nb, int K, int Kp, int q, int n_modes,
                               double *__restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (int64_t)nb * Kp) return;
  const int n = (int)(e / Kp), col = (int)(e % Kp);
  double v = 0.0;
  if (col < K) {
    const int4 d = coldesc[col];
    if (d.x <= 1) {
      const double2 cv = C[(((int64_t)d.y * n_modes + d.z) * nb + n) * q + d.w];
      v = d.x == 0 ? cv.x : cv.y;
    } else {
      const double2 sv = sig[(((int64_t)d.y * nb + n) * n_modes + d.z) * n_modes + d.w];
      v = d.x == 2 ? sv.x : sv.y;
    }
  }
  Y[e] = v;
}

}  // namespace

void launch_proposal_bins(const EvalConsts *c, const double *params, int64_t ld, int64_t b0, int nb, Binary *bins,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_proposal_bins, dim3(grid1(nb, kBlock)), dim3(kBlock), 0, s, c, params, ld, b0, nb, bins);
  RBFL_HIP(hipGetLastError());
}

void launch_rotate_band(const double2 *D, int n_det, int64_t J, int64_t j_lo, int64_t n0, int64_t n_s,
                        double2 *out, hipStream_t s) {
  const int64_t total = (int64_t)n_det * J;
  hipLaunchKernelGGL(k_rotate_band, dim3(grid1(total, kBlock)), dim3(kBlock), 0, s, D, total, J, j_lo, n0, n_s, out);
  RBFL_HIP(hipGetLastError());
}

void launch_outputs_rows(const double2 *C, const double2 *sig, const int4 *coldesc, int nb, int K, int Kp, int q,
                         int n_modes, double *Y, hipStream_t s) {
  hipLaunchKernelGGL(k_outputs_rows, dim3(grid1((int64_t)nb * Kp, kBlock)), dim3(kBlock), 0, s, C, sig, coldesc, nb,
                     K, Kp, q, n_modes, Y);
  RBFL_HIP(hipGetLastError());
}

}  // namespace rbfl
