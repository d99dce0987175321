// Start-up stage kernels (Sec. II C): templates at the nodes, mode overlaps,
// windowed DFT for the overlap time series, SVD post-processing and the RBF
// system assembly.  All FP64.
#include <algorithm>

#include "rbfl_internal.h"

namespace rbfl {

namespace {

constexpr int kBlock = 256;

inline unsigned grid1(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

typedef double d4 __attribute__((ext_vector_type(4)));

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
// conj(h_a) h_b = A_a conj(A_b).  One block of 1024 threads per (node,
// detector), NM modes known at compile time so that the NM (NM + 1) / 2
// running sums stay in registers; each wave adds its lanes' sums in a fixed
// shuffle tree and the block adds its waves' in order (deterministic).  The
// detector's results go to sig[k * det_stride + node_base + node].
constexpr int kSigmaThreads = 1024;

template <int NM>
__global__ void __launch_bounds__(kSigmaThreads) k_sigma(const double2 *__restrict__ A, int nb, int J, int j0,
                                                         int j1, const double *__restrict__ wk, int64_t det_stride,
                                                         int node_base, double2 *__restrict__ sig) {
  constexpr int NP = NM * (NM + 1) / 2;
  constexpr int NW = kSigmaThreads / 64;
  const int i = blockIdx.x;
  const int k = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double2 acc[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = make_double2(0.0, 0.0);
  const double *w = wk + (int64_t)k * J;
  for (int jj = j0 + threadIdx.x; jj < j1; jj += kSigmaThreads) {
    double2 h[NM];
#pragma unroll
    for (int a = 0; a < NM; ++a) h[a] = A[((int64_t)a * nb + i) * J + jj];
    const double ww = w[jj];
    int p = 0;
#pragma unroll
    for (int a = 0; a < NM; ++a)
#pragma unroll
      for (int b = a; b < NM; ++b, ++p) {
        // A_a * conj(A_b)
        acc[p].x += (h[a].x * h[b].x + h[a].y * h[b].y) * ww;
        acc[p].y += (h[a].y * h[b].x - h[a].x * h[b].y) * ww;
      }
  }
  __shared__ double2 red[NW][NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    double2 v = acc[p];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      v.x += __shfl_xor(v.x, m, 64);
      v.y += __shfl_xor(v.y, m, 64);
    }
    if (lane == 0) red[wave][p] = v;
  }
  __syncthreads();
  if (threadIdx.x < NP) {
    const int p = threadIdx.x;
    double2 v = red[0][p];
    for (int wv = 1; wv < NW; ++wv) {
      v.x += red[wv][p].x;
      v.y += red[wv][p].y;
    }
    int a = 0, r = p;
    while (r >= NM - a) {   // pair p = (a, b) in the order a <= b, a slowest
      r -= NM - a;
      ++a;
    }
    const int bm = a + r;
    double2 *out = sig + ((int64_t)k * det_stride + node_base + i) * NM * NM;
    out[a * NM + bm] = v;
    out[bm * NM + a] = make_double2(v.x, -v.y);
  }
}

// Windowed DFT on the FP64 matrix cores:
//   partial[s][i][t] = sum_{jj in split s} A[i][jj] B[jj][t],
//   B[jj][t] = Dk[jj] e^{2 pi i (j_lo + jj) t / n_s},
// where Dk already carries 4 df d_k / S_k and the phase of the window start.
// The complex product is taken as a real one, A'[i][2jj + r] B'[2jj + r][2t + u]:
// A' is A's own memory read as doubles (interleaved re, im) and each complex
// B entry becomes the 2 x 2 real block (Re, Im; -Im, Re), so a real output
// row is the interleaved complex partial row.  Tile: 128 nodes x 128 real
// columns (64 taps) per workgroup of 8 waves, 4 along the nodes x 2 along
// the columns, each wave 32 x 64 from 2 x 4 v_mfma_f64_16x16x4f64 blocks
// (lane l holds A'[l%16][l/16], B'[l/16][l%16]; accumulator element i is
// row l/16 + 4i, column l%16 of its block; at most 128 registers, so two
// workgroups share a CU).  Per step 8 bins (16 real k) go
// through LDS, A' loaded one step ahead; B' is formed in the step, one
// sincospi per (bin, tap) with the phase (j t) mod n_s reduced exactly in
// integers.
constexpr int kDftNodes = 128, kDftTaps = 64, kDftBins = 8, kDftThreads = 512;

__global__ void __launch_bounds__(kDftThreads, 4) k_window_dft(const double2 *__restrict__ A, int nb, int J_mode,
                                                            int J_stride, const double2 *__restrict__ Dk,
                                                            int64_t j_lo, int64_t n_s, int T, int split_len,
                                                            double2 *__restrict__ partial) {
  constexpr int QT = kDftNodes, CW = 2 * kDftTaps, KC = 2 * kDftBins, RT = 2, CT = 4;
  __shared__ double As[KC][QT];
  __shared__ double Bs[KC][CW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave & 3, wc = wave >> 2;
  const int kk = lane >> 4, ll = lane & 15;
  const int node0 = blockIdx.x * QT, tap0 = blockIdx.y * kDftTaps;
  const int split = blockIdx.z;
  const int jb = split * split_len;
  const int je = min(J_mode, jb + split_len);
  d4 acc[RT][CT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < CT; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};
  const double inv_ns2 = 2.0 / (double)n_s;
  // A': QT nodes x 8 bins per step, two entries per thread (bins of one
  // node), loaded one step ahead into registers
  constexpr int LA = QT * kDftBins / kDftThreads;
  double2 ra[LA];
  auto load_a = [&](int j0) {
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int e = tid + u * kDftThreads;
      const int node = node0 + e / kDftBins, jj = j0 + e % kDftBins;
      ra[u] = (node < nb && jj < je) ? A[(int64_t)node * J_stride + jj] : make_double2(0.0, 0.0);
    }
  };
  auto stash = [&](int j0) {
    // keeps the compiler from hoisting these LDS writes (and the wait for
    // their global loads) above the previous step's MFMAs
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int e = tid + u * kDftThreads;
      const int n = e / kDftBins, bb = e % kDftBins;
      As[2 * bb][n] = ra[u].x;
      As[2 * bb + 1][n] = ra[u].y;
    }
    // B': 8 bins x 64 taps, one per thread
    const int bb = tid / kDftTaps, t = tid % kDftTaps;
    const int jj = j0 + bb, tap = tap0 + t;
    double br = 0.0, bi = 0.0;
    if (jj < je && tap < T) {
      const int64_t j = j_lo + jj;
      const int64_t ph = (j * (int64_t)tap) % n_s;
      double sn, cs;
      sincospi((double)ph * inv_ns2, &sn, &cs);
      const double2 d = Dk[jj];
      br = d.x * cs - d.y * sn;
      bi = d.x * sn + d.y * cs;
    }
    Bs[2 * bb][2 * t] = br;
    Bs[2 * bb][2 * t + 1] = bi;
    Bs[2 * bb + 1][2 * t] = -bi;
    Bs[2 * bb + 1][2 * t + 1] = br;
  };
  if (jb < je) load_a(jb);
  for (int j0 = jb; j0 < je; j0 += kDftBins) {
    stash(j0);
    __syncthreads();
    if (j0 + kDftBins < je) load_a(j0 + kDftBins);
#pragma unroll
    for (int st = 0; st < KC / 4; ++st) {
      const int k = 4 * st + kk;
      double a[RT], b[CT];
#pragma unroll
      for (int t = 0; t < RT; ++t) a[t] = As[k][wq * RT * 16 + 16 * t + ll];
#pragma unroll
      for (int u = 0; u < CT; ++u) b[u] = Bs[k][wc * CT * 16 + 16 * u + ll];
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < CT; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
    }
    __syncthreads();
  }
  double *out = reinterpret_cast<double *>(partial);
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int node = node0 + wq * RT * 16 + 16 * t + kk + 4 * i;
      if (node >= nb) continue;
#pragma unroll
      for (int u = 0; u < CT; ++u) {
        const int col = wc * CT * 16 + 16 * u + ll;     // real column: tap col / 2, part col % 2
        const int tap = tap0 + (col >> 1);
        if (tap < T) out[(((int64_t)split * nb + node) * T + tap) * 2 + (col & 1)] = acc[t][u][i];
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
  const dim3 grid(nb, n_det), block(kSigmaThreads);
  switch (n_modes) {
    case 1: hipLaunchKernelGGL(k_sigma<1>, grid, block, 0, s, A, nb, J, j0, j1, wk, det_stride, node_base, sig); break;
    case 2: hipLaunchKernelGGL(k_sigma<2>, grid, block, 0, s, A, nb, J, j0, j1, wk, det_stride, node_base, sig); break;
    case 3: hipLaunchKernelGGL(k_sigma<3>, grid, block, 0, s, A, nb, J, j0, j1, wk, det_stride, node_base, sig); break;
    case 4: hipLaunchKernelGGL(k_sigma<4>, grid, block, 0, s, A, nb, J, j0, j1, wk, det_stride, node_base, sig); break;
    case 5: hipLaunchKernelGGL(k_sigma<5>, grid, block, 0, s, A, nb, J, j0, j1, wk, det_stride, node_base, sig); break;
    default: throw Error(RBFL_E_INVALID_ARG, "mode overlaps: 1 .. 5 modes");
  }
  RBFL_HIP(hipGetLastError());
}

int window_dft_splits(int nb, int T, int64_t len) {
  // as many splits of the bin range as keep the workgroups within one round
  // of the GPU (two 8-wave workgroups per CU, 512 in all: a partly filled
  // second round would leave most CUs idle for its length), and no split
  // shorter than 256 bins
  const int64_t tiles = (int64_t)grid1(nb, kDftNodes) * grid1(T, kDftTaps);
  return (int)std::max<int64_t>(1, std::min<int64_t>(512 / tiles, (len + 255) / 256));
}

void launch_window_dft(const double2 *A_mode, int nb, int J_mode, int J_stride, const double2 *Dk, int64_t j_lo,
                       int64_t n_s, int T, int n_split, double2 *partial, hipStream_t s) {
  int split_len = (J_mode + n_split - 1) / n_split;
  split_len = ((split_len + kDftBins - 1) / kDftBins) * kDftBins;
  dim3 grid(grid1(nb, kDftNodes), grid1(T, kDftTaps), n_split);
  hipLaunchKernelGGL(k_window_dft, grid, dim3(kDftThreads), 0, s, A_mode, nb, J_mode, J_stride, Dk, j_lo, n_s, T,
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
